// chi0_GG'(q, w) of Eq. (RPA) as a contraction over the transition index t.
//
// chi0_GG'(w) = pref * sum_t W_t(w) P_t(G, G'),  P_t(G, G') = R_t(G)^* R_t(G'),
// pref = 2/(N_k V), W_t(w) = 1/(s_t w - D_t + i eta) with s_t = +1, D_t = Delta
// for the resonant rows (v -> c) and s_t = -1, D_t = Delta' for the
// anti-resonant rows.
//
// Each P_t is Hermitian, so with W = Wr + i Wi
//     X(G,G') = sum_t Wr P_t(G,G'),  Y(G,G') = sum_t Wi P_t(G,G')
// over the upper triangle G <= G' gives chi0_GG' = pref (X + iY) and
// chi0_G'G = pref (X^* + i Y^*).  That is one real GEMM
//     C[row][col] = sum_t A[row][t] B[t][col]
// with rows (Re W(w_j), Im W(w_j)) and columns (Re P, Im P) per pair: half the
// multiply-adds of the plain complex product.  A is precomputed per q in the
// MFMA fragment order; B is formed on the fly from R in FP32 (and split into
// bf16 hi + lo for the split path) inside the kernel.
#include <algorithm>
#include <vector>

#include "common.h"

namespace qcx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int KSTEP = 16;

__global__ void k_trans_energy(const double* Ek, const double* Ekq, int n_k, int n_b, int n_occ,
                               double* dt) {
  const int n_c = n_b - n_occ;
  const int nres = n_k * n_occ * n_c;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nres) return;
  const int s = t / nres, r = t % nres;
  const int k = r / (n_occ * n_c), v = (r / n_c) % n_occ, c = r % n_c;
  double d;
  if (s == 0)
    d = Ekq[(size_t)k * n_b + n_occ + c] - Ek[(size_t)k * n_b + v];  // E_c(k+q) - E_v(k)
  else
    d = Ek[(size_t)k * n_b + n_occ + c] - Ekq[(size_t)k * n_b + v];  // E_c(k) - E_v(k+q)
  dt[t] = d / kHartreeEV;
}

// W_t(w_j) in FP64; zero for padded rows or transitions.
__device__ inline cplx weight(const double* w, const double* dt, double eta, int j, int t,
                              int n_w, int n_t) {
  if (j >= n_w || t >= n_t) return {0.0, 0.0};
  const double s = (t < n_t / 2) ? 1.0 : -1.0;
  const double x = s * w[j] - dt[t];
  const double den = 1.0 / (x * x + eta * eta);
  return {x * den, -eta * den};
}

// Fragment order for v_mfma_f32_32x32x2f32: per (row block rb, K step tb) 64
// lanes x 8 floats, element s of lane l = A[rb*32 + l%32][tb*16 + 2s + l/32].
__global__ void k_weights_f32(const double* w, const double* dt, double eta, Chi0Geom g,
                              float* Aw) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ntb = g.n_tp / KSTEP;
  const long total = (long)(g.n_rowsp / 32) * ntb * 64;
  if (i >= total) return;
  const int lane = (int)(i % 64);
  const long fr = i / 64;
  const int tb = (int)(fr % ntb), rb = (int)(fr / ntb);
  const int row = rb * 32 + lane % 32;
  const int j = row >> 1, ri = row & 1;
  float out[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int t = tb * KSTEP + 2 * s + lane / 32;
    const cplx wt = weight(w, dt, eta, j, t, g.n_w, g.n_t);
    out[s] = (float)(ri ? wt.im : wt.re);
  }
  float4* dst = reinterpret_cast<float4*>(Aw + i * 8);
  dst[0] = make_float4(out[0], out[1], out[2], out[3]);
  dst[1] = make_float4(out[4], out[5], out[6], out[7]);
}

__device__ inline uint16_t bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ inline float bf16_val(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// Fragment order for v_mfma_f32_32x32x16_bf16: lane l holds
// A[rb*32 + l%32][tb*16 + 8(l/32) + 0..7]; hi = bf16(x), lo = bf16(x - hi).
// The energy difference s w - D is formed in FP64 (it cancels near resonance),
// the reciprocal in FP32: its error (~1e-7 relative) is far below the 2^-16
// that hi + lo keep.
__global__ void k_weights_bf16(const double* w, const double* dt, double eta, Chi0Geom g,
                               uint16_t* Ahi, uint16_t* Alo) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ntb = g.n_tp / KSTEP;
  const long total = (long)(g.n_rowsp / 32) * ntb * 64;
  if (i >= total) return;
  const int lane = (int)(i % 64);
  const long fr = i / 64;
  const int tb = (int)(fr % ntb), rb = (int)(fr / ntb);
  const int row = rb * 32 + lane % 32;
  const int j = row >> 1, ri = row & 1;
  const bool live_row = j < g.n_w;
  const double wj = live_row ? w[j] : 0.0;
  const float ef = (float)eta;
  uint16_t hi[8], lo[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int t = tb * KSTEP + 8 * (lane / 32) + s;
    float x = 0.0f;
    if (live_row && t < g.n_t) {
      const double sg = (t < g.n_t / 2) ? 1.0 : -1.0;
      const float xf = (float)(sg * wj - dt[t]);
      const float r = 1.0f / (xf * xf + ef * ef);
      x = ri ? -ef * r : xf * r;
    }
    hi[s] = bf16_bits(x);
    lo[s] = bf16_bits(x - bf16_val(hi[s]));
  }
  uint4 h, l;
  h.x = hi[0] | ((uint32_t)hi[1] << 16); h.y = hi[2] | ((uint32_t)hi[3] << 16);
  h.z = hi[4] | ((uint32_t)hi[5] << 16); h.w = hi[6] | ((uint32_t)hi[7] << 16);
  l.x = lo[0] | ((uint32_t)lo[1] << 16); l.y = lo[2] | ((uint32_t)lo[3] << 16);
  l.z = lo[4] | ((uint32_t)lo[5] << 16); l.w = lo[6] | ((uint32_t)lo[7] << 16);
  reinterpret_cast<uint4*>(Ahi)[i] = h;
  reinterpret_cast<uint4*>(Alo)[i] = l;
}

// R32[tb][g][16] complex float.  perm = 1 stores t' = (t%2)*8 + t/2 inside the
// step so that a lane's eight K values of the 32x32x2 f32 MFMA are contiguous.
__global__ void k_pack_r32(const cplx* R, size_t ldt, int n_g, int n_tp, int perm, float* R32) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)n_g * n_tp;
  if (i >= total) return;
  const int t = (int)(i % n_tp), g = (int)(i / n_tp);
  const cplx v = R[(size_t)g * ldt + t];
  const int tb = t / KSTEP, ti = t % KSTEP;
  const int tp = perm ? ((ti & 1) * 8 + (ti >> 1)) : ti;
  float2* dst = reinterpret_cast<float2*>(R32);
  dst[((size_t)tb * n_g + g) * KSTEP + tp] = make_float2((float)v.re, (float)v.im);
}

// ---------------------------------------------------------------------------
// Bulk kernel.  Block = 4 waves; block tile = AF*32 rows x 128 pairs (each
// wave: all AF*32 rows and 32 pairs, i.e. two B fragments, Re P and Im P).
// Per K step (16 transitions) the block stages in LDS, double-buffered through
// registers: the R slab (all G x 16 transitions, complex float; rows padded to
// 144 bytes so that lanes reading consecutive G hit distinct banks) and the
// block's AF A fragments (2 KB each: bf16 hi and lo, or the f32 values).
// grid = (pair tiles, row tiles, K splits).
// ---------------------------------------------------------------------------
// Block scheduling across the 8 XCDs (each with its own L2): workgroup i is
// dispatched to XCD i % 8.  Blocks that share a K range (the same R slab and
// A fragments) are given ids on one XCD, so that their common operands are
// fetched from HBM once per XCD and then served from that XCD's L2.
// Returns (x, y, z) for a logical grid gx * gy * gz with gz % 8 == 0 and the
// z index (K split) kept on one XCD; other shapes map linearly.
struct Blk3 {
  int x, y, z;
};
__device__ inline Blk3 xcd_block(int gx, int gy, int gz) {
  const int id = blockIdx.x;
  if (gz % 8 != 0) return {id % gx, (id / gx) % gy, id / (gx * gy)};
  const int xcd = id & 7, local = id >> 3;
  const int per = gx * gy;
  const int z = xcd + 8 * (local / per);
  const int rem = local % per;
  return {rem % gx, rem / gx, z};
}

constexpr int SLAB_LD4 = 9;  // float4 per padded slab row (8 used)

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Copy one 1 KB chunk (64 lanes x 16 bytes) from global memory straight into
// LDS (gfx950 global_load_lds_dwordx4): lane l's float4 lands at dst + l.
__device__ inline void lds_dma16(const float4* src, float4* dst) {
  __builtin_amdgcn_global_load_lds((const void*)src, (lds_ptr_t)dst, 16, 0, 0);
}

// LDS of one pipeline stage of a bulk block: the R slab (RCH chunks of 1 KB:
// padded rows of 16 complex floats) and the A fragments (NAC chunks).  Each
// stage is its own __shared__ object, so the compiler can see that copies
// into one stage never alias the reads of another: a step issues the copies
// of a later step first and then reads its own stage without waiting.
template <int RCH, int NAC>
struct BulkStage {
  float4 r[RCH * 64];
  float4 a[NAC * 64];
};

// R chunks per wave (template bucket) for n_g slab rows; gather mode stages
// kGatherRows rows
inline int bulk_maxr(int n_g) {
  const int rows = n_g >= kGatherMinNg ? kGatherRows : n_g;
  const int rpw = ((rows * SLAB_LD4 + 63) / 64 + 3) / 4;
  return rpw <= 1 ? 1 : rpw <= 4 ? 4 : 5;
}

// One block tile of the bulk GEMM: pair tile bk.x, row tile bk.y, K split
// bk.z, staged through NST stages s0, s1 (, s2).  Step s issues the copies of
// step s + NST - 1 into the stage freed by step s - 1, then computes from its
// own stage; the end-of-step wait covers only the copies of step s + 1, so
// with NST = 3 the load latency hides behind two steps of MFMA work.
// Only the first NF of the tile's AF 32-row fragments take MFMAs (the others,
// wholly past an item's 2 n_w rows in a batch, keep zero accumulators); the
// copies into LDS do not depend on NF, so every wait counts the same copies.
template <bool BF16, int AF, int MAXR, int NST, bool GATHER, class L, int NF = AF>
__device__ __forceinline__ void bulk_tile(const float4* __restrict__ Ahi,
                                          const float4* __restrict__ Alo,
                                          const float4* __restrict__ R32,
                                          const int* __restrict__ pairs,
                                          const int* __restrict__ rows, const Chi0Geom& g,
                                          float* __restrict__ C, Blk3 bk, L& s0, L& s1, L& s2) {
  constexpr int NAC = 2 * AF;                 // A chunks per step (hi/lo or two f32 quads)
  constexpr int MAXA = (NAC + 3) / 4;         // A chunks per wave
  // the wave index is uniform across the wave: keep it (and everything
  // derived from it alone) in scalar registers
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntb = g.n_tp / KSTEP;
  const int steps = ntb / g.ksplit;
  const int tb0 = bk.z * steps;
  const int rb0 = (g.row_tile0 + bk.y) * AF;  // first 32-row fragment (weights)
  const int rc0 = bk.y * AF;                   // first fragment in the partial buffer
  const int b = bk.x * 128 + wave * 32 + (lane & 31);
  const int pk = pairs[b];
  const int G = pk & 0xffff, Gp = pk >> 16;
  const int nr4 = g.n_g * 8;                  // float4 of one slab in global memory
  // slab rows staged per step: all n_g, or the tile's own rows (gather mode;
  // G and G' above are then indices into the tile's row list)
  const int n_rows_st = GATHER ? kGatherRows : g.n_g;
  const int* trows = GATHER ? rows + (size_t)bk.x * kGatherRows : nullptr;

  // Per-lane source offset of this wave's R chunk i (K step added per step):
  // LDS slot 64c + lane = padded row / column; pad slots read a harmless
  // valid address and are never used.
  int r_off[MAXR];
#pragma unroll
  for (int i = 0; i < MAXR; ++i) {
    const int slot = 64 * (wave + 4 * i) + lane;
    const int row = slot / SLAB_LD4, col = slot - row * SLAB_LD4;
    const bool ok = row < n_rows_st && col < 8;
    r_off[i] = ok ? (GATHER ? trows[row] : row) * 8 + col : 0;
  }
  // A chunk of copy slot i: chunks beyond NAC repeat a real chunk (the same
  // bytes to the same LDS place), so that every wave issues the same number
  // of copies per step and every wait below is an exact compile-time count
  auto a_chunk = [&](int i) {
    const int c = wave + 4 * i;
    return c < NAC ? c : c - NAC;
  };
  const float4* a_src[MAXA];
#pragma unroll
  for (int i = 0; i < MAXA; ++i) {
    const int cc = a_chunk(i);
    const int f = cc >> 1, half = cc & 1;
    const size_t fr = (size_t)(rb0 + f) * ntb * 64 + lane;
    if constexpr (BF16)
      a_src[i] = (half ? Alo : Ahi) + fr;
    else
      a_src[i] = Ahi + fr * 2 + half;
  }
  constexpr int ASTEP = BF16 ? 64 : 128;  // float4 between K steps of one fragment
  // Copies of K step tb into stage d: MAXR + MAXA per wave, always.  R
  // chunks beyond the slab copy a valid row into the unused tail of the
  // stage's R buffer (RCH = 4 MAXR chunks).
  auto stage_r = [&](int tb, L& d) {
#pragma unroll
    for (int i = 0; i < MAXR; ++i)
      lds_dma16(R32 + (size_t)tb * nr4 + r_off[i], d.r + 64 * (wave + 4 * i));
  };
  auto stage_a = [&](int tb, L& d) {
#pragma unroll
    for (int i = 0; i < MAXA; ++i)
      lds_dma16(a_src[i] + (size_t)tb * ASTEP, d.a + 64 * a_chunk(i));
  };
  // RAHEAD (NST = 4): a stage holds the slab of the step after its weights
  auto stage = [&](int tb, L& d) {
    stage_r(NST == 4 ? min(tb + 1, tb0 + steps - 1) : tb, d);
    stage_a(tb, d);
  };
  constexpr int NCOPY = MAXR + MAXA;  // copies per wave per stage (vmcnt of one stage)
  // s_waitcnt with only the vector-memory counter limited (expcnt 7 and
  // lgkmcnt 15 mean "no wait" in the gfx9 encoding)
  constexpr int WAIT_ONE = (NCOPY & 15) | ((NCOPY >> 4) << 14) | (7 << 4) | (15 << 8);
  constexpr int WAIT_ALL = (7 << 4) | (15 << 8);
  const int tb_last = tb0 + steps - 1;

  f32x16 acc[AF][2];
#pragma unroll
  for (int f = 0; f < AF; ++f) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc[f][0][r] = 0.f;
      acc[f][1][r] = 0.f;
    }
  }

  // B operand of one K step: P_t(G, G') for this lane's pair and 8
  // transitions, from the slab held by `src` (FP32, or its bf16 hi/lo split)
  struct Bops {
    float pre[8], pim[8];
    bf16x8 rh, rl, ih, il;
  };
  auto formB = [&](const L& src, Bops& o) {
    const float4* rG = src.r + G * SLAB_LD4 + 4 * h;    // 8 complex = 4 float4
    const float4* rGp = src.r + Gp * SLAB_LD4 + 4 * h;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 xg = rG[i], yg = rGp[i];
      o.pre[2 * i] = xg.x * yg.x + xg.y * yg.y;
      o.pim[2 * i] = xg.x * yg.y - xg.y * yg.x;
      o.pre[2 * i + 1] = xg.z * yg.z + xg.w * yg.w;
      o.pim[2 * i + 1] = xg.z * yg.w - xg.w * yg.z;
    }
    if constexpr (BF16) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const __bf16 rh = (__bf16)o.pre[i];
        const __bf16 ih = (__bf16)o.pim[i];
        o.rh[i] = rh;
        o.ih[i] = ih;
        o.rl[i] = (__bf16)(o.pre[i] - (float)rh);
        o.il[i] = (__bf16)(o.pim[i] - (float)ih);
      }
    }
  };
  // the MFMAs of one K step: A fragments of `cur`, B operand given
  auto mfma = [&](const L& cur, const Bops& B) {
    const float4* As = cur.a;
    if constexpr (BF16) {
      // three sweeps over the 2*NF independent accumulators, so that no MFMA
      // waits on the one issued just before it
      bf16x8 ah[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) ah[f] = __builtin_bit_cast(bf16x8, As[f * 128 + lane]);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], B.rh, acc[f][0], 0, 0, 0);
        acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], B.ih, acc[f][1], 0, 0, 0);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], B.rl, acc[f][0], 0, 0, 0);
        acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], B.il, acc[f][1], 0, 0, 0);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const bf16x8 al = __builtin_bit_cast(bf16x8, As[f * 128 + 64 + lane]);
        acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, B.rh, acc[f][0], 0, 0, 0);
        acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, B.ih, acc[f][1], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const float4 a0 = As[f * 128 + lane], a1 = As[f * 128 + 64 + lane];
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], B.pre[s], acc[f][0], 0, 0, 0);
          acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], B.pim[s], acc[f][1], 0, 0, 0);
        }
      }
    }
  };
  auto compute = [&](const L& cur) {
    Bops B;
    formB(cur, B);
    mfma(cur, B);
  };

  // Workgroup barrier without the release fence of __syncthreads(): that
  // fence would drain every outstanding copy into LDS, including those of
  // step st + 2.  Each wave first waits for its own copies that the next
  // step reads; the memory clobber keeps the compiler from moving LDS
  // accesses across the barrier.
  auto barrier = [] { asm volatile("s_barrier" ::: "memory"); };
  auto one = [&](int st, const L& cur, L& nxt) {
    // copies of step st + NST - 1 (past the end of the tile: the last step
    // again, never read, so that the copy count stays uniform)
    stage(min(tb0 + st + NST - 1, tb_last), nxt);
    compute(cur);
    __builtin_amdgcn_sched_barrier(0);  // issue every MFMA of the step before waiting
    // this wave's copies of step st + 1 landed (with NST = 3 those of st + 2
    // may still be in flight); its LDS reads of `cur` completed
    __builtin_amdgcn_s_waitcnt(NST == 3 ? WAIT_ONE : WAIT_ALL);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    barrier();
  };

  // RAHEAD (NST = 4, three LDS stages): step st issues the weights of st + 2
  // and the slab of st + 3, forms the B operand of st + 1 from its own stage
  // and runs the MFMAs of st with the B operand formed one step earlier, so
  // the VALU work of the next step overlaps the matrix work of this one.
  Bops Bc;
  auto one4 = [&](int st, const L& cur, L& nxt) {
    stage(min(tb0 + st + 2, tb_last), nxt);
    Bops Bn;
    mfma(cur, Bc);
    if (st + 1 < steps) formB(cur, Bn);
    if (st + 1 < steps) Bc = Bn;
    // interleave: each MFMA followed by a few VALU and LDS-read instructions
    // of the next step's B operand
#pragma unroll
    for (int i = 0; i < 6 * AF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
      __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
    }
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(WAIT_ONE);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    barrier();
  };

  if constexpr (NST == 4) {
    stage_r(tb0, s2);                         // slab of the first step
    stage(tb0, s0);
    stage(min(tb0 + 1, tb_last), s1);
    __builtin_amdgcn_s_waitcnt(WAIT_ONE);     // all but the last stage landed
    barrier();
    formB(s2, Bc);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    barrier();                                // s2 is refilled by step 0
  } else {
    stage(tb0, s0);
    if constexpr (NST == 3) {
      stage(min(tb0 + 1, tb_last), s1);
      __builtin_amdgcn_s_waitcnt(WAIT_ONE);
    } else {
      __builtin_amdgcn_s_waitcnt(WAIT_ALL);
    }
    barrier();
  }
  constexpr int NB = NST == 4 ? 3 : NST;  // LDS stages
  for (int st = 0; st < steps; st += NB) {
    if constexpr (NST == 4) {
      one4(st, s0, s2);
      if (st + 1 < steps) one4(st + 1, s1, s0);
      if (st + 2 < steps) one4(st + 2, s2, s1);
    } else if constexpr (NST == 3) {
      one(st, s0, s2);
      if (st + 1 < steps) one(st + 1, s1, s0);
      if (st + 2 < steps) one(st + 2, s2, s1);
    } else {
      one(st, s0, s1);
      if (st + 1 < steps) one(st + 1, s1, s0);
    }
  }
  // the trailing copies must land before the LDS is reused or released
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

  // epilogue: C[((ks*c_rows + row)*2 + ri)*n_bulkp + b], row local to the chunk
#pragma unroll
  for (int f = 0; f < AF; ++f) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (rc0 + f) * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) {
        const size_t o = (((size_t)bk.z * g.c_rows + row) * 2 + ri) * g.n_bulkp + b;
        C[o] = acc[f][ri][r];
      }
    }
  }
}

template <bool BF16, int AF, int MAXR, int NST, bool GATHER>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_bulk(const float4* __restrict__ Ahi, const float4* __restrict__ Alo,
       const float4* __restrict__ R32, const int* __restrict__ pairs,
       const int* __restrict__ rows, Chi0Geom g, float* __restrict__ C) {
  using L = BulkStage<4 * MAXR, 2 * AF>;
  const Blk3 bk = xcd_block(g.n_bulkp / 128, g.c_rows / (32 * AF), g.ksplit);
  if constexpr (NST >= 3) {
    __shared__ L s0, s1, s2;
    bulk_tile<BF16, AF, MAXR, NST, GATHER>(Ahi, Alo, R32, pairs, rows, g, C, bk, s0, s1, s2);
  } else {
    __shared__ L s0, s1;
    bulk_tile<BF16, AF, MAXR, 2, GATHER>(Ahi, Alo, R32, pairs, rows, g, C, bk, s0, s1, s0);
  }
}

// Persistent form for a batch of uneven items: each block takes tiles from a
// global list (ordered by decreasing cost) with an atomic counter until the
// list is exhausted, so items with small N_G or few frequencies fill the gaps
// left by large ones in one launch.
template <bool BF16, int AF, int MAXR, bool GATHER>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_bulk_persistent(const BulkItem* __restrict__ items, const int4* __restrict__ tiles, int n_tiles,
                  int* counter) {
  using L = BulkStage<4 * MAXR, 2 * AF>;
  __shared__ L s0, s1;
  __shared__ int tix;
  for (;;) {
    if (threadIdx.x == 0) tix = atomicAdd(counter, 1);
    __syncthreads();
    const int t = tix;
    if (t >= n_tiles) break;
    const int4 td = tiles[t];
    const BulkItem& it = items[td.x];
    // row fragments of this tile that hold rows of the item's frequencies
    const int nf = min(AF, (it.g.n_rows + 31) / 32 - (it.g.row_tile0 + td.z) * AF);
    const Blk3 bk{td.y, td.z, td.w};
#define QCX_TILE(NFV)                                                                          \
  bulk_tile<BF16, AF, MAXR, 2, GATHER, L, NFV>(it.A, it.Alo, it.R32, it.pairs, it.rows, it.g, \
                                               it.C, bk, s0, s1, s0)
    if (nf >= AF)
      QCX_TILE(AF);
    else if (nf <= 1)
      QCX_TILE(1);
    else if constexpr (AF > 2) {
      if (nf == 2)
        QCX_TILE(2);
      else if constexpr (AF > 3) {
        if (nf == 3)
          QCX_TILE(3);
        else if constexpr (AF > 4)
          QCX_TILE(4);
      }
    }
#undef QCX_TILE
    __syncthreads();  // tix and the LDS stages are reused by the next tile
  }
}

__global__ void k_set_int(int* p, int v) { *p = v; }

size_t lds_bytes_of(int n_g, int af, int nst) {
  const int maxr = bulk_maxr(n_g);
  if (maxr == 0) return (size_t)1 << 40;  // no bucket: never fits
  // nst = 4 is the three-stage pipeline with the slab one step ahead
  return (size_t)(nst == 4 ? 3 : nst) * sizeof(float4) * 64 * (4 * maxr + 2 * af);
}

template <bool BF16, int AF, int NST>
void launch_bulk_t(const void* Ahi, const void* Alo, const float* R32, const int* pairs,
                   const int* rows, const Chi0Geom& g, float* C, hipStream_t st) {
  const dim3 grid((g.n_bulkp / 128) * (g.c_rows / (32 * AF)) * g.ksplit);
  const float4* ah = static_cast<const float4*>(Ahi);
  const float4* al = static_cast<const float4*>(Alo);
  const float4* r = reinterpret_cast<const float4*>(R32);
#define QCX_BULK(MR, GA) \
  hipLaunchKernelGGL((k_bulk<BF16, AF, MR, NST, GA>), grid, dim3(256), 0, st, ah, al, r, pairs, rows, g, C)
  if (g.gather)
    QCX_BULK(5, true);
  else if (bulk_maxr(g.n_g) == 1)
    QCX_BULK(1, false);
  else if (bulk_maxr(g.n_g) == 4)
    QCX_BULK(4, false);
  else
    QCX_BULK(5, false);
#undef QCX_BULK
}

// ---------------------------------------------------------------------------
// FP64 pairs on FP64 MFMA (v_mfma_f64_16x16x4f64): the head and wings (pairs
// (0, G')) or, for the FP64 path, every pair.  Real GEMM
//     out[row][col] = sum_t W[row][t] P[t][col],
// rows (Re W(w_j), Im W(w_j)), columns (Re P, Im P) of the pair-slot table.
// Block = 4 waves = 64 rows x (NCF*16) columns; wave w owns row fragment w and
// all NCF column fragments.  Per chunk of KC transitions the block computes W
// (FP64 reciprocal) and P = R(G)^* R(G') once into LDS.  grid = (column tiles,
// row tiles, K splits); out = [split][n_rowsp][n_colp] partial sums.
// Lane layouts: A 16x4, lane l holds A[l%16][l/16]; B 4x16, lane l holds
// B[l/16][l%16]; D 16x16, lane l holds D[4v + l/16][l%16], v = 0..3.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int KC = 32;          // transitions per LDS chunk
constexpr int NCF = 15;         // column fragments per block
constexpr int COLS64 = NCF * 16;
constexpr int SW_LD = KC + 1;   // padded LDS strides (bank spread)
constexpr int SP_LD = COLS64 + 1;

__global__ void __launch_bounds__(256) k_pairs_mfma64_direct(const cplx* __restrict__ R, size_t ldt,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ dt, double eta,
                                                      int n_w, int n_t,
                                                      const int* __restrict__ pairs, int n_ps,
                                                      int chunk_t, int n_rowsp, int n_colp,
                                                      double* __restrict__ out) {
  __shared__ double sW[64 * SW_LD];
  __shared__ double sP[KC * SP_LD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Blk3 bk = xcd_block(n_colp / COLS64, n_rowsp / 64, gridDim.x / ((n_colp / COLS64) * (n_rowsp / 64)));
  const int row0 = bk.y * 64;                 // first row of the block
  const int j0 = row0 / 2;                    // first frequency
  const int c0 = bk.x * COLS64;               // first column of the block
  const int ps0 = c0 / 2;                     // first pair slot
  f64x4 acc[NCF];
#pragma unroll
  for (int c = 0; c < NCF; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int t_begin = bk.z * chunk_t;
  const int t_end = min(n_t, t_begin + chunk_t);
  for (int t0 = t_begin; t0 < t_end; t0 += KC) {
    __syncthreads();
    // W for 32 frequencies x KC transitions (zero outside the ranges)
    for (int i = threadIdx.x; i < 32 * KC; i += 256) {
      const int jj = i / KC, tt = i % KC;
      const int t = t0 + tt;
      const cplx W = (t < t_end) ? weight(w, dt, eta, j0 + jj, t, n_w, n_t) : cplx{0.0, 0.0};
      sW[(2 * jj) * SW_LD + tt] = W.re;
      sW[(2 * jj + 1) * SW_LD + tt] = W.im;
    }
    // P for KC transitions x COLS64/2 pair slots; consecutive threads walk t
    for (int i = threadIdx.x; i < KC * (COLS64 / 2); i += 256) {
      const int tt = i % KC, pp = i / KC;
      const int t = t0 + tt, ps = ps0 + pp;
      double re = 0.0, im = 0.0;
      if (t < t_end && ps < n_ps) {
        const int pk = pairs[ps];
        const cplx a = R[(size_t)(pk & 0xffff) * ldt + t];
        const cplx b = R[(size_t)(pk >> 16) * ldt + t];
        re = a.re * b.re + a.im * b.im;
        im = a.re * b.im - a.im * b.re;
      }
      sP[tt * SP_LD + 2 * pp] = re;
      sP[tt * SP_LD + 2 * pp + 1] = im;
    }
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < KC / 4; ++s) {
      const int k = 4 * s + (lane >> 4);
      const double a = sW[(16 * wave + (lane & 15)) * SW_LD + k];
#pragma unroll
      for (int c = 0; c < NCF; ++c) {
        const double b = sP[k * SP_LD + 16 * c + (lane & 15)];
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCF; ++c) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + 16 * wave + 4 * v + (lane >> 4);
      const int col = c0 + 16 * c + (lane & 15);
      out[((size_t)bk.z * n_rowsp + row) * n_colp + col] = acc[c][v];
    }
  }
}

// DMA-staged variant for n_g <= NGC: per chunk of KC8 transitions the R rows
// of every G are copied global -> LDS (global_load_lds_dwordx4) into one of
// two named buffers while the MFMAs of the previous chunk run from P and W,
// which live in other named LDS arrays (so the copies need no wait before
// those reads).  Two barriers per chunk.
constexpr int KC8 = 8;
constexpr int SW8_LD = KC8 + 1;

template <int NGC>
__device__ inline void pairs64_stage(const cplx* __restrict__ R, size_t ldt, int n_g, int t0,
                                     float4* buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nch = (n_g + 7) / 8;  // 8 rows of 8 transitions per 1 KB chunk
  for (int c = wave; c < nch; c += 4) {
    const int row = 8 * c + (lane >> 3);
    const int rr = row < n_g ? row : 0;
    const float4* src = reinterpret_cast<const float4*>(R + (size_t)rr * ldt + t0 + (lane & 7));
    lds_dma16(src, buf + 64 * c);
  }
}

template <int NGC>
__device__ inline void pairs64_chunk(const float4* sRc, double* sW, double* sP,
                                     const double* __restrict__ w,
                                     const double* __restrict__ dt, double eta, int n_w,
                                     int n_t, int j0, int t0, int t_end, const int* G_of,
                                     const int* Gp_of, int ps0, int n_ps) {
  // W for 32 frequencies x KC8 transitions
  {
    const int jj = threadIdx.x >> 3, tt = threadIdx.x & 7;
    const int t = t0 + tt;
    const cplx W = (t < t_end) ? weight(w, dt, eta, j0 + jj, t, n_w, n_t) : cplx{0.0, 0.0};
    sW[(2 * jj) * SW8_LD + tt] = W.re;
    sW[(2 * jj + 1) * SW8_LD + tt] = W.im;
  }
  // P for KC8 transitions x COLS64/2 pair slots
  const cplx* R = reinterpret_cast<const cplx*>(sRc);
  for (int i = threadIdx.x; i < KC8 * (COLS64 / 2); i += 256) {
    const int tt = i & 7, pp = i >> 3;
    const int ps = ps0 + pp;
    double re = 0.0, im = 0.0;
    if (ps < n_ps && t0 + tt < t_end) {
      const cplx a = R[G_of[pp] * KC8 + tt];
      const cplx b = R[Gp_of[pp] * KC8 + tt];
      re = a.re * b.re + a.im * b.im;
      im = a.re * b.im - a.im * b.re;
    }
    sP[tt * SP_LD + 2 * pp] = re;
    sP[tt * SP_LD + 2 * pp + 1] = im;
  }
}

template <int NGC>
__global__ void __launch_bounds__(256) k_pairs_mfma64(const cplx* __restrict__ R, size_t ldt,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ dt, double eta,
                                                      int n_w, int n_t, int n_g,
                                                      const int* __restrict__ pairs, int n_ps,
                                                      int chunk_t, int n_rowsp, int n_colp,
                                                      double* __restrict__ out) {
  __shared__ float4 sR0[NGC * KC8];  // [g][KC8] complex
  __shared__ float4 sR1[NGC * KC8];
  __shared__ double sW[64 * SW8_LD];
  __shared__ double sP[KC8 * SP_LD];
  __shared__ int G_of[COLS64 / 2], Gp_of[COLS64 / 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Blk3 bk = xcd_block(n_colp / COLS64, n_rowsp / 64,
                            gridDim.x / ((n_colp / COLS64) * (n_rowsp / 64)));
  const int row0 = bk.y * 64, j0 = row0 / 2;
  const int c0 = bk.x * COLS64, ps0 = c0 / 2;
  for (int i = threadIdx.x; i < COLS64 / 2; i += 256) {
    const int ps = ps0 + i;
    const int pk = ps < n_ps ? pairs[ps] : 0;
    G_of[i] = pk & 0xffff;
    Gp_of[i] = pk >> 16;
  }
  f64x4 acc[NCF];
#pragma unroll
  for (int c = 0; c < NCF; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int t_begin = bk.z * chunk_t;
  const int t_end = min(n_t, t_begin + chunk_t);
  const int nchunk = t_end > t_begin ? (t_end - t_begin + KC8 - 1) / KC8 : 0;

  auto mfma_chunk = [&]() {
#pragma unroll
    for (int s = 0; s < KC8 / 4; ++s) {
      const int k = 4 * s + (lane >> 4);
      const double a = sW[(16 * wave + (lane & 15)) * SW8_LD + k];
#pragma unroll
      for (int c = 0; c < NCF; ++c) {
        const double b = sP[k * SP_LD + 16 * c + (lane & 15)];
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
      }
    }
  };

  if (nchunk > 0) pairs64_stage<NGC>(R, ldt, n_g, t_begin, sR0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int ci = 0; ci < nchunk; ci += 2) {
    // even chunk: R in sR0, prefetch into sR1
    {
      const int t0 = t_begin + ci * KC8;
      pairs64_chunk<NGC>(sR0, sW, sP, w, dt, eta, n_w, n_t, j0, t0, t_end, G_of, Gp_of, ps0, n_ps);
      __syncthreads();
      if (ci + 1 < nchunk) pairs64_stage<NGC>(R, ldt, n_g, t0 + KC8, sR1);
      mfma_chunk();
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
    if (ci + 1 < nchunk) {  // odd chunk: R in sR1, prefetch into sR0
      const int t0 = t_begin + (ci + 1) * KC8;
      pairs64_chunk<NGC>(sR1, sW, sP, w, dt, eta, n_w, n_t, j0, t0, t_end, G_of, Gp_of, ps0, n_ps);
      __syncthreads();
      if (ci + 2 < nchunk) pairs64_stage<NGC>(R, ldt, n_g, t0 + KC8, sR0);
      mfma_chunk();
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
  }
#pragma unroll
  for (int c = 0; c < NCF; ++c) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + 16 * wave + 4 * v + (lane >> 4);
      const int col = c0 + 16 * c + (lane & 15);
      out[((size_t)bk.z * n_rowsp + row) * n_colp + col] = acc[c][v];
    }
  }
}

}  // namespace

size_t bulk_lds_bytes(int n_g, int af, int nst) { return lds_bytes_of(n_g, af, nst); }

void launch_transition_energies(const double* Ek, const double* Ekq, int n_k, int n_b, int n_occ,
                                double* dt, hipStream_t st) {
  const int n = 2 * n_k * n_occ * (n_b - n_occ);
  hipLaunchKernelGGL(k_trans_energy, dim3((n + 255) / 256), dim3(256), 0, st, Ek, Ekq, n_k, n_b,
                     n_occ, dt);
}

void launch_weights_f32(const double* w, const double* dt, double eta, const Chi0Geom& g,
                        float* Aw, hipStream_t st) {
  const long total = (long)(g.n_rowsp / 32) * (g.n_tp / KSTEP) * 64;
  hipLaunchKernelGGL(k_weights_f32, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, w, dt,
                     eta, g, Aw);
}

void launch_weights_bf16(const double* w, const double* dt, double eta, const Chi0Geom& g,
                         uint16_t* Ahi, uint16_t* Alo, hipStream_t st) {
  const long total = (long)(g.n_rowsp / 32) * (g.n_tp / KSTEP) * 64;
  hipLaunchKernelGGL(k_weights_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, w,
                     dt, eta, g, Ahi, Alo);
}

void launch_pack_r32(const cplx* R, size_t ldt, const Chi0Geom& g, int perm, float* R32,
                     hipStream_t st) {
  const long total = (long)g.n_g * g.n_tp;
  hipLaunchKernelGGL(k_pack_r32, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, R, ldt,
                     g.n_g, g.n_tp, perm, R32);
}

int bulk_row_frags(const Chi0Geom& g) {
  // rows per block: 4 or 5 fragments, whichever pads 2 n_w less
  const int r4 = (g.n_rows + 127) / 128 * 128, r5 = (g.n_rows + 159) / 160 * 160;
  return r5 < r4 ? 5 : 4;
}

void launch_bulk_f32(const float* Aw, const float* R32, const int* pairs, const int* rows,
                     const Chi0Geom& g, int nst, float* C, hipStream_t st) {
  const bool af5 = g.n_rowsp % 160 == 0 && bulk_row_frags(g) == 5;
  if (af5 && nst == 4)
    launch_bulk_t<false, 5, 4>(Aw, nullptr, R32, pairs, rows, g, C, st);
  else if (af5 && nst == 3)
    launch_bulk_t<false, 5, 3>(Aw, nullptr, R32, pairs, rows, g, C, st);
  else if (af5)
    launch_bulk_t<false, 5, 2>(Aw, nullptr, R32, pairs, rows, g, C, st);
  else if (nst == 4)
    launch_bulk_t<false, 4, 4>(Aw, nullptr, R32, pairs, rows, g, C, st);
  else if (nst == 3)
    launch_bulk_t<false, 4, 3>(Aw, nullptr, R32, pairs, rows, g, C, st);
  else
    launch_bulk_t<false, 4, 2>(Aw, nullptr, R32, pairs, rows, g, C, st);
}

void launch_bulk_bf16(const uint16_t* Ahi, const uint16_t* Alo, const float* R32,
                      const int* pairs, const int* rows, const Chi0Geom& g, int nst, float* C,
                      hipStream_t st) {
  const bool af5 = g.n_rowsp % 160 == 0 && bulk_row_frags(g) == 5;
  if (af5 && nst == 4)
    launch_bulk_t<true, 5, 4>(Ahi, Alo, R32, pairs, rows, g, C, st);
  else if (af5 && nst == 3)
    launch_bulk_t<true, 5, 3>(Ahi, Alo, R32, pairs, rows, g, C, st);
  else if (af5)
    launch_bulk_t<true, 5, 2>(Ahi, Alo, R32, pairs, rows, g, C, st);
  else if (nst == 4)
    launch_bulk_t<true, 4, 4>(Ahi, Alo, R32, pairs, rows, g, C, st);
  else if (nst == 3)
    launch_bulk_t<true, 4, 3>(Ahi, Alo, R32, pairs, rows, g, C, st);
  else
    launch_bulk_t<true, 4, 2>(Ahi, Alo, R32, pairs, rows, g, C, st);
}

void launch_bulk_persistent(bool bf16, bool gather, const BulkItem* items, const int4* tiles,
                            int n_tiles, int* counter, int max_ng, int grid, hipStream_t st) {
  constexpr int AF = kBatchAF;
#define QCX_PERSIST(B, R, GA)                                                                 \
  hipLaunchKernelGGL((k_bulk_persistent<B, AF, R, GA>), dim3(grid), dim3(256), 0, st, items, \
                     tiles, n_tiles, counter)
  const int maxr = gather ? 5 : bulk_maxr(max_ng);
  if (bf16) {
    if (gather) QCX_PERSIST(true, 5, true);
    else if (maxr == 1) QCX_PERSIST(true, 1, false);
    else if (maxr == 4) QCX_PERSIST(true, 4, false);
    else QCX_PERSIST(true, 5, false);
  } else {
    if (gather) QCX_PERSIST(false, 5, true);
    else if (maxr == 1) QCX_PERSIST(false, 1, false);
    else if (maxr == 4) QCX_PERSIST(false, 4, false);
    else QCX_PERSIST(false, 5, false);
  }
#undef QCX_PERSIST
}

bool bulk_gather_tables(const std::vector<int>& pairs_global, std::vector<int>& pairs_local,
                        std::vector<int>& rows) {
  const size_t nb = pairs_global.size();
  const size_t n_tiles = nb / 128;
  pairs_local.assign(nb, 0);
  rows.assign(n_tiles * kGatherRows, 0);
  std::vector<int> list;
  for (size_t t = 0; t < n_tiles; ++t) {
    list.clear();
    for (size_t b = t * 128; b < (t + 1) * 128; ++b) {
      list.push_back(pairs_global[b] & 0xffff);
      list.push_back(pairs_global[b] >> 16);
    }
    std::sort(list.begin(), list.end());
    list.erase(std::unique(list.begin(), list.end()), list.end());
    if (list.size() > (size_t)kGatherRows) return false;
    for (size_t r = 0; r < (size_t)kGatherRows; ++r)
      rows[t * kGatherRows + r] = list[r < list.size() ? r : 0];
    auto local = [&](int G) {
      return (int)(std::lower_bound(list.begin(), list.end(), G) - list.begin());
    };
    for (size_t b = t * 128; b < (t + 1) * 128; ++b)
      pairs_local[b] = local(pairs_global[b] & 0xffff) | (local(pairs_global[b] >> 16) << 16);
  }
  return true;
}

__global__ void k_reduce_partials(const float* __restrict__ C, int ks, long n, double* C64) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < ks; ++k) s += (double)C[(size_t)k * n + i];
  C64[i] = s;
}

void launch_reduce_partials(const float* C, int ks, int n_rows, int n_bulkp, double* C64,
                            hipStream_t st) {
  const long n = (long)n_rows * 2 * n_bulkp;
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, C, ks,
                     n, C64);
}

void launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
}

void launch_pairs_f64(const cplx* R, size_t ldt, const double* w, const double* dt, double eta,
                      const Geom64& g, const int* pairs, double* out, hipStream_t st) {
  const dim3 grid((g.n_colp / COLS64) * (g.n_rowsp / 64) * g.ksplit);
  if (g.n_g <= 128)
    hipLaunchKernelGGL(k_pairs_mfma64<128>, grid, dim3(256), 0, st, R, ldt, w, dt, eta, g.n_w,
                       g.n_t, g.n_g, pairs, g.n_ps, g.chunk_t, g.n_rowsp, g.n_colp, out);
  else if (g.n_g <= 256)
    hipLaunchKernelGGL(k_pairs_mfma64<256>, grid, dim3(256), 0, st, R, ldt, w, dt, eta, g.n_w,
                       g.n_t, g.n_g, pairs, g.n_ps, g.chunk_t, g.n_rowsp, g.n_colp, out);
  else
    hipLaunchKernelGGL(k_pairs_mfma64_direct, grid, dim3(256), 0, st, R, ldt, w, dt, eta, g.n_w,
                       g.n_t, pairs, g.n_ps, g.chunk_t, g.n_rowsp, g.n_colp, out);
}

// Blocks of the FP64 pairs kernel that the current device holds at once (CUs
// x resident blocks per CU for the variant launch_pairs_f64 picks for n_g).
static int pairs64_slots(int n_g) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e;
  if (n_g <= 128)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pairs_mfma64<128>, 256, 0);
  else if (n_g <= 256)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pairs_mfma64<256>, 256, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pairs_mfma64_direct, 256, 0);
  return e == hipSuccess ? cus * per : 0;
}

// K split of the FP64 pairs kernel: the launch runs in ceil(blocks / slots)
// rounds of blocks that each walk their share of the KC-transition chunks, so
// the split minimises rounds x (chunks per split + a fixed cost of two chunks
// per block: start-up and the partial-sum tile), within the partial-sum
// budget; a split that needs no more splits than a smaller one is skipped.
void geom64_init(Geom64& g, int n_g, int n_w, int n_t, int n_ps, size_t max_bytes) {
  g.n_g = n_g;
  g.n_w = n_w;
  g.n_t = n_t;
  g.n_ps = n_ps;
  g.n_rowsp = (2 * n_w + 63) / 64 * 64;
  g.n_colp = (2 * n_ps + COLS64 - 1) / COLS64 * COLS64;
  const int blocks = (g.n_colp / COLS64) * (g.n_rowsp / 64);
  const int chunks = std::max(1, (n_t + KC - 1) / KC);
  int slots = pairs64_slots(n_g);
  if (slots <= 0) slots = 2048;
  const size_t split_bytes = (size_t)g.n_rowsp * g.n_colp * sizeof(double);
  int best = 1;
  double best_cost = 1e300;
  for (int ks = 1; ks <= std::min(256, chunks); ++ks) {
    const int per = (chunks + ks - 1) / ks;
    if ((chunks + per - 1) / per != ks) continue;
    if (ks > 1 && (size_t)ks * split_bytes > max_bytes) break;
    const long rounds = ((long)blocks * ks + slots - 1) / slots;
    const double cost = (double)rounds * (per + 2);
    if (cost < best_cost) {
      best_cost = cost;
      best = ks;
    }
  }
  g.ksplit = best;
  g.chunk_t = (chunks + best - 1) / best * KC;
}

}  // namespace qcx
