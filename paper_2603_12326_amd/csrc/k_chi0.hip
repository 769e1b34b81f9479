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
// A[rb*32 + l%32][tb*16 + 8(l/32) + 0..7]; hi = bf16(x), lo = bf16(x - hi) with
// the residual taken from the FP64 weight.
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
  uint16_t hi[8], lo[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int t = tb * KSTEP + 8 * (lane / 32) + s;
    const cplx wt = weight(w, dt, eta, j, t, g.n_w, g.n_t);
    const double x = ri ? wt.im : wt.re;
    hi[s] = bf16_bits((float)x);
    lo[s] = bf16_bits((float)(x - (double)bf16_val(hi[s])));
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
// The R slab of the current K step (all G, 16 transitions, complex float) is
// double-buffered in LDS; the A fragments come straight from global memory in
// fragment order.  grid = (pair tiles, row tiles, K splits).
// ---------------------------------------------------------------------------
template <bool BF16, int AF, int MAXF4>
__global__ void __launch_bounds__(256) k_bulk(const void* __restrict__ Ahi_,
                                              const void* __restrict__ Alo_,
                                              const float* __restrict__ R32,
                                              const int* __restrict__ pairs, Chi0Geom g,
                                              float* __restrict__ C) {
  extern __shared__ float4 slab[];  // 2 buffers of n_g * 16 complex floats
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
  const int ntb = g.n_tp / KSTEP;
  const int steps = ntb / g.ksplit;
  const int tb0 = blockIdx.z * steps;
  const int rb0 = blockIdx.y * AF;
  const int b = blockIdx.x * 128 + wave * 32 + (lane & 31);
  const int pk = pairs[b];
  const int G = pk & 0xffff, Gp = pk >> 16;
  const int slab_f4 = g.n_g * KSTEP * 2 / 4;  // float4 per slab
  const float4* src = reinterpret_cast<const float4*>(R32);

  f32x16 acc[AF][2];
#pragma unroll
  for (int f = 0; f < AF; ++f) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc[f][0][r] = 0.f;
      acc[f][1][r] = 0.f;
    }
  }

  // prologue: slab tb0 -> buffer 0
  for (int i = threadIdx.x; i < slab_f4; i += 256) slab[i] = src[(size_t)tb0 * slab_f4 + i];
  __syncthreads();

  for (int st = 0; st < steps; ++st) {
    const int tb = tb0 + st;
    const float4* cur = slab + (st & 1) * slab_f4;
    // prefetch the next slab into registers
    float4 nxt[MAXF4];
    const bool more = st + 1 < steps;
    const float4* nsrc = src + (size_t)(more ? tb + 1 : tb) * slab_f4;
#pragma unroll
    for (int u = 0; u < MAXF4; ++u) {
      const int i = threadIdx.x + u * 256;
      nxt[u] = nsrc[i < slab_f4 ? i : 0];
    }
    // B operand: P_t(G, G') for this lane's pair and 8 transitions
    const float2* s2 = reinterpret_cast<const float2*>(cur);
    float pre[8], pim[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float2 x = s2[G * KSTEP + 8 * h + i];
      const float2 y = s2[Gp * KSTEP + 8 * h + i];
      pre[i] = x.x * y.x + x.y * y.y;
      pim[i] = x.x * y.y - x.y * y.x;
    }
    if constexpr (BF16) {
      bf16x8 bre_hi, bre_lo, bim_hi, bim_lo;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const __bf16 rh = (__bf16)pre[i];
        const __bf16 ih = (__bf16)pim[i];
        bre_hi[i] = rh;
        bim_hi[i] = ih;
        bre_lo[i] = (__bf16)(pre[i] - (float)rh);
        bim_lo[i] = (__bf16)(pim[i] - (float)ih);
      }
      const bf16x8* Ahi = reinterpret_cast<const bf16x8*>(Ahi_);
      const bf16x8* Alo = reinterpret_cast<const bf16x8*>(Alo_);
#pragma unroll
      for (int f = 0; f < AF; ++f) {
        const size_t fi = ((size_t)(rb0 + f) * ntb + tb) * 64 + lane;
        const bf16x8 ah = Ahi[fi], al = Alo[fi];
        acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bre_hi, acc[f][0], 0, 0, 0);
        acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bim_hi, acc[f][1], 0, 0, 0);
        acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bre_lo, acc[f][0], 0, 0, 0);
        acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bim_lo, acc[f][1], 0, 0, 0);
        acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bre_hi, acc[f][0], 0, 0, 0);
        acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bim_hi, acc[f][1], 0, 0, 0);
      }
    } else {
      const float4* A4 = reinterpret_cast<const float4*>(Ahi_);
#pragma unroll
      for (int f = 0; f < AF; ++f) {
        const size_t fi = (((size_t)(rb0 + f) * ntb + tb) * 64 + lane) * 2;
        const float4 a0 = A4[fi], a1 = A4[fi + 1];
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          acc[f][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], pre[s], acc[f][0], 0, 0, 0);
          acc[f][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], pim[s], acc[f][1], 0, 0, 0);
        }
      }
    }
    float4* dst = slab + ((st + 1) & 1) * slab_f4;
#pragma unroll
    for (int u = 0; u < MAXF4; ++u) {
      const int i = threadIdx.x + u * 256;
      if (more && i < slab_f4) dst[i] = nxt[u];
    }
    __syncthreads();
  }

  // epilogue: C[((ks*n_rowsp + row)*2 + ri)*n_bulkp + b]
#pragma unroll
  for (int f = 0; f < AF; ++f) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (rb0 + f) * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) {
        const size_t o = (((size_t)blockIdx.z * g.n_rowsp + row) * 2 + ri) * g.n_bulkp + b;
        C[o] = acc[f][ri][r];
      }
    }
  }
}

template <bool BF16, int AF>
void launch_bulk_t(const void* Ahi, const void* Alo, const float* R32, const int* pairs,
                   const Chi0Geom& g, float* C, hipStream_t st) {
  const dim3 grid(g.n_bulkp / 128, g.n_rowsp / (32 * AF), g.ksplit);
  const size_t lds = 2 * (size_t)g.n_g * KSTEP * 8;
  const int f4 = (g.n_g * KSTEP * 2 / 4 + 255) / 256;
  if (f4 <= 4)
    hipLaunchKernelGGL((k_bulk<BF16, AF, 4>), grid, dim3(256), lds, st, Ahi, Alo, R32, pairs, g, C);
  else if (f4 <= 8)
    hipLaunchKernelGGL((k_bulk<BF16, AF, 8>), grid, dim3(256), lds, st, Ahi, Alo, R32, pairs, g, C);
  else
    hipLaunchKernelGGL((k_bulk<BF16, AF, 24>), grid, dim3(256), lds, st, Ahi, Alo, R32, pairs, g, C);
}

// ---------------------------------------------------------------------------
// FP64 pairs (head/wings, or every pair for the FP64 path).  Block = 256
// threads = 8 frequency groups (4 w each) x 32 pair groups (4 pairs each);
// grid = (pair tiles of 128, frequency tiles of 32, K splits).  Per chunk of
// TC transitions the weights of the block's 32 frequencies and R[g][t] for all
// G are staged in LDS.
// ---------------------------------------------------------------------------
__device__ inline int pair_flat0(int G, int n_g) { return G * n_g - G * (G - 1) / 2; }

__global__ void __launch_bounds__(256) k_pairs_f64(const cplx* __restrict__ R, size_t ldt,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ dt, double eta,
                                                   int n_w, int n_t, int n_g, int pa, int n_pl,
                                                   int tc, int chunk, double* __restrict__ XY) {
  extern __shared__ cplx sm[];
  cplx* sW = sm;              // [32][tc]
  cplx* sR = sm + 32 * tc;    // [n_g][tc]
  const int wg = threadIdx.x >> 5, pg = threadIdx.x & 31;
  const int j0 = blockIdx.y * 32 + wg * 4;
  int Gs[4], Gps[4];
  bool ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int pl = blockIdx.x * 128 + pg * 4 + u;
    ok[u] = pl < n_pl;
    int p = pa + (ok[u] ? pl : 0);
    int G = 0;
    while (G + 1 < n_g && pair_flat0(G + 1, n_g) <= p) ++G;
    Gs[u] = G;
    Gps[u] = G + (p - pair_flat0(G, n_g));
  }
  double acc[4][4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][u][c] = 0.0;

  const int t_begin = blockIdx.z * chunk;
  const int t_end = min(n_t, t_begin + chunk);
  for (int t0 = t_begin; t0 < t_end; t0 += tc) {
    const int tn = min(tc, t_end - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * tc; i += 256) {
      const int jj = i / tc, tt = i % tc;
      sW[i] = (tt < tn) ? weight(w, dt, eta, blockIdx.y * 32 + jj, t0 + tt, n_w, n_t)
                        : cplx{0.0, 0.0};
    }
    for (int i = threadIdx.x; i < n_g * tc; i += 256) {
      const int gg = i / tc, tt = i % tc;
      sR[i] = (tt < tn) ? R[(size_t)gg * ldt + t0 + tt] : cplx{0.0, 0.0};
    }
    __syncthreads();
    for (int tt = 0; tt < tn; ++tt) {
      cplx P[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) P[u] = cmulc(sR[Gs[u] * tc + tt], sR[Gps[u] * tc + tt]);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const cplx W = sW[(wg * 4 + a) * tc + tt];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc[a][u][0] += W.re * P[u].re;
          acc[a][u][1] += W.re * P[u].im;
          acc[a][u][2] += W.im * P[u].re;
          acc[a][u][3] += W.im * P[u].im;
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int j = j0 + a;
    if (j >= n_w) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u]) continue;
      const int pl = blockIdx.x * 128 + pg * 4 + u;
      double* o = XY + (((size_t)blockIdx.z * n_w + j) * n_pl + pl) * 4;
      o[0] = acc[a][u][0];
      o[1] = acc[a][u][1];
      o[2] = acc[a][u][2];
      o[3] = acc[a][u][3];
    }
  }
}

}  // namespace

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

void launch_bulk_f32(const float* Aw, const float* R32, const int* pairs, const Chi0Geom& g,
                     float* C, hipStream_t st) {
  if (g.n_rowsp % 160 == 0 && bulk_row_frags(g) == 5)
    launch_bulk_t<false, 5>(Aw, nullptr, R32, pairs, g, C, st);
  else
    launch_bulk_t<false, 4>(Aw, nullptr, R32, pairs, g, C, st);
}

void launch_bulk_bf16(const uint16_t* Ahi, const uint16_t* Alo, const float* R32,
                      const int* pairs, const Chi0Geom& g, float* C, hipStream_t st) {
  if (g.n_rowsp % 160 == 0 && bulk_row_frags(g) == 5)
    launch_bulk_t<true, 5>(Ahi, Alo, R32, pairs, g, C, st);
  else
    launch_bulk_t<true, 4>(Ahi, Alo, R32, pairs, g, C, st);
}

size_t pairs_f64_tc(int n_g) {
  size_t tc = 65536 / (16 * (size_t)(n_g + 32));
  if (tc > 64) tc = 64;
  if (tc < 1) tc = 1;
  return tc;
}

void launch_pairs_f64(const cplx* R, size_t ldt, const double* w, const double* dt, double eta,
                      int n_w, int n_t, int n_g, int ga, int gb, int ksplit, double* XY,
                      hipStream_t st) {
  auto flat0 = [n_g](int G) { return G * n_g - G * (G - 1) / 2; };
  const int pa = flat0(ga);
  const int n_pl = (gb >= n_g ? n_g * (n_g + 1) / 2 : flat0(gb)) - pa;
  const int tc = (int)pairs_f64_tc(n_g);
  const int chunk = (n_t + ksplit - 1) / ksplit;
  const size_t lds = sizeof(cplx) * (size_t)tc * (32 + n_g);
  const dim3 grid((n_pl + 127) / 128, (n_w + 31) / 32, ksplit);
  hipLaunchKernelGGL(k_pairs_f64, grid, dim3(256), lds, st, R, ldt, w, dt, eta, n_w, n_t, n_g, pa,
                     n_pl, tc, chunk, XY);
}

}  // namespace qcx
