// Kramers-Kronig route of Sec. II.D: the spectral part of Eq. (RPA), binned
// with hat functions, and its transform back to the response at each
// frequency,
//   chi0(w) = sum_b S^r_b K(w - w_b + i eta) - sum_b S^a_b K(w + w_b - i eta),
//   K(x) = (1/d) I(x / d),  I(z) = int_{-1}^{1} (1 - |y|) / (z - y) dy,
// i.e. every hat-shaped piece of the spectral density is carried through the
// energy denominator exactly.  I has the closed form
//   I(z) = (z + 1) log(z + 1) - 2 z log z + (z - 1) log(z - 1)
// (principal logarithm; no branch cut is crossed for Im z != 0), and for
// eta = 0 the limits from above (resonant) and below (anti-resonant) give the
// principal value plus -i pi times the spectral density.  For |z| >= 8 the
// expansion I(z) = sum_n 2 / ((2n+1)(2n+2)) z^-(2n+1) avoids the cancellation
// between the three logarithms.
//
// Binning is a sparse accumulation (two bins per transition), done on the
// FP64 vector units; the transform is a dense FP64 product over the bins on
// FP64 MFMA (k_kk_gemm), with the kernel matrix laid out bin-major so that
// both operands stream in rows of the bin index.
#include "kk.h"

namespace qcx {

namespace {

// ------------------------------------------------------------------ packing
// Rs[rank[t]][g] = R[g][t] (zero for g >= n_g): a tiled transpose, 32
// transitions x 64 G per block, so that the reads walk rows of R and the
// writes walk rows of Rs (rank is the energy order of the transitions).
constexpr int KP_T = 32;
__global__ void __launch_bounds__(256) k_kk_pack(const cplx* __restrict__ R, size_t ldt, int n_g,
                                                 int n_gp, int n_t, const int* __restrict__ rank,
                                                 cplx* __restrict__ Rs) {
  __shared__ cplx tile[KP_T][kKkTile + 1];
  const int t0 = blockIdx.x * KP_T, g0 = blockIdx.y * kKkTile;
  for (int e = threadIdx.x; e < KP_T * kKkTile; e += 256) {
    const int gg = e / KP_T, tt = e % KP_T;
    const int g = g0 + gg, t = t0 + tt;
    tile[tt][gg] = (g < n_g && t < n_t) ? R[(size_t)g * ldt + t] : cplx{0.0, 0.0};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KP_T * kKkTile; e += 256) {
    const int tt = e / kKkTile, gg = e % kKkTile;
    const int t = t0 + tt;
    if (t < n_t) Rs[(size_t)rank[t] * n_gp + g0 + gg] = tile[tt][gg];
  }
}

// ------------------------------------------------------------------ binning
// Block = one 64 x 64 tile (ti <= tj) of the (G, G') plane and one chunk of
// intervals; thread (ty, tx) owns G = g0 + ty + 16 k, G' = h0 + tx + 16 l
// (k, l < 4).  The transitions of the chunk are walked in energy order, 16 at
// a time staged in LDS by direct global-to-LDS loads into one of two buffers
// while the other is consumed (two blocks of 64 KB fit a CU).  Two accumulators per
// pair hold the bins i and i + 1 of the current interval; when the interval
// changes, finished bins are stored (each bin of the chunk exactly once,
// empty bins as zero).  The share of the chunk's last interval in the bin
// after the chunk goes to the chunk's own row of E and is added to that bin
// by k_kk_tail, so every transition is read once, no atomics are needed and
// the result does not depend on the launch.
constexpr int KB_TC = 16;
typedef __attribute__((address_space(3))) void lds_void;

// 16 bytes per lane from g into LDS at l + 16 * lane (l the same for the
// wave).  Written as asm so that the compiler does not order every LDS read
// after it (it cannot tell that the reads use the other buffer); the kernel
// waits for it itself (s_waitcnt vmcnt(0) before the barrier that publishes
// the stage).  It has no register result.
__device__ __forceinline__ void lds_load16(const void* g, lds_void* l) {
  const unsigned base = __builtin_amdgcn_readfirstlane((unsigned)(size_t)l);
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(base)
               : "memory", "m0");
}

// Tile pair p of the upper triangle of T x T tiles: the T (T - 1) / 2
// off-diagonal pairs first, then the T diagonal ones, which hold about 10/16
// of the work, so that the short blocks are the last to be dispatched.
__device__ inline void tile_of(int p, int T, int& ti, int& tj) {
  const int n_off = T * (T - 1) / 2;
  if (p >= n_off) {
    ti = tj = p - n_off;
    return;
  }
  int r = 0, s = T - 1;
  while (p >= s) {  // row r holds the T - 1 - r pairs (r, r + 1 ..)
    p -= s;
    ++r;
    --s;
  }
  ti = r;
  tj = r + 1 + p;
}

// One (chunk, tile) of the binning.  DIAG (a tile on the diagonal, ti = tj):
// a thread's 16 x 16 sub-blocks (k, l) below the diagonal (k > l) hold only
// G > G' and are not computed, and both operands come from one staged slice.
template <bool DIAG>
__device__ __forceinline__ void kk_bin_tile(const cplx* __restrict__ Rs, int n_gp, int n_g,
                                            const int* __restrict__ ib,
                                            const double* __restrict__ xf, const KkChunk ch,
                                            int ti, int tj, double* __restrict__ S,
                                            double* __restrict__ E,
                                            cplx (&sa)[2][KB_TC][kKkTile],
                                            cplx (&sb)[2][KB_TC][kKkTile],
                                            int (&sib)[2][KB_TC], double (&sx)[2][KB_TC]) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int g0 = ti * kKkTile, h0 = tj * kKkTile;
  const size_t n_pairs = (size_t)n_g * (n_g + 1) / 2;

  double lr[4][4], li[4][4], hr[4][4], hi[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int l = 0; l < 4; ++l) lr[k][l] = li[k][l] = hr[k][l] = hi[k][l] = 0.0;

  // row (Re at base, Im at base + n_pairs) <- (vr, vi) for this thread's pairs
  auto store_at = [&](double* __restrict__ base, const double (&vr)[4][4],
                      const double (&vi)[4][4], bool zero) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int G = g0 + ty + 16 * k;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int Gp = h0 + tx + 16 * l;
        if (G < n_g && Gp < n_g && G <= Gp) {
          const size_t p = (size_t)G * n_g - (size_t)G * (G - 1) / 2 + (Gp - G);
          base[p] = zero ? 0.0 : vr[k][l];
          base[n_pairs + p] = zero ? 0.0 : vi[k][l];
        }
      }
    }
  };
  // bin j of the chunk (0 <= j < nb)
  auto store = [&](int j, const double (&vr)[4][4], const double (&vi)[4][4], bool zero) {
    store_at(S + (size_t)(ch.row0 + j) * 2 * n_pairs, vr, vi, zero);
  };
  int wn = 0;  // next bin of the chunk not yet stored
  auto put = [&](int j, const double (&vr)[4][4], const double (&vi)[4][4]) {
    if (j < 0 || j >= ch.nb) return;
    for (; wn < j; ++wn) store(wn, vr, vi, true);
    store(j, vr, vi, false);
    wn = j + 1;
  };

  // Stage at t0 into buffer q: wave w moves the rows tt = w, w + 4, ..
  // (tt < nt) of the tile's 64 G columns (and the 64 G' columns), one
  // 16-byte complex per lane, straight into LDS; rows tt >= nt are not read.
  // The interval and weight of each transition go through registers.
  const int wv = tid >> 6, lane = tid & 63;
  int r_ib = 0;
  double r_x = 0.0;
  auto issue = [&](int t0, int q) {
    const int nt = min(KB_TC, ch.tb - t0);
#pragma unroll
    for (int j = 0; j < KB_TC / 4; ++j) {
      const int tt = wv + 4 * j;
      if (tt < nt) {
        const cplx* row = Rs + (size_t)(t0 + tt) * n_gp;
        lds_load16(row + g0 + lane, (lds_void*)&sa[q][tt][0]);
        if (!DIAG) lds_load16(row + h0 + lane, (lds_void*)&sb[q][tt][0]);
      }
    }
    if (tid < nt) {
      r_ib = ib[t0 + tid];
      r_x = xf[t0 + tid];
    }
  };
  auto put_meta = [&](int q) {
    if (tid < KB_TC) {
      sib[q][tid] = r_ib;
      sx[q][tid] = r_x;
    }
  };

  int cur = ch.k0 - 1;  // interval of the accumulators (bins cur, cur + 1)
  int q = 0;
  if (ch.ta < ch.tb) {
    issue(ch.ta, 0);
    put_meta(0);
  }
  for (int t0 = ch.ta; t0 < ch.tb; t0 += KB_TC) {
    const int nt = min(KB_TC, ch.tb - t0), t1 = t0 + KB_TC;
    // the direct loads of this stage (issued one stage ahead) have landed in
    // every wave, and every wave is done with the buffer the next stage fills
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (t1 < ch.tb) issue(t1, q ^ 1);
    for (int tt = 0; tt < nt; ++tt) {
      const int i = sib[q][tt];
      if (i != cur) {  // the same for every thread of the block
        put(cur - ch.k0, lr, li);
        if (i == cur + 1) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              lr[k][l] = hr[k][l];
              li[k][l] = hi[k][l];
              hr[k][l] = hi[k][l] = 0.0;
            }
        } else {
          put(cur + 1 - ch.k0, hr, hi);
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int l = 0; l < 4; ++l) lr[k][l] = li[k][l] = hr[k][l] = hi[k][l] = 0.0;
        }
        cur = i;
      }
      const double x = sx[q][tt], wl = 1.0 - x;
      cplx a[4], b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = sa[q][tt][ty + 16 * k];
        b[k] = DIAG ? sa[q][tt][tx + 16 * k] : sb[q][tt][tx + 16 * k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          if (DIAG && k > l) continue;
          const double pr = a[k].re * b[l].re + a[k].im * b[l].im;  // conj(a) b
          const double pi = a[k].re * b[l].im - a[k].im * b[l].re;
          lr[k][l] += wl * pr;
          li[k][l] += wl * pi;
          hr[k][l] += x * pr;
          hi[k][l] += x * pi;
        }
    }
    if (t1 < ch.tb) put_meta(q ^ 1);
    q ^= 1;
  }
  put(cur - ch.k0, lr, li);
  put(cur + 1 - ch.k0, hr, hi);  // bin nb (past the chunk) is not stored here
  for (; wn < ch.nb; ++wn) store(wn, lr, li, true);
  // bin nb: zero unless the last interval of the chunk held transitions
  store_at(E + (size_t)blockIdx.x * 2 * n_pairs, hr, hi, cur + 1 != ch.k0 + ch.nb);
}

__global__ void __launch_bounds__(256) k_kk_bin(const cplx* __restrict__ Rs, int n_gp, int n_g,
                                                const int* __restrict__ ib,
                                                const double* __restrict__ xf,
                                                const KkChunk* __restrict__ chunks,
                                                double* __restrict__ S, double* __restrict__ E) {
  __shared__ cplx sa[2][KB_TC][kKkTile], sb[2][KB_TC][kKkTile];
  __shared__ int sib[2][KB_TC];
  __shared__ double sx[2][KB_TC];
  int ti, tj;
  tile_of(blockIdx.y, n_gp / kKkTile, ti, tj);
  const KkChunk ch = chunks[blockIdx.x];
  if (ti == tj)  // the same for the whole block
    kk_bin_tile<true>(Rs, n_gp, n_g, ib, xf, ch, ti, tj, S, E, sa, sb, sib, sx);
  else
    kk_bin_tile<false>(Rs, n_gp, n_g, ib, xf, ch, ti, tj, S, E, sa, sb, sib, sx);
}

// Bin tail of every chunk: S[tail] = E[chunk] (+ S[tail] when the next chunk
// of the side has stored its own share of that bin).  Rows are distinct per
// chunk, so the order of the additions is fixed.
__global__ void __launch_bounds__(256) k_kk_tail(const KkChunk* __restrict__ chunks,
                                                 size_t row_len, const double* __restrict__ E,
                                                 double* __restrict__ S) {
  const KkChunk ch = chunks[blockIdx.y];
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= row_len) return;
  double* dst = S + (size_t)ch.tail_row * row_len + i;
  const double e = E[(size_t)blockIdx.y * row_len + i];
  *dst = ch.tail_add ? *dst + e : e;
}

// ---------------------------------------------------------------- transform
struct c64 {
  double re, im;
};
__device__ inline c64 cm(c64 a, c64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline c64 clog_(c64 z) { return {0.5 * log(z.re * z.re + z.im * z.im), atan2(z.im, z.re)}; }
// z log z, with 0 log 0 = 0
__device__ inline c64 zlogz(c64 z) {
  if (z.re == 0.0 && z.im == 0.0) return {0.0, 0.0};
  return cm(z, clog_(z));
}

__device__ inline c64 hat_kernel(c64 z) {
  const double r2 = z.re * z.re + z.im * z.im;
  if (r2 >= 64.0) {
    // 1/z + 1/(6 z^3) + 1/(15 z^5) + ...: terms fall by |z|^-2 <= 1/64
    const double inv = 1.0 / r2;
    const c64 iz = {z.re * inv, -z.im * inv};
    const c64 iz2 = cm(iz, iz);
    c64 p = iz, s = {0.0, 0.0};
#pragma unroll
    for (int n = 0; n < 9; ++n) {
      const double c = 2.0 / ((2.0 * n + 1.0) * (2.0 * n + 2.0));
      s.re += c * p.re;
      s.im += c * p.im;
      p = cm(p, iz2);
    }
    return s;
  }
  const c64 a = zlogz({z.re + 1.0, z.im}), b = zlogz(z), c = zlogz({z.re - 1.0, z.im});
  return {a.re - 2.0 * b.re + c.re, a.im - 2.0 * b.im + c.im};
}

// Kb[c][row] (bin-major, rows_p bins x ldm rows, zero past the last bin and
// past row 2 n_w): row 2j + ri is the real (ri = 0) or imaginary part of the
// transform of bin c at frequency j.
__global__ void k_kk_matrix(const double* __restrict__ w, int n_w, double eta, double d, int nr,
                            int na, int br, int ba, int rows_p, int ldm, double* __restrict__ Kb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)rows_p * ldm) return;
  const int c = (int)(i / ldm), row = (int)(i % ldm);
  const int j = row >> 1, ri = row & 1;
  double v = 0.0;
  if (c < nr + na && row < 2 * n_w) {
    c64 k;
    if (c < nr) {  // resonant: K(w - w_b + i eta), limit from above at eta = 0
      const double wb = (br + c) * d;
      k = hat_kernel({(w[j] - wb) / d, eta / d});
    } else {       // anti-resonant: -K(w + w_b - i eta), limit from below
      const double wb = (ba + c - nr) * d;
      k = hat_kernel({(w[j] + wb) / d, eta > 0.0 ? -eta / d : -0.0});
      k = {-k.re, -k.im};
    }
    v = (ri ? k.im : k.re) / d;
  }
  Kb[i] = v;
}

// --------------------------------------------------------------- transform
// C[m][n] = sum_k Kb[k][m] S[k][n] on FP64 MFMA (v_mfma_f64_16x16x4f64):
// m < M = 2 n_w rows (frequency, re/im), n < N = 2 pairs columns, k over
// rows_p bins (a multiple of KG_K; Kb and S are zero in the padding).  A
// block of 256 threads owns KG_M x KG_N of C; its four waves own KG_M / 2 x
// KG_N / 2 each (5 x 4 MFMA tiles of 16 x 16).  Tiles of KG_K bins of both
// operands go through LDS in two buffers: the copies of the next tile into
// one are issued before the MFMAs on the other, one barrier per tile.  LDS
// rows are padded by 16 doubles so that the 16-lane groups of a fragment
// read hit different banks.  Blocks are
// placed so that the KG_M-row tiles sharing a column tile of S run on one
// XCD (S, the large operand, is then read from memory once).
// MFMA layouts: A 16x4, lane l holds A[l%16][l/16]; B 4x16, lane l holds
// B[l/16][l%16]; D 16x16, lane l holds D[4r + l/16][l%16], r = 0..3.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int KG_M = 160, KG_N = 128, KG_K = 16;
constexpr int KG_LA = KG_M + 16, KG_LB = KG_N + 16;  // padded LDS rows (doubles)
constexpr int KG_FA = KG_M / 32, KG_FB = KG_N / 32;   // fragments per wave: 5 x 4
constexpr int KG_VA = KG_K * KG_M / 2 / 256;          // 16-byte loads per thread: 5

// The next tile of bins k0 .. k0 + KG_K - 1, copied from memory straight into
// LDS (global_load_lds_dwordx4: one wave instruction moves 1 KB, lane l's 16
// bytes landing at the destination + 16 l): rows of S (KG_N doubles = 1 KB)
// and the first 128 columns of the Kb rows go one row per instruction into
// padded rows; the last 32 columns of the Kb rows (256 B each) go four rows
// per instruction into an unpadded block.
constexpr int KG_M1 = 128, KG_M2 = KG_M - KG_M1;
constexpr int KG_LA1 = KG_M1 + 16;
typedef __attribute__((address_space(3))) void* kg_lds_t;
__device__ __forceinline__ void kg_issue(const double* __restrict__ Kb, int ldm,
                                         const double* __restrict__ S, int N, int m0, int n0, int k0,
                                         int lane, int wave, double* sA1, double* sA2, double* sB) {
#pragma unroll
  for (int i = 0; i < KG_K / 4; ++i) {
    const int r = wave + 4 * i;
    __builtin_amdgcn_global_load_lds((const void*)(S + (size_t)(k0 + r) * N + n0 + 2 * lane),
                                     (kg_lds_t)(sB + r * KG_LB), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(Kb + (size_t)(k0 + r) * ldm + m0 + 2 * lane),
                                     (kg_lds_t)(sA1 + r * KG_LA1), 16, 0, 0);
  }
  const int r2 = 4 * wave + (lane >> 4);
  __builtin_amdgcn_global_load_lds(
      (const void*)(Kb + (size_t)(k0 + r2) * ldm + m0 + KG_M1 + 2 * (lane & 15)),
      (kg_lds_t)(sA2 + 4 * wave * KG_M2), 16, 0, 0);
}

__global__ void __launch_bounds__(256) k_kk_gemm(const double* __restrict__ Kb, int ldm,
                                                 const double* __restrict__ S, int N, int rows_p,
                                                 int M, int n_mt, int n_nt,
                                                 double* __restrict__ C) {
  __shared__ __attribute__((aligned(16))) double sA1[2][KG_K * KG_LA1];
  __shared__ __attribute__((aligned(16))) double sA2[2][KG_K * KG_M2];
  __shared__ __attribute__((aligned(16))) double sB[2][KG_K * KG_LB];
  // XCD-aware placement: consecutive logical tiles on one XCD share n
  const int total = n_mt * n_nt, per = (total + 7) / 8;
  const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= total) return;
  const int nt = logical / n_mt, mt = logical % n_mt;
  const int m0 = mt * KG_M, n0 = nt * KG_N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (KG_M / 2), wn = (wave & 1) * (KG_N / 2);
  f64x4 acc[KG_FA][KG_FB];
#pragma unroll
  for (int a = 0; a < KG_FA; ++a)
#pragma unroll
    for (int b = 0; b < KG_FB; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nk = rows_p / KG_K;
  kg_issue(Kb, ldm, S, N, m0, n0, 0, lane, wave, sA1[0], sA2[0], sB[0]);
  __syncthreads();  // its fence waits for the copies into LDS as well
  for (int s = 0; s < nk; ++s) {
    const int buf = s & 1;
    if (s + 1 < nk)
      kg_issue(Kb, ldm, S, N, m0, n0, (s + 1) * KG_K, lane, wave, sA1[buf ^ 1], sA2[buf ^ 1],
               sB[buf ^ 1]);
#pragma unroll
    for (int kk = 0; kk < KG_K; kk += 4) {
      const int k = kk + (lane >> 4);
      double fa[KG_FA], fb[KG_FB];
#pragma unroll
      for (int a = 0; a < KG_FA; ++a) {
        const int mm = wm + 16 * a;  // wave-uniform: which block holds the fragment
        fa[a] = mm < KG_M1 ? sA1[buf][k * KG_LA1 + mm + (lane & 15)]
                           : sA2[buf][k * KG_M2 + mm - KG_M1 + (lane & 15)];
      }
#pragma unroll
      for (int b = 0; b < KG_FB; ++b) fb[b] = sB[buf][k * KG_LB + wn + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < KG_FA; ++a)
#pragma unroll
        for (int b = 0; b < KG_FB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();  // the fence also waits for this wave's copies of the next tile
  }
#pragma unroll
  for (int a = 0; a < KG_FA; ++a)
#pragma unroll
    for (int b = 0; b < KG_FB; ++b) {
      const int n = n0 + wn + 16 * b + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * a + 4 * r + (lane >> 4);
        if (m < M && n < N) C[(size_t)m * N + n] = acc[a][b][r];
      }
    }
}

}  // namespace

void launch_kk_pack(const cplx* R, size_t ldt, int n_g, int n_gp, int n_t, const int* rank,
                    cplx* Rs, hipStream_t st) {
  const dim3 grid((unsigned)((n_t + KP_T - 1) / KP_T), (unsigned)(n_gp / kKkTile));
  hipLaunchKernelGGL(k_kk_pack, grid, dim3(256), 0, st, R, ldt, n_g, n_gp, n_t, rank, Rs);
}

void launch_kk_bin(const cplx* Rs, int n_gp, int n_g, const int* ib, const double* xf,
                   const KkChunk* chunks, int n_chunks, double* S, double* E, hipStream_t st) {
  const int T = n_gp / kKkTile;
  hipLaunchKernelGGL(k_kk_bin, dim3((unsigned)n_chunks, (unsigned)(T * (T + 1) / 2)), dim3(256), 0,
                     st, Rs, n_gp, n_g, ib, xf, chunks, S, E);
  const size_t row_len = (size_t)n_g * (n_g + 1);  // 2 n_pairs
  hipLaunchKernelGGL(k_kk_tail, dim3((unsigned)((row_len + 255) / 256), (unsigned)n_chunks),
                     dim3(256), 0, st, chunks, row_len, E, S);
}

void launch_kk_matrix(const double* w, int n_w, double eta, double d, int nr, int na, int br,
                      int ba, int rows_p, int ldm, double* Kb, hipStream_t st) {
  const long total = (long)rows_p * ldm;
  hipLaunchKernelGGL(k_kk_matrix, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, w, n_w,
                     eta, d, nr, na, br, ba, rows_p, ldm, Kb);
}

int kk_rows_padded(int rows) { return (rows + KG_K - 1) / KG_K * KG_K; }
int kk_ldm(int n_w) { return (2 * n_w + KG_M - 1) / KG_M * KG_M; }
size_t kk_s_slack() { return KG_N; }

void launch_kk_transform(const double* Kb, int ldm, const double* S, int N, int rows_p, int M,
                         double* C, hipStream_t st) {
  const int n_mt = ldm / KG_M, n_nt = (N + KG_N - 1) / KG_N;
  const int total = n_mt * n_nt;
  hipLaunchKernelGGL(k_kk_gemm, dim3((unsigned)(8 * ((total + 7) / 8))), dim3(256), 0, st, Kb, ldm,
                     S, N, rows_p, M, n_mt, n_nt, C);
}

}  // namespace qcx
