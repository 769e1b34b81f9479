// Kramers-Kronig route of Sec. II.D: the spectral part of Eq. (RPA) is binned
// (k_bulk with hat-function weights, see launch_hat_weights) and the full
// response at each frequency follows from the binned spectral function by a
// linear transform:
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
#include "common.h"

namespace qcx {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

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

// Transform matrix Kt[2 n_w (padded m_p)][n_rowsp]: row 2j = Re, 2j + 1 = Im of
// the kernel of frequency w_j for bin column c (resonant bins, then
// anti-resonant bins, then zero padding).
__global__ void k_kk_matrix(const double* __restrict__ w, int n_w, double eta, double d, int nr,
                            int na, int b0r, int b0a, int n_cols, int m_p, double* __restrict__ Kt) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)m_p * n_cols) return;
  const int row = (int)(i / n_cols), c = (int)(i % n_cols);
  const int j = row >> 1, ri = row & 1;
  double v = 0.0;
  if (j < n_w && c < nr + na) {
    c64 k;
    if (c < nr) {  // resonant: K(w - w_b + i eta), limit from above at eta = 0
      const double wb = (b0r + c) * d;
      k = hat_kernel({(w[j] - wb) / d, eta / d});
    } else {       // anti-resonant: -K(w + w_b - i eta), limit from below
      const double wb = (b0a + c - nr) * d;
      k = hat_kernel({(w[j] + wb) / d, eta > 0.0 ? -eta / d : -0.0});
      k = {-k.re, -k.im};
    }
    v = (ri ? k.im : k.re) / d;
  }
  Kt[i] = v;
}

// C[M][N] = A[M][K] B[K][N] (row-major FP64) on FP64 MFMA 16x16x4: block
// 64 x 64 of C, wave 32 x 32 (2 x 2 tiles), K staged 16 at a time k-major in
// LDS.  Layouts: A 16x4, lane l holds A[l%16][l/16]; B 4x16, lane l holds
// B[l/16][l%16]; D 16x16, lane l holds D[4r + l/16][l%16].
__global__ void __launch_bounds__(256) k_gemm64(const double* __restrict__ A, int lda,
                                                const double* __restrict__ B, int ldb,
                                                double* __restrict__ C, int ldc, int M, int N, int K) {
  __shared__ double sA[16][65], sB[16][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = 32 * (w >> 1), wn = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += 256) {
      const int m = e >> 4, kk = e & 15;  // A: consecutive threads along k
      const int gm = m0 + m, gk = k0 + kk;
      sA[kk][m] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.0;
      const int kb = e >> 6, n = e & 63;  // B: consecutive threads along n
      const int gkb = k0 + kb, gn = n0 + n;
      sB[kb][n] = (gkb < K && gn < N) ? B[(size_t)gkb * ldb + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[kk + lk][wm + 16 * t + li];
        b[t] = sB[kk + lk][wn + 16 * t + li];
      }
#pragma unroll
      for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[ra][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ra], b[cb], acc[ra][cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ra = 0; ra < 2; ++ra)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * ra + 4 * r + lk, gn = n0 + wn + 16 * cb + li;
        if (gm < M && gn < N) C[(size_t)gm * ldc + gn] = acc[ra][cb][r];
      }
}

}  // namespace

void launch_kk_matrix(const double* w, int n_w, double eta, double d, int nr, int na, int b0r,
                      int b0a, int n_cols, int m_p, double* Kt, hipStream_t st) {
  const long total = (long)m_p * n_cols;
  hipLaunchKernelGGL(k_kk_matrix, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, w, n_w,
                     eta, d, nr, na, b0r, b0a, n_cols, m_p, Kt);
}

void launch_gemm64(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int M,
                   int N, int K, hipStream_t st) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K);
}

}  // namespace qcx
