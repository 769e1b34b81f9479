// Head and wings of chi0 (the pairs (0, G'), Eq. (RPA)) in FP64 for the
// mixed-precision paths: the contraction over the transitions as one FP64
// GEMM on MFMA with a per-q table of the pair products.
#include <algorithm>

#include "common.h"

namespace qcx {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------- head and wings, FP64
// The head/wing pairs (0, G') as one FP64 GEMM over the transitions,
//   XY[z][row][col] = sum over t in split z of A[t][row] P[t][col],
// rows (Re W(w_j), Im W(w_j)), columns (Re P, Im P) of each pair.  P is laid
// out per q as a table [t][col] (k_hw_ptable), so that its tiles stream in
// 1 KB rows straight into LDS; A is formed from the energies in FP64 while the
// previous tile's MFMAs run (frequencies loaded once, transition energies
// one tile ahead).  A block of 256 threads owns HW_M rows x HW_N
// columns of one split; its four waves own HW_M / 2 x HW_N / 2 each (5 x 4
// tiles of v_mfma_f64_16x16x4f64, 160 accumulator registers), tiles of HW_K
// transitions go through two LDS buffers with one barrier each, LDS rows
// padded by 16 doubles against bank conflicts; two blocks per CU.  Blocks of
// one split are placed on one XCD, so its P rows are read from memory once.
constexpr int HW_M = 160, HW_N = 128, HW_K = 16;
constexpr int HW_LA = HW_M + 16, HW_LB = HW_N + 16;
constexpr int HW_FA = HW_M / 32, HW_FB = HW_N / 32;
constexpr int HW_WA = HW_K * HW_M / 2 / 256;  // weights per thread per tile: 5
typedef __attribute__((address_space(3))) void* hw_lds_t;

// P[t][2p + ri] for t < n_tk (zero past n_t) and columns < n_colp (a
// multiple of 64; zero past 2 n_ps): a block does 64 transitions x 32 pairs,
// reading both R rows of each pair along t and writing P rows along the
// columns.
__global__ void __launch_bounds__(256) k_hw_ptable(const cplx* __restrict__ R, size_t ldt,
                                                   const int* __restrict__ pairs, int n_ps,
                                                   int n_t, int n_tk, int n_colp,
                                                   double* __restrict__ P) {
  __shared__ double tile[64][65];
  const int t0 = blockIdx.x * 64, p0 = blockIdx.y * 32;
  const int tt = threadIdx.x & 63;
  for (int pp = threadIdx.x >> 6; pp < 32; pp += 4) {
    const int p = p0 + pp, t = t0 + tt;
    double re = 0.0, im = 0.0;
    if (p < n_ps && t < n_t) {
      const int pk = pairs[p];
      const cplx a = R[(size_t)(pk & 0xffff) * ldt + t];
      const cplx b = R[(size_t)(pk >> 16) * ldt + t];
      re = a.re * b.re + a.im * b.im;
      im = a.re * b.im - a.im * b.re;
    }
    tile[tt][2 * pp] = re;
    tile[tt][2 * pp + 1] = im;
  }
  __syncthreads();
  const int c = threadIdx.x & 63;
  for (int r = threadIdx.x >> 6; r < 64 && t0 + r < n_tk; r += 4)
    P[(size_t)(t0 + r) * n_colp + 2 * p0 + c] = tile[r][c];
}

// 1/d from a single-precision estimate refined by two Newton steps in FP64
// (24 -> 48 -> 96 bits: the FP64 reciprocal to within an ulp) with fewer
// dependent FP64 instructions than the IEEE division, which here shares the
// FP64 pipe with the MFMAs; outside the single-precision range, the division.
__device__ inline double recip_nr(double d) {
  if (!(d > 1e-30 && d < 1e30)) return 1.0 / d;
  double r = (double)__builtin_amdgcn_rcpf((float)d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Two waves per SIMD (two blocks per CU): the register budget is 256, so the
// accumulators sit in the same file as the operands.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_hw_gemm(const double* __restrict__ w, const double* __restrict__ dt, double eta, int n_w, int n_t,
          const double* __restrict__ P, int n_rowsp, int n_colp, int kper, int ks,
          double* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) double sA[2][HW_K * HW_LA];
  __shared__ __attribute__((aligned(16))) double sB[2][HW_K * HW_LB];
  const int n_mt = n_rowsp / HW_M, n_nt = n_colp / HW_N, tiles = n_mt * n_nt;
  const int total = tiles * ks, per = (total + 7) / 8;
  const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= total) return;
  const int z = logical / tiles, tile = logical % tiles;
  const int m0 = (tile % n_mt) * HW_M, n0 = (tile / n_mt) * HW_N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (HW_M / 2), wn = (wave & 1) * (HW_N / 2);
  const int kb = z * kper;
  f64x4 acc[HW_FA][HW_FB];
#pragma unroll
  for (int a = 0; a < HW_FA; ++a)
#pragma unroll
    for (int b = 0; b < HW_FB; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // This thread's weights of a tile: (tt, jj) = (e / 80, e % 80) for
  // e = tid + 256 i, the same positions in every tile; w_j is loaded once,
  // the transition energies one tile ahead.
  double wj[HW_WA], dn[HW_WA];
  const int th = n_t / 2;
#pragma unroll
  for (int i = 0; i < HW_WA; ++i) {
    const int e = tid + 256 * i, jj = e % (HW_M / 2);
    wj[i] = m0 / 2 + jj < n_w ? w[m0 / 2 + jj] : 0.0;
  }
  auto load_dt = [&](int k0) {
#pragma unroll
    for (int i = 0; i < HW_WA; ++i) {
      const int t = k0 + (tid + 256 * i) / (HW_M / 2);
      dn[i] = t < n_t ? dt[t] : 0.0;
    }
  };
  // tile k0 into buffer buf: P rows by DMA (one 1 KB row per wave
  // instruction), the weights from dn (the energies of tile k0)
  auto fill = [&](int k0, int buf) {
#pragma unroll
    for (int i = 0; i < HW_K / 4; ++i) {
      const int r = wave + 4 * i;
      __builtin_amdgcn_global_load_lds((const void*)(P + (size_t)(k0 + r) * n_colp + n0 + 2 * lane),
                                       (hw_lds_t)(&sB[buf][r * HW_LB]), 16, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < HW_WA; ++i) {
      const int e = tid + 256 * i, tt = e / (HW_M / 2), jj = e % (HW_M / 2);
      const int t = k0 + tt;
      double re = 0.0, im = 0.0;
      if (t < n_t && m0 / 2 + jj < n_w) {  // W_t(w_j) = 1 / (s_t w_j - D_t + i eta)
        const double x = (t < th ? wj[i] : -wj[i]) - dn[i];
        const double r = recip_nr(x * x + eta * eta);
        re = x * r;
        im = -eta * r;
      }
      *reinterpret_cast<double2*>(&sA[buf][tt * HW_LA + 2 * jj]) = make_double2(re, im);
    }
  };
  const int nk = kper / HW_K;
  load_dt(kb);
  fill(kb, 0);
  if (nk > 1) load_dt(kb + HW_K);
  __syncthreads();  // its fence waits for the copies into LDS as well
  for (int s = 0; s < nk; ++s) {
    const int buf = s & 1;
    if (s + 1 < nk) {
      fill(kb + (s + 1) * HW_K, buf ^ 1);
      if (s + 2 < nk) load_dt(kb + (s + 2) * HW_K);
    }
#pragma unroll
    for (int kk = 0; kk < HW_K; kk += 4) {
      const int k = kk + (lane >> 4);
      double fa[HW_FA], fb[HW_FB];
#pragma unroll
      for (int a = 0; a < HW_FA; ++a) fa[a] = sA[buf][k * HW_LA + wm + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < HW_FB; ++b) fb[b] = sB[buf][k * HW_LB + wn + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < HW_FA; ++a)
#pragma unroll
        for (int b = 0; b < HW_FB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  double* o = out + (size_t)z * n_rowsp * n_colp;
#pragma unroll
  for (int a = 0; a < HW_FA; ++a)
#pragma unroll
    for (int b = 0; b < HW_FB; ++b) {
      const int n = n0 + wn + 16 * b + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * a + 4 * r + (lane >> 4);
        o[(size_t)m * n_colp + n] = acc[a][b][r];
      }
    }
}

}  // namespace

void geom_hw_init(Geom64& g, int n_g, int n_w, int n_t, int n_ps, size_t max_bytes) {
  g.n_g = n_g;
  g.n_w = n_w;
  g.n_t = n_t;
  g.n_ps = n_ps;
  g.n_rowsp = (2 * n_w + HW_M - 1) / HW_M * HW_M;
  g.n_colp = (2 * n_ps + HW_N - 1) / HW_N * HW_N;
  const int tiles = (g.n_rowsp / HW_M) * (g.n_colp / HW_N);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int slots = 2 * cus;                       // two blocks per CU (80 KB of LDS each)
  const int steps = std::max(1, (n_t + HW_K - 1) / HW_K);
  const size_t split_bytes = (size_t)g.n_rowsp * g.n_colp * sizeof(double);
  // fill the slots in one round, at least 8 tiles of HW_K per split
  int ks = std::max(1, std::min(slots / std::max(1, tiles), steps / 8));
  while (ks > 1 && (size_t)ks * split_bytes > max_bytes) --ks;
  const int per = (steps + ks - 1) / ks;
  g.ksplit = (steps + per - 1) / per;
  g.chunk_t = per * HW_K;
}

size_t hw_ptable_doubles(const Geom64& g) { return (size_t)g.ksplit * g.chunk_t * g.n_colp; }

void launch_headwings_f64(const cplx* R, size_t ldt, const double* w, const double* dt, double eta,
                          const Geom64& g, const int* pairs, double* P, double* out,
                          hipStream_t st) {
  const int n_tk = g.ksplit * g.chunk_t;
  hipLaunchKernelGGL(k_hw_ptable, dim3((unsigned)((n_tk + 63) / 64), (unsigned)(g.n_colp / 64)),
                     dim3(256), 0, st, R, ldt, pairs, g.n_ps, g.n_t, n_tk, g.n_colp, P);
  const int tiles = (g.n_rowsp / HW_M) * (g.n_colp / HW_N);
  const int total = tiles * g.ksplit;
  hipLaunchKernelGGL(k_hw_gemm, dim3((unsigned)(8 * ((total + 7) / 8))), dim3(256), 0, st, w, dt,
                     eta, g.n_w, g.n_t, P, g.n_rowsp, g.n_colp, g.chunk_t, g.ksplit, out);
}

}  // namespace qcx
