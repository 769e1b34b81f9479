// FP64 dielectric matrix, its inverse diagonal and the loss (Eq. eps_LFE,
// Eq. eps_noLFE).
//
// eps_GG' = delta_GG' - v_G v_G' chi0_GG' with v_G = sqrt(4 pi)/|q+G| (the
// symmetrised Coulomb factor of Eq. RPA).  [eps^-1]_GG for every G comes from
// an in-place Gauss-Jordan inversion with partial pivoting on column moduli
// |re| + |im|.  Rows are not swapped: step k picks pivot row p_k among the rows
// not yet used, and at the end [eps^-1]_kk = B[p_k][k'] where k' is the step at
// which row k served as pivot.
#include <limits.h>

#include "common.h"

namespace qcx {

namespace {

// Upper-triangle pair index p -> (G, G'), G <= G', row-major.  Row g starts
// at s(g) = g n - g (g - 1) / 2; the quadratic is inverted in double and the
// rounding fixed by at most a step either way.
__device__ inline void pair_decode(int p, int n_g, int& G, int& Gp) {
  auto start = [&](long gg) { return gg * n_g - gg * (gg - 1) / 2; };
  const double b = 2.0 * n_g + 1.0;
  int g = (int)floor(0.5 * (b - sqrt(fmax(b * b - 8.0 * p, 0.0))));
  g = max(0, min(g, n_g - 1));
  while (g > 0 && start(g) > p) --g;
  while (g + 1 < n_g && start(g + 1) <= p) ++g;
  G = g;
  Gp = g + (int)(p - start(g));
}

// mode 0: eps; mode 1: chi0
__global__ void k_assemble(AsmArgs a, Chi0Geom g, int mode, cplx* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)g.n_w * g.n_pairs) return;
  const int j = (int)(i / g.n_pairs), p = (int)(i % g.n_pairs);
  int G, Gp;
  pair_decode(p, g.n_g, G, Gp);
  double Xr = 0.0, Xi = 0.0, Yr = 0.0, Yi = 0.0;
  if (p < a.n_pairs64) {
    for (int ks = 0; ks < a.ks64; ++ks) {
      const double* x0 = a.XY + ((size_t)ks * a.n_rowsp64 + 2 * j) * a.n_colp64 + 2 * p;
      const double* x1 = x0 + a.n_colp64;
      Xr += x0[0];
      Xi += x0[1];
      Yr += x1[0];
      Yi += x1[1];
    }
  } else if (a.C64) {
    const int b = p - g.p0;
    const size_t r0 = (size_t)(2 * j) * 2, r1 = r0 + 2;
    Xr = a.C64[(r0 + 0) * g.n_bulkp + b];
    Xi = a.C64[(r0 + 1) * g.n_bulkp + b];
    Yr = a.C64[(r1 + 0) * g.n_bulkp + b];
    Yi = a.C64[(r1 + 1) * g.n_bulkp + b];
  } else {
    const int b = p - g.p0;
    for (int ks = 0; ks < a.ks; ++ks) {
      const size_t r0 = ((size_t)ks * g.n_rowsp + 2 * j) * 2;  // row 2j: Re W
      const size_t r1 = r0 + 2;                                 // row 2j+1: Im W
      Xr += (double)a.C[(r0 + 0) * g.n_bulkp + b];
      Xi += (double)a.C[(r0 + 1) * g.n_bulkp + b];
      Yr += (double)a.C[(r1 + 0) * g.n_bulkp + b];
      Yi += (double)a.C[(r1 + 1) * g.n_bulkp + b];
    }
  }
  if (G == Gp) {  // P_t(G, G) = |R_t(G)|^2 is real
    Xi = 0.0;
    Yi = 0.0;
  }
  cplx cab = {a.pref * (Xr - Yi), a.pref * (Xi + Yr)};  // chi0_{G G'}
  cplx cba = {a.pref * (Xr + Yi), a.pref * (Yr - Xi)};  // chi0_{G' G}
  const size_t base = (size_t)j * g.n_g * g.n_g;
  if (mode == 0) {
    const double vv = a.vq[G] * a.vq[Gp];
    cab = {(G == Gp ? 1.0 : 0.0) - vv * cab.re, -vv * cab.im};
    cba = {(G == Gp ? 1.0 : 0.0) - vv * cba.re, -vv * cba.im};
  }
  out[base + (size_t)G * g.n_g + Gp] = cab;
  if (G != Gp) out[base + (size_t)Gp * g.n_g + G] = cba;
}

__device__ inline cplx cinv(cplx a) {
  const double d = 1.0 / (a.re * a.re + a.im * a.im);
  return {a.re * d, -a.im * d};
}

// Register-resident Gauss-Jordan for n <= NTR*RP and n <= 32*CP with 32*NTR
// threads: thread (tr, tc) = (tid / 32, tid % 32) owns rows tr + NTR a and
// columns tc + 32 b; wave w holds row groups 2w and 2w + 1.  Step k (column
// block kb = k / 32 known at compile time):
//   1. the owners of column k propose the largest |re| + |im| among their
//      unused rows; the two proposals of a wave are combined by a shuffle and
//      written to LDS (one entry per wave);
//   -- barrier --
//   2. every wave reduces the proposals itself (same result everywhere, ties
//      to the smaller row), which gives the pivot row p;
//   3. the 32 owners of row p divide it by the pivot (the pivot value comes by
//      shuffle from its owner) and publish w = row p / piv with w_k = 1 / piv;
//      the owners of column k publish u = column k with u_p = piv - 1 and
//      replace column k by e_p;
//   -- barrier --
//   4. every thread applies m <- m - u w^T to its RP x CP block.
// Two barriers per step; the used-row marks live in registers.
template <int RP, int CP, int NTR>
__global__ void __launch_bounds__(32 * NTR) k_gj_reg(const cplx* __restrict__ eps, int n,
                                                     cplx* __restrict__ diag, int* sing) {
  constexpr int NWV = NTR / 2;  // waves
  __shared__ cplx colk[NTR * RP], rowp[32 * CP];
  __shared__ int piv[NTR * RP], sor[NTR * RP];
  __shared__ double cand_v[NWV];
  __shared__ int cand_i[NWV];
  const int tid = threadIdx.x, tr = tid >> 5, tc = tid & 31, lane = tid & 63;
  const cplx* A = eps + (size_t)blockIdx.x * n * n;
  cplx m[RP][CP];
#pragma unroll
  for (int a = 0; a < RP; ++a)
#pragma unroll
    for (int b = 0; b < CP; ++b) {
      const int i = tr + NTR * a, j = tc + 32 * b;
      m[a][b] = (i < n && j < n) ? A[(size_t)i * n + j] : cplx{0.0, 0.0};
    }
  unsigned used = 0;  // bit a: row tr + NTR a already served as pivot
  bool singular = false;
#pragma unroll
  for (int kb = 0; kb < CP; ++kb) {
    for (int kk = 0; kk < 32; ++kk) {
      const int k = 32 * kb + kk;
      if (k >= n) break;
      // 1. proposals from the owners of column k
      double best = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int a = 0; a < RP; ++a) {
        const int i = tr + NTR * a;
        if (i < n && !((used >> a) & 1u)) {
          double mag = fabs(m[a][kb].re) + fabs(m[a][kb].im);
          if (mag != mag) mag = INFINITY;  // a NaN entry still selects a row
          if (mag > best) {
            best = mag;
            bi = i;
          }
        }
      }
      {
        const double ob = __shfl_xor(best, 32, 64);
        const int oi = __shfl_xor(bi, 32, 64);
        if (oi != INT_MAX && (bi == INT_MAX || ob > best || (ob == best && oi < bi))) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == kk) {
        cand_v[tid >> 6] = best;
        cand_i[tid >> 6] = bi;
      }
      __syncthreads();
      // 2. every wave reduces the proposals
      double cb = lane < NWV ? cand_v[lane] : -1.0;
      int ci = lane < NWV ? cand_i[lane] : INT_MAX;
#pragma unroll
      for (int off = NWV / 2; off > 0; off >>= 1) {
        const double ob = __shfl_xor(cb, off, 64);
        const int oi = __shfl_xor(ci, off, 64);
        if (oi != INT_MAX && (ci == INT_MAX || ob > cb || (ob == cb && oi < ci))) {
          cb = ob;
          ci = oi;
        }
      }
      int p = __shfl(ci, 0, 64);
      if (p == INT_MAX) p = 0;  // unreachable: some row is always unused
      const int pa = p / NTR, pt = p - pa * NTR;
      // 3. publish w (row p / piv) and u (column k, u_p = piv - 1)
      if (tr == pt) {
        cplx pv = m[0][kb];
#pragma unroll
        for (int a = 1; a < RP; ++a)
          if (a == pa) pv = m[a][kb];
        // the pivot sits in column k, i.e. with lane tc == kk of this half-wave
        pv.re = __shfl(pv.re, (lane & 32) + kk, 64);
        pv.im = __shfl(pv.im, (lane & 32) + kk, 64);
        if (pv.re == 0.0 && pv.im == 0.0) singular = true;
        const cplx inv = cinv(pv);
#pragma unroll
        for (int b = 0; b < CP; ++b) {
          const int j = tc + 32 * b;
          cplx v = m[0][b];
#pragma unroll
          for (int a = 1; a < RP; ++a)
            if (a == pa) v = m[a][b];
          if (j < n) rowp[j] = (j == k) ? inv : cmul(v, inv);
        }
        if (tc == kk) {
          colk[p] = {pv.re - 1.0, pv.im};
          piv[k] = p;
          sor[p] = k;
        }
      }
      if (tc == kk) {
#pragma unroll
        for (int a = 0; a < RP; ++a) {
          const int i = tr + NTR * a;
          if (i < n && i != p) colk[i] = m[a][kb];
          m[a][kb] = {i == p ? 1.0 : 0.0, 0.0};
        }
      }
      if (pt == tr) used |= 1u << pa;
      __syncthreads();
      // 4. rank-1 update
      cplx wv[CP];
#pragma unroll
      for (int b = 0; b < CP; ++b) {
        const int j = tc + 32 * b;
        wv[b] = j < n ? rowp[j] : cplx{0.0, 0.0};
      }
#pragma unroll
      for (int a = 0; a < RP; ++a) {
        const int i = tr + NTR * a;
        const cplx u = i < n ? colk[i] : cplx{0.0, 0.0};
#pragma unroll
        for (int b = 0; b < CP; ++b) {
          m[a][b].re -= u.re * wv[b].re - u.im * wv[b].im;
          m[a][b].im -= u.re * wv[b].im + u.im * wv[b].re;
        }
      }
    }
  }
  __syncthreads();
  // [eps^-1]_kk = B[piv[k]][sor[k]]
  for (int k = 0; k < n; ++k) {
    const int i = piv[k], j = sor[k];
    if (i % NTR == tr && (j & 31) == tc) {
      cplx v = {0.0, 0.0};
#pragma unroll
      for (int a = 0; a < RP; ++a)
#pragma unroll
        for (int b = 0; b < CP; ++b)
          if (a == i / NTR && b == (j >> 5)) v = m[a][b];
      diag[(size_t)blockIdx.x * n + k] = v;
    }
  }
  if (singular) atomicMin(sing, (int)blockIdx.x);
}

// Blocked Gauss-Jordan for n > 128 (one block of 256 threads per matrix; the
// matrix stays in global memory).  Columns are processed in panels of MB: the
// MB pivot steps are applied to the n x MB panel in LDS only (same pivots as the
// unblocked sweep, which depends on the panel columns alone), the panel is
// written back, and the remaining columns J receive the combined rank-MB
// update  T[:, J] += Z Y  with Y = T[P][J] (pivot rows, before the update) and
// Z = panel with 1 subtracted at (p_a, a), which turns the pivot rows into
// B^-1 Y and the others into T - T[:,K] B^-1 Y.
constexpr int GJ_YT = 32;  // trailing-update column tile

__device__ inline void block_argmax(double v, int i, double* redv, int* redi, int* out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (oi != INT_MAX && (i == INT_MAX || ov > v || (ov == v && oi < i))) {
      v = ov;
      i = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    redv[wave] = v;
    redi[wave] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = -1.0;
    int bi = INT_MAX;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      if (redi[w] == INT_MAX) continue;
      if (bi == INT_MAX || redv[w] > b || (redv[w] == b && redi[w] < bi)) {
        b = redv[w];
        bi = redi[w];
      }
    }
    *out = bi == INT_MAX ? 0 : bi;
  }
}

template <int MB>
__global__ void __launch_bounds__(256) k_gj_blocked(cplx* __restrict__ eps, int n,
                                                    cplx* __restrict__ diag, int* sing) {
  extern __shared__ char smem[];
  cplx* panel = reinterpret_cast<cplx*>(smem);  // [n][MB]
  cplx* ucol = panel + (size_t)n * MB;            // [n]
  cplx* wrow = ucol + n;                          // [MB]
  cplx* ytile = wrow + MB;                        // [MB][GJ_YT]
  int* used = reinterpret_cast<int*>(ytile + MB * GJ_YT);
  int* piv = used + n;
  int* sor = piv + n;
  int* pb = sor + n;  // [MB] pivot rows of the current panel
  __shared__ double redv[4];
  __shared__ int redi[4];
  __shared__ int pivrow;
  cplx* A = eps + (size_t)blockIdx.x * n * n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n; i += 256) used[i] = 0;
  bool singular = false;
  for (int k0 = 0; k0 < n; k0 += MB) {
    const int mb = min(MB, n - k0);
    __syncthreads();
    for (int e = tid; e < n * mb; e += 256) {
      const int i = e / mb, c = e % mb;
      panel[i * MB + c] = A[(size_t)i * n + k0 + c];
    }
    __syncthreads();
    for (int kk = 0; kk < mb; ++kk) {
      double best = -1.0;
      int bi = INT_MAX;
      for (int i = tid; i < n; i += 256) {
        if (used[i]) continue;
        const cplx v = panel[i * MB + kk];
        double mag = fabs(v.re) + fabs(v.im);
        if (mag != mag) mag = INFINITY;
        if (mag > best) {
          best = mag;
          bi = i;
        }
      }
      block_argmax(best, bi, redv, redi, &pivrow);
      if (tid == 0) {
        const int p = pivrow;
        used[p] = 1;
        piv[k0 + kk] = p;
        sor[p] = k0 + kk;
        pb[kk] = p;
      }
      __syncthreads();
      const int p = pivrow;
      for (int i = tid; i < n; i += 256) ucol[i] = panel[i * MB + kk];
      for (int c = tid; c < mb; c += 256) wrow[c] = panel[p * MB + c];
      __syncthreads();
      const cplx pv = wrow[kk];
      if (pv.re == 0.0 && pv.im == 0.0) singular = true;
      const cplx inv = cinv(pv);
      for (int e = tid; e < n * mb; e += 256) {
        const int i = e / mb, c = e % mb;
        cplx u = ucol[i];
        if (i == p) u.re -= 1.0;
        const cplx w = (c == kk) ? inv : cmul(wrow[c], inv);
        cplx v = (c == kk) ? cplx{i == p ? 1.0 : 0.0, 0.0} : panel[i * MB + c];
        v.re -= u.re * w.re - u.im * w.im;
        v.im -= u.re * w.im + u.im * w.re;
        panel[i * MB + c] = v;
      }
      __syncthreads();
    }
    // write the swept panel back, then form Z in LDS
    for (int e = tid; e < n * mb; e += 256) {
      const int i = e / mb, c = e % mb;
      A[(size_t)i * n + k0 + c] = panel[i * MB + c];
    }
    __syncthreads();
    if (tid < mb) panel[pb[tid] * MB + tid].re -= 1.0;
    __syncthreads();
    // trailing update over column tiles outside the panel
    const int c = lane & 31;                 // column inside the tile
    const int g = 2 * wave + (lane >> 5);    // row group 0..7
    for (int jt = 0; jt < n; jt += GJ_YT) {
      const int j = jt + c;
      const bool col_ok = j < n && (j < k0 || j >= k0 + mb);
      {  // tiles that overlap the panel are processed with those columns masked
        for (int e = tid; e < mb * GJ_YT; e += 256) {
          const int a = e / GJ_YT, cc = e % GJ_YT;
          const int jj = jt + cc;
          ytile[e] = (jj < n) ? A[(size_t)pb[a] * n + jj] : cplx{0.0, 0.0};
        }
        __syncthreads();
        for (int i0 = 0; i0 < n; i0 += 32) {
          cplx acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
          for (int a = 0; a < mb; ++a) {
            const cplx y = ytile[a * GJ_YT + c];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = i0 + g + 8 * r;
              const cplx z = (i < n) ? panel[i * MB + a] : cplx{0.0, 0.0};
              acc[r].re += z.re * y.re - z.im * y.im;
              acc[r].im += z.re * y.im + z.im * y.re;
            }
          }
          if (col_ok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = i0 + g + 8 * r;
              if (i < n) {
                cplx t = A[(size_t)i * n + j];
                t.re += acc[r].re;
                t.im += acc[r].im;
                A[(size_t)i * n + j] = t;
              }
            }
          }
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256) diag[(size_t)blockIdx.x * n + k] = A[(size_t)piv[k] * n + sor[k]];
  if (singular && tid == 0) atomicMin(sing, (int)blockIdx.x);
}

size_t gj_blocked_lds(int n, int mb) {
  return sizeof(cplx) * ((size_t)n * mb + n + mb + (size_t)mb * GJ_YT) + sizeof(int) * (3 * (size_t)n + mb);
}

__global__ void k_nolfe(const cplx* eps, int n, int n_w, cplx* diag, int* sing) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * n_w) return;
  const int j = (int)(i / n), G = (int)(i % n);
  const cplx e = eps[((size_t)j * n + G) * n + G];
  if (e.re == 0.0 && e.im == 0.0) atomicMin(sing, j);
  diag[i] = cinv(e);
}

__global__ void k_loss(const cplx* diag, int n, int n_w, double* loss, cplx* epsM) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * n_w) return;
  const cplx d = diag[i];
  loss[i] = -d.im;
  if (i % n == 0) epsM[i / n] = cinv(d);
}

__global__ void k_rho_export(const cplx* R, size_t ldt, int n_g, int n_t, cplx* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_g * n_t) return;
  const int t = (int)(i / n_g), g = (int)(i % n_g);
  out[i] = R[(size_t)g * ldt + t];
}

}  // namespace

void launch_eps_assemble(const AsmArgs& a, const Chi0Geom& g, cplx* eps, hipStream_t st) {
  const long total = (long)g.n_w * g.n_pairs;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, g, 0,
                     eps);
}

void launch_chi0_export(const AsmArgs& a, const Chi0Geom& g, cplx* chi, hipStream_t st) {
  const long total = (long)g.n_w * g.n_pairs;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, g, 1,
                     chi);
}

void launch_gj_diag(cplx* eps, int n_g, int n_w, cplx* diag, int* sing, hipStream_t st) {
  if (n_g <= 64)
    hipLaunchKernelGGL((k_gj_reg<2, 2, 32>), dim3(n_w), dim3(1024), 0, st, eps, n_g, diag, sing);
  else if (n_g <= 128)
    hipLaunchKernelGGL((k_gj_reg<4, 4, 32>), dim3(n_w), dim3(1024), 0, st, eps, n_g, diag, sing);
  else if (gj_blocked_lds(n_g, 32) <= 160 * 1024)
    hipLaunchKernelGGL(k_gj_blocked<32>, dim3(n_w), dim3(256), gj_blocked_lds(n_g, 32), st, eps,
                       n_g, diag, sing);
  else if (gj_blocked_lds(n_g, 16) <= 160 * 1024)
    hipLaunchKernelGGL(k_gj_blocked<16>, dim3(n_w), dim3(256), gj_blocked_lds(n_g, 16), st, eps,
                       n_g, diag, sing);
  else
    hipLaunchKernelGGL(k_gj_blocked<8>, dim3(n_w), dim3(256), gj_blocked_lds(n_g, 8), st, eps,
                       n_g, diag, sing);
}

void launch_nolfe_diag(const cplx* eps, int n_g, int n_w, cplx* diag, int* sing, hipStream_t st) {
  const long total = (long)n_g * n_w;
  hipLaunchKernelGGL(k_nolfe, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, eps, n_g,
                     n_w, diag, sing);
}

void launch_loss(const cplx* diag, int n_g, int n_w, double* loss, cplx* epsM, hipStream_t st) {
  const long total = (long)n_g * n_w;
  hipLaunchKernelGGL(k_loss, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, diag, n_g,
                     n_w, loss, epsM);
}

void launch_rho_export(const cplx* R, size_t ldt, int n_g, int n_t, cplx* out, hipStream_t st) {
  const long total = (long)n_g * n_t;
  hipLaunchKernelGGL(k_rho_export, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, R, ldt,
                     n_g, n_t, out);
}

}  // namespace qcx
