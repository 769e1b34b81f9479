// Pair densities of Eq. (RPA) from Gaussian-type-orbital Bloch states.
//
// rho_vck(Q) = <c,k+q| e^{iQ.r} |v,k> = sum_{mu nu} C_mu,c(k+q)^* M_mu,nu(k;Q) C_nu,v(k),
// M_mu,nu(k;Q) = sum_T e^{ik.T} F_mu,nu(Q,T),
// F_mu,nu(Q,T) = int chi_mu(r - A_mu) e^{iQ.r} chi_nu(r - A_nu - T) d^3r.
//
// F is evaluated by the McMurchie-Davidson Hermite expansion: per axis the
// product of the two Cartesian Gaussians is K_x sum_t E^{ij}_t Lambda_t(x) with
// Lambda_t = d^t/dP^t e^{-p (x-P)^2}, whose Fourier transform is
// sqrt(pi/p) e^{-Q^2/4p} (iQ)^t e^{iQP}.
//
// Per q: cell_ft (one thread per shell pair, Q and cell, G-major output); then
// the Bloch sum and the band
// contraction in one pass (k_rho_fused.hip, M in LDS only) whenever the
// basis and the valence bands fit its tiles.  Otherwise the 27-cell Bloch sum
// M(k;Q) runs here (phase_sum, also used for the overlaps S(k)) in k chunks,
// followed by the band contraction (one block per k and G tile; C(k), C(k+q)
// and M(k;Q) tiles staged in LDS), valence side first (k_band_vf) or ket side
// first (k_band_contract), whichever needs fewer multiply-adds.
#include <algorithm>
#include <utility>

#include "common.h"

namespace qcx {

namespace {

// Cartesian monomials per l: l=0: 1; l=1: x, y, z; l=2: xx, xy, xz, yy, yz, zz.
__device__ __constant__ int kCartPow[10][3] = {
    {0, 0, 0},                                                    // s
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},                              // p
    {2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}  // d
};

template <int L>
struct Shape;
template <>
struct Shape<0> {
  static constexpr int ncart = 1, nsph = 1, first = 0;
};
template <>
struct Shape<1> {
  static constexpr int ncart = 3, nsph = 3, first = 1;
};
template <>
struct Shape<2> {
  static constexpr int ncart = 6, nsph = 5, first = 4;
};

// Real solid harmonics as combinations of the Cartesian monomials above,
// without the radial normalisation.
__device__ inline double sph_coef(int l, int m, int c) {
  if (l < 2) return (m == c) ? 1.0 : 0.0;
  const double h = 0.28867513459481288225;  // 1/(2 sqrt 3)
  switch (m) {
    case 0: return c == 1 ? 1.0 : 0.0;                              // xy
    case 1: return c == 4 ? 1.0 : 0.0;                              // yz
    case 2: return c == 5 ? 2.0 * h : ((c == 0 || c == 3) ? -h : 0.0);  // 2zz - xx - yy
    case 3: return c == 2 ? 1.0 : 0.0;                              // xz
    default: return c == 0 ? 0.5 : (c == 3 ? -0.5 : 0.0);           // (xx - yy)/2
  }
}

// Normalisation of a unit-norm primitive of angular momentum l.
__device__ inline double prim_norm(int l, double a) {
  double g = pow(2.0 * a / kPi, 0.75);
  if (l == 1) return g * sqrt(4.0 * a);
  if (l == 2) return g * 4.0 * a;
  return g;
}

// Hermite coefficients E^{ij}_t for one axis, i <= LA, j <= LB, t <= LA+LB,
// and the per-axis integral J[i][j] = sum_t E^{ij}_t (iQ)^t (without the
// common Gaussian factors).
template <int LA, int LB>
__device__ inline void axis_j(double xpa, double xpb, double i2p, double qx,
                              cplx (&J)[LA + 1][LB + 1]) {
  constexpr int TM = LA + LB + 1;
  double E[LA + 1][LB + 1][TM + 1];
#pragma unroll
  for (int i = 0; i <= LA; ++i)
#pragma unroll
    for (int j = 0; j <= LB; ++j)
#pragma unroll
      for (int t = 0; t <= TM; ++t) E[i][j][t] = 0.0;
  E[0][0][0] = 1.0;
#pragma unroll
  for (int i = 0; i <= LA; ++i) {
#pragma unroll
    for (int j = 0; j <= LB; ++j) {
      if (i == 0 && j == 0) continue;
      if (j == 0) {  // raise i
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          double v = xpa * E[i - 1][0][t] + (t + 1) * E[i - 1][0][t + 1];
          if (t > 0) v += i2p * E[i - 1][0][t - 1];
          E[i][0][t] = v;
        }
      } else {  // raise j
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          double v = xpb * E[i][j - 1][t] + (t + 1) * E[i][j - 1][t + 1];
          if (t > 0) v += i2p * E[i][j - 1][t - 1];
          E[i][j][t] = v;
        }
      }
    }
  }
  // (iQ)^t: 1, iQ, -Q^2, -iQ^3, Q^4
  double qp[TM];
  qp[0] = 1.0;
#pragma unroll
  for (int t = 1; t < TM; ++t) qp[t] = qp[t - 1] * qx;
#pragma unroll
  for (int i = 0; i <= LA; ++i)
#pragma unroll
    for (int j = 0; j <= LB; ++j) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int t = 0; t <= i + j; ++t) {
        double v = E[i][j][t] * qp[t];
        switch (t & 3) {
          case 0: re += v; break;
          case 1: im += v; break;
          case 2: re -= v; break;
          default: im -= v; break;
        }
      }
      J[i][j] = {re, im};
    }
}

template <int LA, int LB>
__device__ void pair_block(double a, double b, const double* A, const double* B, const double* Q,
                           cplx* out, int ld) {
  const double p = a + b, ip = 1.0 / p, i2p = 0.5 * ip;
  double P[3], ab2 = 0.0, q2 = 0.0, qp = 0.0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    P[x] = (a * A[x] + b * B[x]) * ip;
    double d = A[x] - B[x];
    ab2 += d * d;
    q2 += Q[x] * Q[x];
    qp += Q[x] * P[x];
  }
  // common factor (pi/p)^{3/2} K e^{-Q^2/4p} e^{iQ.P}
  double mag = pow(kPi * ip, 1.5) * exp(-a * b * ip * ab2 - 0.25 * q2 * ip);
  double s, c;
  sincos(qp, &s, &c);
  const cplx pref = {mag * c, mag * s};

  cplx Jx[LA + 1][LB + 1], Jy[LA + 1][LB + 1], Jz[LA + 1][LB + 1];
  axis_j<LA, LB>(P[0] - A[0], P[0] - B[0], i2p, Q[0], Jx);
  axis_j<LA, LB>(P[1] - A[1], P[1] - B[1], i2p, Q[1], Jy);
  axis_j<LA, LB>(P[2] - A[2], P[2] - B[2], i2p, Q[2], Jz);

  constexpr int NCA = Shape<LA>::ncart, NCB = Shape<LB>::ncart;
  constexpr int NSA = Shape<LA>::nsph, NSB = Shape<LB>::nsph;
  cplx cart[NCA][NCB];
#pragma unroll
  for (int ca = 0; ca < NCA; ++ca) {
    const int* pa = kCartPow[Shape<LA>::first + ca];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int* pb = kCartPow[Shape<LB>::first + cb];
      cart[ca][cb] = cmul(cmul(Jx[pa[0]][pb[0]], Jy[pa[1]][pb[1]]), Jz[pa[2]][pb[2]]);
    }
  }
  const double nn = prim_norm(LA, a) * prim_norm(LB, b);
#pragma unroll
  for (int ma = 0; ma < NSA; ++ma) {
    cplx tmp[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int ca = 0; ca < NCA; ++ca) {
        double w = sph_coef(LA, ma, ca);
        re += w * cart[ca][cb].re;
        im += w * cart[ca][cb].im;
      }
      tmp[cb] = {re, im};
    }
#pragma unroll
    for (int mb = 0; mb < NSB; ++mb) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        double w = sph_coef(LB, mb, cb);
        re += w * tmp[cb].re;
        im += w * tmp[cb].im;
      }
      cplx r = cmul({re * nn, im * nn}, pref);
      out[ma * ld + mb] = r;
    }
  }
}

// One thread per (shell pair, Q, cell T), cells fastest: F[Q][T][mu][nu]
// (G-major, the layout the Bloch sum reads per G).  The Hermite evaluation of
// a d-d pair needs the whole register file, so the kernel runs one wave per
// SIMD; staging whole slabs through LDS (one block per (Q, T)) left most
// lanes idle at the barrier and took 4x longer, so every thread writes its
// shell pair's block directly.
__global__ void __launch_bounds__(256) k_cell_ft(ShellTab sh, const int* __restrict__ pair_order,
                                                 const double* __restrict__ tvec, int n_t,
                                                 const double* __restrict__ Q, int n_q,
                                                 cplx* __restrict__ F) {
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per_pair = (long)n_t * n_q;
  if (tid >= per_pair * sh.n_sh * sh.n_sh) return;
  const int sp = pair_order[tid / per_pair];
  const int rem = (int)(tid % per_pair);
  const int g = rem / n_t, it = rem % n_t;
  const int sa = sp / sh.n_sh, sb = sp % sh.n_sh;
  const double a = sh.ex[sa], b = sh.ex[sb];
  double A[3], B[3], q[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    A[x] = sh.ctr[3 * sa + x];
    B[x] = sh.ctr[3 * sb + x] + tvec[3 * it + x];
    q[x] = Q[3 * g + x];
  }
  const int n = sh.n_ao;
  cplx* out = F + ((size_t)g * n_t + it) * n * n + (size_t)sh.off[sa] * n + sh.off[sb];
  switch (sh.l[sa] * 3 + sh.l[sb]) {
    case 0: pair_block<0, 0>(a, b, A, B, q, out, n); break;
    case 1: pair_block<0, 1>(a, b, A, B, q, out, n); break;
    case 2: pair_block<0, 2>(a, b, A, B, q, out, n); break;
    case 3: pair_block<1, 0>(a, b, A, B, q, out, n); break;
    case 4: pair_block<1, 1>(a, b, A, B, q, out, n); break;
    case 5: pair_block<1, 2>(a, b, A, B, q, out, n); break;
    case 6: pair_block<2, 0>(a, b, A, B, q, out, n); break;
    case 7: pair_block<2, 1>(a, b, A, B, q, out, n); break;
    default: pair_block<2, 2>(a, b, A, B, q, out, n); break;
  }
}

// Gradient integrals of App. C, <chi_mu| d/dr_c |chi_nu(. - T)>: at Q = 0 the
// axis integrals are the Hermite overlaps S[i][j] = E^{ij}_0 (times the common
// factor), and d/dx of the ket's (x - B_x)^j e^{-b (x - B_x)^2} gives the
// axis factor j S[i][j-1] - 2 b S[i][j+1]; the other axes keep S.
template <int LA, int LB>
__device__ void pair_grad(double a, double b, const double* A, const double* B, double* out,
                          int ld, size_t cstride) {
  const double p = a + b, ip = 1.0 / p, i2p = 0.5 * ip;
  double P[3], ab2 = 0.0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    P[x] = (a * A[x] + b * B[x]) * ip;
    const double d = A[x] - B[x];
    ab2 += d * d;
  }
  const double mag = pow(kPi * ip, 1.5) * exp(-a * b * ip * ab2);
  double S[3][LA + 1][LB + 2], G[3][LA + 1][LB + 1];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    cplx J[LA + 1][LB + 2];
    axis_j<LA, LB + 1>(P[x] - A[x], P[x] - B[x], i2p, 0.0, J);
#pragma unroll
    for (int i = 0; i <= LA; ++i) {
#pragma unroll
      for (int j = 0; j <= LB + 1; ++j) S[x][i][j] = J[i][j].re;
#pragma unroll
      for (int j = 0; j <= LB; ++j) G[x][i][j] = (j > 0 ? j * S[x][i][j - 1] : 0.0) - 2.0 * b * S[x][i][j + 1];
    }
  }
  constexpr int NCA = Shape<LA>::ncart, NCB = Shape<LB>::ncart;
  constexpr int NSA = Shape<LA>::nsph, NSB = Shape<LB>::nsph;
  const double nn = prim_norm(LA, a) * prim_norm(LB, b) * mag;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double cart[NCA][NCB];
#pragma unroll
    for (int ca = 0; ca < NCA; ++ca) {
      const int* pa = kCartPow[Shape<LA>::first + ca];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int* pb = kCartPow[Shape<LB>::first + cb];
        double v = 1.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) v *= (x == c) ? G[x][pa[x]][pb[x]] : S[x][pa[x]][pb[x]];
        cart[ca][cb] = v;
      }
    }
#pragma unroll
    for (int ma = 0; ma < NSA; ++ma) {
      double tmp[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        double r = 0.0;
#pragma unroll
        for (int ca = 0; ca < NCA; ++ca) r += sph_coef(LA, ma, ca) * cart[ca][cb];
        tmp[cb] = r;
      }
#pragma unroll
      for (int mb = 0; mb < NSB; ++mb) {
        double r = 0.0;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) r += sph_coef(LB, mb, cb) * tmp[cb];
        // stored as complex (imaginary part 0) so the Bloch sum of the
        // overlap path applies unchanged
        out[2 * (c * cstride + (size_t)ma * ld + mb)] = r * nn;
        out[2 * (c * cstride + (size_t)ma * ld + mb) + 1] = 0.0;
      }
    }
  }
}

// One thread per (shell pair, cell): D[c][T][mu][nu], c = x, y, z (the
// components take the place of the G list of F).
__global__ void __launch_bounds__(256) k_grad_ft(ShellTab sh, const double* tvec, int n_t,
                                                 cplx* D) {
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)n_t * sh.n_sh * sh.n_sh;
  if (tid >= total) return;
  const int sp = (int)(tid / n_t), it = (int)(tid % n_t);
  const int sa = sp / sh.n_sh, sb = sp % sh.n_sh;
  const double a = sh.ex[sa], b = sh.ex[sb];
  double A[3], B[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    A[x] = sh.ctr[3 * sa + x];
    B[x] = sh.ctr[3 * sb + x] + tvec[3 * it + x];
  }
  const int n = sh.n_ao;
  const size_t cs = (size_t)n * n * n_t;  // component stride: D[c][T][mu][nu]
  double* out = reinterpret_cast<double*>(D + (size_t)it * n * n + (size_t)sh.off[sa] * n + sh.off[sb]);
  switch (sh.l[sa] * 3 + sh.l[sb]) {
    case 0: pair_grad<0, 0>(a, b, A, B, out, n, cs); break;
    case 1: pair_grad<0, 1>(a, b, A, B, out, n, cs); break;
    case 2: pair_grad<0, 2>(a, b, A, B, out, n, cs); break;
    case 3: pair_grad<1, 0>(a, b, A, B, out, n, cs); break;
    case 4: pair_grad<1, 1>(a, b, A, B, out, n, cs); break;
    case 5: pair_grad<1, 2>(a, b, A, B, out, n, cs); break;
    case 6: pair_grad<2, 0>(a, b, A, B, out, n, cs); break;
    case 7: pair_grad<2, 1>(a, b, A, B, out, n, cs); break;
    default: pair_grad<2, 2>(a, b, A, B, out, n, cs); break;
  }
}

// G = 0 row of the pair densities divided by |q| in the optical limit:
// Rp[c][t] holds <c|d/dr_c|v> (resonant t) or <v|d/dr_c|c> (anti-resonant t)
// at the same k; the row is -i qhat.P / D or +i qhat.P / D, D = dt[t] > 0.
__global__ void k_optical_row(const cplx* __restrict__ Rp, size_t ldt, const double* __restrict__ dt,
                              int n_t, double q0, double q1, double q2, cplx* __restrict__ R0) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_t) return;
  const cplx a = Rp[t], b = Rp[ldt + t], c = Rp[2 * ldt + t];
  const double pr = q0 * a.re + q1 * b.re + q2 * c.re, pi = q0 * a.im + q1 * b.im + q2 * c.im;
  const double id = 1.0 / dt[t];
  R0[t] = t < n_t / 2 ? cplx{pi * id, -pr * id} : cplx{-pi * id, pr * id};
}

__global__ void k_bloch_phase(const double* kf, int n_k, double s0, double s1, double s2,
                              const int* cells, int n_t, cplx* ph) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_k * n_t) return;
  const int k = i / n_t, t = i % n_t;
  // e^{2 pi i kf.n}; sincospi keeps the argument reduction exact for rational kf
  double arg = (kf[3 * k] + s0) * cells[3 * t] + (kf[3 * k + 1] + s1) * cells[3 * t + 1] +
               (kf[3 * k + 2] + s2) * cells[3 * t + 2];
  double s, c;
  sincospi(2.0 * arg, &s, &c);
  ph[i] = {c, s};
}

// M[k][e] = sum_T ph[k0+k][T] F[T][e] for the n_q*n_ao^2 elements e.
// grid = (element tiles of 256, k chunks of kch): each thread keeps its n_t
// lattice terms in registers (n_t <= 27) and walks its k chunk; the phases of
// the chunk are broadcast from LDS.  Consecutive threads write consecutive e.
template <int NT>
__global__ void __launch_bounds__(256) k_phase_sum(const cplx* __restrict__ F,
                                                   const cplx* __restrict__ ph, long n_el, int n_e,
                                                   int k0, int nk, int kch,
                                                   cplx* __restrict__ M) {
  extern __shared__ cplx sph[];  // [kch][NT]
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int kb = blockIdx.y * kch;
  const int kn = min(kch, nk - kb);
  for (int i = threadIdx.x; i < kn * NT; i += blockDim.x) sph[i] = ph[(size_t)(k0 + kb) * NT + i];
  __syncthreads();
  if (e >= n_el) return;
  // element e of the G list is (G, mu nu) = (e / n_e, e % n_e); F is G-major
  const cplx* Fe = F + (size_t)(e / n_e) * NT * n_e + e % n_e;
  cplx f[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) f[t] = Fe[(size_t)t * n_e];
  for (int kk = 0; kk < kn; ++kk) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const cplx p = sph[kk * NT + t];
      re += p.re * f[t].re - p.im * f[t].im;
      im += p.re * f[t].im + p.im * f[t].re;
    }
    M[(size_t)(kb + kk) * n_el + e] = {re, im};
  }
}

// Generic lattice range: loop over cells from global memory.
__global__ void __launch_bounds__(256) k_phase_sum_any(const cplx* __restrict__ F,
                                                       const cplx* __restrict__ ph, int n_t,
                                                       long n_el, int n_e, int k0, int nk,
                                                       cplx* __restrict__ M) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_el) return;
  const cplx* Fe = F + (size_t)(e / n_e) * n_t * n_e + e % n_e;
  for (int kk = 0; kk < nk; ++kk) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < n_t; ++t) {
      const cplx p = ph[(size_t)(k0 + kk) * n_t + t];
      const cplx f = Fe[(size_t)t * n_e];
      re += p.re * f.re - p.im * f.im;
      im += p.re * f.im + p.im * f.re;
    }
    M[(size_t)kk * n_el + e] = {re, im};
  }
}

// Band contraction in the ket-first order (used when 2 n_occ >= n_b, where it
// needs fewer multiply-adds than the valence-first kernel below, and when no
// tile of that kernel fits).  A block owns one k and a contiguous range of G tiles
// (GT vectors each); C(k) and C(k+q) are staged in LDS once and read as
// broadcasts.  Per tile:
//   step 1: T1_G[mu][b] = sum_nu M_G[mu][nu] C_k[nu][b]; a thread owns
//           (G, mu, BQ consecutive b) and keeps its BQ sums in registers, so
//           one LDS read of M feeds BQ complex multiply-adds.  M rows are
//           padded to n_ao + 1 in LDS (consecutive rows then start in
//           different banks);
//   step 2: rho_G[v][c] = sum_mu conj(C_kq[mu][n_occ+c]) T1_G[mu][v] and
//           sigma_G[v][c] = sum_mu conj(C_kq[mu][v]) T1_G[mu][n_occ+c],
//           written to R[g][t], t = ((s*n_k + k)*n_occ + v)*n_cond + c.
// The next tile's M is loaded into registers while the current one is
// computed (MPF = per-thread capacity in complex values; when a tile does
// not fit, the remainder is loaded synchronously).
// ALIAS: every thread owns at most one step-1 item, so T1 overwrites the M
// tile after a barrier (less LDS, larger tiles).
constexpr int kBQ = 10;
constexpr int kMPF = 16;

template <int GT, bool ALIAS>
__global__ void __launch_bounds__(256) k_band_contract(const cplx* __restrict__ M,
                                                       const cplx* __restrict__ Ck,
                                                       const cplx* __restrict__ Ckq, int n_ao,
                                                       int n_b, int n_occ, int n_k, int k0,
                                                       int n_g, int tiles_per_block,
                                                       cplx* __restrict__ R, size_t ldt) {
  extern __shared__ cplx lds[];
  const int kk = blockIdx.x;   // index inside the chunk
  const int k = k0 + kk;
  const int n_tiles = (n_g + GT - 1) / GT;
  const int tile0 = blockIdx.y * tiles_per_block;
  const int tile1 = min(n_tiles, tile0 + tiles_per_block);
  const int n_c = n_b - n_occ;
  const int nab = n_ao * n_b, naa = n_ao * n_ao, lda = n_ao + 1;
  const int nthr = blockDim.x, tid = threadIdx.x;
  cplx* sCk = lds;
  cplx* sCq = sCk + nab;
  cplx* sM = sCq + nab;                                   // [GT][n_ao][lda]
  cplx* sT = ALIAS ? sM : sM + (size_t)GT * n_ao * lda;   // [GT][n_ao][n_b]
  for (int i = tid; i < nab; i += nthr) {
    sCk[i] = Ck[(size_t)kk * nab + i];   // Ck, Ckq already offset to the chunk
    sCq[i] = Ckq[(size_t)kk * nab + i];
  }
  const int nbq = (n_b + kBQ - 1) / kBQ;
  const int nvc = n_occ * n_c;
  const size_t t_res = (size_t)k * nvc;
  const size_t t_anti = ((size_t)n_k + k) * nvc;

  // register prefetch of a tile's M (element i of the tile = tid + j*nthr)
  cplx pf[kMPF];
  auto fetch = [&](int tile) {
    const int g0 = tile * GT, ng = min(GT, n_g - g0);
    const cplx* Mk = M + ((size_t)kk * n_g + g0) * naa;
#pragma unroll
    for (int j = 0; j < kMPF; ++j) {
      const int i = tid + j * nthr;
      if (i < ng * naa) pf[j] = Mk[i];
    }
  };
  auto put = [&](int tile) {
    const int g0 = tile * GT, ng = min(GT, n_g - g0);
    const cplx* Mk = M + ((size_t)kk * n_g + g0) * naa;
    auto store = [&](int i, cplx v) {
      const int g = i / naa, e = i - g * naa;
      const int mu = e / n_ao, nu = e - mu * n_ao;
      sM[(g * n_ao + mu) * lda + nu] = v;
    };
#pragma unroll
    for (int j = 0; j < kMPF; ++j) {
      const int i = tid + j * nthr;
      if (i < ng * naa) store(i, pf[j]);
    }
    for (int i = tid + kMPF * nthr; i < ng * naa; i += nthr) store(i, Mk[i]);
  };
  if (tile0 < tile1) fetch(tile0);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int g0 = tile * GT, ng = min(GT, n_g - g0);
    __syncthreads();  // the previous tile's step 2 has finished with the LDS
    put(tile);
    __syncthreads();
    if (tile + 1 < tile1) fetch(tile + 1);  // in flight during this tile's work
    // step 1
    const int n_items = ng * n_ao * nbq;
    for (int w0 = 0; w0 < n_items; w0 += nthr) {
      const int w = w0 + tid;
      const bool live = w < n_items;
      const int g = live ? w / (n_ao * nbq) : 0, rem = live ? w - g * n_ao * nbq : 0;
      const int mu = rem / nbq, b0 = (rem - mu * nbq) * kBQ;
      double re[kBQ], im[kBQ];
#pragma unroll
      for (int j = 0; j < kBQ; ++j) re[j] = im[j] = 0.0;
      const cplx* mrow = sM + (g * n_ao + mu) * lda;
      for (int nu = 0; nu < (live ? n_ao : 0); ++nu) {
        const cplx m = mrow[nu];
        const cplx* crow = sCk + nu * n_b + b0;
#pragma unroll
        for (int j = 0; j < kBQ; ++j) {
          if (b0 + j < n_b) {
            const cplx c = crow[j];
            re[j] += m.re * c.re - m.im * c.im;
            im[j] += m.re * c.im + m.im * c.re;
          }
        }
      }
      if (ALIAS) __syncthreads();  // every read of M done before T1 overwrites it
      cplx* trow = sT + (g * n_ao + mu) * n_b + b0;
#pragma unroll
      for (int j = 0; j < kBQ; ++j)
        if (live && b0 + j < n_b) trow[j] = {re[j], im[j]};
    }
    __syncthreads();
    // step 2
    for (int w = tid; w < ng * 2 * nvc; w += nthr) {
      const int g = w / (2 * nvc), i = w - g * 2 * nvc;
      const int s = i / nvc, vc = i - s * nvc;
      const int v = vc / n_c, c = vc - v * n_c;
      const int bra = s == 0 ? n_occ + c : v;
      const int ket = s == 0 ? v : n_occ + c;
      const cplx* T = sT + (size_t)g * n_ao * n_b;
      double re = 0.0, im = 0.0;
      for (int mu = 0; mu < n_ao; ++mu) {
        const cplx a = sCq[mu * n_b + bra], t = T[mu * n_b + ket];
        re += a.re * t.re + a.im * t.im;
        im += a.re * t.im - a.im * t.re;
      }
      R[(size_t)(g0 + g) * ldt + (s == 0 ? t_res : t_anti) + vc] = {re, im};
    }
  }
}

// Valence-first band contraction.  The pair densities need only the n_occ
// valence columns on one side of M_G, so with C_v / C_c the valence /
// conduction columns:
//   X_G = M_G C_v(k)         [mu][v]   (ket side)
//   U_G = C_v(k+q)^H M_G     [v][nu]   (bra side)
//   rho_G[v][c]   = sum_mu conj(C_c(k+q)[mu][c]) X_G[mu][v]
//   sigma_G[v][c] = sum_nu U_G[v][nu] C_c(k)[nu][c]
// i.e. 2 n_ao^2 n_occ + 2 n_occ n_c n_ao complex multiply-adds per (k, G)
// against n_ao^2 n_b + 2 n_occ n_c n_ao in the ket-first order above.
// Both halves of each step run the same branch-free loop (an item picks its
// operand strides and the conjugation sign), so a wave never splits between
// them.  Step 1 item: one row of X or column of U for 4 valence bands; step 2
// item: one conduction band c for 2 valence bands, lanes along c.
// ALIAS: X and U overwrite the M tile after a barrier (every thread owns at
// most one step-1 item).
constexpr int kVB1 = 4;
constexpr int kVB2 = 2;

template <int GT, bool ALIAS>
__global__ void __launch_bounds__(256) k_band_vf(const cplx* __restrict__ M,
                                                 const cplx* __restrict__ Ck,
                                                 const cplx* __restrict__ Ckq, int n_ao, int n_b,
                                                 int n_occ, int n_k, int k0, int n_g,
                                                 int tiles_per_block, cplx* __restrict__ R,
                                                 size_t ldt) {
  extern __shared__ cplx lds[];
  const int kk = blockIdx.x;
  const int k = k0 + kk;
  const int n_tiles = (n_g + GT - 1) / GT;
  const int tile0 = blockIdx.y * tiles_per_block;
  const int tile1 = min(n_tiles, tile0 + tiles_per_block);
  const int n_c = n_b - n_occ;
  const int nab = n_ao * n_b, naa = n_ao * n_ao, lda = n_ao + 1;
  const int nthr = blockDim.x, tid = threadIdx.x;
  cplx* sCk = lds;
  cplx* sCq = sCk + nab;
  cplx* sM = sCq + nab;                                   // [GT][n_ao][lda]
  cplx* sX = ALIAS ? sM : sM + (size_t)GT * n_ao * lda;   // [GT][n_ao][n_occ]
  cplx* sU = sX + (size_t)GT * n_ao * n_occ;              // [GT][n_occ][n_ao]
  for (int i = tid; i < nab; i += nthr) {
    sCk[i] = Ck[(size_t)kk * nab + i];
    sCq[i] = Ckq[(size_t)kk * nab + i];
  }
  const int nvc = n_occ * n_c;
  const size_t t_res = (size_t)k * nvc;
  const size_t t_anti = ((size_t)n_k + k) * nvc;
  const int nvg = (n_occ + kVB1 - 1) / kVB1;
  const int nvp = (n_occ + kVB2 - 1) / kVB2;

  cplx pf[kMPF];
  auto fetch = [&](int tile) {
    const int g0 = tile * GT, ng = min(GT, n_g - g0);
    const cplx* Mk = M + ((size_t)kk * n_g + g0) * naa;
#pragma unroll
    for (int j = 0; j < kMPF; ++j) {
      const int i = tid + j * nthr;
      if (i < ng * naa) pf[j] = Mk[i];
    }
  };
  auto put = [&](int tile) {
    const int g0 = tile * GT, ng = min(GT, n_g - g0);
    const cplx* Mk = M + ((size_t)kk * n_g + g0) * naa;
    auto store = [&](int i, cplx v) {
      const int g = i / naa, e = i - g * naa;
      const int mu = e / n_ao, nu = e - mu * n_ao;
      sM[(g * n_ao + mu) * lda + nu] = v;
    };
#pragma unroll
    for (int j = 0; j < kMPF; ++j) {
      const int i = tid + j * nthr;
      if (i < ng * naa) store(i, pf[j]);
    }
    for (int i = tid + kMPF * nthr; i < ng * naa; i += nthr) store(i, Mk[i]);
  };
  if (tile0 < tile1) fetch(tile0);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int g0 = tile * GT, ng = min(GT, n_g - g0);
    __syncthreads();  // the previous tile's step 2 has finished with the LDS
    put(tile);
    __syncthreads();
    if (tile + 1 < tile1) fetch(tile + 1);
    // step 1: item (g, side, vg, row); side 0: X row mu = row, side 1: U
    // column nu = row
    const int per_g1 = 2 * nvg * n_ao;
    const int n1 = ng * per_g1;
    for (int w0 = 0; w0 < n1; w0 += nthr) {
      const int w = w0 + tid;
      const bool live = w < n1;
      const int ww = live ? w : 0;
      const int g = ww / per_g1, r = ww - g * per_g1;
      const int side = r / (nvg * n_ao), r2 = r - side * nvg * n_ao;
      const int vg = r2 / n_ao, row = r2 - vg * n_ao;
      const int v0 = vg * kVB1;
      // X: M[g][row][i] C_k[i][v];  U: M[g][i][row] conj(C_kq[i][v])
      const cplx* mp = sM + g * n_ao * lda + (side ? row : row * lda);
      const int ms = side ? lda : 1;
      const cplx* cp = side ? sCq : sCk;
      const double sg = side ? -1.0 : 1.0;
      int vc[kVB1];
#pragma unroll
      for (int j = 0; j < kVB1; ++j) vc[j] = min(v0 + j, n_occ - 1);
      double re[kVB1], im[kVB1];
#pragma unroll
      for (int j = 0; j < kVB1; ++j) re[j] = im[j] = 0.0;
#pragma unroll 4
      for (int i = 0; i < n_ao; ++i) {
        const cplx m = mp[i * ms];
#pragma unroll
        for (int j = 0; j < kVB1; ++j) {
          const cplx c = cp[i * n_b + vc[j]];
          const double ci = sg * c.im;
          re[j] += m.re * c.re - m.im * ci;
          im[j] += m.re * ci + m.im * c.re;
        }
      }
      if (ALIAS) __syncthreads();  // every read of M done before X and U overwrite it
      if (live) {
#pragma unroll
        for (int j = 0; j < kVB1; ++j) {
          if (v0 + j < n_occ) {
            if (side)
              sU[(g * n_occ + v0 + j) * n_ao + row] = {re[j], im[j]};
            else
              sX[(g * n_ao + row) * n_occ + v0 + j] = {re[j], im[j]};
          }
        }
      }
    }
    __syncthreads();
    // step 2: item (g, side, vp, c); side 0: rho with conj(C_kq[i][n_occ+c])
    // and X[g][i][v], side 1: sigma with C_k[i][n_occ+c] and U[g][v][i]
    const int per_g2 = 2 * nvp * n_c;
    const int n2 = ng * per_g2;
    for (int w = tid; w < n2; w += nthr) {
      const int g = w / per_g2, r = w - g * per_g2;
      const int side = r / (nvp * n_c), r2 = r - side * nvp * n_c;
      const int vp = r2 / n_c, c = r2 - vp * n_c;
      const int v0 = vp * kVB2;
      const cplx* ap = (side ? sCk : sCq) + n_occ + c;
      const double sg = side ? 1.0 : -1.0;
      const cplx* bp[kVB2];
#pragma unroll
      for (int j = 0; j < kVB2; ++j) {
        const int v = min(v0 + j, n_occ - 1);
        bp[j] = side ? sU + (g * n_occ + v) * n_ao : sX + g * n_ao * n_occ + v;
      }
      const int bs = side ? 1 : n_occ;
      double re[kVB2], im[kVB2];
#pragma unroll
      for (int j = 0; j < kVB2; ++j) re[j] = im[j] = 0.0;
#pragma unroll 4
      for (int i = 0; i < n_ao; ++i) {
        const cplx a = ap[i * n_b];
        const double ai = sg * a.im;
#pragma unroll
        for (int j = 0; j < kVB2; ++j) {
          const cplx b = bp[j][i * bs];
          re[j] += a.re * b.re - ai * b.im;
          im[j] += a.re * b.im + ai * b.re;
        }
      }
      const size_t tb = (side ? t_anti : t_res) + c;
#pragma unroll
      for (int j = 0; j < kVB2; ++j)
        if (v0 + j < n_occ) R[(size_t)(g0 + g) * ldt + tb + (size_t)(v0 + j) * n_c] = {re[j], im[j]};
    }
  }
}

// dev[k] = max |C^H S C - I| (one block per k)
__global__ void __launch_bounds__(256) k_orth_check(const cplx* __restrict__ S,
                                                    const cplx* __restrict__ C, int n_ao,
                                                    int n_b, double* dev) {
  extern __shared__ cplx lds[];
  const int k = blockIdx.x;
  const int nab = n_ao * n_b, naa = n_ao * n_ao;
  cplx* sS = lds;
  cplx* sC = sS + naa;
  cplx* sT = sC + nab;
  __shared__ double red[256];
  for (int i = threadIdx.x; i < naa; i += blockDim.x) sS[i] = S[(size_t)k * naa + i];
  for (int i = threadIdx.x; i < nab; i += blockDim.x) sC[i] = C[(size_t)k * nab + i];
  __syncthreads();
  for (int i = threadIdx.x; i < nab; i += blockDim.x) {
    const int mu = i / n_b, b = i % n_b;
    cplx acc = {0.0, 0.0};
    for (int nu = 0; nu < n_ao; ++nu) acc = cadd(acc, cmul(sS[mu * n_ao + nu], sC[nu * n_b + b]));
    sT[i] = acc;
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = threadIdx.x; i < n_b * n_b; i += blockDim.x) {
    const int a = i / n_b, b = i % n_b;
    cplx acc = {a == b ? -1.0 : 0.0, 0.0};
    for (int mu = 0; mu < n_ao; ++mu) acc = cadd(acc, cmulc(sC[mu * n_b + a], sT[mu * n_b + b]));
    double m = fabs(acc.re) + fabs(acc.im);
    if (!(m <= mx)) mx = m;  // NaN propagates
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double o = red[threadIdx.x + s];
      if (!(o <= red[threadIdx.x])) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) dev[k] = red[0];
}

}  // namespace

void launch_cell_ft(const ShellTab& sh, const int* pair_order, const double* tvec, int n_t,
                    const double* Q, int n_q, cplx* F, hipStream_t st) {
  const long total = (long)sh.n_sh * sh.n_sh * n_t * n_q;
  hipLaunchKernelGGL(k_cell_ft, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, sh,
                     pair_order, tvec, n_t, Q, n_q, F);
}

void launch_grad_ft(const ShellTab& sh, const double* tvec, int n_t, cplx* D, hipStream_t st) {
  const long total = (long)sh.n_sh * sh.n_sh * n_t;
  hipLaunchKernelGGL(k_grad_ft, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, sh, tvec,
                     n_t, D);
}

void launch_optical_row(const cplx* Rp, size_t ldt, const double* dt, int n_t, const double qhat[3],
                        cplx* R0, hipStream_t st) {
  hipLaunchKernelGGL(k_optical_row, dim3((unsigned)((n_t + 255) / 256)), dim3(256), 0, st, Rp, ldt,
                     dt, n_t, qhat[0], qhat[1], qhat[2], R0);
}

void launch_bloch_phase(const double* k_frac, int n_k, const double shift[3], const int* cells,
                        int n_t, cplx* ph, hipStream_t st) {
  const int n = n_k * n_t;
  hipLaunchKernelGGL(k_bloch_phase, dim3((n + 255) / 256), dim3(256), 0, st, k_frac, n_k,
                     shift[0], shift[1], shift[2], cells, n_t, ph);
}

void launch_phase_sum(const cplx* F, const cplx* ph, int n_t, int n_q, int n_e, int k0, int nk,
                      cplx* M, hipStream_t st) {
  const long n_el = (long)n_q * n_e;
  const long etiles = (n_el + 255) / 256;
  if (n_t == 27 || n_t == 1) {
    // k chunk: enough blocks to fill the device, at most 64 k per thread
    long kch = (etiles * nk + 1023) / 1024;
    kch = kch < 4 ? 4 : (kch > 64 ? 64 : kch);
    if (kch > nk) kch = nk;
    const dim3 grid((unsigned)etiles, (unsigned)((nk + kch - 1) / kch));
    const size_t lds = sizeof(cplx) * kch * n_t;
    if (n_t == 27)
      hipLaunchKernelGGL(k_phase_sum<27>, grid, dim3(256), lds, st, F, ph, n_el, n_e, k0, nk,
                         (int)kch, M);
    else
      hipLaunchKernelGGL(k_phase_sum<1>, grid, dim3(256), lds, st, F, ph, n_el, n_e, k0, nk,
                         (int)kch, M);
  } else {
    hipLaunchKernelGGL(k_phase_sum_any, dim3((unsigned)etiles), dim3(256), 0, st, F, ph, n_t, n_el,
                       n_e, k0, nk, M);
  }
}

static size_t band_lds(int n_ao, int n_b, int gt, bool alias) {
  const size_t m = (size_t)gt * n_ao * (n_ao + 1), t = (size_t)gt * n_ao * n_b;
  return sizeof(cplx) * (2 * (size_t)n_ao * n_b + (alias ? std::max(m, t) : m + t));
}

// the single-G tile without aliasing is the floor: the configuration check
// uses it
size_t band_contract_lds(int n_ao, int n_b, int /*n_occ*/) {
  return band_lds(n_ao, n_b, 1, false);
}

static size_t band_vf_lds(int n_ao, int n_b, int n_occ, int gt, bool alias) {
  const size_t m = (size_t)gt * n_ao * (n_ao + 1), xu = 2 * (size_t)gt * n_ao * n_occ;
  return sizeof(cplx) * (2 * (size_t)n_ao * n_b + (alias ? std::max(m, xu) : m + xu));
}

void launch_band_contract(const cplx* M, const cplx* Ck, const cplx* Ckq, int n_ao, int n_b,
                          int n_occ, int n_k, int k0, int nk, int n_g, cplx* R, size_t ldt,
                          hipStream_t st) {
  const cplx* ck = Ck + (size_t)k0 * n_ao * n_b;
  const cplx* cq = Ckq + (size_t)k0 * n_ao * n_b;
  const int nbq = (n_b + kBQ - 1) / kBQ;
  const size_t cap = 80 * 1024;  // two blocks per CU
  // G tiles of each k shared out over enough blocks to fill the chip
  auto grid_y = [&](int gt) {
    const int n_tiles = (n_g + gt - 1) / gt;
    const int want = std::max(1, std::min(n_tiles, (2048 + nk - 1) / nk));
    return std::make_pair((n_tiles + want - 1) / want, want);
  };
  // the largest G tile that keeps one step-1 item per thread and two blocks
  // per CU; otherwise single-G tiles
#define QCX_BC(GT, AL)                                                                          \
  do {                                                                                          \
    const auto tb = grid_y(GT);                                                                 \
    hipLaunchKernelGGL((k_band_contract<GT, AL>), dim3(nk, (unsigned)((n_g + GT - 1) / GT +    \
                                                                      tb.first - 1) / tb.first), \
                       dim3(256), band_lds(n_ao, n_b, GT, AL), st, M, ck, cq, n_ao, n_b, n_occ,   \
                       n_k, k0, n_g, tb.first, R, ldt);                                         \
  } while (0)
  // the valence-first order when it needs fewer multiply-adds (2 n_occ < n_b)
  // and a tile of at least one G fits two blocks per CU
  const int nvg = (n_occ + kVB1 - 1) / kVB1;
  const bool vf = 2 * n_occ < n_b;
#define QCX_VF(GT, AL)                                                                          \
  do {                                                                                          \
    const auto tb = grid_y(GT);                                                                 \
    hipLaunchKernelGGL((k_band_vf<GT, AL>), dim3(nk, (unsigned)((n_g + GT - 1) / GT +          \
                                                                tb.first - 1) / tb.first),       \
                       dim3(256), band_vf_lds(n_ao, n_b, n_occ, GT, AL), st, M, ck, cq, n_ao,    \
                       n_b, n_occ, n_k, k0, n_g, tb.first, R, ldt);                             \
  } while (0)
  auto vf_alias = [&](int gt) {
    return gt * 2 * nvg * n_ao <= 256 && band_vf_lds(n_ao, n_b, n_occ, gt, true) <= cap;
  };
  if (vf && vf_alias(4))
    QCX_VF(4, true);
  else if (vf && vf_alias(2))
    QCX_VF(2, true);
  else if (vf && vf_alias(1))
    QCX_VF(1, true);
  else if (4 * n_ao * nbq <= 256 && band_lds(n_ao, n_b, 4, true) <= cap)
    QCX_BC(4, true);
  else if (2 * n_ao * nbq <= 256 && band_lds(n_ao, n_b, 2, true) <= cap)
    QCX_BC(2, true);
  else if (n_ao * nbq <= 256 && band_lds(n_ao, n_b, 1, true) <= cap)
    QCX_BC(1, true);
  else if (vf && band_vf_lds(n_ao, n_b, n_occ, 1, false) <= 160 * 1024)
    QCX_VF(1, false);
  else if (n_ao * nbq <= 256)
    QCX_BC(1, true);
  else
    QCX_BC(1, false);
#undef QCX_BC
#undef QCX_VF
}

// Device-side state checks (deferred reporting): flags[0] = smallest k whose
// energies are non-finite or whose empty bands do not all lie above its
// occupied bands (at k and at k+q); flags[1] = smallest index i of dev (k,
// then n_k + k for k+q) with max|C^H S C - I| above tol.  Both stay INT_MAX
// when the states pass, and accumulate (minimum) until read and reset.
__global__ void k_band_check(const double* __restrict__ Ek, const double* __restrict__ Ekq,
                             int n_k, int n_b, int n_occ, int* flags) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_k) return;
  double vmax = -1e300, cmin = 1e300;
  bool bad = false;
  for (int b = 0; b < n_b; ++b) {
    const double e1 = Ek[(size_t)k * n_b + b], e2 = Ekq[(size_t)k * n_b + b];
    if (!isfinite(e1) || !isfinite(e2)) bad = true;
    if (b < n_occ)
      vmax = fmax(vmax, fmax(e1, e2));
    else
      cmin = fmin(cmin, fmin(e1, e2));
  }
  if (bad || !(cmin > vmax)) atomicMin(&flags[0], k);
}

__global__ void k_orth_flag(const double* __restrict__ dev, int n, double tol, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(dev[i] <= tol)) atomicMin(&flags[1], i);
}

void launch_state_flags(const double* Ek, const double* Ekq, int n_k, int n_b, int n_occ,
                        const double* dev, double tol, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_band_check, dim3((n_k + 255) / 256), dim3(256), 0, st, Ek, Ekq, n_k, n_b,
                     n_occ, flags);
  hipLaunchKernelGGL(k_orth_flag, dim3((2 * n_k + 255) / 256), dim3(256), 0, st, dev, 2 * n_k,
                     tol, flags);
}

// Q = q + G in Cartesian coordinates (G = sum_j n_j b_j, the reciprocal
// vectors b_j being the rows of rec) and the symmetrised Coulomb factor
// v_G = sqrt(4 pi)/|q + G| of every row (Eq. RPA).  In the optical limit the
// G = 0 row keeps sqrt(4 pi) alone: its 1/|q| goes into the k.p row.  The
// host rejects a vanishing q + G before enqueueing; such a row would get 0.
__global__ void k_q_plus_g(const double* __restrict__ q, const int* __restrict__ G, Mat3 rec,
                           int n_g, int optical, double* __restrict__ Q, double* __restrict__ vq) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_g) return;
  double n2 = 0.0;
  for (int x = 0; x < 3; ++x) {
    double v = q[x];
    for (int j = 0; j < 3; ++j) v += G[3 * g + j] * rec.m[3 * j + x];
    Q[3 * g + x] = v;
    n2 += v * v;
  }
  const double s4pi = sqrt(4.0 * kPi);
  vq[g] = (optical && g == 0) ? s4pi : (n2 > 0.0 ? s4pi / sqrt(n2) : 0.0);
}

// Zero the columns n_t..ldt-1 of every row of R[n_g][ldt] (readers that work
// in K chunks run past n_t into them)
__global__ void k_zero_tail(cplx* R, size_t ldt, int n_t, int n_g) {
  const size_t tail = ldt - n_t;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tail * n_g) return;
  R[(i / tail) * ldt + n_t + i % tail] = cplx{0.0, 0.0};
}

void launch_q_plus_g(const double* q, const int* G, const double rec[9], int n_g, bool optical,
                     double* Q, double* vq, hipStream_t st) {
  Mat3 r;
  for (int i = 0; i < 9; ++i) r.m[i] = rec[i];
  hipLaunchKernelGGL(k_q_plus_g, dim3((n_g + 255) / 256), dim3(256), 0, st, q, G, r, n_g,
                     optical ? 1 : 0, Q, vq);
}

void launch_zero_tail(cplx* R, size_t ldt, int n_t, int n_g, hipStream_t st) {
  const size_t n = (ldt - n_t) * (size_t)n_g;
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_tail, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, R, ldt, n_t,
                     n_g);
}

void launch_orth_check(const cplx* S, const cplx* C, int n_ao, int n_b, int n_k, double* dev,
                       hipStream_t st) {
  const size_t lds = sizeof(cplx) * ((size_t)n_ao * n_ao + 2 * (size_t)n_ao * n_b);
  hipLaunchKernelGGL(k_orth_check, dim3(n_k), dim3(256), lds, st, S, C, n_ao, n_b, dev);
}

}  // namespace qcx
