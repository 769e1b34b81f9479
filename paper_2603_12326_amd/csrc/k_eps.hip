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

#include <utility>

#include "common.h"

namespace qcx {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

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

// 1/a = conj(a) / |a|^2 with a first scaled by the binary exponent of
// max(|re|, |im|) (exact), so that |a|^2 neither underflows nor overflows for
// any finite nonzero a; zero and non-finite a take the plain formula (they
// are reported as singular pivots).
__device__ inline cplx cinv(cplx a) {
  const double s = fmax(fabs(a.re), fabs(a.im));
  if (!(s > 0.0 && s < INFINITY)) {
    const double d = 1.0 / (a.re * a.re + a.im * a.im);
    return {a.re * d, -a.im * d};
  }
  int e;
  (void)frexp(s, &e);
  const double x = ldexp(a.re, -e), y = ldexp(a.im, -e);
  const double d = 1.0 / (x * x + y * y);
  return {ldexp(x * d, -e), ldexp(-y * d, -e)};
}

// A pivot of modulus zero, or a non-finite one (NaN or infinite entries, e.g.
// eta = 0 with w on a transition energy), makes the matrix count as singular.
__device__ inline bool bad_pivot(cplx v) {
  const double m = fabs(v.re) + fabs(v.im);
  return !(m > 0.0 && m < INFINITY);
}

// 64-bit pivot key for a wave maximum: the modulus |re| + |im| in the high
// bits (non-negative doubles order like their bit patterns), the complement
// of the row index in the low 12 bits, so that moduli equal to 40 mantissa
// bits go to the smaller row.  A NaN entry counts as infinite so that it still selects a
// row (and poisons the result instead of hiding).  Every key is > 0.
__device__ inline unsigned long long pivot_key(cplx v, int row) {
  double mag = fabs(v.re) + fabs(v.im);
  if (mag != mag) mag = INFINITY;
  const unsigned long long b = (unsigned long long)__double_as_longlong(mag);
  return (b & ~0xFFFull) | (unsigned long long)(0xFFF - row);
}

// An empty asm statement makes x opaque, so that choosing one element of a
// register array by a run-time index (a == pa, b == jt / 16) stays a choice
// between values instead of becoming an indexed load that would move the
// whole array to scratch memory.
__device__ inline cplx opaque(cplx x) {
  asm volatile("" : "+v"(x.re), "+v"(x.im));
  return x;
}

// The same for an integer: row indices derived from it inside a loop are then
// recomputed there instead of being hoisted (and spilled) as RP constants.
__device__ inline int opaque_i(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Element pa (wave-uniform) of a per-lane register array, as held by lane pl:
// one scalar branch per slot, so that only the readlanes of slot pa run and
// they read the registers in place (no VALU copy of the chosen element).
template <int RP>
__device__ inline cplx readlane_slot(const cplx (&c)[RP], int pa, int pl) {
  cplx r = {0.0, 0.0};
#pragma unroll
  for (int a = 0; a < RP; ++a)
    if (a == pa) r = {readlane_d(c[a].re, pl), readlane_d(c[a].im, pl)};
  return r;
}

// Maximum of a 64-bit value over the wave: butterflies inside each row of 16
// lanes by DPP (lane xor 1, xor 2, half-row mirror, row mirror), then the four
// row results by readlane.  Needs every lane active.
__device__ inline unsigned long long wave_max_u64(unsigned long long x) {
  auto step = [&](auto ctrl) {
    constexpr int c = decltype(ctrl)::value;
    const int lo = __builtin_amdgcn_update_dpp((int)x, (int)x, c, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(x >> 32), (int)(x >> 32), c, 0xF, 0xF, false);
    const unsigned long long o = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    x = o > x ? o : x;
  };
  step(std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
  step(std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
  step(std::integral_constant<int, 0x141>{});  // row_half_mirror
  step(std::integral_constant<int, 0x140>{});  // row_mirror
  unsigned long long r = 0ull;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)x, 16 * row);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), 16 * row);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    r = o > r ? o : r;
  }
  return r;
}

// 32-bit pivot key: the high word of the modulus |re| + |im| as a double (its
// exponent and 8 mantissa bits; non-negative doubles order like their bit
// patterns, over the whole double range) with the low 12 bits replaced by the
// complement of the row index, so that moduli equal to that precision go to
// the smaller row.  Partial pivoting then takes a pivot within a factor
// 1 - 2^-8 of the largest modulus.  A NaN entry counts as infinite.  Every key
// of a live row is > 0 except for modulus 0.
__device__ inline unsigned pivot_key32(cplx v, int row) {
  double mag = fabs(v.re) + fabs(v.im);
  if (mag != mag) mag = INFINITY;
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(mag) >> 32);
  return (hi & ~0xFFFu) | (unsigned)(0xFFF - row);
}

// Maximum of a 32-bit value over the wave: DPP butterflies inside each row of
// 16 lanes, then the four row results by readlane.  Needs every lane active.
__device__ inline unsigned wave_max_u32(unsigned x) {
  auto step = [&](auto ctrl) {
    constexpr int c = decltype(ctrl)::value;
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, c, 0xF, 0xF, false);
    x = o > x ? o : x;
  };
  step(std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
  step(std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
  step(std::integral_constant<int, 0x141>{});  // row_half_mirror
  step(std::integral_constant<int, 0x140>{});  // row_mirror
  unsigned r = 0u;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const unsigned o = (unsigned)__builtin_amdgcn_readlane((int)x, 16 * row);
    r = o > r ? o : r;
  }
  return r;
}

// 1/a as cinv, with 1/|a|^2 of the scaled a (in [1/4, 2)) from a
// single-precision estimate refined by two Newton steps in FP64 (24 -> 48 ->
// 96 bits: within an ulp of the FP64 reciprocal), a shorter chain of
// dependent instructions than the IEEE division.
__device__ inline cplx cinv_nr(cplx a) {
  const double s = fmax(fabs(a.re), fabs(a.im));
  if (!(s > 0.0 && s < INFINITY)) {
    const double d = 1.0 / (a.re * a.re + a.im * a.im);
    return {a.re * d, -a.im * d};
  }
  int e;
  (void)frexp(s, &e);
  const double x = ldexp(a.re, -e), y = ldexp(a.im, -e);
  const double d = x * x + y * y;
  double r = (double)__builtin_amdgcn_rcpf((float)d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return {ldexp(x * r, -e), ldexp(-y * r, -e)};
}

// Register-resident Gauss-Jordan for n <= 64 RP and n <= 16 CP with 16 waves:
// lane l of wave v owns rows l + 64 a and columns v + 16 b, so column k lives
// in wave k % 16 alone.  Step k applies m <- m - u w^T with the pivot folded
// into u: u_i = c_i / piv (u_p = (piv - 1) / piv) and w = row p as it stands
// except w_k = piv + 1, where c = column k and piv = m[p][k].  This is the
// Gauss-Jordan sweep (row p / piv, column k -c / piv, pivot 1 / piv, the rest
// m - c row_p / piv) with no per-element fix-ups.
//
// One barrier per step.  Between two barriers the wave that owns column k + 1
// runs the chain that bounds the step: read p and u, update column k + 1,
// choose its pivot (largest unused modulus by pivot_key32 and DPP maxima),
// publish u and p through LDS.  It runs that chain before any of its other
// columns, while the other waves do their FMAs.  Every wave then reads row p
// of its columns from lane p % 64 with readlane (scalar registers, no LDS
// traffic: the LDS pipe is shared by all 16 waves); the row slot p / 64 is
// dispatched once per step by a scalar branch, so the readlanes take the
// registers in place instead of a VALU copy of the chosen slot.  u and p are
// double-buffered by the parity of k; u is zero past row n; used-row marks
// live in registers.
// Body of one 1024-thread block: matrix A (n x n), diagonal of the inverse
// into drow[n]; a zero pivot sets *sing to at most widx.
template <int RP, int CP>
__device__ __forceinline__ void gj_reg_body(const cplx* __restrict__ A, int n,
                                            cplx* __restrict__ drow, int* sing, int widx) {
  constexpr int NW = 16;
  __shared__ cplx ucol[2][64 * RP];
  __shared__ int prow[2], sor[64 * RP];
  const int tid = threadIdx.x, l = tid & 63;
  const int v = __builtin_amdgcn_readfirstlane(tid >> 6);
  cplx m[RP][CP];
#pragma unroll
  for (int a = 0; a < RP; ++a)
#pragma unroll
    for (int b = 0; b < CP; ++b) {
      const int i = l + 64 * a, j = v + NW * b;
      m[a][b] = (i < n && j < n) ? A[(size_t)i * n + j] : cplx{0.0, 0.0};
    }
  for (int e = tid; e < 2 * 64 * RP; e += 1024) (&ucol[0][0])[e] = {0.0, 0.0};
  __syncthreads();
  unsigned used = 0;       // bit a: row l + 64 a already served as pivot
  bool singular = false;
  cplx wk = {0.0, 0.0};    // piv + 1 of the column this wave owns next

  // Owner wave of column kc (current values c): choose the pivot, publish u
  // into buffer pb, p and sor[p].
  auto choose = [&](const cplx (&c)[RP], int kc, int pb) {
    unsigned best = 0u;
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = l + 64 * a;
      if (i < n && !((used >> a) & 1u)) best = max(best, pivot_key32(c[a], i));
    }
    best = wave_max_u32(best);
    const int p = __builtin_amdgcn_readfirstlane(0xFFF - (int)(best & 0xFFFu));
    const int pl = p & 63, pa = p >> 6;
    const cplx pv = readlane_slot<RP>(c, pa, pl);
    if (bad_pivot(pv)) singular = true;
    const cplx inv = cinv_nr(pv);
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = l + 64 * a;
      cplx x = c[a];
      if (i == p) x.re -= 1.0;
      if (i < n) ucol[pb][i] = cmul(x, inv);
    }
    if (l == 0) {
      prow[pb] = p;
      sor[p] = kc;
    }
    wk = {pv.re + 1.0, pv.im};
  };

  if (v == 0) {
    cplx c[RP];
#pragma unroll
    for (int a = 0; a < RP; ++a) c[a] = m[a][0];
    choose(c, 0, 0);
  }
  // Step k = 16 kb + kk; with kb, t and the row slot unrolled every register
  // index is static.  The owner of column k + 1 (slot kb, or kb + 1 when
  // kk = 15) updates it and chooses before its other columns.
#pragma unroll
  for (int kb = 0; kb < CP; ++kb) {
    for (int kk = 0; kk < NW; ++kk) {
      const int k = NW * kb + kk;
      if (k >= n) break;
      const int par = k & 1;
      // the owner of column k + 1 runs at raised wave priority until it has
      // published, so that its chain is issued ahead of the other waves' FMAs
      if (v == (k + 1) % NW) __builtin_amdgcn_s_setprio(3);
      __syncthreads();  // u, p of column k published
      const int p = __builtin_amdgcn_readfirstlane(prow[par]);
      const int pl = p & 63, pa = p >> 6;
      cplx u[RP];
#pragma unroll
      for (int a = 0; a < RP; ++a) u[a] = ucol[par][l + 64 * a];
      if (l == pl) used |= 1u << pa;
      const int k1 = k + 1;
      const bool owner1 = k1 < n && v == k1 % NW;  // owns column k + 1
      const bool next = kk == NW - 1;               // column k + 1 in slot kb + 1
      // m[.][b] -= u w^T for one column
      auto update = [&](int b, cplx w) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < RP; ++a) {
          m[a][b].re = fma(-u[a].re, w.re, m[a][b].re);
          m[a][b].re = fma(u[a].im, w.im, m[a][b].re);
          m[a][b].im = fma(-u[a].re, w.im, m[a][b].im);
          m[a][b].im = fma(-u[a].im, w.re, m[a][b].im);
        }
      };
      if (owner1) {
        auto update_choose = [&](int b) __attribute__((always_inline)) {
          cplx c[RP];
#pragma unroll
          for (int a = 0; a < RP; ++a) c[a] = m[a][b];
          update(b, readlane_slot<RP>(c, pa, pl));  // column k + 1 is never column k
#pragma unroll
          for (int a = 0; a < RP; ++a) c[a] = m[a][b];
          choose(c, k1, par ^ 1);
        };
        if (!next)
          update_choose(kb);
        else
          update_choose(kb + 1 < CP ? kb + 1 : CP - 1);  // k1 < n keeps kb + 1 < CP
      }
      __builtin_amdgcn_s_setprio(0);
      cplx wr[CP];  // row p of this wave's columns (lane pl), wave-uniform
      // pa is wave-uniform: one scalar branch per row slot, and inside it
      // the readlanes take the registers in place (no VALU copies)
#pragma unroll
      for (int a = 0; a < RP; ++a)
        if (a == pa) {
#pragma unroll
          for (int b = 0; b < CP; ++b) wr[b] = {readlane_d(m[a][b].re, pl), readlane_d(m[a][b].im, pl)};
        }
      if (v == kk) wr[kb] = wk;  // owner of column k: w_k = piv + 1
#pragma unroll
      for (int t = 0; t < CP; ++t) {
        const int b = (kb + t) % CP;
        const bool done = owner1 && ((t == 0 && !next) || (t == 1 && next));
        if (v + NW * b < n && !done) update(b, wr[b]);
      }
    }
  }
  __syncthreads();
  // [eps^-1]_kk sits at row piv[k] (the row whose sor is k) and column sor[k]
#pragma unroll
  for (int a = 0; a < RP; ++a) {
    const int i = l + 64 * a;
    if (i >= n) continue;
    const int k = sor[i], jt = sor[k];
    if (jt % NW != v) continue;
#pragma unroll
    for (int b = 0; b < CP; ++b)
      if (b == jt / NW) drow[k] = opaque(m[a][b]);
  }
  if (singular) atomicMin(sing, widx);
}

// Blocked Gauss-Jordan for 128 < n <= 64 RP (RP <= 16) with 1024 threads per
// matrix; the matrix stays in global memory and is swept in panels of MB
// columns, made of one or two sub-panels of 16.  For each panel:
//  1. lane l of wave v holds rows l + 64 a of sub-panel column s0 + v in
//     registers, and the sub-panel's 16 pivot steps run as in k_gj_reg (one
//     barrier per step, the next column's owner chooses its pivot while the
//     others update), restricted to the sub-panel's columns;
//  2. with two sub-panels, the second one's columns first receive the first
//     one's rank-16 update, and after their own sweep the first one's columns
//     receive theirs (the same deferred update as below, on 16 columns), so
//     that the panel holds what 32 single steps would leave there;
//  3. every other column j receives the deferred rank-MB update
//     T[:, j] += Z Y[:, j]  with Y = T[P][j] (the MB pivot rows before this
//     update) and Z = swept panel with 1 subtracted at (p_a, a), one chunk of
//     ZR rows of Z at a time.  With several chunks the pivot rows are left
//     out of the chunk passes and updated in a last pass of their own, so
//     that every chunk pass reads their old values; with one chunk they are
//     updated with the other rows.
// The update runs on FP64 MFMA (v_mfma_f64_16x16x4f64) as two real products
// with K = 2 MB:  Re T += [Re Z | Im Z] [Re Y ; -Im Y],
//                 Im T += [Re Z | Im Z] [Im Y ;  Re Y].
// Z (chunks of ZR rows) and a JT-column tile of Y are staged in LDS k-major
// (lane-consecutive rows / columns); each wave owns a 32 x 16 output block
// (2 MFMA tiles, re and im) per tile and updates it in place.  Each Y tile is
// loaded into registers while the previous tile's MFMAs run and stored into
// the other of two LDS buffers: one barrier per column tile.
// MFMA layouts: A 16x4, lane l holds A[l%16][l/16]; B 4x16, lane l holds
// B[l/16][l%16]; D 16x16, lane l holds D[4r + l/16][l%16], r = 0..3.
// Panel shape by row class: up to 320 rows (RP <= 5) a panel is one sub-panel
// of 16 columns and Z is staged in one chunk of every row (one pass per
// panel); larger matrices take two sub-panels per panel (rank-32 updates,
// half the passes over the matrix, which bound them) and Z in chunks of 128
// rows, which is what fits the LDS with the wider panel.
__host__ __device__ constexpr int gjp_nsub(int rp) { return rp <= 5 ? 1 : 2; }
__host__ __device__ constexpr int gjp_zr(int rp) { return rp <= 5 ? 64 * rp : 128; }
constexpr int GJP_MS = 16, GJP_JT = 64;

template <int RP>
__device__ __forceinline__ void gj_panel_body(cplx* __restrict__ A, int n,
                                              cplx* __restrict__ drow, int* sing, int widx) {
  constexpr int NW = 16, MS = GJP_MS, MB = gjp_nsub(RP) * MS, JT = GJP_JT, KR = 2 * MB,
                ZR = gjp_zr(RP);
  extern __shared__ __align__(16) char smem[];
  double* Zt = reinterpret_cast<double*>(smem);    // [KR][ZR]: k' < MB Re Z, else Im Z
  cplx* ucol = reinterpret_cast<cplx*>(smem);      // [2][64 RP] during the pivot steps
  cplx* Ys = reinterpret_cast<cplx*>(Zt + (size_t)KR * ZR);  // [2][MB][JT]: Y tiles
  int* piv = reinterpret_cast<int*>(Ys + 2 * MB * JT);  // [n] pivot row of step k
  int* sor = piv + n;                               // [n] step of pivot row i
  __shared__ int prow[2];
  const int tid = threadIdx.x, l = tid & 63;
  const int v = __builtin_amdgcn_readfirstlane(tid >> 6);
  unsigned used = 0;  // bit a: row l + 64 a already served as pivot
  bool singular = false;
  cplx wk = {0.0, 0.0};

  auto choose = [&](const cplx (&c)[RP], int kc, int pb) {
    const int lo = opaque_i(l);
    unsigned long long best = 0ull;
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = lo + 64 * a;
      if (i < n && !((used >> a) & 1u)) best = max(best, pivot_key(c[a], i));
    }
    best = wave_max_u64(best);
    const int p = __builtin_amdgcn_readfirstlane(0xFFF - (int)(best & 0xFFFull));
    const int pl = p & 63, pa = p >> 6;
    cplx x = c[0];
#pragma unroll
    for (int a = 1; a < RP; ++a)
      if (a == pa) x = opaque(c[a]);
    const cplx pv = {readlane_d(x.re, pl), readlane_d(x.im, pl)};
    if (bad_pivot(pv)) singular = true;
    const cplx inv = cinv(pv);
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = lo + 64 * a;
      cplx y = c[a];
      if (i == p) y.re -= 1.0;
      if (i < n) ucol[pb * 64 * RP + i] = cmul(y, inv);
    }
    if (l == 0) {
      prow[pb] = p;
      piv[kc] = p;
      sor[p] = kc;
    }
    wk = {pv.re + 1.0, pv.im};
  };
  // Up to five row slots (N_G <= 320) the sweep takes the register kernel's
  // short pivot chain (32-bit keys, the pivot read under a scalar branch on its
  // slot, Newton-refined reciprocal, the owner at raised priority); the larger
  // classes keep the form above, which spills fewer registers there.
  constexpr bool SHORT = RP <= 5;
  auto choose_short = [&](const cplx (&c)[RP], int kc, int pb) {
    const int lo = opaque_i(l);
    unsigned best = 0u;
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = lo + 64 * a;
      if (i < n && !((used >> a) & 1u)) best = max(best, pivot_key32(c[a], i));
    }
    best = wave_max_u32(best);
    const int p = __builtin_amdgcn_readfirstlane(0xFFF - (int)(best & 0xFFFu));
    const int pl = p & 63, pa = p >> 6;
    const cplx pv = readlane_slot<RP>(c, pa, pl);
    if (bad_pivot(pv)) singular = true;
    const cplx inv = cinv_nr(pv);
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = lo + 64 * a;
      cplx y = c[a];
      if (i == p) y.re -= 1.0;
      if (i < n) ucol[pb * 64 * RP + i] = cmul(y, inv);
    }
    if (l == 0) {
      prow[pb] = p;
      piv[kc] = p;
      sor[p] = kc;
    }
    wk = {pv.re + 1.0, pv.im};
  };

  auto load_col = [&](cplx (&pm)[RP], int jc) {
    const int lo = opaque_i(l);
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = lo + 64 * a;
      pm[a] = i < n ? A[(size_t)i * n + jc] : cplx{0.0, 0.0};
    }
  };
  auto store_col = [&](const cplx (&pm)[RP], int jc) {
    const int lo = opaque_i(l);
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = lo + 64 * a;
      if (i < n) A[(size_t)i * n + jc] = pm[a];
    }
  };
  // The deferred update of one column jc held in pm by the steps z0 .. z0 +
  // zs - 1 (already swept, their columns in A):
  //   pm[i] += sum_b (A[i][z0 + b] - [i == piv[z0 + b]]) A[piv[z0 + b]][jc],
  // the second factor read from A, which still holds the column before it.
  auto defer = [&](cplx (&pm)[RP], int jc, int z0, int zs) {
    const int lo = opaque_i(l);
    for (int b0 = 0; b0 < zs; b0 += 4) {
      cplx y[4];
      int pr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = b0 + q;
        pr[q] = b < zs ? piv[z0 + b] : -1;
        y[q] = b < zs ? A[(size_t)pr[q] * n + jc] : cplx{0.0, 0.0};
      }
#pragma unroll
      for (int a = 0; a < RP; ++a) {
        const int i = lo + 64 * a;
        if (i >= n) continue;
        cplx acc = pm[a];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (b0 + q >= zs) continue;
          cplx z = A[(size_t)i * n + z0 + b0 + q];
          if (i == pr[q]) z.re -= 1.0;
          acc.re = fma(z.re, y[q].re, acc.re);
          acc.re = fma(-z.im, y[q].im, acc.re);
          acc.im = fma(z.re, y[q].im, acc.im);
          acc.im = fma(z.im, y[q].re, acc.im);
        }
        pm[a] = acc;
      }
    }
  };
  // The pivot steps s0 .. s0 + ms - 1 on their columns, held by waves v < ms
  // in pm; each wave's column goes back to A afterwards.
  auto sweep = [&](cplx (&pm)[RP], int s0, int ms) {
    const bool hascol = v < ms;
    if (v == 0) {
      if constexpr (SHORT)
        choose_short(pm, s0, s0 & 1);
      else
        choose(pm, s0, s0 & 1);
    }
    for (int kk = 0; kk < ms; ++kk) {
      const int k = s0 + kk, par = k & 1;
      // the owner of column k + 1 at raised priority until it has published
      if (SHORT && v == kk + 1) __builtin_amdgcn_s_setprio(3);
      __syncthreads();  // u, p of column k published
      const int p = __builtin_amdgcn_readfirstlane(prow[par]);
      const int pl = p & 63, pa = p >> 6;
      if (l == pl) used |= 1u << pa;
      if (hascol) {
        const int lo = opaque_i(l);
        cplx x = pm[0];
#pragma unroll
        for (int a = 1; a < RP; ++a)
          if (!SHORT && a == pa) x = opaque(pm[a]);
        cplx w = {readlane_d(x.re, pl), readlane_d(x.im, pl)};
        if constexpr (SHORT) w = readlane_slot<RP>(pm, pa, pl);
        if (v == kk) w = wk;  // owner of column k: w_k = piv + 1
#pragma unroll
        for (int a = 0; a < RP; ++a) {
          const int i = lo + 64 * a;
          const cplx u = i < n ? ucol[par * 64 * RP + i] : cplx{0.0, 0.0};
          pm[a].re = fma(-u.re, w.re, pm[a].re);
          pm[a].re = fma(u.im, w.im, pm[a].re);
          pm[a].im = fma(-u.re, w.im, pm[a].im);
          pm[a].im = fma(-u.im, w.re, pm[a].im);
          // keep the scheduler from hoisting all RP loads of u at once
          if ((a & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        if (kk + 1 < ms && v == kk + 1) {
          if constexpr (SHORT)
            choose_short(pm, k + 1, par ^ 1);
          else
            choose(pm, k + 1, par ^ 1);
        }
      }
      if (SHORT) __builtin_amdgcn_s_setprio(0);
    }
    if (hascol) store_col(pm, s0 + v);
  };

  for (int k0 = 0; k0 < n; k0 += MB) {
    const int mb = min(MB, n - k0);
    const int ms1 = min(MS, mb), ms2 = mb - ms1;
    __syncthreads();  // the previous panel's update is complete
    cplx pm[RP];
    // first sub-panel
    if (v < ms1) load_col(pm, k0 + v);
    sweep(pm, k0, ms1);
    if (ms2 > 0) {
      __syncthreads();  // its swept columns in A; pivot buffers free
      // second sub-panel: the first one's update, then its own steps
      if (v < ms2) {
        load_col(pm, k0 + ms1 + v);
        defer(pm, k0 + ms1 + v, k0, ms1);
      }
      sweep(pm, k0 + ms1, ms2);
      __syncthreads();  // its swept columns in A
      // the first sub-panel's columns: the second one's update
      if (v < ms1) {
        load_col(pm, k0 + v);
        defer(pm, k0 + v, k0 + ms1, ms2);
        store_col(pm, k0 + v);
      }
    }
    __syncthreads();  // swept panel in memory; pivot buffers free
    // ---- deferred rank-mb update of every column outside the panel
    const int nch = (n + ZR - 1) / ZR;
    // With several chunks the panel's pivot rows are left out of the chunk
    // passes (their Z rows are zero there) and updated in a pass of their own
    // at the end, so every chunk pass reads Y = the pivot rows before this
    // update straight from the matrix, and each Z chunk is staged once per
    // panel.  With one chunk, a column tile's Y is staged before any of its
    // columns changes, so the pivot rows take their update in the same pass
    // (Z with 1 subtracted at (p_a, a)).
    const bool one = nch == 1;
    auto is_piv = [&](int i) {
      bool f = false;
      for (int a = 0; a < mb; ++a) f |= piv[k0 + a] == i;
      return f;
    };
    auto load_z = [&](int r0) {
      for (int e = tid; e < ZR * MB; e += 1024) {
        const int r = e / MB, a = e % MB, i = r0 + r;
        cplx z = {0.0, 0.0};
        if (i < n && a < mb && (one || !is_piv(i))) {
          z = A[(size_t)i * n + k0 + a];
          if (i == piv[k0 + a]) z.re -= 1.0;
        }
        Zt[a * ZR + r] = z.re;
        Zt[(MB + a) * ZR + r] = z.im;
      }
    };
    // Z of the pivot rows: row r < mb is the pivot row of step k0 + r, with 1
    // subtracted at (r, r)
    auto load_zp = [&]() {
      for (int e = tid; e < ZR * MB; e += 1024) {
        const int r = e / MB, a = e % MB;
        cplx z = {0.0, 0.0};
        if (r < mb && a < mb) {
          z = A[(size_t)piv[k0 + r] * n + k0 + a];
          if (a == r) z.re -= 1.0;
        }
        Zt[a * ZR + r] = z.re;
        Zt[(MB + a) * ZR + r] = z.im;
      }
    };
    // Y tile of columns jt ..: two elements per thread, loaded into registers
    // a tile ahead and stored into the other buffer after this tile's MFMAs
    constexpr int YE = MB * JT / 1024;
    cplx yreg[YE];
    auto y_load = [&](int jt) {
#pragma unroll
      for (int q = 0; q < YE; ++q) {
        const int e = tid + 1024 * q, a = e / JT, c = e % JT, j = jt + c;
        yreg[q] = (a < mb && j < n) ? A[(size_t)piv[k0 + a] * n + j] : cplx{0.0, 0.0};
      }
    };
    auto y_store = [&](int buf) {
#pragma unroll
      for (int q = 0; q < YE; ++q) Ys[buf * MB * JT + tid + 1024 * q] = yreg[q];
    };
    const int li = l & 15, lk = l >> 4;
    // one 32 x 16 output block: rows r0 + 32 rb .. (the pivot rows of steps
    // k0 + 32 rb .. in the pivot pass), columns jt + 16 cb ..  The B operands
    // come from the stored Y: rows kr < MB give Re Y (for Re T) and Im Y (for
    // Im T), rows kr >= MB give -Im Y and Re Y.
    auto block = [&](int r0, int rb, int jt, int cb, int buf, bool pivot_pass) {
      f64x4 acc[2][2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        acc[rt][0] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc[rt][1] = f64x4{0.0, 0.0, 0.0, 0.0};
      }
      const cplx* Yb = Ys + buf * MB * JT;
#pragma unroll 2
      for (int s = 0; s < KR / 4; ++s) {
        const int kr = 4 * s + lk;
        const cplx y = Yb[(kr % MB) * JT + 16 * cb + li];
        const bool lower = 4 * s < MB;  // wave-uniform
        const double br = lower ? y.re : -y.im, bi = lower ? y.im : y.re;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const double za = Zt[kr * ZR + 32 * rb + 16 * rt + li];
          acc[rt][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(za, br, acc[rt][0], 0, 0, 0);
          acc[rt][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(za, bi, acc[rt][1], 0, 0, 0);
        }
      }
      const int j = jt + 16 * cb + li;
      if (j >= n || (j >= k0 && j < k0 + mb)) return;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = 32 * rb + 16 * rt + 4 * r + lk;
          if (pivot_pass ? rr >= mb : (rr >= ZR || r0 + rr >= n)) continue;
          const int i = pivot_pass ? piv[k0 + rr] : r0 + rr;
          cplx t = A[(size_t)i * n + j];
          t.re += acc[rt][0][r];
          t.im += acc[rt][1][r];
          A[(size_t)i * n + j] = t;
        }
    };
    // the column tiles of one pass (rows r0 .. of Z in Zt, or the pivot
    // rows): Y of the first tile staged beforehand, one barrier per tile
    auto pass = [&](int r0, bool pivot_pass) {
      y_load(0);
      y_store(0);
      __syncthreads();  // Z and the first Y tile staged
      int buf = 0;
      for (int jt = 0; jt < n; jt += JT) {
        const bool more = jt + JT < n;
        if (more) y_load(jt + JT);
        constexpr int NRB = ZR / 32, NU = NRB * (JT / 16);
        if (pivot_pass) {
          for (int u = v; u < JT / 16; u += NW) block(0, 0, jt, u, buf, true);
        } else {
          for (int u = v; u < NU; u += NW) block(r0, u % NRB, jt, u / NRB, buf, false);
        }
        if (more) y_store(buf ^ 1);
        __syncthreads();  // this tile's Y reads and updates done; the next Y staged
        buf ^= 1;
      }
    };
    for (int c = 0; c < nch; ++c) {
      load_z(c * ZR);
      pass(c * ZR, false);
    }
    if (!one) {
      load_zp();
      pass(0, true);
    }
  }
  __syncthreads();
  for (int k = tid; k < n; k += 1024) drow[k] = A[(size_t)piv[k] * n + sor[k]];
  if (singular) atomicMin(sing, widx);
}

template <int RP, int CP>
__global__ void __launch_bounds__(1024) k_gj_reg(const cplx* __restrict__ eps, int n,
                                                 cplx* __restrict__ diag, int* sing, int w_base) {
  gj_reg_body<RP, CP>(eps + (size_t)blockIdx.x * n * n, n, diag + (size_t)blockIdx.x * n, sing,
                      w_base + (int)blockIdx.x);
}

template <int RP>
__global__ void __launch_bounds__(1024) k_gj_panel(cplx* __restrict__ eps, int n,
                                                   cplx* __restrict__ diag, int* sing, int w_base) {
  gj_panel_body<RP>(eps + (size_t)blockIdx.x * n * n, n, diag + (size_t)blockIdx.x * n, sing,
                    w_base + (int)blockIdx.x);
}

// The job of this block in a multi-item launch: blocks [block0, block0 +
// n_w) of a launch belong to job j (jobs sorted by block0).
__device__ inline GjJob find_job(const GjJob* __restrict__ jobs, int n_jobs, int& w) {
  int j = 0;
  while (j + 1 < n_jobs && (int)blockIdx.x >= jobs[j + 1].block0) ++j;
  w = (int)blockIdx.x - jobs[j].block0;
  return jobs[j];
}

template <int RP, int CP>
__global__ void __launch_bounds__(1024) k_gj_reg_jobs(const GjJob* __restrict__ jobs, int n_jobs) {
  int w;
  const GjJob J = find_job(jobs, n_jobs, w);
  gj_reg_body<RP, CP>(J.eps + (size_t)w * J.n * J.n, J.n, J.diag + (size_t)w * J.n, J.sing, w);
}

template <int RP>
__global__ void __launch_bounds__(1024) k_gj_panel_jobs(const GjJob* __restrict__ jobs, int n_jobs) {
  int w;
  const GjJob J = find_job(jobs, n_jobs, w);
  gj_panel_body<RP>(J.eps + (size_t)w * J.n * J.n, J.n, J.diag + (size_t)w * J.n, J.sing, w);
}

size_t gj_panel_lds(int n, int rp) {
  const int mb = gjp_nsub(rp) * GJP_MS;
  return sizeof(double) * (size_t)(2 * mb) * gjp_zr(rp) + sizeof(cplx) * 2 * mb * GJP_JT +
         sizeof(int) * 2 * (size_t)n;
}

__global__ void k_nolfe(const cplx* eps, int n, int n_w, cplx* diag, int* sing, int w_base) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * n_w) return;
  const int j = (int)(i / n), G = (int)(i % n);
  const cplx e = eps[((size_t)j * n + G) * n + G];
  if (bad_pivot(e)) atomicMin(sing, w_base + j);
  diag[i] = cinv(e);
}

__global__ void k_loss(const cplx* diag, int n, int n_w, double* loss, cplx* epsM) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n * n_w) return;
  const cplx d = diag[i];
  loss[i] = -d.im;
  if (epsM && i % n == 0) epsM[i / n] = cinv(d);
}

// noLFE loss of Eq. (eps_noLFE) for a list of G from diagonal-only partial
// sums: chi0_GG = pref (Xr + i Yr) with Xr, Yr the Re W and Im W rows of the
// G-th diagonal pair (P_t(G, G) = |R_t(G)|^2 is real), eps_GG = 1 - v_G^2
// chi0_GG, loss = Im(-1 / eps_GG) = Im eps_GG / |eps_GG|^2.  Partials come
// from the bulk (a.C, [ks][n_rowsp][2][n_bulkp]) or the FP64 pairs kernel
// (a.XY, [ks64][n_rowsp64][n_colp64]); column b of chunk G-index b.
__global__ void k_diag_loss(AsmArgs a, Chi0Geom g, int n_g, int n_w, double* __restrict__ loss,
                            cplx* __restrict__ inv, int ldl, int g0) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_w * n_g) return;
  const int j = (int)(i / n_g), b = (int)(i % n_g);
  double Xr = 0.0, Yr = 0.0;
  if (a.XY) {
    for (int ks = 0; ks < a.ks64; ++ks) {
      const double* x0 = a.XY + ((size_t)ks * a.n_rowsp64 + 2 * j) * a.n_colp64 + 2 * b;
      Xr += x0[0];
      Yr += x0[a.n_colp64];
    }
  } else {
    for (int ks = 0; ks < a.ks; ++ks) {
      const size_t r0 = ((size_t)ks * g.n_rowsp + 2 * j) * 2;
      Xr += (double)a.C[r0 * g.n_bulkp + b];
      Yr += (double)a.C[(r0 + 2) * g.n_bulkp + b];
    }
  }
  const double vv = a.vq[b] * a.vq[b];
  const double er = 1.0 - vv * a.pref * Xr, ei = -vv * a.pref * Yr;
  const double d2 = er * er + ei * ei;
  loss[(size_t)j * ldl + g0 + b] = ei / d2;
  if (inv) inv[(size_t)j * ldl + g0 + b] = {er / d2, -ei / d2};  // 1 / eps_GG
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

int gj_class(int n_g) {
  if (n_g <= 64) return 0;
  if (n_g <= 128) return 1;
  if (n_g <= 192) return 2;
  if (n_g <= 256) return 3;
  if (n_g <= 320) return 4;
  if (n_g <= 512) return 5;
  if (n_g <= 768) return 6;
  if (n_g <= 1024) return 7;
  return 8;  // beyond the inversion kernels: callers reject n_g > 1024
}

void launch_gj_diag(cplx* eps, int n_g, int n_w, cplx* diag, int* sing, hipStream_t st,
                    int w_base) {
  const dim3 g(n_w), b(1024);
  switch (gj_class(n_g)) {
    case 0: hipLaunchKernelGGL((k_gj_reg<1, 4>), g, b, 0, st, eps, n_g, diag, sing, w_base); return;
    case 1: hipLaunchKernelGGL((k_gj_reg<2, 8>), g, b, 0, st, eps, n_g, diag, sing, w_base); return;
    case 2: hipLaunchKernelGGL(k_gj_panel<3>, g, b, gj_panel_lds(n_g, 3), st, eps, n_g, diag, sing, w_base); return;
    case 3: hipLaunchKernelGGL(k_gj_panel<4>, g, b, gj_panel_lds(n_g, 4), st, eps, n_g, diag, sing, w_base); return;
    case 4: hipLaunchKernelGGL(k_gj_panel<5>, g, b, gj_panel_lds(n_g, 5), st, eps, n_g, diag, sing, w_base); return;
    case 5: hipLaunchKernelGGL(k_gj_panel<8>, g, b, gj_panel_lds(n_g, 8), st, eps, n_g, diag, sing, w_base); return;
    case 6: hipLaunchKernelGGL(k_gj_panel<12>, g, b, gj_panel_lds(n_g, 12), st, eps, n_g, diag, sing, w_base); return;
    case 7: hipLaunchKernelGGL(k_gj_panel<16>, g, b, gj_panel_lds(n_g, 16), st, eps, n_g, diag, sing, w_base); return;
    default: break;
  }
  // callers keep n_g <= 1024 (class 7); nothing is launched beyond
}

void launch_gj_jobs(int cls, const GjJob* jobs, int n_jobs, int n_blocks, int max_n, hipStream_t st) {
  const dim3 g(n_blocks), b(1024);
  switch (cls) {
    case 0: hipLaunchKernelGGL((k_gj_reg_jobs<1, 4>), g, b, 0, st, jobs, n_jobs); return;
    case 1: hipLaunchKernelGGL((k_gj_reg_jobs<2, 8>), g, b, 0, st, jobs, n_jobs); return;
    case 2: hipLaunchKernelGGL(k_gj_panel_jobs<3>, g, b, gj_panel_lds(max_n, 3), st, jobs, n_jobs); return;
    case 3: hipLaunchKernelGGL(k_gj_panel_jobs<4>, g, b, gj_panel_lds(max_n, 4), st, jobs, n_jobs); return;
    case 4: hipLaunchKernelGGL(k_gj_panel_jobs<5>, g, b, gj_panel_lds(max_n, 5), st, jobs, n_jobs); return;
    case 5: hipLaunchKernelGGL(k_gj_panel_jobs<8>, g, b, gj_panel_lds(max_n, 8), st, jobs, n_jobs); return;
    case 6: hipLaunchKernelGGL(k_gj_panel_jobs<12>, g, b, gj_panel_lds(max_n, 12), st, jobs, n_jobs); return;
    case 7: hipLaunchKernelGGL(k_gj_panel_jobs<16>, g, b, gj_panel_lds(max_n, 16), st, jobs, n_jobs); return;
    default: return;
  }
}

void launch_nolfe_diag(const cplx* eps, int n_g, int n_w, cplx* diag, int* sing, hipStream_t st,
                       int w_base) {
  const long total = (long)n_g * n_w;
  hipLaunchKernelGGL(k_nolfe, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, eps, n_g,
                     n_w, diag, sing, w_base);
}

void launch_loss(const cplx* diag, int n_g, int n_w, double* loss, cplx* epsM, hipStream_t st) {
  const long total = (long)n_g * n_w;
  hipLaunchKernelGGL(k_loss, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, diag, n_g,
                     n_w, loss, epsM);
}

void launch_diag_loss(const AsmArgs& a, const Chi0Geom& g, int n_g, int n_w, double* loss,
                      cplx* inv, int ldl, int g0, hipStream_t st) {
  const long total = (long)n_g * n_w;
  hipLaunchKernelGGL(k_diag_loss, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, g,
                     n_g, n_w, loss, inv, ldl, g0);
}

void launch_rho_export(const cplx* R, size_t ldt, int n_g, int n_t, cplx* out, hipStream_t st) {
  const long total = (long)n_g * n_t;
  hipLaunchKernelGGL(k_rho_export, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, R, ldt,
                     n_g, n_t, out);
}

}  // namespace qcx
