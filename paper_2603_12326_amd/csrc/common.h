// Internal declarations shared by the translation units of libqcx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "qcx.h"

namespace qcx {

constexpr double kHartreeEV = 27.211386245988;  // CODATA 2018
constexpr double kPi = 3.14159265358979323846;

struct cplx {
  double re, im;
};

__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }

// Device buffer owned by a context; grows, never shrinks, freed on destroy.
// With a budget attached, a growth that would take the budget's total above
// its limit (limit 0: none) fails with hipErrorOutOfMemory and keeps the old
// buffer.
struct DevBudget {
  size_t used = 0, limit = 0;
};
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBudget* budget = nullptr;
  hipError_t reserve(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (budget && budget->limit && budget->used - bytes + n > budget->limit)
      return hipErrorOutOfMemory;
    release();
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) {
      bytes = n;
      if (budget) budget->used += n;
    } else {
      p = nullptr;
    }
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    if (budget) budget->used -= bytes;
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ---------------------------------------------------------------- launchers
// Gaussian Fourier integrals F[T][g][mu][nu] for every shell pair.
struct ShellTab {
  const int* l;        // [n_sh]
  const double* ex;    // [n_sh]
  const double* ctr;   // [n_sh][3]
  const int* off;      // [n_sh] first AO of the shell
  int n_sh;
  int n_ao;
};
// F[g][T][mu][nu] (G-major); pair_order lists the shell pairs sa * n_sh + sb
// sorted by (l_a, l_b)
void launch_cell_ft(const ShellTab& sh, const int* pair_order, const double* tvec, int n_t,
                    const double* Q, int n_q, cplx* F, hipStream_t st);
// Pair densities in one pass (Bloch sum on FP64 MFMA, valence-first band
// contraction, M in LDS only) into R[g][t] (stride ldt) for every k and the
// n_g rows of F[g][T][mu][nu]; Cb holds the bra states.  rho_fused_fits:
// N_AO <= 32, n_occ <= 4, at most 28 cells.
bool rho_fused_fits(int n_ao, int n_occ, int n_t);
void launch_rho_fused(const cplx* F, const cplx* ph, const cplx* Ck, const cplx* Cb, int n_ao,
                      int n_b, int n_occ, int n_k, int n_t, int n_g, cplx* R, size_t ldt,
                      hipStream_t st);
// optical limit (App. C): D[c][T][mu][nu] = <chi_mu| d/dr_c |chi_nu(. - T)>
// (real values in complex storage), and the G = 0 row R0[t] = -/+ i qhat.P / dt
// from the band matrices Rp[c][t] (stride ldt) of the resonant / anti-resonant
// transitions
void launch_grad_ft(const ShellTab& sh, const double* tvec, int n_t, cplx* D, hipStream_t st);
void launch_optical_row(const cplx* Rp, size_t ldt, const double* dt, int n_t, const double qhat[3],
                        cplx* R0, hipStream_t st);
// e^{2 pi i kf.n_T} for kf = k_frac[k] + shift
void launch_bloch_phase(const double* k_frac, int n_k, const double shift[3], const int* cells,
                        int n_t, cplx* ph, hipStream_t st);
// M[k][g][e] = sum_T ph[k0+k][T] F[g][T][e], e = mu*n_ao+nu, for k in [0, nk)
void launch_phase_sum(const cplx* F, const cplx* ph, int n_t, int n_q, int n_e, int k0, int nk,
                      cplx* M, hipStream_t st);
// R64[g][t] (t fastest, stride ldt) for k in [k0, k0+nk) from M chunk, in the
// valence-first order when 2 n_occ < n_b and a tile fits, else ket-first
void launch_band_contract(const cplx* M, const cplx* Ck, const cplx* Ckq, int n_ao, int n_b,
                          int n_occ, int n_k, int k0, int nk, int n_g, cplx* R, size_t ldt,
                          hipStream_t st);
// max_k |C^H S C - I| per k
// deferred state checks: flags[0] band order / finiteness (first bad k),
// flags[1] orthonormality (first bad index of dev[2 n_k]); INT_MAX when fine
void launch_state_flags(const double* Ek, const double* Ekq, int n_k, int n_b, int n_occ,
                        const double* dev, double tol, int* flags, hipStream_t st);
void launch_orth_check(const cplx* S, const cplx* C, int n_ao, int n_b, int n_k, double* dev,
                       hipStream_t st);
size_t band_contract_lds(int n_ao, int n_b, int n_occ);
// 3x3 matrix passed by value to a kernel
struct Mat3 {
  double m[9];
};
// Q[g] = q + G_g (G_int[g] in reciprocal-vector units, rec rows b_j) and
// vq[g] = sqrt(4 pi)/|Q[g]| (the G = 0 row sqrt(4 pi) in the optical limit);
// q is read from device memory
void launch_q_plus_g(const double* q, const int* G_int, const double rec[9], int n_g, bool optical,
                     double* Q, double* vq, hipStream_t st);
// zero columns n_t .. ldt-1 of the n_g rows of R
void launch_zero_tail(cplx* R, size_t ldt, int n_t, int n_g, hipStream_t st);

// chi0 pieces
struct Chi0Geom {
  int n_g, n_t, n_tp;       // transitions, padded to the K tile
  int n_w, n_rows, n_rowsp; // rows = 2 n_w (Re W, Im W), padded
  int n_pairs;              // n_g (n_g + 1) / 2 upper-triangle pairs, row-major
  int p0;                   // first bulk pair (n_g when head/wings run in FP64)
  int n_bulk, n_bulkp;      // bulk pairs and padded count
  int ksplit;
  int gather;               // 1: per-tile row lists (N_G >= kGatherMinNg)
  int row_tile0;            // first row tile of this launch (row chunks)
  int c_rows;               // rows held by the partial buffer C (n_rowsp unless chunked)
};
// transition energies Delta_t (Ha) and signs for t in [0, n_t)
void launch_transition_energies(const double* Ek, const double* Ekq, int n_k, int n_b, int n_occ,
                                double* dt, hipStream_t st);
// Weights in fragment order for the MFMA A operand
void launch_weights_f32(const double* w, const double* dt, double eta, const Chi0Geom& g,
                        float* Aw, hipStream_t st);
void launch_weights_bf16(const double* w, const double* dt, double eta, const Chi0Geom& g,
                         uint16_t* Ahi, uint16_t* Alo, hipStream_t st);
// R64[g][t] -> R32 slabs [t/16][g][16] (complex float)
void launch_pack_r32(const cplx* R, size_t ldt, const Chi0Geom& g, int perm, float* R32,
                     hipStream_t st);
constexpr int KSTEP_T = 16;  // transitions per bulk K step (one MFMA K block)
// Largest K split of a bulk launch; the bulk's operands are padded to
// KSTEP_T * kMaxKsplit transitions, and the pair-density rows R[g][t] have a
// stride (ldt) of at least n_t + 16 rounded up to that padding, with zeros past
// n_t, so that every padded or chunked reader stays inside its own row.
constexpr int kMaxKsplit = 64;
constexpr int kLdtAlign = KSTEP_T * kMaxKsplit;
// Row-gather mode of the bulk kernel: a tile of 128 consecutive upper-triangle
// pairs touches at most 129 distinct G (checked when the tables are built),
// so for large N_G each tile stages only its own slab rows, listed in
// rows[tile][kGatherRows], and the pair table holds tile-local indices.
constexpr int kGatherRows = 129;
constexpr int kGatherMinNg = 129;
// Fill the local pair table and the per-tile row lists from the global pair
// table (G | G' << 16 per bulk column, n_bulkp columns).  Returns false if a
// tile needs more than kGatherRows rows (it cannot: see above).
bool bulk_gather_tables(const std::vector<int>& pairs_global, std::vector<int>& pairs_local,
                        std::vector<int>& rows);
int bulk_row_frags(const Chi0Geom& g);
// LDS bytes of one bulk block: nst pipeline stages of the R slab (n_g rows)
// and af A fragment pairs
size_t bulk_lds_bytes(int n_g, int af, int nst);
// bulk launches; nst = 2 or 3 LDS pipeline stages
void launch_bulk_f32(const float* Aw, const float* R32, const int* pairs, const int* rows,
                     const Chi0Geom& g, int nst, float* C, hipStream_t st);
void launch_bulk_bf16(const uint16_t* Ahi, const uint16_t* Alo, const float* R32,
                      const int* pairs, const int* rows, const Chi0Geom& g, int nst, float* C,
                      hipStream_t st);
// One item of a batched bulk launch (its own weights, R, pairs and partials).
struct BulkItem {
  const float4* A;
  const float4* Alo;
  const float4* R32;
  const int* pairs;
  const int* rows;   // per-tile row lists (gather mode) or NULL
  Chi0Geom g;
  float* C;
};
// Persistent bulk kernel over tiles {item, pair tile, row tile, K split};
// AF = 4 row fragments; max_ng sizes the LDS.
void launch_bulk_persistent(bool bf16, bool gather, const BulkItem* items, const int4* tiles,
                            int n_tiles, int* counter, int max_ng, int grid, hipStream_t st);
void launch_set_int(int* p, int v, hipStream_t st);
// C64[r][ri][b] = sum over ks splits of C[ks][r][ri][b] for the rows of one
// chunk (C holds n_rows rows; C64 points at the chunk's first row)
void launch_reduce_partials(const float* C, int ks, int n_rows, int n_bulkp, double* C64,
                            hipStream_t st);
constexpr int kBatchAF = 4;

// FP64 pairs on FP64 MFMA: out[split][row][col], rows (Re W, Im W) per
// frequency, columns (Re P, Im P) per pair slot; slot ps holds (G | G' << 16).
struct Geom64 {
  int n_g, n_w, n_t, n_ps;
  int n_rowsp, n_colp;
  int ksplit, chunk_t;
};
void geom64_init(Geom64& g, int n_g, int n_w, int n_t, int n_ps, size_t max_bytes);
void launch_pairs_f64(const cplx* R, size_t ldt, const double* w, const double* dt, double eta,
                      const Geom64& g, const int* pairs, double* out, hipStream_t st);
// Head and wings (few pairs, all transitions): the same partials XY from an
// FP64 GEMM over a per-q table P[t][col] of the pair products (held in P,
// hw_ptable_doubles(g) doubles).  Geometry: rows padded to 160, columns to
// 128, K split to fill the device in one round.
void geom_hw_init(Geom64& g, int n_g, int n_w, int n_t, int n_ps, size_t max_bytes);
size_t hw_ptable_doubles(const Geom64& g);
void launch_headwings_f64(const cplx* R, size_t ldt, const double* w, const double* dt, double eta,
                          const Geom64& g, const int* pairs, double* P, double* out,
                          hipStream_t st);
// eps assembly (symmetrised Coulomb, prefactor 2/(N_k V))
struct AsmArgs {
  const float* C;       // bulk partials [ks][n_rowsp][2][n_bulkp] or null
  const double* C64;    // or: reduced FP64 partials [n_rowsp][2][n_bulkp] (row chunks)
  const double* XY;     // FP64 partials [ks64][n_rowsp64][n_colp64] or null
  int ks, ks64;
  int n_rowsp64, n_colp64;
  int n_pairs64;        // pairs (flat indices 0..n_pairs64-1) held by XY
  const double* vq;     // sqrt(4 pi)/|q+G|
  double pref;
};
void launch_eps_assemble(const AsmArgs& a, const Chi0Geom& g, cplx* eps, hipStream_t st);
// Gauss-Jordan diag(eps^-1) of n_w matrices; a zero or non-finite pivot in
// matrix j sets *sing to at most w_base + j (atomic minimum)
void launch_gj_diag(cplx* eps, int n_g, int n_w, cplx* diag, int* sing, hipStream_t st,
                    int w_base = 0);
// noLFE loss from diagonal-only partials of n_g G (chunk columns 0..n_g-1)
// into loss[j * ldl + g0 + b]
// loss[w][g0 + b] (and, if inv is not null, inv[w][g0 + b] = 1 / eps_GG) for
// the n_g diagonal entries of one chunk; row stride ldl
void launch_diag_loss(const AsmArgs& a, const Chi0Geom& g, int n_g, int n_w, double* loss,
                      cplx* inv, int ldl, int g0, hipStream_t st);
// One item of a multi-item inversion launch: its n_w matrices are blocks
// [block0, block0 + n_w) of the launch.
struct GjJob {
  cplx* eps;   // [n_w][n][n], overwritten
  cplx* diag;  // [n_w][n] diagonal of the inverse
  int* sing;   // lowest frequency index with a zero pivot (atomic minimum)
  int n, n_w, block0;
};
// Kernel class of an inversion of size n_g (items of one class share a
// launch); class 8 has no multi-item form.
int gj_class(int n_g);
void launch_gj_jobs(int cls, const GjJob* jobs, int n_jobs, int n_blocks, int max_n, hipStream_t st);
void launch_nolfe_diag(const cplx* eps, int n_g, int n_w, cplx* diag, int* sing, hipStream_t st,
                       int w_base = 0);
// loss = -Im diag and, if epsM is not null, eps_M = 1 / diag[w][0]
void launch_loss(const cplx* diag, int n_g, int n_w, double* loss, cplx* epsM, hipStream_t st);
void launch_chi0_export(const AsmArgs& a, const Chi0Geom& g, cplx* chi, hipStream_t st);
void launch_rho_export(const cplx* R, size_t ldt, int n_g, int n_t, cplx* out, hipStream_t st);

}  // namespace qcx
