// Kramers-Kronig route of Sec. II.D (internal launchers).
//
// The spectral part of Eq. (RPA) is binned on a uniform grid w_b = b d with
// hat functions: a transition at energy D = (i + x) d (i = floor(D / d),
// 0 <= x < 1) puts weight 1 - x on bin i and x on bin i + 1, so that
//   S_b(G, G') = sum_t h_b(D_t) conj(R_t(G)) R_t(G')          (per side)
// is a piecewise-linear spectral density carrying the zeroth and first
// energy moments of every transition exactly.  The full response follows
// from S by the exact transform of each hat piece through the energy
// denominator (see k_kk.hip), one dense FP64 product over the bins on FP64
// MFMA.
#pragma once

#include "common.h"

namespace qcx {

// One run of consecutive intervals [k0, k0 + nb) of one side and their
// transitions [ta, tb) (energy order).  The chunk stores the bins k0 ..
// k0 + nb - 1 (rows row0 + (0..nb) of S; bin k0 without the share of
// interval k0 - 1) and leaves the share of its last interval in bin k0 + nb
// in its row of E, which the tail pass adds to S row tail_row (tail_add = 1:
// the next chunk has stored its share of that bin) or stores there
// (tail_add = 0: the side's last bin).
struct KkChunk {
  int row0, k0, nb, ta, tb, tail_row, tail_add;
};

constexpr int kKkTile = 64;  // G and G' rows of one binning block

// Rs[rank[t]][n_gp] = R[G][t] (zero for G >= n_g); rank = energy order of t
void launch_kk_pack(const cplx* R, size_t ldt, int n_g, int n_gp, int n_t, const int* rank,
                    cplx* Rs, hipStream_t st);
// S[row][2][n_pairs] (Re, Im) for every bin and upper-triangle pair
// (G <= G'): the binning, then the tail pass; E holds n_chunks rows of
// 2 n_pairs doubles of scratch
void launch_kk_bin(const cplx* Rs, int n_gp, int n_g, const int* ib, const double* xf,
                   const KkChunk* chunks, int n_chunks, double* S, double* E, hipStream_t st);
// Kb[rows_p][ldm] (bin-major): entry (c, 2j) = Re, (c, 2j + 1) = Im of the
// transform kernel of w_j for bin c: resonant bins c < nr at (br + c) d,
// anti-resonant bins nr <= c < nr + na at (ba + c - nr) d; zero for
// c >= nr + na and for rows >= 2 n_w
void launch_kk_matrix(const double* w, int n_w, double eta, double d, int nr, int na, int br,
                      int ba, int rows_p, int ldm, double* Kb, hipStream_t st);
// Padded sizes of the transform: bins rounded up to the K tile, the row
// length of Kb (2 n_w rounded up to the M tile), and the slack S needs past
// its last row (the last column tile reads up to one tile beyond N).
int kk_rows_padded(int rows);
int kk_ldm(int n_w);
size_t kk_s_slack();
// C[M][N] = Kb^T S over rows_p bins (S: rows_p x N, row-major, rows past the
// last bin zero, kk_s_slack() doubles of addressable memory after it)
void launch_kk_transform(const double* Kb, int ldm, const double* S, int N, int rows_p, int M,
                         double* C, hipStream_t st);

}  // namespace qcx
