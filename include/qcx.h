/*
 * qcx.h - C ABI of the MI355X library for all-electron RPA screening with
 * local field effects (pair densities -> chi0 -> FP64 eps inversion -> loss).
 *
 * The calls follow the statement of the problem in Sec. II.D of the paper:
 * Eq. (RPA) defines eps_GG'(w, q) from Kohn-Sham states at k and k' = k + q,
 * Eq. (eps_LFE) the finite-momentum eps(w, q+G) = 1/[eps^-1]_GG (G = 0 gives
 * the macroscopic eps_M) and Eq. (eps_noLFE) the variant without local field
 * effects.  Sec. III fixes the Gaussian-type-orbital basis and the shifted k
 * grid.
 *
 * Conventions for every entry point
 *   - Return value: QCX_OK (0) or a negative QCX_E* code; qcx_last_error()
 *     then holds a message.  Errors leave the context's previous results
 *     untouched unless stated otherwise.
 *   - Units: lengths in bohr, momenta in bohr^-1, energies (band energies,
 *     frequencies, broadening) in eV.  Internally Hartree atomic units with
 *     1 Ha = 27.211386245988 eV, so the 4 pi alpha of Eq. (RPA) is 4 pi.
 *   - Complex numbers are interleaved (re, im) pairs of doubles (c128) or of
 *     floats (c64).  All arrays are C order (last index fastest).
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership.  Device pointers are borrowed for the duration of the
 *     call only, unless stated otherwise.
 *   - All device work is enqueued on the HIP stream given to qcx_create (for
 *     PyTorch: torch.cuda.current_stream().cuda_stream).  The library never
 *     creates or destroys that stream.  Calls that return results on the host
 *     synchronise it; all others are asynchronous.
 *   - Calls that stage host data (qcx_set_cell_basis, qcx_set_states,
 *     qcx_pair_density*, qcx_chi0, qcx_chi0_kk, qcx_loss_diag, qcx_qbin_add /
 *     _finish / _rate_halo, and qcx_run_batch[_rho] when it builds a plan) return
 *     QCX_EINVAL while the context's stream is being captured into a graph.
 *   - A context is not thread-safe; use one context per host thread.
 *   - The call order is qcx_set_cell_basis -> qcx_set_states ->
 *     qcx_pair_density -> qcx_chi0 -> qcx_eps_inv -> qcx_loss.  A call made
 *     before its inputs exist returns QCX_ESTATE.  Setting new inputs
 *     invalidates everything downstream of them.
 */
#ifndef QCX_H
#define QCX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qcx_ctx qcx_ctx;

enum {
  QCX_OK = 0,
  QCX_EINVAL = -1,     /* bad shape or value                                */
  QCX_ESTATE = -2,     /* call order violated                               */
  QCX_ENONORTH = -3,   /* C^H S(k) C != I, or S(k) not positive definite    */
  QCX_ESINGULAR = -4,  /* zero pivot in the eps inversion                   */
  QCX_EDEVICE = -5,    /* HIP runtime error, or the library is not built for
                          the device                                        */
  QCX_ENOMEM = -6      /* device allocation failed                          */
};

enum { QCX_MEM_HOST = 0, QCX_MEM_DEVICE = 1 };

/* Arithmetic of the chi0 bulk (the G, G' != 0 entries).  The head and wings
 * (G = 0 row and column) and the eps inversion are FP64 unless requested
 * otherwise (see qcx_chi0). */
enum {
  QCX_FP64 = 0,        /* FP64 throughout                                   */
  QCX_FP32 = 1,        /* FP32 operands on FP32 MFMA, FP32 accumulation     */
  QCX_SPLIT_BF16 = 2   /* x = hi + lo (bf16 each), hi*hi + hi*lo + lo*hi on
                          BF16 MFMA with FP32 accumulation                  */
};

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL means the default stream).  *out receives the
 * context.  The library uses whichever HIP runtime (libamdhip64.so.7) the
 * process has loaded; a process that also uses PyTorch must load PyTorch's
 * first, since two HIP runtimes in one process cannot share the device.
 * Errors: QCX_EINVAL (out NULL, device out of range), QCX_EDEVICE (HIP
 * runtime not usable, or device is not gfx950). */
int qcx_create(qcx_ctx** out, int device, void* hip_stream);

/* Free every device buffer the context owns.  The stream is not touched.
 * Safe on NULL. */
int qcx_destroy(qcx_ctx* ctx);

/* Message describing the last error on this context (static storage owned
 * by the context, valid until the next call).  ctx may be NULL for errors of
 * qcx_create. */
const char* qcx_last_error(const qcx_ctx* ctx);

/* Wait for all work enqueued by this context and report errors detected on
 * the device since the last call: QCX_EINVAL / QCX_ENONORTH for device-input
 * states that failed their checks (qcx_set_states), QCX_ESINGULAR if an eps
 * matrix had a zero pivot (qcx_last_error names the index). */
int qcx_sync(qcx_ctx* ctx);

/* Crystal cell and Gaussian basis (Sec. III: Gaussian-type orbitals; one
 * band per AO).
 *   lat[9]        rows a1, a2, a3 of the primitive cell (bohr)
 *   xyz           [n_atoms][3] atomic positions (bohr)
 *   shell_atom    [n_shells] atom index of each shell
 *   shell_l       [n_shells] angular momentum, 0, 1 or 2
 *   shell_exp     [n_shells] Gaussian exponent (bohr^-2), > 0; one primitive
 *                 per shell, normalised to unit self-overlap
 *   pure_d        must be 1: d shells are the five real solid harmonics in
 *                 the order xy, yz, (2z^2-x^2-y^2)/(2 sqrt 3), xz, (x^2-y^2)/2
 *                 (times the normalised radial Gaussian); p shells are x, y, z
 *   lattice_range L >= 0: Bloch sums run over cells n1 a1 + n2 a2 + n3 a3 with
 *                 n in {-L..L}^3 (L = 1: 27 cells) with phase e^{ik.T}
 * AOs are numbered shell by shell in the given order.  All inputs are host
 * pointers and are copied.  Invalidates states and all results.
 * Errors: QCX_EINVAL (l > 2, exponent <= 0, atom index out of range,
 * singular lattice, pure_d != 1, L > 3). */
int qcx_set_cell_basis(qcx_ctx* ctx, const double lat[9], int n_atoms, const double* xyz,
                       int n_shells, const int* shell_atom, const int* shell_l,
                       const double* shell_exp, int pure_d, int lattice_range);

/* Kohn-Sham states at k and at k + q for one momentum q (Eq. RPA with
 * k' = k + q; Sec. III: final states on the shifted grid).
 *   q_cart[3]  q in Cartesian bohr^-1 (host)
 *   k_frac     [n_k][3] k in reciprocal-basis coordinates (host or device)
 *   n_occ      bands 0..n_occ-1 are occupied (f = 2), the rest empty (f = 0)
 *   n_bands    bands per k, n_occ < n_bands <= N_AO
 *   C_k, C_kq  [n_k][N_AO][n_bands] c128 coefficients of the states at k and
 *              at k + q on the Bloch sums of the AOs
 *   E_k, E_kq  [n_k][n_bands] band energies (eV); every empty band must lie
 *              above every occupied band at each k and k + q
 *   mem        QCX_MEM_HOST or QCX_MEM_DEVICE for k_frac, C_*, E_*
 * The states are copied to the device and checked: finite energies with the
 * band order above, and |C^H S C - I| <= 1e-10 at every k and k + q with S(k)
 * the library's own overlap.  Host inputs (QCX_MEM_HOST) are checked before
 * this call returns (it synchronises the stream).  Device inputs are checked
 * on the stream without a round trip: a failure is reported (QCX_EINVAL or
 * QCX_ENONORTH, results computed from those states being invalid) by the
 * context's next synchronising call: qcx_sync, qcx_loss to host memory or
 * qcx_batch_sync.  Invalidates pair densities and all results.
 * Errors: QCX_ESTATE (no basis), QCX_EINVAL (sizes, band order),
 * QCX_ENONORTH, QCX_ENOMEM. */
int qcx_set_states(qcx_ctx* ctx, const double q_cart[3], int n_k, const double* k_frac,
                   int n_occ, int n_bands, const double* C_k, const double* E_k,
                   const double* C_kq, const double* E_kq, int mem);

/* Pair densities of Eq. (RPA) for the G list (Sec. II.D; Gaussian Fourier
 * integrals summed over the lattice cells):
 *   rho_vck(G)   = <c, k+q| e^{i(q+G).r} |v, k>      (resonant,      s = 0)
 *   sigma_vck(G) = <v, k+q| e^{i(q+G).r} |c, k>      (anti-resonant, s = 1)
 *   n_G      number of G vectors, 1 <= n_G <= 4096
 *   G_int    [n_G][3] host, integer reciprocal-basis coefficients;
 *            G_int[0] must be (0,0,0) and no q + G may vanish
 *   rho_out  NULL (kept on the device for qcx_chi0) or a device buffer of
 *            [2][n_k][n_occ][n_cond][n_G] c128 receiving (s, k, v, c, G)
 * Errors: QCX_ESTATE (no states), QCX_EINVAL, QCX_ENOMEM. */
int qcx_pair_density(qcx_ctx* ctx, int n_G, const int* G_int, void* rho_out);

/* Pair densities in the optical limit q -> 0 (App. C) for the head and wings
 * of eps: the states must have been set with q_cart = (0, 0, 0); the k states
 * serve on both sides (the k+q states are not read).  Rows G != 0 are the
 * pair densities of qcx_pair_density at q = 0; the G = 0 row, which vanishes
 * like |q|, is replaced by its limit divided by |q| from k.p perturbation
 * theory,
 *   rho_vck(0) / |q|   -> -i qhat.<c k|grad|v k> / (E_c(k) - E_v(k)),
 *   sigma_vck(0) / |q| -> +i qhat.<v k|grad|c k> / (E_c(k) - E_v(k)),
 * with the momentum matrix elements from Gaussian gradient integrals (the
 * same 27-cell Bloch sum), and the Coulomb factor of that row becomes
 * sqrt(4 pi) (|q| cancels).  qcx_chi0 / qcx_chi0_kk / qcx_eps_inv / qcx_loss
 * then give eps and the loss as q -> 0 along qhat (the G = 0 loss is the
 * optical loss function).  Transition energies are recomputed at the same k.
 *   qhat  host [3], any nonzero length (normalised)
 * Other arguments as for qcx_pair_density.
 * Errors: QCX_ESTATE, QCX_EINVAL (q != 0, qhat zero, G list). */
int qcx_pair_density_optical(qcx_ctx* ctx, int n_G, const int* G_int, const double* qhat,
                             void* rho_out);

/* Independent-particle response of Eq. (RPA) at finite broadening:
 *   chi0_GG'(w) = 1/(N_k V) sum_{k,v,c} [ 2 rho(G)^* rho(G') / (w - D + i eta)
 *                                        - 2 sigma(G)^* sigma(G') / (w + D' - i eta) ]
 * with D = E_c(k+q) - E_v(k), D' = E_c(k) - E_v(k+q), V the cell volume; the
 * row index G carries the conjugate.
 *   n_w, w_eV      frequencies (host, eV), 1 <= n_w <= 65536
 *   eta_eV         broadening >= 0 (0 allowed for symmetry checks)
 *   precision      QCX_FP64, QCX_FP32 or QCX_SPLIT_BF16 for the bulk
 *   headwings_fp64 1: the G = 0 row and column are computed in FP64 whatever
 *                  the precision; 0: they use the bulk precision
 *   chi0_out       NULL, or a device buffer [n_w][n_G][n_G] c128 that receives
 *                  chi0 (diagnostic; costs an extra pass)
 * Errors: QCX_ESTATE (no pair densities), QCX_EINVAL, QCX_ENOMEM. */
int qcx_chi0(qcx_ctx* ctx, int n_w, const double* w_eV, double eta_eV, int precision,
             int headwings_fp64, void* chi0_out);

/* FP64 dielectric matrix eps_GG' = delta_GG' - 4 pi chi0_GG' / (|q+G||q+G'|)
 * (the symmetrised form of Eq. RPA) and, per frequency:
 *   lfe = 1: d_G = [eps^-1]_GG by Gauss-Jordan inversion with partial
 *            pivoting (Eq. eps_LFE), for n_G <= 1024;
 *   lfe = 0: d_G = 1 / eps_GG (Eq. eps_noLFE).
 *   diag_out  NULL or device [n_w][n_G] c128 receiving d
 *   epsM_out  NULL or device [n_w] c128 receiving eps_M = 1/d_0
 * A zero or non-finite pivot is reported by qcx_sync / qcx_loss as
 * QCX_ESINGULAR.
 * Errors: QCX_ESTATE (no chi0), QCX_EINVAL (lfe with n_G > 1024), QCX_ENOMEM. */
int qcx_eps_inv(qcx_ctx* ctx, int lfe, void* diag_out, void* epsM_out);

/* Diagonal of the inverse of caller-supplied dielectric matrices (Eq.
 * eps_LFE with lfe = 1, Gauss-Jordan with partial pivoting in FP64 as in
 * qcx_eps_inv; Eq. eps_noLFE, d_G = 1 / eps_GG, with lfe = 0) and the loss
 * -Im d_G: for an eps formed outside the library, e.g. from a model of the
 * screening or another response route.  The context supplies the device,
 * the stream and its working buffers; its pair densities, chi0 and results
 * of qcx_eps_inv are not used (qcx_loss afterwards needs qcx_eps_inv again).
 *   n_w, n_G   matrices and their size, 1 <= n_w <= 65536, 1 <= n_G <= 1024
 *              (lfe = 1) or 65536 (lfe = 0), at most 2^33 elements
 *   eps        device [n_w][n_G][n_G] c128 (read only; copied to a working
 *              buffer of the context)
 *   loss_out   device [n_w][n_G] float64
 *   diag_out   NULL or device [n_w][n_G] c128 receiving d
 *   epsM_out   NULL or device [n_w] c128 receiving eps_M = 1 / d_0
 * Asynchronous.  A zero or non-finite pivot (or eps_GG for lfe = 0) is
 * reported by the next qcx_sync as QCX_ESINGULAR naming the lowest such
 * frequency index.
 * Accuracy: the elimination folds each pivot into its rank-1 update (u_p =
 * (piv - 1) / piv, w_k = piv + 1), which keeps FP64 accuracy for pivots of
 * order one or below, as in eps = 1 - v chi0, at any scale down to the
 * smallest normal doubles; pivots far above one lose about eps |piv|
 * relative accuracy in their row, so such matrices should be scaled first.
 * Errors: QCX_EINVAL (sizes, NULL buffers), QCX_ENOMEM. */
int qcx_eps_inv_given(qcx_ctx* ctx, int n_w, int n_G, const void* eps, int lfe, double* loss_out,
                      void* diag_out, void* epsM_out);

/* qcx_eps_inv_given without any device allocation, for callers that cannot
 * allocate (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as qcx_eps_inv_given (the
 * same kernels, identical bits), except that the singular check is reported
 * in status_out instead of through qcx_sync:
 *   status_out  device int, set to INT_MAX, or to the lowest frequency index
 *               with a zero or non-finite pivot (eps_GG for lfe = 0)
 * The working copy of eps and, when diag_out is NULL, the diagonal live in a
 * 64 MiB array the library holds on each GPU for the life of the process;
 * frequencies run in chunks that fit it (for lfe = 1 a frequency takes
 * 16 n_G^2 bytes, plus 16 n_G without diag_out).  Only kernels and
 * device-to-device copies are enqueued on the context's stream: no
 * allocation, no memset, no synchronisation.  All calls on one GPU share its
 * array, so calls that overlap on one GPU (other streams or contexts) race.
 * Errors: QCX_EINVAL (sizes as qcx_eps_inv_given; a frequency that does not
 * fit 64 MiB; NULL eps, loss_out or status_out), QCX_EDEVICE. */
int qcx_eps_inv_given_noalloc(qcx_ctx* ctx, int n_w, int n_G, const void* eps, int lfe,
                              double* loss_out, void* diag_out, void* epsM_out, int* status_out);

/* Cap the device memory the context's own buffers may hold (all of them but
 * a batch plan's, a surrogate's and a q-binning table's): a call that would
 * grow them beyond `bytes` returns QCX_ENOMEM and keeps the buffers it had;
 * 0 removes the cap (the default).  qcx_memory_used reports their current
 * total.  Errors: QCX_EINVAL (NULL). */
int qcx_set_memory_limit(qcx_ctx* ctx, size_t bytes);
int qcx_memory_used(const qcx_ctx* ctx, size_t* bytes);

/* Loss function at momentum q + G: out[w][G] = Im(-1/eps(w, q+G)) = -Im d_G
 * (Eq. eps_LFE, or Eq. eps_noLFE when qcx_eps_inv ran with lfe = 0).
 *   out  [n_w][n_G] doubles, host (mem = QCX_MEM_HOST: synchronises and
 *        reports deferred errors as qcx_sync does) or device (QCX_MEM_DEVICE:
 *        asynchronous).
 * Errors: QCX_ESTATE (no eps_inv), QCX_EINVAL, QCX_ESINGULAR. */
int qcx_loss(qcx_ctx* ctx, double* out, int mem);

/* chi0 by way of the spectral part (Sec. II.D, Eq. eRPA_spectral and the
 * Kramers-Kronig relations): the pair products of every transition are
 * binned by energy with hat functions of width bin_eV on the grid
 * w_b = b * bin_eV (resonant and anti-resonant transitions separately; a
 * transition at (i + x) bin_eV, 0 <= x < 1, weighs 1 - x on bin i and x on
 * bin i + 1),
 *   S_b(G, G') = sum_t h_b(D_t) rho_t(G)^* rho_t(G'),
 * and the response at each frequency follows from the binned spectral
 * function carried through the energy denominator exactly:
 *   chi0_GG'(w) = 2/(N_k V) sum_b [ S^r_b K(w - w_b + i eta) - S^a_b K(w + w_b - i eta) ],
 *   K(x) = int h(x') / (x - x') dx' / bin_eV (closed form; at eta = 0 the
 *   principal value minus i pi times the binned spectral density).
 * As bin_eV -> 0 this converges to qcx_chi0 at the same eta (error of order
 * (bin_eV / eta)^2); at eta = 0 its imaginary part is the binned spectral
 * part and its real part the Kramers-Kronig transform of it.  Everything
 * runs in FP64: the binning on the vector units over energy-sorted
 * transitions (each bin written once, no atomics: the result does not depend
 * on the launch), the transform as one FP64 matrix product on FP64 MFMA
 * of the [2 n_w][bins] kernel matrix with the [bins][2 n_pairs] spectral
 * function.
 * Afterwards qcx_eps_inv / qcx_loss work as after qcx_chi0.  The transition
 * energies are read back to the host (the call synchronises the stream).
 *   n_w, w_eV, eta_eV (>= 0), chi0_out as for qcx_chi0; bin_eV > 0
 * Device memory: S takes bins x n_G (n_G + 1) x 8 bytes (bins = the energy
 * span of the transitions / bin_eV, both sides).
 * Errors: QCX_ESTATE (no pair densities), QCX_EINVAL (sizes, non-finite
 * values, more than 2^20 bins per side or S above 16 GB: widen bin_eV),
 * QCX_ENOMEM. */
int qcx_chi0_kk(qcx_ctx* ctx, int n_w, const double* w_eV, double eta_eV, double bin_eV,
                void* chi0_out);

/* Loss without local field effects, Eq. (eps_noLFE), for a G list of any
 * length (Sec. III: the high-momentum part of the composite dielectric
 * function, where only the diagonal of Eq. (RPA) is needed):
 *   chi0_GG(w) = 1/(N_k V) sum_{k,v,c} [ 2 |rho(G)|^2 / (w - D + i eta)
 *                                        - 2 |sigma(G)|^2 / (w + D' - i eta) ],
 *   eps_GG = 1 - 4 pi chi0_GG / |q + G|^2,  loss_G(w) = Im(-1 / eps_GG).
 * Works on the states of qcx_set_states; the G list is processed in chunks of
 * 4096 (pair densities, then the diagonal contraction on MFMA in FP32 or
 * split-BF16, or on FP64 MFMA for QCX_FP64).
 *   n_G        >= 1; G_int [n_G][3] host, reciprocal-basis coefficients; no
 *              q + G may vanish; G = 0 is not required
 *   n_w, w_eV, eta_eV, precision as for qcx_chi0
 *   loss_out   device [n_w][n_G] float64
 *   inv_out    NULL or device [n_w][n_G] c128 receiving 1 / eps_GG (the
 *              value qcx_qbin_add bins with kind QCX_QBIN_INV)
 * Asynchronous.  Replaces the context's pair densities (qcx_pair_density
 * must be called again before qcx_chi0).
 * Errors: QCX_ESTATE (no states), QCX_EINVAL, QCX_ENOMEM. */
int qcx_loss_diag(qcx_ctx* ctx, int n_G, const int* G_int, int n_w, const double* w_eV,
                  double eta_eV, int precision, double* loss_out, void* inv_out);

/* One item of a batch: the frequencies of one context's q point. */
typedef struct qcx_item {
  int ctx;              /* index into the context array; its pair densities are used */
  int n_w;              /* number of frequencies, 1..65536 */
  const double* w_eV;   /* host [n_w] frequencies (eV) */
  double eta_eV;        /* broadening (eV), >= 0 */
  double* loss_out;     /* device [n_w][n_G of that context]: the loss of Eq. (eps_LFE) */
} qcx_item;

/* Batched chi0 -> eps -> loss for uneven items (different cells, q points,
 * frequency lists and N_G; Eq. RPA per item).  Every context in ctxs must have
 * current pair densities (qcx_pair_density) and all must be on one device; the
 * work is enqueued on the stream of ctxs[0].  The chi0 bulk of all items runs
 * in one persistent launch over a shared tile list; the FP64 head/wings,
 * assembly, inversion and loss of every item follow.  The sequence is captured
 * once per batch signature (items, frequencies, buffers) into a hipGraph owned
 * by ctxs[0] and replayed on later calls with the same signature; new states
 * or pair densities of the same shapes are picked up by the replay.
 *   precision, headwings_fp64, lfe as for qcx_chi0 / qcx_eps_inv.
 * The K split of each item follows from a target number of MFMA steps (16
 * transitions each) per split, never more than 1024 steps per split in FP32
 * (splits are added in FP64).  With autotuning on (qcx_set_autotune, FP32 and
 * split-BF16), the first call of a signature builds a plan for each target in
 * {128, 256, 512, 1024}, replays and times each with HIP events on ctxs[0]'s
 * stream and keeps the fastest (that call synchronises the stream).  Every
 * replay computes the complete result, so the outputs are those of the kept
 * plan.  Contexts may use different streams: the batch waits on ctxs[0]'s
 * stream for the work already queued on the others, and the others wait for
 * the batch before any later work of theirs.  Asynchronous otherwise;
 * qcx_batch_sync(ctxs[0]) waits and reports QCX_ESINGULAR, and the deferred
 * state checks (QCX_EINVAL / QCX_ENONORTH, as qcx_sync) of every context of
 * the batch, which must all stay alive until then.  With timing on (qcx_set_timing on ctxs[0]),
 * qcx_stage_times reports t[1] the persistent bulk launch, t[4] head/wings +
 * assembly + inversion + loss, t[3] the whole batch.
 * Errors: QCX_EINVAL (sizes, devices, NULL loss_out), QCX_ESTATE (a context
 * without pair densities), QCX_ENOMEM, QCX_EDEVICE. */
int qcx_run_batch(qcx_ctx* const* ctxs, int n_ctx, const qcx_item* items, int n_items,
                  int precision, int headwings_fp64, int lfe);
/* qcx_run_batch with the pair densities of Eq. (RPA) computed inside the
 * batch: for every context c, the G list G_int[c] (host [n_G[c]][3] integer
 * coordinates in the reciprocal basis, G = 0 first, 1 <= n_G[c] <= 1024 with
 * lfe, 4096 without) replaces a qcx_pair_density call.  Every context needs
 * states (qcx_set_states, host or device) and may appear only once in ctxs.
 * q + G, the Coulomb factors, the cell Fourier integrals and the densities
 * (27-cell Bloch sum and band contraction of Sec. III) are part of the
 * captured plan; the q of each context is read from the device copy that
 * qcx_set_states makes, so new states of the same shapes, including a new q,
 * are picked up by the replay.  The G lists and the shapes of the states are
 * part of the plan's signature.  A vanishing q + G is rejected on the host
 * (QCX_EINVAL) from the q last set.  On return (and on success) each
 * context holds the pair densities of its G list, as after qcx_pair_density
 * (usable by qcx_chi0 etc. once the batch has run on the device).  With
 * timing on, t[0] is the pair densities of all contexts.  Arrays n_G and
 * G_int have n_ctx entries; the rest is as for qcx_run_batch.
 * Errors: as qcx_run_batch, and QCX_ESTATE (a context without states),
 * QCX_EINVAL (G lists, a context listed twice). */
int qcx_run_batch_rho(qcx_ctx* const* ctxs, int n_ctx, const int* n_G, const int* const* G_int,
                      const qcx_item* items, int n_items, int precision, int headwings_fp64,
                      int lfe);
int qcx_batch_sync(qcx_ctx* ctx);
/* Plan of the last batch run on ctx (the ctxs[0] of qcx_run_batch):
 * cfg = {target MFMA steps per K split, tiles in the persistent list, blocks
 * launched}, and the wall time spent tuning when the plan was built (ms, 0
 * without tuning).  Errors: QCX_ESTATE (no batch yet). */
int qcx_batch_config(qcx_ctx* ctx, int cfg[3], double* tune_ms);

/* ---------------------------------------------------------------------------
 * Surrogate of the loss (not part of the paper's method): an ensemble of
 * small networks mapping a momentum transfer and an energy to
 * log Im[-1/eps_LFE](Q, w), the quantity of Eq. (eps_LFE) that the rate
 * integral sweeps.  Each member is 49 -> 256 -> 256 -> 256 -> 256 -> 1 with
 * SiLU after the hidden layers (the 49 inputs are the features that
 * qcx_mlp_encode forms); FP32 master weights, bf16 copies for the
 * products (v_mfma_f32_32x32x16_bf16, FP32 accumulation), Adam training on
 * the mean squared error.  Members run on the device and stream of the
 * context they were created from; errors are reported through
 * qcx_last_error of that context.
 *
 * Parameter vector (QCX_MLP_NPARAM floats): per layer l = 1..5 the weight
 * matrix W_l[n_out][n_in] (row-major), then the bias b_l[n_out].
 * ------------------------------------------------------------------------ */
#define QCX_MLP_NIN 49
#define QCX_MLP_NPARAM 210433
typedef struct qcx_mlp qcx_mlp;

/* Create n_members (1..16) networks with zero parameters on ctx. */
int qcx_mlp_create(qcx_mlp** out, qcx_ctx* ctx, int n_members);
/* Free the networks (synchronises the context's stream).  Safe on NULL. */
int qcx_mlp_destroy(qcx_mlp* m);
/* Copy host params[QCX_MLP_NPARAM] into member `member` and reset its Adam
 * state.  Synchronous.  Errors: QCX_EINVAL (index, NULL, non-finite). */
int qcx_mlp_set_params(qcx_mlp* m, int member, const float* params);
/* Copy member `member`'s FP32 parameters to host params.  Synchronous. */
int qcx_mlp_get_params(qcx_mlp* m, int member, float* params);
/* Network output y[i] for device inputs x[n][QCX_MLP_NIN] (device y[n]).
 * Async. */
int qcx_mlp_forward(qcx_mlp* m, int member, int n, const float* x, float* y);
/* Gradient of mean_i (y_i - t_i)^2 over device x[n][QCX_MLP_NIN], t[n] (n <= 16384)
 * into host grad[QCX_MLP_NPARAM]; the loss into *loss if not NULL.  No
 * update.  Synchronous. */
int qcx_mlp_grad(qcx_mlp* m, int member, int n, const float* x, const float* t, float* grad,
                 float* loss);
/* n_steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on
 * mini-batches: step s uses samples order[s*batch .. (s+1)*batch) of the
 * device data x[n_data][QCX_MLP_NIN], t[n_data]; order is a device int array of
 * n_steps*batch indices in [0, n_data) (checked before the first step).
 * Learning rate lr1 + (lr0 - lr1)(1 + cos(pi s / n_steps))/2.  batch
 * 1..16384.  Per-step losses into host loss_hist[n_steps] if not NULL (then
 * synchronous; otherwise asynchronous). */
int qcx_mlp_train(qcx_mlp* m, int member, int n_data, const float* x, const float* t, int batch,
                  int n_steps, const int* order, float lr0, float lr1, float* loss_hist);
/* Input and output scaling shared by qcx_mlp_encode and qcx_mlp_query.
 * The QCX_MLP_NIN features of a query (Q, w), formed in FP64 and rounded to
 * FP32, are
 *   2|Q|/q_max - 1;  Q/|Q| (zero for Q = 0);  2w/w_max - 1;
 *   sin, cos of pi 2^(j/2) w/w_max for j = 0..7;
 *   sin, cos of pi 2^(j/2) |Q|/q_max for j = 0..7;
 *   sin, cos of h Q.a_i for i = 1..3, h = 1, 2,
 * with a_i the primitive vectors lattice[3i .. 3i+2] (host, bohr) of the
 * crystal the loss belongs to; the target is
 * t = (log max(L, 1e-30) - mu)/sigma; the error estimate of a query is
 * calib * sigma * (sample standard deviation of the members' outputs), an
 * estimate of the relative error of the returned loss.  Errors: QCX_EINVAL
 * (non-positive scales or sigma, negative calib, non-finite values, NULL
 * lattice). */
int qcx_mlp_set_encoding(qcx_mlp* m, double q_max, double w_max_eV, const double* lattice,
                         double mu, double sigma, double calib);
/* Features x[n][QCX_MLP_NIN] (device float) of device queries qw[n][4] = (Qx, Qy, Qz
 * in bohr^-1, w in eV), and, if loss (device double [n]) and t are not
 * NULL, the training targets t[n].  Errors: QCX_ESTATE before
 * qcx_mlp_set_encoding.  Async. */
int qcx_mlp_encode(qcx_mlp* m, int n, const double* qw, const double* loss, float* x, float* t);
/* Surrogate answer for device queries qw[n][4]: loss[n] = exp(mu + sigma *
 * mean of the members), err[n] (may be NULL) the error estimate.  If
 * reject_idx is not NULL (then err and n_reject must be too), the indices
 * with err > tol are written to reject_idx in ascending order and their
 * number to the host *n_reject; the caller recomputes those points with the
 * method itself (qcx_chi0 / qcx_eps_inv / qcx_loss).  Synchronous when
 * rejecting, otherwise asynchronous. */
int qcx_mlp_query(qcx_mlp* m, int n, const double* qw, double* loss, double* err, double tol,
                  int* reject_idx, int* n_reject);
/* Surrogate answer with fallback to the method for one momentum: the loss at
 * Q = q + G (q of the states last set on ctx, G the list G_int[n_G][3] in
 * the reciprocal basis with G_int[0] = (0,0,0), as for qcx_pair_density) and
 * the frequencies w_eV (host [n_w], eV), into loss_out (device double
 * [n_w][n_G]).  The networks answer every point.  Accuracy is measured per
 * loss curve along frequency (one curve per G over this call's frequencies):
 * the error of a point in units of its curve's maximum, |L - L_method| /
 * max_w |L_method|; a point's estimate in these units is its relative
 * estimate (qcx_mlp_query) times its predicted loss over the largest
 * predicted loss of its curve.  Every frequency with a point whose estimate
 * exceeds tol is recomputed by the method on ctx (qcx_pair_density for G_int,
 * qcx_chi0 at those frequencies with `precision` and FP64 head/wings,
 * qcx_eps_inv with LFE, qcx_loss) and its row replaced.  err_out (device
 * double [n_w][n_G], may be NULL) receives the estimates in curve units (a
 * non-finite estimate or prediction counts as infinite); *n_fallback (may be
 * NULL) the number of recomputed frequencies.  ctx's pair densities and results are overwritten
 * when a fallback runs.  The networks and ctx must be on one device.
 * The call waits for the networks' answers and the rejections (on the
 * networks' stream); the fallback rows are then enqueued on ctx's stream and
 * the call returns: loss_out is complete once ctx's stream has run them, and
 * their deferred state checks and a singular eps are reported by the next
 * synchronising call on ctx (qcx_sync).  Errors: as the calls above;
 * QCX_EINVAL beyond 2^26 points, QCX_ESTATE before qcx_mlp_set_encoding or
 * qcx_set_states. */
int qcx_mlp_infer(qcx_mlp* m, qcx_ctx* ctx, int n_G, const int* G_int, int n_w,
                  const double* w_eV, double eta_eV, double tol, int precision, double* loss_out,
                  double* err_out, int* n_fallback);

/* ------------------------------------------------------------------------
 * From the dielectric function to scattering rates (Sec. III binning, Eq.
 * dynamic_structure_factor, Eq. general_rate with the nonrelativistic cross
 * section of Eq. cross_section).
 *
 * A qcx_qbin accumulates the finite-momentum dielectric function
 * eps(w, q + G) of any number of (q, G) entries into a three-dimensional
 * momentum grid: n_shell spherical shells of width dq (bohr^-1 = alpha m_e;
 * shell s holds s dq <= |q| < (s + 1) dq), each split into n_theta x n_phi
 * angular bins uniform in theta = acos(q_z / |q|) on [0, pi] and in
 * phi = atan2(q_y, q_x) on [0, 2 pi); bin (s, i, j) has index
 * (s n_theta + i) n_phi + j.  The paper uses n_theta = 9, n_phi = 16,
 * dq = 0.02.  A bin's value is the mean of the complex eps of its entries.
 * Work runs on the context's device and stream; errors are reported through
 * qcx_last_error of that context.
 * ------------------------------------------------------------------------ */
typedef struct qcx_qbin qcx_qbin;
enum { QCX_QBIN_EPS = 0, QCX_QBIN_INV = 1 };

/* Empty table for n_w frequencies (1..65536), n_shell >= 1, dq > 0,
 * 1 <= n_theta <= 360, 1 <= n_phi <= 720, at most 2^26 bins and 32 GB
 * (n_w x bins x 16 bytes of device memory).  Errors: QCX_EINVAL, QCX_ENOMEM. */
int qcx_qbin_create(qcx_qbin** out, qcx_ctx* ctx, int n_w, int n_shell, double dq, int n_theta,
                    int n_phi);
/* Free the table (synchronises the stream).  Safe on NULL. */
int qcx_qbin_destroy(qcx_qbin* b);
/* Forget every entry. */
int qcx_qbin_reset(qcx_qbin* b);
/* Add n entries: momenta qvec[n][3] (host, Cartesian, bohr^-1) and values
 * vals (device c128, vals[w * ld + e], ld >= n): eps itself
 * (kind = QCX_QBIN_EPS) or 1/eps (kind = QCX_QBIN_INV: [eps^-1]_GG of
 * qcx_eps_inv's diag_out, or inv_out of qcx_loss_diag).  Entries with
 * |q| >= n_shell dq are skipped.  The bins of the entries are found on the
 * host; the sums run on the device, deterministically.  Asynchronous
 * (vals must stay valid until the stream reaches the call).
 * Errors: QCX_EINVAL (sizes, kind, non-finite momenta). */
int qcx_qbin_add(qcx_qbin* b, int n, const double* qvec, const void* vals, int ld, int kind);
/* Bin means, interpolation of bins without entries, and the isotropic
 * dynamic structure factor.  Interpolation runs in sweeps: every empty bin
 * with at least one filled neighbour among its 26 adjacent bins (phi
 * periodic; shell and theta not) takes the mean of those neighbours, using
 * only bins filled before the sweep, until no bin changes.  Then
 *   S_out[w][s] = solid-angle weighted mean over the filled bins of shell s
 *                 of q_s^2 / (2 pi alpha) Im(-1 / eps),  q_s = (s + 1/2) dq
 * in (alpha m_e)^2 (NaN for a shell no sweep reaches).
 *   eps_out    NULL or device [n_w][bins] c128 (the binned eps)
 *   S_out      device [n_w][n_shell] float64
 *   state_out  NULL or host [bins]: 1 entries, 2 interpolated, 0 empty
 * The table keeps its entries (more may be added and finish called again).
 * Errors: QCX_EINVAL, QCX_ENOMEM. */
int qcx_qbin_finish(qcx_qbin* b, void* eps_out, double* S_out, int* state_out);

/* Dark-matter halo and interaction for qcx_qbin_rate_halo: the standard
 * truncated Maxwell-Boltzmann halo (Galactic dispersion v0, escape speed
 * vesc, Earth speed vE, local density rho_chi) and a mediator of mass m_med
 * (F_DM(q) = ((alpha m_e)^2 + m_med^2) / (q^2 + m_med^2), Eq. F_DM;
 * m_med = INFINITY: heavy limit F_DM = 1; m_med = 0: light limit). */
typedef struct qcx_halo {
  double m_chi_eV;         /* dark-matter mass */
  double m_med_eV;         /* mediator mass, >= 0 or INFINITY */
  double sigma_e_cm2;      /* reference cross section */
  double rho_T_g_cm3;      /* target mass density */
  double rho_chi_GeV_cm3;  /* 0.3 in the paper */
  double v0_kms;           /* 238 */
  double vE_kms;           /* 250.2 in the paper */
  double vesc_kms;         /* 544 in the paper */
} qcx_halo;

/* Halo scattering rate per unit target mass (events / kg / year / eV) at
 * the n_w frequencies w_eV (host, >= 0) of the table, from S_iso (device
 * [n_w][n_shell], qcx_qbin_finish's S_out):
 *   dR/dw = rho_chi / (m_chi rho_T) sigma_e / (4 pi mu^2)
 *           sum_s dq q_s |F_DM(q_s)|^2 S(w, q_s) eta(v_min(q_s, w)),
 * v_min = q / (2 m_chi) + w / q, eta(v) = int d^3u f(u) / |u| over |u| > v
 * (the halo's mean inverse speed, closed form), mu the DM-electron reduced
 * mass; shells where S is NaN contribute nothing.  Natural units inside;
 * CODATA 2018 constants, year = 365.25 days.  rate_out: device [n_w].
 * Asynchronous.  Errors: QCX_EINVAL (non-positive parameters). */
int qcx_qbin_rate_halo(qcx_qbin* b, const double* w_eV, const double* S_iso, const qcx_halo* h,
                       double* rate_out);

/* Tile selection of the chi0 bulk kernel (qcx_chi0 with FP32 or split-BF16).
 * mode 1 (default): on the first qcx_chi0 of each shape (device, precision,
 * N_G, padded N_T, padded rows), every candidate configuration - K split
 * (a power of two up to 64, at least enough that no split sums more than
 * 1024 MFMA steps of 16 transitions in FP32: the splits are added in FP64)
 * and the LDS pipeline (2 or 3 stages, or 3 stages with the transition slab
 * one step ahead of the weights), within 160 KB of LDS - is timed on the
 * real operands with HIP events and the fastest is kept for the process;
 * that call synchronises the stream.  Shapes whose FP32 partial sums would
 * exceed 8 GB run in chunks of frequency rows reduced into FP64.  The
 * result used is always computed with the chosen configuration.  mode 0: a
 * fixed heuristic.  Tuning is skipped for shapes whose single launch is
 * estimated above 0.5 s.
 * Errors: QCX_EINVAL (mode). */
int qcx_set_autotune(qcx_ctx* ctx, int mode);
/* Configuration of the last bulk launch: cfg = {K split, pipeline (2 or 3 LDS stages;
 * 4: three stages with the transition slab one step ahead of the weights),
 * row fragments per wave} (zeros if there was no bulk), and the time spent
 * tuning in that call (ms, 0 when the shape was cached).  Errors:
 * QCX_ESTATE before qcx_chi0. */
int qcx_bulk_config(qcx_ctx* ctx, int cfg[3], double* tune_ms);
/* Force the LDS pipeline of the chi0 bulk kernel (2, 3 or 4 as reported by
 * qcx_bulk_config; the K split stays heuristic and tuning is skipped), or
 * restore the tuned / heuristic choice with 0.  For tests and experiments.
 * Errors: QCX_EINVAL (other values; at qcx_chi0 if the pipeline does not fit
 * the shape). */
int qcx_set_bulk_pipeline(qcx_ctx* ctx, int nst);

/* Per-stage device time of the most recent calls, in milliseconds, measured
 * with HIP events on the context's stream (enabled by qcx_set_timing):
 * t[0] pair_density, t[1] chi0 bulk kernel, t[2] chi0 FP64 head/wings,
 * t[3] chi0 total, t[4] eps assembly + inversion, t[5] launches of the bulk
 * kernel counted (after qcx_chi0_kk: t[1] is the binning kernel), t[6] the
 * FP64 transform product of qcx_chi0_kk.  Synchronises the stream.  Values accumulate until
 * qcx_set_timing is called again. */
int qcx_stage_times(qcx_ctx* ctx, double t[7]);
int qcx_set_timing(qcx_ctx* ctx, int enable);

/* Library build description (kernel variants compiled in). */
const char* qcx_build_info(void);

#ifdef __cplusplus
}
#endif

#endif /* QCX_H */
