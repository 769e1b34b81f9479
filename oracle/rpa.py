"""RPA response, dielectric matrix, inverse and loss (oracle, FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Written from Sec. II.D of the paper:

* Eq. (RPA): eps_GG'(w, q) = delta_GG' - 4 pi alpha / (V |q+G||q+G'|)
  sum_{ik, jk'} (f_ik - f_jk') <ik|e^{-i(q+G)r}|jk'><jk'|e^{i(q+G')r}|ik>
  / (w - (w_jk' - w_ik) + i sgn(w_jk' - w_ik) eta), with k' = k + q and
  T = 0 occupations f = 2 (occupied) or 0 (empty).
* Eq. (eps_LFE): eps(w, q+G) = 1 / [eps^{-1}]_GG; the macroscopic eps_M is
  the G = 0 entry.
* Eq. (eps_noLFE): off-diagonal entries dropped, eps^noLFE = eps_GG; for the
  many high-momentum G of the composite dielectric function of Sec. III only
  the diagonal of chi0 is formed (loss_diag, loss_composite).
* The loss is Im(-1/eps) (Eq. dynamic_structure_factor uses it).

Readings of points the paper leaves open (each also listed in the design doc):

* Hartree atomic units, so 4 pi alpha -> 4 pi; eV at the boundary with
  1 Ha = 27.211386245988 eV.
* The k sum carries the weight 1/N_k (crystal volume N_k V), the standard
  Adler-Wiser normalisation, so chi0 does not grow with the k grid.
* Finite eta, evaluated as written by chi0(): the time-ordered
  prescription, +i eta on the resonant (v -> c) term and -i eta on the
  anti-resonant (c -> v) term.  chi0_kk() is the binned spectral route of
  Sec. II.D (hat-function bins, exact transform; at eta = 0 the
  Kramers-Kronig form).
* Synthetic states are not time-reversal symmetric, so the anti-resonant
  pair density sigma_vck(Q) = <v,k+q|e^{iQr}|c,k> is kept explicitly.
* The row index G carries the complex conjugate.

Transition index t = ((s * n_k + k) * n_occ + v) * n_cond + c with s = 0 for
the resonant pair density rho_vck(Q) = <c,k+q|e^{iQr}|v,k> and s = 1 for
sigma_vck(Q); both rows are stored in R[t][G].
"""
from __future__ import annotations

import math

import numpy as np

from . import gto

HARTREE_EV = 27.211386245988


def q_plus_g(lat, q_cart, G_int) -> np.ndarray:
    """Cartesian Q_G = q + G for integer reciprocal-basis triples G_int."""
    b = gto.reciprocal_basis(lat)
    return np.asarray(q_cart, np.float64)[None, :] + np.asarray(G_int, np.float64) @ b


def pair_densities(M: np.ndarray, C_k: np.ndarray, C_kq: np.ndarray, n_occ: int) -> np.ndarray:
    """R[2][k][v][c][G] from the AO matrix M[k][G][mu][nu].

    rho_vck(G)   = sum_{mu nu} C_mu,c(k+q)^* M_mu,nu(k; Q_G) C_nu,v(k)
    sigma_vck(G) = sum_{mu nu} C_mu,v(k+q)^* M_mu,nu(k; Q_G) C_nu,c(k)
    Parity: pinned by orthonormality at Q = 0 and by the all-band sum identity.
    """
    nk, ng, nao, _ = M.shape
    nb = C_k.shape[2]
    nc = nb - n_occ
    MC = np.matmul(M, C_k[:, None, :, :])                  # [k][G][mu][b]
    CqH = np.conj(np.swapaxes(C_kq, 1, 2))[:, None]        # [k][1][b][mu]
    B = np.matmul(CqH, MC)                                 # [k][G][b'][b] = <b',k+q|..|b,k>
    R = np.empty((2, nk, n_occ, nc, ng), np.complex128)
    # resonant: bra c at k+q, ket v at k
    R[0] = np.transpose(B[:, :, n_occ:, :n_occ], (0, 3, 2, 1))
    # anti-resonant: bra v at k+q, ket c at k
    R[1] = np.transpose(B[:, :, :n_occ, n_occ:], (0, 2, 3, 1))
    return R


def pair_densities_from_workload(wl_cell, wl_basis, lattice_range, k_frac, q_cart, G_int,
                                 C_k, C_kq, n_occ, k_chunk: int = 64) -> np.ndarray:
    """R for one q, the AO matrix built in k chunks to bound memory."""
    Q = q_plus_g(wl_cell.lat, q_cart, G_int)
    F = gto.cell_ft(wl_cell.lat, wl_cell.xyz, wl_basis.shell_atom, wl_basis.shell_l,
                    wl_basis.shell_exp, lattice_range, Q)
    nT, nG, nao, _ = F.shape
    Ff = F.reshape(nT, -1)
    nk = len(k_frac)
    nc = C_k.shape[2] - n_occ
    R = np.empty((2, nk, n_occ, nc, nG), np.complex128)
    for k0 in range(0, nk, k_chunk):
        k1 = min(nk, k0 + k_chunk)
        ph = gto.bloch_phases(k_frac[k0:k1], lattice_range)
        M = (ph @ Ff).reshape(k1 - k0, nG, nao, nao)
        R[:, k0:k1] = pair_densities(M, C_k[k0:k1], C_kq[k0:k1], n_occ)
    return R


def transition_energies(E_k, E_kq, n_occ):
    """Delta[k][v][c] = E_c(k+q) - E_v(k) and Delta'[k][v][c] = E_c(k) - E_v(k+q) (Ha)."""
    ek = np.asarray(E_k, np.float64) / HARTREE_EV
    ekq = np.asarray(E_kq, np.float64) / HARTREE_EV
    d_res = ekq[:, None, n_occ:] - ek[:, :n_occ, None]
    d_anti = ek[:, None, n_occ:] - ekq[:, :n_occ, None]
    return d_res, d_anti


def transition_weights(E_k, E_kq, n_occ, w_eV, eta_eV, volume) -> np.ndarray:
    """W[w][t]: the occupation factor, energy denominator and 1/(N_k V) of Eq. (RPA).

    resonant     (i = v at k, j = c at k+q):  2 / (N_k V (w - Delta + i eta))
    anti-resonant(i = c at k, j = v at k+q): -2 / (N_k V (w + Delta' - i eta))
    """
    nk = np.asarray(E_k).shape[0]
    d_res, d_anti = transition_energies(E_k, E_kq, n_occ)
    w = np.asarray(w_eV, np.float64)[:, None] / HARTREE_EV
    eta = float(eta_eV) / HARTREE_EV
    norm = 1.0 / (nk * float(volume))
    wr = 2.0 * norm / (w - d_res.reshape(1, -1) + 1j * eta)
    wa = -2.0 * norm / (w + d_anti.reshape(1, -1) - 1j * eta)
    return np.concatenate([wr, wa], axis=1)


def chi0(R: np.ndarray, W: np.ndarray) -> np.ndarray:
    """chi0[w][G][G'] = sum_t R[t][G]^* W[w][t] R[t][G'] (row G conjugated).

    Parity: pinned by Hermiticity at w = 0, eta = 0; the sign of the
    anti-Hermitian part; the large-w moments; k-grid independence of the
    first moment; a one-transition closed form.
    """
    Rt = R.reshape(-1, R.shape[-1])
    out = np.empty((W.shape[0], Rt.shape[1], Rt.shape[1]), np.complex128)
    RH = np.conj(Rt).T
    for iw in range(W.shape[0]):
        out[iw] = (RH * W[iw][None, :]) @ Rt
    return out


def coulomb_sqrt(Qc: np.ndarray) -> np.ndarray:
    """sqrt(4 pi) / |q + G| (the symmetrised Coulomb factor)."""
    qn = np.linalg.norm(np.asarray(Qc, np.float64), axis=1)
    if np.any(qn == 0.0):
        raise ValueError("q + G = 0")
    return math.sqrt(4.0 * math.pi) / qn


def epsilon(chi: np.ndarray, Qc: np.ndarray) -> np.ndarray:
    """eps_GG' = delta_GG' - 4 pi chi0_GG' / (|q+G| |q+G'|)."""
    v = coulomb_sqrt(Qc)
    ng = len(v)
    return np.eye(ng)[None] - v[None, :, None] * chi * v[None, None, :]


def inverse_diagonal(eps: np.ndarray) -> np.ndarray:
    """[eps^{-1}]_GG for each frequency (LAPACK getrf/getri through numpy)."""
    inv = np.linalg.inv(eps)
    return np.diagonal(inv, axis1=1, axis2=2).copy()


def loss_lfe(eps: np.ndarray) -> np.ndarray:
    """loss[w][G] = Im(-1/eps(w, q+G)) = -Im [eps^{-1}]_GG (Eq. eps_LFE)."""
    return -np.imag(inverse_diagonal(eps))


def loss_nolfe(eps: np.ndarray) -> np.ndarray:
    """loss[w][G] = Im(-1/eps_GG) (Eq. eps_noLFE)."""
    d = np.diagonal(eps, axis1=1, axis2=2)
    return np.imag(-1.0 / d)


def chi0_diagonal(R: np.ndarray, W: np.ndarray) -> np.ndarray:
    """chi0[w][G] = sum_t W[w][t] |R[t][G]|^2, the diagonal of Eq. (RPA) alone
    (what Eq. eps_noLFE needs).  Parity: equals the diagonal of chi0()."""
    Rt = R.reshape(-1, R.shape[-1])
    return W @ (np.abs(Rt) ** 2)


def eps_diag(cell, basis, lattice_range, k_frac, n_occ, G_int, states, w_eV, eta_eV):
    """eps_GG = 1 - 4 pi chi0_GG / |q + G|^2 for any G list (Eq. eps_noLFE's
    diagonal; no G = 0 needed), complex [n_w][n_G]."""
    R = pair_densities_from_workload(cell, basis, lattice_range, k_frac, states.q_cart, G_int,
                                     states.C_k, states.C_kq, n_occ)
    volume = abs(float(np.linalg.det(np.asarray(cell.lat, np.float64))))
    W = transition_weights(states.E_k, states.E_kq, n_occ, w_eV, eta_eV, volume)
    chi = chi0_diagonal(R, W)
    v = coulomb_sqrt(q_plus_g(cell.lat, states.q_cart, G_int))
    return 1.0 - (v * v)[None, :] * chi


def loss_diag(cell, basis, lattice_range, k_frac, n_occ, G_int, states, w_eV, eta_eV):
    """noLFE loss for any G list (Eq. eps_noLFE; no G = 0 needed):
    Im(-1 / eps_GG) with eps_GG = 1 - 4 pi chi0_GG / |q + G|^2.
    Parity: equals loss_nolfe() of the full path on the same G."""
    return np.imag(-1.0 / eps_diag(cell, basis, lattice_range, k_frac, n_occ, G_int, states, w_eV,
                                   eta_eV))


def composite_split(lat, q_cart, G_int, q_lfe: float):
    """Indices of the G with |q + G| <= q_lfe (the LFE block, in the given
    order; it must start with G = 0) and of the rest (Sec. III, the composite
    dielectric function)."""
    qn = np.linalg.norm(q_plus_g(lat, q_cart, G_int), axis=1)
    inner = np.nonzero(qn <= q_lfe)[0]
    outer = np.nonzero(qn > q_lfe)[0]
    if len(inner) == 0 or inner[0] != 0 or np.any(np.asarray(G_int)[0] != 0):
        raise ValueError("the LFE block must start with G = 0")
    return inner, outer


def loss_composite(cell, basis, lattice_range, k_frac, n_occ, G_int, states, w_eV, eta_eV,
                   q_lfe: float):
    """Composite loss (Sec. III): Eq. (eps_LFE) from the inverse of eps over
    the G with |q + G| <= q_lfe, Eq. (eps_noLFE) for the G beyond; result in
    the order of G_int."""
    G = np.asarray(G_int)
    inner, outer = composite_split(cell.lat, states.q_cart, G, q_lfe)
    out = np.empty((len(w_eV), len(G)))
    out[:, inner] = solve(cell, basis, lattice_range, k_frac, n_occ, G[inner], states, w_eV,
                          eta_eV, lfe=True)
    if len(outer):
        out[:, outer] = loss_diag(cell, basis, lattice_range, k_frac, n_occ, G[outer], states,
                                  w_eV, eta_eV)
    return out


# --------------------------------------------------------------------------
# Kramers-Kronig route (Sec. II.D, Eq. eRPA_spectral): the spectral part of
# Eq. (RPA) binned by transition energy, then carried back to every
# frequency.  Each transition's delta function is shared between its two
# nearest bins with hat weights h_b(x) = max(0, 1 - |x - w_b| / d); the binned
# spectral density is the piecewise-linear function sum_b S_b h_b(x) / d, and
# its response at w is the integral of that density against the energy
# denominator, which for one hat is K(x) = I(x / d) / d with
#     I(z) = int_{-1}^{1} (1 - |y|) / (z - y) dy.
# --------------------------------------------------------------------------
def hat_kernel(z) -> np.ndarray:
    """I(z) in closed form: (z + 1) log(z + 1) - 2 z log z + (z - 1) log(z - 1),
    principal complex logarithm (Im z != 0 keeps the segment [z - 1, z + 1]
    off the branch cut); on the real axis the sign of the zero imaginary part
    selects the limit from above (+0) or below (-0); 0 log 0 = 0.  The three
    terms grow like |z| log|z| while I(z) falls like 1/z, so the sum loses
    about log10(|z|^2 log|z|) digits: it is evaluated in extended precision
    (x86 long double, 64-bit mantissa) and returned in complex128.
    Parity: pinned by numerical quadrature of the defining integral."""
    z = np.asarray(z, np.clongdouble)

    def xlogx(u):
        out = np.zeros_like(u)
        nz = u != 0
        out[nz] = u[nz] * np.log(u[nz])
        return out

    def shift(u, a):  # u + a with the imaginary part (and the sign of a zero) kept
        v = np.empty_like(u)
        v.real = u.real + a
        v.imag = u.imag
        return v

    return (xlogx(shift(z, 1.0)) - 2.0 * xlogx(z) + xlogx(shift(z, -1.0))).astype(np.complex128)


def spectral_bins(E: np.ndarray, bin_eV: float):
    """Bin centres b d (Ha) covering every energy of E (Ha) and hat weights
    H[b][t] (each column sums to 1)."""
    d = bin_eV / HARTREE_EV
    b_lo = int(np.floor(E.min() / d)) - 1
    b_hi = int(np.floor(E.max() / d)) + 2
    centres = np.arange(b_lo, b_hi + 1) * d
    H = np.maximum(0.0, 1.0 - np.abs(E[None, :] - centres[:, None]) / d)
    return centres, H


def chi0_kk(R, E_k, E_kq, n_occ, w_eV, eta_eV, bin_eV, volume) -> np.ndarray:
    """chi0[w][G][G'] from the binned spectral part:
    sum_b S^r_b K(w - w_b + i eta) - sum_b S^a_b K(w + w_b - i eta), with
    S_b = 2/(N_k V) sum_t h_b(D_t) R_t(G)^* R_t(G') per side (D = E_c(k+q) -
    E_v(k) resonant, D' = E_c(k) - E_v(k+q) anti-resonant).  eta = 0 gives the
    spectral part as the imaginary part and its Kramers-Kronig transform as
    the real part.
    Parity: tends to chi0() at the same eta as bin_eV -> 0 (second order)."""
    nk = np.asarray(E_k).shape[0]
    d = bin_eV / HARTREE_EV
    eta = float(eta_eV) / HARTREE_EV
    w = np.asarray(w_eV, np.float64) / HARTREE_EV
    d_res, d_anti = transition_energies(E_k, E_kq, n_occ)
    ng = R.shape[-1]
    norm = 2.0 / (nk * float(volume))
    out = np.zeros((len(w), ng, ng), np.complex128)
    for side, E, sgn in ((0, d_res.reshape(-1), 1.0), (1, d_anti.reshape(-1), -1.0)):
        Rs = R[side].reshape(-1, ng)
        centres, H = spectral_bins(E, bin_eV)
        RH = np.conj(Rs).T
        S = np.stack([(RH * H[b][None, :]) @ Rs for b in range(len(centres))]) * norm
        # resonant K(w - w_b + i eta), limit from above at eta = 0;
        # anti-resonant -K(w + w_b - i eta), limit from below at eta = 0
        x = (w[:, None] - sgn * centres[None, :]) / d
        z = np.empty(x.shape, np.complex128)
        z.real = x
        z.imag = sgn * eta / d if eta > 0 else sgn * 0.0   # signed zero picks the side
        K = hat_kernel(z) / d
        out += sgn * np.einsum("wb,bgh->wgh", K, S)
    return out


# --------------------------------------------------------------------------
# Optical limit (App. C): for q -> 0 the G = 0 pair densities vanish like
# |q|, and by first-order k.p perturbation
#     <i k| e^{-iq.r} |j k+q>  ->  -(i/m) q.<i k|grad|j k> / (w_jk - w_ik),
# so rho_vck(q) / |q| -> -i qhat.P_cv / D and sigma_vck(q) / |q| ->
# +i qhat.P_vc / D with P_ab = <a k|grad|b k> (anti-Hermitian), D = E_c - E_v
# at the same k, m = 1.  With these as the G = 0 row (and the Coulomb factor
# of that row sqrt(4 pi), |q| cancelled) the head and wings of Eq. (RPA) are
# their q -> 0 limits; the G != 0 rows are the pair densities at q = 0.
# --------------------------------------------------------------------------
def momentum_bands(cell, basis, lattice_range, k_frac, C_k) -> np.ndarray:
    """P[k][c][a][b] = <a k| d/dr_c |b k> in the band basis (bohr^-1)."""
    D = gto.grad_matrix(cell.lat, cell.xyz, basis.shell_atom, basis.shell_l, basis.shell_exp,
                        lattice_range, k_frac)
    C = np.asarray(C_k)
    return np.einsum("kma,kcmn,knb->kcab", np.conj(C), D, C)


def optical_row(P, E_k, n_occ, qhat) -> np.ndarray:
    """R0[s][k][v][c]: the G = 0 pair densities divided by |q| in the limit
    (s = 0: -i qhat.P_cv / D, s = 1: +i qhat.P_vc / D)."""
    qh = np.asarray(qhat, np.float64) / np.linalg.norm(qhat)
    Pq = np.einsum("c,kcab->kab", qh, P)                       # qhat . P
    ek = np.asarray(E_k, np.float64) / HARTREE_EV
    D = ek[:, None, n_occ:] - ek[:, :n_occ, None]              # [k][v][c]
    res = -1j * np.transpose(Pq[:, n_occ:, :n_occ], (0, 2, 1)) / D    # P_cv -> [k][v][c]
    anti = 1j * Pq[:, :n_occ, n_occ:] / D                              # P_vc
    return np.stack([res, anti])


def pair_densities_optical(cell, basis, lattice_range, k_frac, G_int, C_k, E_k, n_occ, qhat):
    """R[s][k][v][c][G] for q -> 0: G != 0 from Eq. (RPA) at q = 0 (states at k
    on both sides), G = 0 (must be G_int[0]) from optical_row."""
    G = np.asarray(G_int).reshape(-1, 3)
    if np.any(G[0] != 0):
        raise ValueError("G_int[0] must be 0")
    R = pair_densities_from_workload(cell, basis, lattice_range, k_frac, np.zeros(3), G, C_k, C_k,
                                     n_occ)
    P = momentum_bands(cell, basis, lattice_range, k_frac, C_k)
    R[..., 0] = optical_row(P, E_k, n_occ, qhat)
    return R


def coulomb_sqrt_optical(lat, G_int) -> np.ndarray:
    """sqrt(4 pi) / |G| with the G = 0 entry sqrt(4 pi) (its |q| went into R)."""
    Qc = q_plus_g(lat, np.zeros(3), G_int)
    n = np.linalg.norm(Qc, axis=1)
    v = np.full(len(n), math.sqrt(4.0 * math.pi))
    v[1:] = v[1:] / n[1:]
    return v


def epsilon_optical(chi: np.ndarray, lat, G_int) -> np.ndarray:
    """eps_GG' = delta - v_G v_G' chi_GG' with coulomb_sqrt_optical."""
    v = coulomb_sqrt_optical(lat, G_int)
    n = chi.shape[-1]
    return np.eye(n)[None] - v[None, :, None] * chi * v[None, None, :]


def optical_head_wings(P, E_k, n_occ, w_eV, eta_eV, qhat, volume, rho, gnorm):
    """App. C's head eps_00 and wings eps_0G', eps_G0 written out as sums over
    (k, v, c) and both orderings (i, j) of each transition, with 1/N_k (R1).
    Signs: the wing eps_0G' as printed; the head and eps_G0 with the signs
    that Eq. (RPA) gives in the limit (the appendix prints + in front of the
    head sum, which makes Im eps_00 < 0 for w > 0, and - in front of eps_G0,
    which breaks eps_G0 = conj(eps_0G) for real w below the gap at eta -> 0).
    rho: [2][k][v][c][G] pair densities at q = 0 of the G != 0 columns
    (<c|e^{iGr}|v>, <v|e^{iGr}|c>), gnorm [G] their |G|.
    Returns (eps00[w], eps0G[w][G], epsG0[w][G])."""
    qh = np.asarray(qhat, np.float64) / np.linalg.norm(qhat)
    Pq = np.einsum("c,kcab->kab", qh, P)
    ek = np.asarray(E_k, np.float64) / HARTREE_EV
    D = ek[:, None, n_occ:] - ek[:, :n_occ, None]              # [k][v][c]
    w = np.asarray(w_eV, np.float64)[:, None, None, None] / HARTREE_EV
    eta = float(eta_eV) / HARTREE_EV
    nk = ek.shape[0]
    pre = 4.0 * math.pi / (float(volume) * nk)
    Pcv = np.transpose(Pq[:, n_occ:, :n_occ], (0, 2, 1))      # qhat.<c|grad|v> as [k][v][c]
    Pvc = Pq[:, :n_occ, n_occ:]                                # qhat.<v|grad|c>
    # (i, j) = (v, c): f_i - f_j = 2, w_j - w_i = D, denominator w - D + i eta;
    # (i, j) = (c, v): f_i - f_j = -2, w_j - w_i = -D, denominator w + D - i eta
    dr = 1.0 / (w - D[None] + 1j * eta)
    da = 1.0 / (w + D[None] - 1j * eta)
    head = 1.0 - pre * np.sum(2.0 * np.abs(Pvc[None]) ** 2 / D[None] ** 2 * (dr - da), axis=(1, 2, 3))
    # eps_0G' = 4 pi i / (V |G'|) sum (f_i - f_j)/(w_j - w_i) qhat.<i|grad|j> <j|e^{iG'r}|i> / den
    t_r = (2.0 / D)[None, ..., None] * Pvc[None, ..., None] * rho[0][None] * dr[..., None]
    t_a = (2.0 / D)[None, ..., None] * Pcv[None, ..., None] * rho[1][None] * da[..., None]
    w0G = 1j * pre * np.sum(t_r + t_a, axis=(1, 2, 3)) / gnorm[None, :]
    # eps_G0 = 4 pi i / (V |G|) sum (f_i - f_j)/(w_j - w_i) <i|e^{-iGr}|j> qhat.<j|grad|i> / den
    u_r = (2.0 / D)[None, ..., None] * np.conj(rho[0])[None] * Pcv[None, ..., None] * dr[..., None]
    u_a = (2.0 / D)[None, ..., None] * np.conj(rho[1])[None] * Pvc[None, ..., None] * da[..., None]
    wG0 = 1j * pre * np.sum(u_r + u_a, axis=(1, 2, 3)) / gnorm[None, :]
    return head, w0G, wG0


def eps_macro(eps: np.ndarray) -> np.ndarray:
    """eps_M(w) = 1 / [eps^{-1}]_00."""
    return 1.0 / inverse_diagonal(eps)[:, 0]


def solve(cell, basis, lattice_range, k_frac, n_occ, G_int, states, w_eV, eta_eV, lfe=True,
          return_all=False):
    """The full path for one q: R -> W -> chi0 -> eps -> loss."""
    R = pair_densities_from_workload(cell, basis, lattice_range, k_frac, states.q_cart, G_int,
                                     states.C_k, states.C_kq, n_occ)
    volume = abs(float(np.linalg.det(np.asarray(cell.lat, np.float64))))
    W = transition_weights(states.E_k, states.E_kq, n_occ, w_eV, eta_eV, volume)
    chi = chi0(R, W)
    Qc = q_plus_g(cell.lat, states.q_cart, G_int)
    eps = epsilon(chi, Qc)
    L = loss_lfe(eps) if lfe else loss_nolfe(eps)
    if return_all:
        return dict(R=R, W=W, chi0=chi, eps=eps, loss=L, Q=Qc)
    return L


def solve_workload(wl, iq=0, w_idx=None, lfe=True, return_all=False):
    st = wl.states(iq)
    w = wl.w_eV if w_idx is None else np.asarray(wl.w_eV)[w_idx]
    return solve(wl.cell, wl.basis, wl.lattice_range, wl.k_frac, wl.n_occ, wl.G_int, st, w,
                 wl.eta_eV, lfe=lfe, return_all=return_all)


def rel_err_normwise(L: np.ndarray, Lref: np.ndarray) -> float:
    """max over G of  max_w |L - Lref| / max_w |Lref|  (per-(q,G) curve, normwise)."""
    num = np.max(np.abs(L - Lref), axis=0)
    den = np.max(np.abs(Lref), axis=0)
    den = np.where(den == 0.0, 1.0, den)
    return float(np.max(num / den))
