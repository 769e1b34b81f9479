"""Pins for the oracle's pair densities, chi0, eps, inverse and loss (CPU only).

Each test checks a property that the paper's definitions (Eq. RPA,
Eq. eps_LFE, Eq. eps_noLFE) or plain mathematics fix, chosen so that a
dropped term, a swapped index, a wrong sign or a wrong normalisation fails.
"""
import math

import numpy as np
import pytest

from oracle import gto, rpa
from synth import make_tiny
from synth.generator import Basis, Cell, QStates


def _vol(cell):
    return abs(np.linalg.det(cell.lat))


# ---------------------------------------------------------------- pair densities
def test_pair_density_orthonormality_at_q0(tiny):
    """q = 0, G = 0 with all bands: <b', k|b, k> = delta (C^H S C = I)."""
    st = tiny.states(0)
    bs = tiny.basis
    S = gto.overlap_matrix(tiny.cell.lat, tiny.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1,
                           tiny.k_frac)
    # all-band matrix: pair densities with states at k on both sides
    n = tiny.n_bands
    for split in (1, tiny.n_occ):
        R = rpa.pair_densities(S[:, None], st.C_k, st.C_k, split)
        assert np.max(np.abs(R)) < 1e-12     # off-diagonal bands only
    # diagonal: duplicate band b in front so that "c" runs over every band
    for b in (0, n - 1):
        Cp = np.concatenate([st.C_k[:, :, b:b + 1], st.C_k], axis=2)
        R = rpa.pair_densities(S[:, None], Cp, Cp, 1)
        want = np.zeros(n)
        want[b] = 1.0
        assert np.max(np.abs(R[0][:, 0, :, 0] - want[None, :])) < 1e-12


def test_band_sum_identity(tiny):
    """sum_j |<j,k+q|e^{iQr}|b,k>|^2 over ALL bands j = m^H S(k+q)^{-1} m, m = M C_b.

    The right side uses a linear solve with the oracle's S(k+q) and no bra
    coefficients, so it checks conjugation and index order of the band
    contraction and the completeness of the Lowdin states.
    """
    st = tiny.states(0)
    bs = tiny.basis
    Q = rpa.q_plus_g(tiny.cell.lat, st.q_cart, tiny.G_int)
    M = gto.ao_matrix(tiny.cell.lat, tiny.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1,
                      tiny.k_frac, Q)
    qf = tiny.cell.lat @ st.q_cart / (2 * math.pi)
    Skq = gto.overlap_matrix(tiny.cell.lat, tiny.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1,
                             tiny.k_frac + qf)
    for b in (0, 3, tiny.n_bands - 1):
        Cp = np.concatenate([st.C_k[:, :, b:b + 1], st.C_k], axis=2)
        Cq = np.concatenate([st.C_kq[:, :, b:b + 1], st.C_kq], axis=2)
        R = rpa.pair_densities(M, Cp, Cq, 1)            # R[0][k][0][j][G]: bra j at k+q, ket b at k
        lhs = np.sum(np.abs(R[0][:, 0]) ** 2, axis=1)   # [k][G]
        m = np.einsum("kgmn,kn->kgm", M, st.C_k[:, :, b])
        rhs = np.real(np.einsum("kgm,kgm->kg", m.conj(), np.linalg.solve(Skq[:, None], m[..., None])[..., 0]))
        assert np.max(np.abs(lhs - rhs)) < 1e-11 * max(1.0, np.max(np.abs(rhs)))


# ---------------------------------------------------------------- chi0
def _chi_parts(wl, w_eV, eta_eV):
    st = wl.states(0)
    R = rpa.pair_densities_from_workload(wl.cell, wl.basis, 1, wl.k_frac, st.q_cart, wl.G_int,
                                         st.C_k, st.C_kq, wl.n_occ)
    W = rpa.transition_weights(st.E_k, st.E_kq, wl.n_occ, w_eV, eta_eV, _vol(wl.cell))
    return st, R, W, None


def test_chi0_hermitian_at_zero_frequency_zero_eta(tiny):
    st, R, W, _ = _chi_parts(tiny, np.array([0.0]), 0.0)
    chi = rpa.chi0(R, W)[0]
    assert np.max(np.abs(chi - chi.conj().T)) < 1e-14 * np.max(np.abs(chi))


def test_chi0_antihermitian_part_negative(tiny):
    """For w >= 0 both prescriptions give Im W_t <= 0, so (chi0 - chi0^H)/2i <= 0."""
    st, R, W, _ = _chi_parts(tiny, np.linspace(0.0, 40.0, 9), tiny.eta_eV)
    chi = rpa.chi0(R, W)
    for c in chi:
        A = (c - c.conj().T) / 2j
        ev = np.linalg.eigvalsh(A)
        assert ev.max() < 1e-12 * np.abs(ev).max()
        assert ev.min() < 0


def test_chi0_large_frequency_moments(tiny):
    """chi0(w) = m1/w + m2/w^2 + O(w^-3) with
    m1 = 2/(N_k V) [sum_res P_t - sum_anti P_t],
    m2 = 2/(N_k V) [sum_res (Delta - i eta) P_t + sum_anti (Delta' - i eta) P_t],
    P_t = rho_t(G)^* rho_t(G'), Delta = E_c(k+q) - E_v(k), Delta' = E_c(k) - E_v(k+q)."""
    st = tiny.states(0)
    wbig = 2.0e4  # Ha
    eta = tiny.eta_eV / rpa.HARTREE_EV
    _, R, W, _ = _chi_parts(tiny, np.array([wbig * rpa.HARTREE_EV]), tiny.eta_eV)
    chi = rpa.chi0(R, W)[0]
    nk = tiny.n_k
    ha = rpa.HARTREE_EV
    dres = np.array([[[st.E_kq[k, tiny.n_occ + c] - st.E_k[k, v] for c in range(tiny.n_cond)]
                      for v in range(tiny.n_occ)] for k in range(nk)]) / ha
    dant = np.array([[[st.E_k[k, tiny.n_occ + c] - st.E_kq[k, v] for c in range(tiny.n_cond)]
                      for v in range(tiny.n_occ)] for k in range(nk)]) / ha
    pref = 2.0 / (nk * _vol(tiny.cell))
    P0 = np.einsum("kvcg,kvch->gh", R[0].conj(), R[0])
    P1 = np.einsum("kvcg,kvch->gh", R[1].conj(), R[1])
    m1 = pref * (P0 - P1)
    m2 = pref * (np.einsum("kvc,kvcg,kvch->gh", dres - 1j * eta, R[0].conj(), R[0])
                 + np.einsum("kvc,kvcg,kvch->gh", dant - 1j * eta, R[1].conj(), R[1]))
    assert np.max(np.abs(wbig * chi - m1)) < 1e-3 * np.max(np.abs(m1)) + 1e-14
    est_m2 = wbig * wbig * (chi - m1 / wbig)
    assert np.max(np.abs(est_m2 - m2)) < 2e-3 * np.max(np.abs(m2))


def test_chi0_tail_independent_of_kgrid():
    """At large w, Im chi0_GG -> -(2 eta / (N_k V w^2)) sum_t |R_t(G)|^2: a
    Brillouin-zone average of a smooth function of k, so it must agree
    between k grids (this fixes the 1/N_k weight; without it the two grids
    differ by 512/216)."""
    tails = []
    wbig = 1.0e5
    for n in (6, 8):
        wl = make_tiny(kgrid=n, n_g=9)
        st, R, W, _ = _chi_parts(wl, np.array([wbig * rpa.HARTREE_EV]), wl.eta_eV)
        tails.append(wbig * wbig * np.diagonal(rpa.chi0(R, W)[0]).imag)
    assert np.all(tails[0] < 0)
    rel = np.max(np.abs(tails[0] - tails[1]) / np.abs(tails[1]))
    assert rel < 2e-2, rel


def test_chi0_single_transition_conjugates_row():
    R = np.zeros((2, 1, 1, 1, 3), np.complex128)
    rho = np.array([0.3 + 0.1j, -0.2 + 0.5j, 0.05 - 0.4j])
    R[0, 0, 0, 0] = rho
    W = np.array([[0.7 - 0.2j, 0.0]])
    chi = rpa.chi0(R, W)[0]
    assert np.allclose(chi, (0.7 - 0.2j) * np.outer(rho.conj(), rho), atol=1e-15, rtol=0)


# ---------------------------------------------------------------- eps
def test_eps_length_scaling():
    """Scale every length by s (cell, centres; exponents by 1/s^2; q by 1/s).
    Pair densities of normalised orbitals are unchanged, chi0 ~ 1/V ~ s^-3 and
    the Coulomb factor ~ s^2, so (eps - 1) ~ 1/s exactly."""
    wl = make_tiny(kgrid=2, n_g=9, n_w=5)
    st = wl.states(0)
    base = rpa.solve(wl.cell, wl.basis, 1, wl.k_frac, wl.n_occ, wl.G_int, st, wl.w_eV, wl.eta_eV,
                     return_all=True)["eps"]
    s = 1.37
    cell = Cell(wl.cell.name, wl.cell.a * s, wl.cell.lat * s, wl.cell.xyz * s, wl.cell.species)
    basis = Basis(wl.basis.shell_atom, wl.basis.shell_l, wl.basis.shell_exp / s ** 2)
    st2 = QStates(st.q_cart / s, st.C_k, st.E_k, st.C_kq, st.E_kq)
    sc = rpa.solve(cell, basis, 1, wl.k_frac, wl.n_occ, wl.G_int, st2, wl.w_eV, wl.eta_eV,
                   return_all=True)["eps"]
    I = np.eye(len(wl.G_int))[None]
    assert np.max(np.abs((sc - I) * s - (base - I))) < 1e-10 * np.max(np.abs(base - I))


def test_eps_tends_to_one_at_large_q(small_oracle):
    eps = small_oracle["eps"]
    R = small_oracle["R"].reshape(-1, eps.shape[1])
    W = small_oracle["W"]
    Q = small_oracle["Q"]
    q2 = np.sum(Q * Q, axis=1)
    bound = 4 * math.pi / q2[None, :] * (np.abs(W) @ (np.abs(R) ** 2))
    dev = np.abs(np.diagonal(eps, axis1=1, axis2=2) - 1.0)
    assert np.all(dev <= bound * (1 + 1e-12) + 1e-15)
    # and the bound itself falls with |q+G|: largest |q+G| deviates far less than G = 0
    assert dev[:, np.argmax(q2)].max() < 0.1 * dev[:, 0].max()


def test_eps_antihermitian_part_psd(small_oracle):
    for e in small_oracle["eps"][::8]:
        ev = np.linalg.eigvalsh((e - e.conj().T) / 2j)
        assert ev.min() > -1e-12 * np.abs(ev).max()


# ---------------------------------------------------------------- inverse and loss
def test_lfe_equals_nolfe_without_offdiagonals(small_oracle):
    eps = small_oracle["eps"]
    d = np.einsum("wgg->wg", eps)
    diag_only = np.zeros_like(eps)
    idx = np.arange(eps.shape[1])
    diag_only[:, idx, idx] = d
    assert np.max(np.abs(rpa.loss_lfe(diag_only) - rpa.loss_nolfe(eps))) < 1e-14
    one = eps[:, :1, :1]
    assert np.max(np.abs(rpa.loss_lfe(one) - rpa.loss_nolfe(one))) < 1e-15


def test_loss_nonnegative(small_oracle):
    assert small_oracle["loss"].min() > -1e-15
    assert rpa.loss_nolfe(small_oracle["eps"]).min() > -1e-15


def test_inverse_diagonal_invariances(small_oracle):
    """diag(eps^-1) is unchanged by transposition and by the non-symmetric
    Coulomb form eps' = 1 - v(q+G) chi0 (a similar matrix)."""
    eps = small_oracle["eps"][::16]
    chi = small_oracle["chi0"][::16]
    Q = small_oracle["Q"]
    d = rpa.inverse_diagonal(eps)
    assert np.max(np.abs(rpa.inverse_diagonal(np.swapaxes(eps, 1, 2)) - d)) < 1e-12
    v = 4 * math.pi / np.sum(Q * Q, axis=1)
    eps_ns = np.eye(len(Q))[None] - v[None, :, None] * chi
    assert np.max(np.abs(rpa.inverse_diagonal(eps_ns) - d)) < 1e-11
    X = np.linalg.inv(eps)
    for e, x in zip(eps, X):
        res = np.linalg.norm(e @ x - np.eye(len(e))) / (np.linalg.norm(e) * np.linalg.norm(x))
        assert res < 1e-13


def test_macroscopic_eps_is_inverse_head(small_oracle):
    eps = small_oracle["eps"]
    em = rpa.eps_macro(eps)
    assert np.allclose(em, 1.0 / np.linalg.inv(eps)[:, 0, 0], rtol=1e-14, atol=0)
    # loss at G = 0 is Im(-1/eps_M)
    assert np.allclose(small_oracle["loss"][:, 0], np.imag(-1.0 / em), rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- noLFE diagonal and composite
def test_chi0_diagonal_is_diagonal_of_chi0(small_oracle):
    d = rpa.chi0_diagonal(small_oracle["R"], small_oracle["W"])
    full = np.einsum("wgg->wg", small_oracle["chi0"])
    assert np.max(np.abs(d - full)) <= 1e-14 * np.max(np.abs(full))


def test_loss_diag_matches_nolfe_of_full_path(small_wl, small_oracle):
    st = small_wl.states(0)
    L = rpa.loss_diag(small_wl.cell, small_wl.basis, small_wl.lattice_range, small_wl.k_frac, small_wl.n_occ,
                      small_wl.G_int, st, small_wl.w_eV, small_wl.eta_eV)
    ref = rpa.loss_nolfe(small_oracle["eps"])
    assert np.max(np.abs(L - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_loss_diag_per_g_independent_of_list(small_wl):
    """Each G's diagonal depends on that G alone: any subset, order or
    duplication (no G = 0) gives the same columns."""
    st = small_wl.states(0)
    G = np.asarray(small_wl.G_int)
    args = (small_wl.cell, small_wl.basis, small_wl.lattice_range, small_wl.k_frac, small_wl.n_occ)
    w = small_wl.w_eV[::16]
    full = rpa.loss_diag(*args, G, st, w, small_wl.eta_eV)
    pick = np.array([5, 3, 26, 5, 11])
    sub = rpa.loss_diag(*args, G[pick], st, w, small_wl.eta_eV)
    assert np.max(np.abs(sub - full[:, pick])) <= 1e-13 * np.max(np.abs(full))


def test_composite_limits(small_wl, small_oracle):
    """q_lfe above every |q+G|: the LFE loss; q_lfe between |q| and the next
    |q+G|: a 1 x 1 LFE block, i.e. the noLFE loss everywhere."""
    st = small_wl.states(0)
    args = (small_wl.cell, small_wl.basis, small_wl.lattice_range, small_wl.k_frac, small_wl.n_occ, small_wl.G_int, st,
            small_wl.w_eV, small_wl.eta_eV)
    qn = np.linalg.norm(small_oracle["Q"], axis=1)
    hi = rpa.loss_composite(*args, q_lfe=qn.max() * 1.01)
    assert np.max(np.abs(hi - small_oracle["loss"])) <= 1e-13 * np.max(np.abs(small_oracle["loss"]))
    lo = rpa.loss_composite(*args, q_lfe=0.5 * (qn[0] + np.sort(qn)[1]))
    ref = rpa.loss_nolfe(small_oracle["eps"])
    assert np.max(np.abs(lo - ref)) <= 1e-13 * np.max(np.abs(ref))
    with pytest.raises(ValueError):
        rpa.composite_split(small_wl.cell.lat, st.q_cart, np.asarray(small_wl.G_int)[1:], qn.max())


# ---------------------------------------------------------------- Kramers-Kronig route
def _quad_hat(z):
    """int_{-1}^{1} (1 - |y|) / (z - y) dy by adaptive quadrature (Cauchy
    principal value for real z inside (-1, 1))."""
    from scipy.integrate import quad
    if z.imag != 0.0:
        f = lambda y, part: getattr((1 - abs(y)) / (z - y), part)
        return sum(quad(f, a, b, args=(p,), limit=400)[0] * (1 if p == "real" else 1j)
                   for a, b in ((-1, 0), (0, 1)) for p in ("real", "imag"))
    x = z.real
    # PV int g(y)/(x - y) = -PV int g(y)/(y - x): quad's weight 'cauchy' computes PV int f/(y - x)
    pv = 0.0
    for a, b, g in ((-1.0, 0.0, lambda y: 1 + y), (0.0, 1.0, lambda y: 1 - y)):
        if a < x < b:
            pv -= quad(g, a, b, weight="cauchy", wvar=x)[0]
        else:
            pv += quad(lambda y: g(y) / (x - y), a, b)[0]
    return pv


def test_hat_kernel_against_quadrature():
    for z in (2 + 0.5j, -0.3 + 0.01j, 0.4 - 0.2j, 30 + 0.1j, -7 - 3j, 1e-3 + 1e-3j):
        assert abs(rpa.hat_kernel(np.array([z]))[0] - _quad_hat(z)) < 1e-12 * max(1.0, abs(z) ** -1)
    # real axis: principal value, and -/+ i pi (1 - |x|) from above / below
    for x in (-0.5, 0.3, 0.999, 1.7, -3.0):
        up = rpa.hat_kernel(np.array([complex(x, 0.0)]))[0]
        dn = rpa.hat_kernel(np.array([complex(x, -0.0)]))[0]
        pv = _quad_hat(complex(x, 0.0))
        spec = -np.pi * max(0.0, 1 - abs(x))
        assert abs(up.real - pv) < 1e-10 and abs(dn.real - pv) < 1e-10
        assert abs(up.imag - spec) < 1e-12 and abs(dn.imag + spec) < 1e-12


def test_hat_kernel_far_field_series():
    """Far from the hat, 1/(z - y) = sum_m y^m / z^(m+1) integrates term by
    term to I(z) = sum_n 2 / ((2n+1)(2n+2)) z^-(2n+1); the closed form must
    keep that to near working precision where its three terms nearly cancel."""
    for z in (12.0 + 0.2j, -40.0 + 1.0j, 500.0 + 0.3j, -1800.0 - 0.05j, 3000.0 + 0.0j):
        n = np.arange(12)
        ser = np.sum(2.0 / ((2 * n + 1) * (2 * n + 2)) * complex(z) ** (-(2 * n + 1)))
        got = rpa.hat_kernel(np.array([z]))[0]
        assert abs(got - ser) < 1e-11 * abs(ser), (z, got, ser)


def test_spectral_bins_partition_of_unity():
    E = np.random.default_rng(1).uniform(0.05, 0.9, 500)
    c, H = rpa.spectral_bins(E, 0.3)
    assert np.max(np.abs(H.sum(axis=0) - 1.0)) < 1e-13
    assert np.max(np.abs(c @ H - E)) < 1e-13       # first moment kept too


def test_chi0_kk_converges_to_direct(small_oracle, small_wl):
    """At fixed eta the binned route tends to Eq. (RPA) at second order in the
    bin width: halving the width divides the error by about four."""
    st = small_wl.states(0)
    vol = _vol(small_wl.cell)
    w = small_wl.w_eV[::8]
    W = rpa.transition_weights(st.E_k, st.E_kq, small_wl.n_occ, w, small_wl.eta_eV, vol)
    direct = rpa.chi0(small_oracle["R"], W)
    errs = []
    for b in (0.08, 0.04, 0.02):
        kk = rpa.chi0_kk(small_oracle["R"], st.E_k, st.E_kq, small_wl.n_occ, w, small_wl.eta_eV, b, vol)
        errs.append(np.max(np.abs(kk - direct)) / np.max(np.abs(direct)))
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs
    assert errs[2] < 2e-3


def test_chi0_kk_zero_eta_is_kramers_kronig_pair(small_oracle, small_wl):
    """eta = 0: Im chi0 is -pi times the binned spectral density, and Re chi0
    is its Kramers-Kronig (Hilbert) transform, checked for the head by an
    independent quadrature over the piecewise-linear density."""
    from scipy.integrate import quad
    st = small_wl.states(0)
    vol = _vol(small_wl.cell)
    b = 0.1
    w = np.array([3.03, 7.57, 12.01, 20.04])   # poles inside segments, not on bin centres
    kk = rpa.chi0_kk(small_oracle["R"], st.E_k, st.E_kq, small_wl.n_occ, w, 0.0, b, vol)[:, 0, 0]
    # spectral densities (per Ha) of the head, both sides, as piecewise-linear functions
    d_res, d_anti = rpa.transition_energies(st.E_k, st.E_kq, small_wl.n_occ)
    norm = 2.0 / (len(small_wl.k_frac) * vol)
    dens = []
    for side, E in ((0, d_res.reshape(-1)), (1, d_anti.reshape(-1))):
        c, H = rpa.spectral_bins(E, b)
        S = norm * (H @ (np.abs(small_oracle["R"][side].reshape(-1, 27)[:, 0]) ** 2))
        dens.append((c, S / (b / rpa.HARTREE_EV)))
    wh = w / rpa.HARTREE_EV
    for j in range(len(w)):
        c, s = dens[0]
        assert abs(kk[j].imag + np.pi * np.interp(wh[j], c, s, left=0, right=0)) < 1e-10 * np.max(np.abs(kk))
        re = 0.0
        for side, sgn in ((0, 1.0), (1, -1.0)):
            c, s = dens[side]
            x0 = sgn * wh[j]                          # pole of 1/(w - x) or -1/(w + x)
            for a, bb, sa, sb in zip(c[:-1], c[1:], s[:-1], s[1:]):   # linear on each segment
                f = lambda x: sa + (sb - sa) * (x - a) / (bb - a)
                if a < x0 < bb:     # PV int f/(w - x) = -PV int f/(x - w)
                    re -= sgn * quad(f, a, bb, weight="cauchy", wvar=x0)[0]
                else:
                    re += quad(lambda x: sgn * f(x) / (wh[j] - sgn * x), a, bb)[0]
        assert abs(kk[j].real - re) < 1e-9 * np.max(np.abs(kk)), (j, kk[j].real, re)
