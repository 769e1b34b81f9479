"""Pins of oracle/rates.py (q binning, S(w, q), halo rate) against what the
paper and the mathematics fix, independently of the oracle's own code."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import rates

ND = dict(dq=0.1, n_shell=6, n_theta=9, n_phi=16)


def test_bin_index_ranges():
    rng = np.random.default_rng(5)
    q = rng.normal(size=(4000, 3)) * 0.3
    b = rates.bin_index(q, **ND)
    r = np.linalg.norm(q, axis=1)
    assert np.all((b >= 0) == (r < ND["n_shell"] * ND["dq"]))
    na = ND["n_theta"] * ND["n_phi"]
    for qq, bb, rr in zip(q, b, r):
        if bb < 0:
            continue
        s, rem = divmod(int(bb), na)
        i, j = divmod(rem, ND["n_phi"])
        assert s * ND["dq"] <= rr < (s + 1) * ND["dq"]
        th = math.acos(qq[2] / rr)
        ph = math.atan2(qq[1], qq[0]) % (2 * math.pi)
        assert i * math.pi / 9 <= th <= (i + 1) * math.pi / 9
        assert j * 2 * math.pi / 16 <= ph <= (j + 1) * 2 * math.pi / 16


def _eps_with_loss(g):
    """eps with Im(-1/eps) = g: -1/eps = i g."""
    return 1j / np.asarray(g, np.complex128)


def test_isotropic_average_weights():
    """Bin values equal to the exact bin averages of f(theta, phi) must give
    the exact sphere average of f: 1/3 for cos^2, 0 for sin cos(phi) shifted."""
    nt, nph = 9, 16
    t = np.arange(nt + 1) * math.pi / nt
    p = np.arange(nph + 1) * 2 * math.pi / nph
    om = rates.solid_angles(nt, nph)
    assert abs(om.sum() - 4 * math.pi) < 1e-13
    c1, c2 = np.cos(t[:-1]), np.cos(t[1:])
    avg_cos2 = (c1 ** 3 - c2 ** 3) / (3 * (c1 - c2))                        # per theta bin
    # f = 2 + sin(theta) cos(phi): bin mean of sin over d(cos), of cos over phi
    sin_mean = (((t[1:] - t[:-1]) - (np.sin(2 * t[1:]) - np.sin(2 * t[:-1])) / 2) / 2) / (c1 - c2)
    cos_mean = (np.sin(p[1:]) - np.sin(p[:-1])) / (p[1:] - p[:-1])
    for vals, exact in ((np.repeat(avg_cos2, nph), 1.0 / 3.0),
                        (2.0 + np.outer(sin_mean, cos_mean).reshape(-1), 2.0)):
        eps = _eps_with_loss(np.tile(vals, 1))[None, :]
        state = np.ones(nt * nph, np.int64)
        qs, S = rates.isotropic_s(eps, state, 1.0, 1, nt, nph)
        assert abs(S[0, 0] - qs[0] ** 2 / (2 * math.pi * rates.ALPHA) * exact) < 1e-12 * S[0, 0]


def test_fill_missing_rule():
    ns, nt, nph = 3, 3, 4
    nb = ns * nt * nph
    rng = np.random.default_rng(2)
    val = rng.normal(size=(2, nb)) + 1j * rng.normal(size=(2, nb))
    cnt = np.ones(nb, np.int64)
    hole = (1 * nt + 1) * nph + 0           # shell 1, theta 1, phi 0 (phi wraps to 3)
    cnt[hole] = 0
    eps, state = rates.fill_missing(np.where(cnt > 0, val, 0), cnt, ns, nt, nph)
    nbrs = []
    for ds in (-1, 0, 1):
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if (ds, di, dj) != (0, 0, 0):
                    nbrs.append(((1 + ds) * nt + 1 + di) * nph + (0 + dj) % nph)
    assert len(set(nbrs)) == 26
    assert np.allclose(eps[:, hole], val[:, nbrs].mean(axis=1), rtol=0, atol=1e-14)
    assert state[hole] == 2 and np.all(np.delete(state, hole) == 1)
    # a whole empty shell 0 is reached in one sweep from shell 1, shell 0's
    # values only from shell-1 bins (no empty bin feeds another in a sweep)
    cnt = np.ones(nb, np.int64)
    cnt[: nt * nph] = 0
    eps, state = rates.fill_missing(np.where(cnt > 0, val, 0), cnt, ns, nt, nph)
    assert np.all(state[: nt * nph] == 2)
    b = 0 * nt * nph + 0 * nph + 0           # shell 0, theta 0, phi 0
    expect = [(1 * nt + i) * nph + j % nph for i in (0, 1) for j in (-1, 0, 1)]
    assert np.allclose(eps[:, b], val[:, expect].mean(axis=1), rtol=0, atol=1e-14)


def test_structure_factor_f_sum_rule():
    """Drude eps = 1 - wp^2 / (w (w + i g)): int_0^inf w Im(-1/eps) dw = pi wp^2 / 2,
    and with wp^2 = 4 pi alpha n_e / m_e (natural units) the f-sum rule of the
    dynamic structure factor reads int w S(w, q) dw = pi n_e q^2 / m_e."""
    n_e, m_e, q = 0.03, 1.0, 0.7          # units where only ratios matter
    wp2 = 4 * math.pi * rates.ALPHA * n_e / m_e
    g = 0.05

    def ws(w):
        eps = 1.0 - wp2 / (w * (w + 1j * g))
        return w * rates.structure_factor(eps, q)

    wp = math.sqrt(wp2)
    val = sum(integrate.quad(ws, a, b, epsabs=0, epsrel=1e-12, limit=400)[0]
              for a, b in ((1e-12, wp - 20 * g), (wp - 20 * g, wp + 20 * g), (wp + 20 * g, np.inf)))
    ref = math.pi * n_e * q * q / m_e
    assert abs(val - ref) < 1e-9 * ref, (val, ref)


def _eta_closed(vmin, v0, vE, vesc):
    x, y, z = vmin / v0, vE / v0, vesc / v0
    N = special.erf(z) - 2 * z * math.exp(-z * z) / math.sqrt(math.pi)
    if x < z - y:
        r = special.erf(x + y) - special.erf(x - y) - 4 * y * math.exp(-z * z) / math.sqrt(math.pi)
    elif x < z + y:
        r = special.erf(z) - special.erf(x - y) - 2 * (z + y - x) * math.exp(-z * z) / math.sqrt(math.pi)
    else:
        return 0.0
    return r / (2 * N * y * v0)


def test_eta_against_closed_form():
    h = rates.HALO
    v = np.array([0.0, 50.0, 200.0, 293.0, 293.9, 294.5, 500.0, 790.0, 794.1, 800.0])
    got = rates.eta_shm(v)
    for vm, g in zip(v, got):
        ref = _eta_closed(vm, h["v0"], h["vE"], h["vesc"])
        assert abs(g - ref) <= 1e-9 * max(ref, 1e-6), (vm, g, ref)


def test_rate_units_against_si():
    """The natural-units evaluation against the same formula in SI, restored
    with hbar and c (dR/dw = n/rho_T sigma/(8 pi^2 alpha) int dq q^3 |F|^2 L eta
    / (mu^2 hbar^3 c), q in kg m/s, mu in kg) and an independent constant set."""
    hbar, c, eV, me_kg, a0 = 1.054571817e-34, 299792458.0, 1.602176634e-19, 9.1093837015e-31, 5.29177210903e-11
    qs = (np.arange(40) + 0.5) * 0.25              # alpha m_e
    w = np.array([3.0, 12.0, 25.0])
    L = np.exp(-((qs[None, :] - 4.0) ** 2) / 6.0) * (0.2 + w[:, None] / 30.0)
    S = qs[None, :] ** 2 / (2 * math.pi * rates.ALPHA) * L
    m_chi, sig, rhoT = 1e8, 1e-39, 2.33
    for m_med in (math.inf, 0.0):
        got = rates.rate_halo(w, qs, S, 0.25, m_chi, m_med, sig, rhoT)
        n = 0.3e9 * eV / (m_chi * eV / c ** 2 * c ** 2) * 1e6            # m^-3
        rho = rhoT * 1e3                                                 # kg / m^3
        mchi_kg = m_chi * eV / c ** 2
        mu = mchi_kg * me_kg / (mchi_kg + me_kg)
        q_si = qs * hbar / a0
        F = np.ones_like(qs) if math.isinf(m_med) else (hbar / a0) ** 2 / q_si ** 2
        for a in range(len(w)):
            vmin = q_si / (2 * mchi_kg) + w[a] * eV / q_si                 # m/s
            eta = np.array([_eta_closed(v / 1e3, 238.0, 250.2, 544.0) for v in vmin]) / 1e3   # s/m
            integ = np.sum(0.25 * hbar / a0 * q_si ** 3 * F ** 2 * L[a] * eta)
            x = n / rho * sig * 1e-4 / (8 * math.pi ** 2 * rates.ALPHA) * integ / (mu ** 2 * hbar ** 3 * c)
            ref = x * eV * 365.25 * 86400.0                              # per kg per year per eV
            assert abs(got[a] - ref) < 1e-8 * abs(ref), (m_med, a, got[a], ref)


# --------------------------------------------------------------------------
# Independent route to the halo rate: the relativistic isotropic cross section
# of Eq. (cross_section_iso) with the vector-mediator H_V of Eq. (H), E_chi =
# gamma m_chi and E_chi' = E_chi - w, v_min of Eq. (v_min) with gamma, fed
# through the first form of Eq. (general_rate), i.e. an explicit integral of
# f_chi(v) v dsigma/dw(v) over three-dimensional velocity space (no mean
# inverse speed, no closed form).  Written from Sec. II.B alone, with its own
# constants (SI values converted here) and Gauss-Legendre quadrature.
# --------------------------------------------------------------------------
_C_SI = 299792458.0
_EV_J = 1.602176634e-19
_HBAR_SI = 1.054571817e-34
_ME_KG = 9.1093837015e-31
_A0_M = 5.29177210903e-11


def _gl(a, b, n=48):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _pieces(a, b, cuts, n=48):
    pts = [a] + sorted(c for c in cuts if a < c < b) + [b]
    xs, ws = [], []
    for lo, hi in zip(pts[:-1], pts[1:]):
        x, w = _gl(lo, hi, n)
        xs.append(x)
        ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def _rate_from_flux(w_eV, qs_ame, S, dq_ame, m_chi_eV, m_med_eV, sigma_cm2, rho_T_g_cm3,
                    v0=238.0, vE=250.2, vesc=544.0, rho_chi=0.3):
    """dR/dw per unit target mass (events / kg / year / eV):
    (1 / m_T) (rho_chi / m_chi) int d^3v f(v) v dsigma/dw(v), with dsigma/dw of
    Eq. (cross_section_iso) at each speed, the q integral by the midpoint rule
    over the shells (as the oracle) and Theta(v - v_min(q, gamma(v))) kept
    exactly.  m_med_eV = inf is the heavy limit of the mediator factor."""
    me_eV = _ME_KG * _C_SI ** 2 / _EV_J
    ame_eV = _HBAR_SI * _C_SI / _A0_M / _EV_J          # alpha m_e c^2 = hbar c / a0
    alpha = ame_eV / me_eV
    mu = m_chi_eV * me_eV / (m_chi_eV + me_eV)
    hbarc_cm = _HBAR_SI * _C_SI / _EV_J * 100.0          # eV cm
    n_chi = rho_chi * 1e9 / m_chi_eV * hbarc_cm ** 3     # eV^3
    rhoT = rho_T_g_cm3 * 1e-3 * _C_SI ** 2 / _EV_J * hbarc_cm ** 3   # eV^4
    sig = sigma_cm2 / hbarc_cm ** 2
    heavy = math.isinf(m_med_eV)
    kms = 1e3 / _C_SI
    v0, vE, vesc = v0 * kms, vE * kms, vesc * kms
    # Galactic-frame distribution exp(-u^2/v0^2) for u < vesc, normalised
    ug, uw = _gl(0.0, vesc, 96)
    norm = 4 * math.pi * np.sum(uw * ug * ug * np.exp(-ug * ug / (v0 * v0)))
    out = np.zeros(len(w_eV))
    for a, w in enumerate(w_eV):
        tot = 0.0
        for s, qa in enumerate(qs_ame):
            if not np.isfinite(S[a, s]):
                continue
            q = qa * ame_eV
            # threshold speed: v = q / (2 gamma(v) m_chi) + w / q
            vs = q / (2 * m_chi_eV) + w / q
            for _ in range(60):
                vs = q * math.sqrt(1.0 - min(vs * vs, 0.25)) / (2 * m_chi_eV) + w / q
            if vs >= vesc + vE:
                continue

            def h(v):   # H_V / (E_chi E_chi') at speed v
                E = m_chi_eV / np.sqrt(1.0 - v * v)
                Ep = E - w
                return ((E + Ep) ** 2 - q * q) / (E * Ep)

            # int d^3v f(v) v (1/v^2) h(v) Theta(v - vs) with v = |u - v_E| (lab
            # velocity = Galactic velocity minus the Earth's); over the angle
            # between u and v_E: int dc g(v) = int v dv g(v) / (u vE)
            uq, uwq = _pieces(0.0, vesc, [vE, vE + vs, vE - vs, vs - vE], 64)
            lo, hi = np.maximum(np.abs(uq - vE), vs), uq + vE
            live = hi > lo
            uq, uwq, lo, hi = uq[live], uwq[live], lo[live], hi[live]
            x, xw = np.polynomial.legendre.leggauss(24)
            vq = 0.5 * (hi - lo)[:, None] * x[None, :] + 0.5 * (hi + lo)[:, None]
            inner = 0.5 * (hi - lo) * (h(vq) @ xw) / (uq * vE)
            acc = np.sum(uwq * 2 * math.pi * uq * uq * np.exp(-uq * uq / (v0 * v0)) * inner) / norm
            if heavy:
                med = 1.0          # (m_A^2 + (alpha m_e)^2)^2 / (w^2 - q^2 - m_A^2)^2 -> 1
            else:
                mA = m_med_eV
                med = (mA * mA + ame_eV ** 2) ** 2 / (w * w - q * q - mA * mA) ** 2
            # S on the shells is q^2/(2 pi alpha) Im(-1/eps) in (alpha m_e)^2
            tot += dq_ame * ame_eV * q * med * S[a, s] * ame_eV ** 2 * acc
        x = n_chi / rhoT * sig / (16 * math.pi * mu * mu) * tot       # eV^-1
        out[a] = x * _EV_J / _HBAR_SI / (_EV_J / _C_SI ** 2) * 365.25 * 86400.0
    assert abs(alpha / rates.ALPHA - 1.0) < 1e-8   # two CODATA routes to alpha
    return out


@pytest.mark.parametrize("m_chi", [1e9, 1e7])
@pytest.mark.parametrize("m_med", [math.inf, 0.0])
def test_rate_halo_against_flux_integral(m_chi, m_med):
    """oracle rate_halo (the nonrelativistic Eq. cross_section through the mean
    inverse speed) against the relativistic Eq. (cross_section_iso) integrated
    over the halo's velocity distribution in three dimensions.  They differ
    only by what the nonrelativistic limit drops (gamma - 1 in E_chi and
    v_min, q^2/m_chi^2 in H_V, (w/q)^2 in the light propagator), all of order
    v^2 <= (v_esc + v_E)^2 = 7e-6.  Scaling every halo speed by 1/lam, the
    momenta by 1/lam and the energies by 1/lam^2 keeps the kinematics and
    shrinks those terms by lam^2: at lam = 1 the two agree to 3e-5, at lam = 8
    to 1e-6, and the difference falls like lam^-2."""
    dq0 = 0.25
    qs0 = (np.arange(56) + 0.5) * dq0
    w0 = np.array([3.0, 12.0, 25.0])
    L = np.exp(-((qs0[None, :] - 4.0) ** 2) / 6.0) * (0.2 + w0[:, None] / 30.0)
    S = qs0[None, :] ** 2 / (2 * math.pi * rates.ALPHA) * L
    rel = {}
    for lam in (1.0, 8.0):
        h = {k: v / lam for k, v in rates.HALO.items() if k != "rho_chi"}
        h["rho_chi"] = rates.HALO["rho_chi"]
        qs, dq, w = qs0 / lam, dq0 / lam, w0 / lam ** 2
        mm = m_med if math.isinf(m_med) else m_med / lam
        ref = _rate_from_flux(w, qs, S, dq, m_chi, mm, 1e-39, 2.33, v0=h["v0"], vE=h["vE"],
                              vesc=h["vesc"], rho_chi=h["rho_chi"])
        got = rates.rate_halo(w, qs, S, dq, m_chi, mm, 1e-39, 2.33, halo=h)
        assert np.all(ref > 0)
        rel[lam] = np.abs(got / ref - 1.0)
    print("rate_halo vs flux integral", m_chi, m_med, rel)
    assert np.all(rel[1.0] < 3e-5), rel
    assert np.all(rel[8.0] < 1e-6), rel
    big = rel[1.0] > 1e-7
    ratio = rel[1.0][big] / rel[8.0][big]
    assert np.all((ratio > 64 / 2) & (ratio < 64 * 2)), ratio
