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
