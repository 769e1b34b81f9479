"""From the dielectric function to dark-matter-electron scattering rates
(oracle, FP64, numpy/scipy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Written from the paper:

* Eq. (dynamic_structure_factor): S(w, q) = q^2 / (2 pi alpha) Im(-1/eps(w, q)).
* Sec. III (binning): the finite-momentum dielectric function eps(w, q + G) of
  every q and G is binned in three-dimensional q space: spherical shells of
  width dq, each split into N_theta x N_phi angular bins (N_theta = 9,
  N_phi = 16, dq = 0.02 alpha m_e in the paper); bins that received no entry
  are filled by interpolation from the surrounding bins; the isotropic
  approximation averages over the directions of q to obtain S(w, q).
* Eq. (general_rate) with the halo flux, and the nonrelativistic cross
  section of Eq. (cross_section) / App. A: per unit target mass
      dR/dw = rho_chi / (m_chi rho_T) * sigma_e / (8 pi^2 alpha mu^2)
              * int dq q^3 |F_DM(q)|^2 Im(-1/eps(w, q)) eta(v_min(q, w)),
  v_min = q / (2 m_chi) + w / q (Eq. v_min with gamma = 1), eta the mean
  inverse speed above v_min, F_DM of Eq. (F_DM); halo parameters v_esc =
  544 km/s, v_E = 250.2 km/s, rho_chi = 0.3 GeV / cm^3 (footnote of Sec. IV).

Readings of points the paper leaves open (each also listed in the design doc):

* Angular bins uniform in theta in [0, pi] and in phi in [0, 2 pi) (phi from
  atan2, negative angles shifted by 2 pi); shell s holds s dq <= |q| <
  (s + 1) dq.  A bin's value is the plain mean of the complex eps of its
  entries; S of a bin is evaluated at the shell centre (s + 1/2) dq.
* Interpolation: sweeps; in each sweep every empty bin with at least one
  non-empty neighbour (the 26 bins adjacent in shell, theta and phi; phi is
  periodic, shell and theta are not) takes the mean of those neighbours'
  eps, using only bins filled before the sweep; repeated until no bin
  changes.  Bins that no sweep reaches stay empty.
* The isotropic S(w, q) of a shell is the solid-angle weighted mean of S
  over its non-empty bins (weights (2 pi / N_phi)(cos theta_i - cos
  theta_{i+1})), i.e. the average over directions.
* The q integral is the midpoint rule over shells with data.
* Halo: the standard truncated Maxwell-Boltzmann distribution in the
  Galactic frame, f(u) ~ exp(-u^2 / v0^2) for u < v_esc, boosted by the
  Earth's velocity, with v0 = 238 km/s (the paper cites the recommended
  parameters but prints only v_esc, v_E and rho_chi).  eta(v_min) is its
  definition, int d^3v f(v) / v over v > v_min, by quadrature.
* Units: q in alpha m_e (= bohr^-1), w in eV, S in (alpha m_e)^2; rates in
  events per kg per year per eV (year = 365.25 days); CODATA 2018 constants.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

ALPHA = 7.2973525693e-3              # fine-structure constant
ME_EV = 510998.95000                  # electron mass (eV)
AME_EV = ALPHA * ME_EV                # alpha m_e (eV) = 1 bohr^-1 in momentum
HBARC_EV_CM = 1.973269804e-5          # hbar c (eV cm)
HBAR_EV_S = 6.582119569e-16           # hbar (eV s)
EV_KG = 1.782661921e-36               # 1 eV / c^2 in kg
C_KMS = 299792.458                    # speed of light (km/s)
YEAR_S = 365.25 * 86400.0

HALO = dict(v0=238.0, vE=250.2, vesc=544.0, rho_chi=0.3)   # km/s, GeV / cm^3


# ----------------------------------------------------------------- binning
def bin_index(qvec, dq: float, n_shell: int, n_theta: int, n_phi: int) -> np.ndarray:
    """Bin of each momentum q (rows of qvec, alpha m_e): (s * n_theta + i) * n_phi
    + j, or -1 when |q| >= n_shell dq (or q = 0)."""
    q = np.asarray(qvec, np.float64)
    r = np.sqrt(q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1] + q[:, 2] * q[:, 2])
    out = np.full(len(q), -1, np.int64)
    ok = (r > 0.0) & (r < n_shell * dq)
    s = np.floor(r[ok] / dq).astype(np.int64)
    s = np.minimum(s, n_shell - 1)
    th = np.arccos(np.clip(q[ok, 2] / r[ok], -1.0, 1.0))
    ph = np.arctan2(q[ok, 1], q[ok, 0])
    ph = np.where(ph < 0.0, ph + 2.0 * math.pi, ph)
    i = np.minimum(np.floor(th / (math.pi / n_theta)).astype(np.int64), n_theta - 1)
    j = np.minimum(np.floor(ph / (2.0 * math.pi / n_phi)).astype(np.int64), n_phi - 1)
    out[ok] = (s * n_theta + i) * n_phi + j
    return out


def bin_eps(entries, n_w: int, dq: float, n_shell: int, n_theta: int, n_phi: int):
    """Mean eps per bin over all (qvec[n][3], eps[n_w][n]) pairs of entries:
    returns (eps_bin[n_w][n_bins] complex, count[n_bins])."""
    nb = n_shell * n_theta * n_phi
    tot = np.zeros((n_w, nb), np.complex128)
    cnt = np.zeros(nb, np.int64)
    for qvec, eps in entries:
        b = bin_index(qvec, dq, n_shell, n_theta, n_phi)
        keep = b >= 0
        for e in np.nonzero(keep)[0]:
            tot[:, b[e]] += eps[:, e]
            cnt[b[e]] += 1
    out = np.zeros_like(tot)
    has = cnt > 0
    out[:, has] = tot[:, has] / cnt[has]
    return out, cnt


def neighbours(b: int, n_shell: int, n_theta: int, n_phi: int):
    """The bins adjacent to bin b (26-neighbourhood, phi periodic)."""
    s, rem = divmod(b, n_theta * n_phi)
    i, j = divmod(rem, n_phi)
    out = []
    for ds in (-1, 0, 1):
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if ds == 0 and di == 0 and dj == 0:
                    continue
                s2, i2 = s + ds, i + di
                if not (0 <= s2 < n_shell and 0 <= i2 < n_theta):
                    continue
                j2 = (j + dj) % n_phi
                nb = (s2 * n_theta + i2) * n_phi + j2
                if nb not in out:      # n_phi <= 2 folds neighbours together
                    out.append(nb)
    return out


def fill_missing(eps_bin, count, n_shell: int, n_theta: int, n_phi: int):
    """Interpolate empty bins (sweeps of neighbour means).  Returns
    (eps, state) with state 1 = data, 2 = interpolated, 0 = still empty."""
    eps = eps_bin.copy()
    state = np.where(count > 0, 1, 0).astype(np.int64)
    while True:
        filled = state > 0
        updates = []
        for b in np.nonzero(~filled)[0]:
            nbs = [n for n in neighbours(int(b), n_shell, n_theta, n_phi) if filled[n]]
            if nbs:
                updates.append((b, nbs))
        if not updates:
            return eps, state
        for b, nbs in updates:
            eps[:, b] = np.mean(eps[:, nbs], axis=1)
            state[b] = 2


def structure_factor(eps, q):
    """S = q^2 / (2 pi alpha) Im(-1/eps) (Eq. dynamic_structure_factor); q in
    alpha m_e, S in (alpha m_e)^2."""
    return np.asarray(q) ** 2 / (2.0 * math.pi * ALPHA) * np.imag(-1.0 / eps)


def solid_angles(n_theta: int, n_phi: int) -> np.ndarray:
    """Solid angle of each angular bin [n_theta * n_phi] (uniform theta, phi)."""
    t = np.arange(n_theta + 1) * (math.pi / n_theta)
    w = (2.0 * math.pi / n_phi) * (np.cos(t[:-1]) - np.cos(t[1:]))
    return np.repeat(w, n_phi)


def isotropic_s(eps, state, dq: float, n_shell: int, n_theta: int, n_phi: int):
    """S(w, q_s) on the shell centres q_s = (s + 1/2) dq: solid-angle weighted
    mean of S over each shell's non-empty bins; NaN for a shell without any."""
    n_w = eps.shape[0]
    na = n_theta * n_phi
    om = solid_angles(n_theta, n_phi)
    qs = (np.arange(n_shell) + 0.5) * dq
    out = np.full((n_w, n_shell), np.nan)
    for s in range(n_shell):
        sl = slice(s * na, (s + 1) * na)
        ok = state[sl] > 0
        if not ok.any():
            continue
        S = structure_factor(eps[:, sl][:, ok], qs[s])
        out[:, s] = S @ om[ok] / om[ok].sum()
    return qs, out


# -------------------------------------------------------------------- halo
def eta_shm(vmin_kms, v0=HALO["v0"], vE=HALO["vE"], vesc=HALO["vesc"]) -> np.ndarray:
    """eta(v_min) = int d^3v f(v) / v over |v| > v_min (s/km), f the truncated
    Maxwell-Boltzmann distribution of Galactic velocities u = v + v_E,
    normalised over |u| < v_esc.  Plain quadrature of the definition: the
    angle between v and v_E, then the speed."""
    norm = 4.0 * math.pi * integrate.quad(lambda u: u * u * math.exp(-u * u / (v0 * v0)), 0.0, vesc,
                                          epsabs=0.0, epsrel=1e-13)[0]

    def angular(s):  # int_{-1}^{1} dc exp(-|u|^2/v0^2) [|u| < vesc], |u|^2 = s^2 + vE^2 + 2 s vE c
        # the cut |u| < vesc is c < c_max
        c_max = (vesc * vesc - s * s - vE * vE) / (2.0 * s * vE) if s > 0 else (1.0 if s * s + vE * vE < vesc * vesc else -1.0)
        hi = min(1.0, c_max)
        if hi <= -1.0:
            return 0.0
        return integrate.quad(lambda c: math.exp(-(s * s + vE * vE + 2.0 * s * vE * c) / (v0 * v0)),
                              -1.0, hi, epsabs=0.0, epsrel=1e-13)[0]

    vmax = vesc + vE
    out = []
    for vm in np.atleast_1d(np.asarray(vmin_kms, np.float64)):
        if vm >= vmax:
            out.append(0.0)
            continue
        lo = max(vm, 0.0)
        # 2 pi int ds s^2 (1/s) angular(s); the cut enters the angular range at vesc - vE
        pts = [p for p in (vesc - vE,) if lo < p < vmax]
        val = integrate.quad(lambda s: s * angular(s), lo, vmax, points=pts or None,
                             epsabs=0.0, epsrel=1e-12, limit=200)[0]
        out.append(2.0 * math.pi * val / norm)
    return np.array(out)


def form_factor(q, m_med_eV: float) -> np.ndarray:
    """F_DM(q) = ((alpha m_e)^2 + m^2) / (q^2 + m^2) (Eq. F_DM), q in alpha m_e;
    m = inf: heavy mediator (F = 1); m = 0: light mediator ((alpha m_e / q)^2)."""
    q = np.asarray(q, np.float64)
    if math.isinf(m_med_eV):
        return np.ones_like(q)
    m = m_med_eV / AME_EV
    return (1.0 + m * m) / (q * q + m * m)


def rate_halo(w_eV, qs, S_iso, dq: float, m_chi_eV: float, m_med_eV: float, sigma_e_cm2: float,
              rho_T_g_cm3: float, halo=HALO) -> np.ndarray:
    """dR/dw (events / kg / year / eV) per frequency, from the isotropic S on
    the shell centres qs (alpha m_e), midpoint rule over shells with data.
    Natural units inside (hbar = c = 1, eV)."""
    w = np.asarray(w_eV, np.float64)
    mu = m_chi_eV * ME_EV / (m_chi_eV + ME_EV)
    n_chi = halo["rho_chi"] * 1e9 / m_chi_eV * HBARC_EV_CM ** 3        # eV^3
    rho_T = rho_T_g_cm3 * 1e-3 / EV_KG * HBARC_EV_CM ** 3               # eV^4
    sigma = sigma_e_cm2 / HBARC_EV_CM ** 2                              # eV^-2
    q_ev = np.asarray(qs) * AME_EV
    F2 = form_factor(qs, m_med_eV) ** 2
    out = np.zeros(len(w))
    for a in range(len(w)):
        tot = 0.0
        for s in range(len(qs)):
            S = S_iso[a, s]
            if not np.isfinite(S):
                continue
            vmin = (q_ev[s] / (2.0 * m_chi_eV) + w[a] / q_ev[s]) * C_KMS    # km/s
            eta = eta_shm(vmin, halo["v0"], halo["vE"], halo["vesc"])[0] * C_KMS   # 1/c
            # int dq q |F|^2 S eta / (4 pi): S in eV^2 = S (alpha m_e)^2 * AME_EV^2
            tot += dq * AME_EV * q_ev[s] * F2[s] * S * AME_EV ** 2 * eta
        x = n_chi / rho_T * sigma / (4.0 * math.pi * mu * mu) * tot     # eV^-1 (natural)
        out[a] = x / HBAR_EV_S / EV_KG * YEAR_S
    return out
