"""Seeded generator of synthetic, silicon-shaped RPA workloads.

Everything here is input data: the crystal cell, single-primitive Gaussian
shells, Gamma-centred k grids, the q list, the G list (closed shells sorted
by |G|^2), the frequency grid and, for each k and k+q, Lowdin-orthonormal
random coefficients with sorted random band energies.

Units follow the library boundary: lengths in bohr, energies in eV.

The coefficients must satisfy C^H S(k) C = I (the states of Eq. RPA are
orthonormal Kohn-Sham states).  A DFT code builds S(k) with its own integral
routines; so does this generator, with the real-space Obara-Saika overlap
recursion, a route used by neither the oracle (Fourier moments) nor the HIP
kernels (Hermite expansion).  Both of those recompute S(k) and reject states
that are not orthonormal, so a mistake here cannot pass silently.

Random coefficients are a smooth function of k (a few lattice harmonics), so
that pair densities between different bands vanish as q -> 0 as they do for
real insulators; `smooth=False` gives independent draws per k instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

HARTREE_EV = 27.211386245988  # CODATA 2018
BASE_SEED = 20260312


# --------------------------------------------------------------------------
# cells, reciprocal lattice, grids
# --------------------------------------------------------------------------
@dataclass
class Cell:
    name: str
    a: float
    lat: np.ndarray          # rows a1, a2, a3 (bohr)
    xyz: np.ndarray          # [n_atoms][3] bohr
    species: List[str]

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.lat)))


def fcc_cell(a: float, name: str = "diamond", species=("X", "X")) -> Cell:
    """Diamond / zincblende primitive cell: fcc vectors, atoms at 0 and a/4(1,1,1)."""
    lat = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    xyz = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    return Cell(name=name, a=a, lat=lat, xyz=xyz, species=list(species))


def reciprocal_rows(lat: np.ndarray) -> np.ndarray:
    """Rows b1, b2, b3 with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(lat).T


def gamma_grid(n: int) -> np.ndarray:
    """Gamma-centred n^3 grid in fractional (reciprocal-basis) coordinates."""
    m = np.arange(n) / n
    g = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3)
    return np.ascontiguousarray(g)


def _sorted_g(ints: np.ndarray, lat: np.ndarray) -> np.ndarray:
    b = reciprocal_rows(lat)
    g2 = np.einsum("ni,ij->nj", ints.astype(np.float64), b)
    g2 = np.round(np.sum(g2 * g2, axis=1), 9)
    order = np.lexsort((ints[:, 2], ints[:, 1], ints[:, 0], g2))
    return np.ascontiguousarray(ints[order].astype(np.int32))


def g_cube(lat: np.ndarray) -> np.ndarray:
    """The 27 G with reciprocal-basis coefficients in {-1,0,1}^3, G=0 first."""
    r = np.arange(-1, 2)
    ints = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    return _sorted_g(ints, lat)


def g_shells(lat: np.ndarray, n_g: int, nmax: int = 8) -> np.ndarray:
    """First n_g reciprocal vectors by |G|; n_g must close a shell."""
    r = np.arange(-nmax, nmax + 1)
    ints = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    srt = _sorted_g(ints, lat)
    b = reciprocal_rows(lat)
    g2 = np.sum((srt.astype(np.float64) @ b) ** 2, axis=1)
    if n_g < len(srt) and abs(g2[n_g] - g2[n_g - 1]) < 1e-9 * max(1.0, g2[n_g]):
        raise ValueError(f"n_g={n_g} does not close a shell")
    return np.ascontiguousarray(srt[:n_g])


# --------------------------------------------------------------------------
# basis
# --------------------------------------------------------------------------
@dataclass
class Basis:
    shell_atom: np.ndarray   # int32 [n_shells]
    shell_l: np.ndarray      # int32 [n_shells]
    shell_exp: np.ndarray    # float64 [n_shells] (bohr^-2)

    @property
    def n_ao(self) -> int:
        return int(sum(1 if l == 0 else 3 if l == 1 else 5 for l in self.shell_l))


def _logu_spaced(rng, n, lo, hi, ratio=1.5, tries=10000):
    """n exponents log-uniform in [lo, hi] with neighbours at least `ratio` apart."""
    for _ in range(tries):
        e = np.sort(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n)))
        if n < 2 or np.all(e[1:] / e[:-1] >= ratio):
            return e[::-1].copy()
    raise RuntimeError("could not draw well-separated exponents")


def _basis_small(rng, n_atoms, species):
    """Two s shells (0.5 and 2.0, +/-10% jitter) and one p shell (0.8) per atom;
    atoms of one species share their exponents."""
    per_species = {}
    for sp in species:
        if sp not in per_species:
            j = rng.uniform(-0.1, 0.1, size=2)
            per_species[sp] = [(0, 0.5 * (1 + j[0])), (0, 2.0 * (1 + j[1])), (1, 0.8)]
    sa, sl, se = [], [], []
    for ia in range(n_atoms):
        for l, e in per_species[species[ia]]:
            sa.append(ia)
            sl.append(l)
            se.append(e)
    return Basis(np.array(sa, np.int32), np.array(sl, np.int32), np.array(se, np.float64))


def _basis_ranges(rng, n_atoms, species, spec):
    """spec: list of (l, count, lo, hi); exponents log-uniform, same-l ratio >= 1.5."""
    per_species = {}
    for sp in species:
        if sp not in per_species:
            shells = []
            for l, cnt, lo, hi in spec:
                for e in _logu_spaced(rng, cnt, lo, hi):
                    shells.append((l, float(e)))
            per_species[sp] = shells
    sa, sl, se = [], [], []
    for ia in range(n_atoms):
        for l, e in per_species[species[ia]]:
            sa.append(ia)
            sl.append(l)
            se.append(e)
    return Basis(np.array(sa, np.int32), np.array(sl, np.int32), np.array(se, np.float64))


# Real solid harmonics used as the AO functions, as Cartesian monomial lists.
# Normalised so that each primitive has unit self-overlap.
def _ao_terms(l: int, alpha: float):
    base = (2.0 * alpha / math.pi) ** 0.75
    if l == 0:
        return [[(base, (0, 0, 0))]]
    if l == 1:
        n = base * math.sqrt(4.0 * alpha)
        return [[(n, (1, 0, 0))], [(n, (0, 1, 0))], [(n, (0, 0, 1))]]
    if l == 2:
        n = 4.0 * alpha * base
        c = n / (2.0 * math.sqrt(3.0))
        return [
            [(n, (1, 1, 0))],
            [(n, (0, 1, 1))],
            [(2 * c, (0, 0, 2)), (-c, (2, 0, 0)), (-c, (0, 2, 0))],
            [(n, (1, 0, 1))],
            [(0.5 * n, (2, 0, 0)), (-0.5 * n, (0, 2, 0))],
        ]
    raise ValueError("l > 2 not supported")


def _os_table(a, b, xa, xb, imax, jmax):
    """1D Obara-Saika overlap table of (x-xa)^i e^{-a(x-xa)^2} (x-xb)^j e^{-b(x-xb)^2}."""
    p = a + b
    px = (a * xa + b * xb) / p
    s = np.zeros((imax + 2, jmax + 2))
    s[0, 0] = math.sqrt(math.pi / p) * math.exp(-a * b / p * (xa - xb) ** 2)
    for i in range(imax + 1):
        for j in range(jmax + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                v = (px - xa) * s[i - 1, j]
                if i > 1:
                    v += (i - 1) * s[i - 2, j] / (2 * p)
                if j > 0:
                    v += j * s[i - 1, j - 1] / (2 * p)
            else:
                v = (px - xb) * s[i, j - 1]
                if j > 1:
                    v += (j - 1) * s[i, j - 2] / (2 * p)
            s[i, j] = v
    return s


def real_space_overlaps(cell: Cell, basis: Basis, lattice_range: int = 1):
    """s[T][mu][nu] = int chi_mu(r-A_mu) chi_nu(r-A_nu-T) d^3r and the cell index list."""
    rr = np.arange(-lattice_range, lattice_range + 1)
    tn = np.stack(np.meshgrid(rr, rr, rr, indexing="ij"), axis=-1).reshape(-1, 3)
    tvec = tn @ cell.lat
    aos = []
    for s in range(len(basis.shell_l)):
        for terms in _ao_terms(int(basis.shell_l[s]), float(basis.shell_exp[s])):
            aos.append((s, terms))
    n = len(aos)
    out = np.zeros((len(tn), n, n))
    for it, t in enumerate(tvec):
        for m, (sm, tm) in enumerate(aos):
            am = float(basis.shell_exp[sm])
            ca = cell.xyz[basis.shell_atom[sm]]
            for v, (sv, tv) in enumerate(aos):
                bv = float(basis.shell_exp[sv])
                cb = cell.xyz[basis.shell_atom[sv]] + t
                tabs = [_os_table(am, bv, ca[x], cb[x], 2, 2) for x in range(3)]
                acc = 0.0
                for cm, pm in tm:
                    for cv, pv in tv:
                        acc += cm * cv * tabs[0][pm[0], pv[0]] * tabs[1][pm[1], pv[1]] * tabs[2][pm[2], pv[2]]
                out[it, m, v] = acc
    return tn, out


def bloch_overlap(s_t: np.ndarray, tn: np.ndarray, k_frac: np.ndarray) -> np.ndarray:
    """S(k) = sum_T exp(2 pi i kf.n_T) s_T for each row of k_frac."""
    ph = np.exp(2j * math.pi * (k_frac @ tn.T))       # [nk][nT]
    return np.einsum("kt,tmn->kmn", ph, s_t)


# --------------------------------------------------------------------------
# states
# --------------------------------------------------------------------------
def _smooth_x(rng, n_ao, n_bands, amp=0.35):
    """Seven lattice harmonics: X(k) = X0 + amp * sum_{i,+-} X_{i+-} e^{+-2 pi i kf_i}."""
    shp = (7, n_ao, n_bands)
    coef = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / math.sqrt(2.0)
    coef[1:] *= amp
    harm = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    return coef, harm


def _lowdin_once(x: np.ndarray, s: np.ndarray) -> np.ndarray:
    m = x.conj().T @ s @ x
    m = 0.5 * (m + m.conj().T)
    w, u = np.linalg.eigh(m)
    if w.min() <= 1e-12 * w.max():
        raise RuntimeError("rank-deficient random coefficients")
    return x @ (u * (1.0 / np.sqrt(w))) @ u.conj().T


def lowdin(x: np.ndarray, s: np.ndarray) -> np.ndarray:
    """C = X (X^H S X)^{-1/2} for one k, applied twice: where X is nearly
    singular the first pass leaves C^H S C - I at ~eps cond(X)^2; the second
    pass starts from the well-conditioned C and brings it to ~eps."""
    return _lowdin_once(_lowdin_once(x, s), s)


@dataclass
class QStates:
    """States at k and at k+q for one q (the inputs of one pair-density call)."""
    q_cart: np.ndarray       # [3] bohr^-1
    C_k: np.ndarray          # [n_k][n_ao][n_bands] complex128
    E_k: np.ndarray          # [n_k][n_bands] eV
    C_kq: np.ndarray
    E_kq: np.ndarray


@dataclass
class Workload:
    name: str
    cell: Cell
    basis: Basis
    lattice_range: int
    n_occ: int
    n_bands: int
    k_frac: np.ndarray
    G_int: np.ndarray
    w_eV: np.ndarray
    eta_eV: float
    q_list: List[np.ndarray]
    seed: int
    energy_ranges: Sequence = ()
    smooth: bool = True
    smooth_bands: bool = False
    _x: Optional[tuple] = field(default=None, repr=False)
    _s: Optional[tuple] = field(default=None, repr=False)
    _ek: Optional[np.ndarray] = field(default=None, repr=False)
    _ck: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def n_k(self):
        return len(self.k_frac)

    @property
    def n_ao(self):
        return self.basis.n_ao

    @property
    def n_cond(self):
        return self.n_bands - self.n_occ

    @property
    def n_t(self):
        return 2 * self.n_occ * self.n_cond * self.n_k

    def states(self, iq: int) -> QStates:
        return draw_states(self, iq)


def _energies(rng, n_k, ranges):
    cols = []
    for cnt, lo, hi in ranges:
        cols.append(np.sort(rng.uniform(lo, hi, size=(n_k, cnt)), axis=1))
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


def _band_model(rng, ranges, amp=0.06):
    """Smooth periodic bands: per band a level drawn in its range plus three
    cosine harmonics e^{2 pi i kf.h} (h = unit vectors) with amplitude amp x
    the range width and random phases."""
    levels, amps, phases = [], [], []
    for cnt, lo, hi in ranges:
        levels.append(np.sort(rng.uniform(lo, hi, size=cnt)))
        amps.append(amp * (hi - lo) * rng.uniform(0.5, 1.0, size=(cnt, 3)))
        phases.append(rng.uniform(0.0, 2 * math.pi, size=(cnt, 3)))
    return levels, amps, phases


def _band_energies(model, ranges, k_frac):
    """E_n(k) of the band model, sorted within each group and kept in range."""
    levels, amps, phases = model
    cols = []
    for (cnt, lo, hi), lv, am, ph in zip(ranges, levels, amps, phases):
        arg = 2 * math.pi * k_frac[:, None, :] + ph[None, :, :]        # [nk][cnt][3]
        e = lv[None, :] + np.sum(am[None] * np.cos(arg), axis=2)
        cols.append(np.sort(np.clip(e, lo, hi), axis=1))
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


def _coeffs(wl: Workload, k_frac: np.ndarray, rng_iid=None):
    if wl._s is None:
        wl._s = real_space_overlaps(wl.cell, wl.basis, wl.lattice_range)
    tn, s_t = wl._s
    s_k = bloch_overlap(s_t, tn, k_frac)
    out = np.empty((len(k_frac), wl.n_ao, wl.n_bands), np.complex128)
    if wl.smooth:
        coef, harm = wl._x
        ph = np.exp(2j * math.pi * (k_frac @ harm.T))    # [nk][7]
        xs = np.einsum("kh,hab->kab", ph, coef)
    else:
        shp = (len(k_frac), wl.n_ao, wl.n_bands)
        xs = (rng_iid.standard_normal(shp) + 1j * rng_iid.standard_normal(shp)) / math.sqrt(2.0)
    for i in range(len(k_frac)):
        out[i] = lowdin(xs[i], s_k[i])
    return out


def draw_states(wl: Workload, iq: int) -> QStates:
    ss = np.random.SeedSequence(wl.seed)
    kids = ss.spawn(3 + len(wl.q_list))
    if wl._x is None:
        wl._x = _smooth_x(np.random.default_rng(kids[0]), wl.n_ao, wl.n_bands)
    bands = _band_model(np.random.default_rng(kids[2]), wl.energy_ranges) if wl.smooth_bands else None
    if wl._ck is None:
        rk = np.random.default_rng(kids[1])
        if bands is not None:
            wl._ek = _band_energies(bands, wl.energy_ranges, wl.k_frac)
        else:
            wl._ek = _energies(rk, wl.n_k, wl.energy_ranges)
        wl._ck = _coeffs(wl, wl.k_frac, rk)
    q = np.asarray(wl.q_list[iq], np.float64)
    qf = wl.cell.lat @ q / (2.0 * math.pi)
    rq = np.random.default_rng(kids[3 + iq])
    if bands is not None:
        e_kq = _band_energies(bands, wl.energy_ranges, wl.k_frac + qf[None, :])
    else:
        e_kq = _energies(rq, wl.n_k, wl.energy_ranges)
    c_kq = _coeffs(wl, wl.k_frac + qf[None, :], rq)
    return QStates(q_cart=q, C_k=wl._ck, E_k=wl._ek, C_kq=c_kq, E_kq=e_kq)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def make_smallest(smooth: bool = True) -> Workload:
    """Smallest FP64 instance: 10 GTOs, 4+6 bands, 4^3 k, one q, 27 G, 128 w."""
    seed = BASE_SEED + 1
    cell = fcc_cell(10.26, "Si-like")
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    basis = _basis_small(rng, 2, cell.species)
    a = cell.a
    return Workload(
        name="c1_diamond_ng27", cell=cell, basis=basis, lattice_range=1, n_occ=4, n_bands=10,
        k_frac=gamma_grid(4), G_int=g_cube(cell.lat), w_eV=np.linspace(0.0, 40.0, 128),
        eta_eV=0.2, q_list=[np.array([0.1 * 2 * math.pi / a, 0.0, 0.0])], seed=seed,
        energy_ranges=[(4, -12.0, 0.0), (6, 1.1, 15.0)], smooth=smooth)


SI_SPEC = [(0, 3, 0.1, 50.0), (1, 2, 0.1, 50.0), (2, 1, 0.1, 50.0)]


def make_si_ng113(n_q: int = 10, n_w: int = 400, kgrid: int = 8, smooth: bool = True) -> Workload:
    """Si-scale precision study: 28 AO, 4+16 bands, 8^3 k, 10 q on [100], N_G=113, 400 w."""
    seed = BASE_SEED + 2
    cell = fcc_cell(10.26, "Si-like")
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    basis = _basis_ranges(rng, 2, cell.species, SI_SPEC)
    a = cell.a
    qs = [np.array([(i / 10.0) * 2 * math.pi / a, 0.0, 0.0]) for i in range(1, n_q + 1)]
    return Workload(
        name="c2_si_ng113", cell=cell, basis=basis, lattice_range=1, n_occ=4, n_bands=20,
        k_frac=gamma_grid(kgrid), G_int=g_shells(cell.lat, 113), w_eV=np.linspace(0.0, 60.0, n_w),
        eta_eV=0.1, q_list=qs, seed=seed,
        energy_ranges=[(4, -12.0, 0.0), (16, 1.1, 15.0)], smooth=smooth)


MIXED_CELLS = [
    ("diamond-like", 6.74, ("C", "C")),
    ("Si-like", 10.26, ("Si", "Si")),
    ("Ge-like", 10.69, ("Ge", "Ge")),
    ("GaAs-like", 10.68, ("Ga", "As")),
    ("SiC-like", 8.24, ("Si", "C")),
]
MIXED_NG = [59, 113, 181, 259]


def make_mixed_batch_items(n_items: int = 20, kgrid_override: Optional[int] = None) -> List[Workload]:
    """Mixed batch: item i uses cell i mod 5, N_G = [59,113,181,259][i div 5],
    an n^3 k grid with n = 6 + (3i mod 5), q = (0.1+0.04 i) 2pi/a along x,
    n_w = 10 i + 5 frequencies over 0-60 eV, eta = 0.1 eV."""
    items = []
    for i in range(n_items):
        name, a, species = MIXED_CELLS[i % 5]
        seed = BASE_SEED + 300 + i
        cell = fcc_cell(a, name, species)
        rng = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 3 + 1000 * (i % 5)).spawn(3)[2])
        basis = _basis_small(rng, 2, species)
        n = kgrid_override if kgrid_override else 6 + (3 * i) % 5
        items.append(Workload(
            name=f"c3_item{i}_{name}", cell=cell, basis=basis, lattice_range=1, n_occ=4, n_bands=10,
            k_frac=gamma_grid(n), G_int=g_shells(cell.lat, MIXED_NG[(i // 5) % 4]),
            w_eV=np.linspace(0.0, 60.0, 10 * i + 5), eta_eV=0.1,
            q_list=[np.array([(0.1 + 0.04 * i) * 2 * math.pi / a, 0.0, 0.0])], seed=seed,
            energy_ranges=[(4, -12.0, 0.0), (6, 1.1, 15.0)]))
    return items


def make_all_electron(n_w: int = 1000, kgrid: int = 12, q_list=None) -> Workload:
    """High-momentum all-electron case: 6s+5p+1d per atom (26 AO), 5 core + 4 valence
    + 28 conduction bands, 12^3 k, N_G = 749, 1000 w over 0-100 eV."""
    seed = BASE_SEED + 4
    cell = fcc_cell(10.26, "Si-like")
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    spec = [(0, 6, 0.1, 1.0e4), (1, 5, 0.1, 50.0), (2, 1, 0.1, 50.0)]
    basis = _basis_ranges(rng, 2, cell.species, spec)
    a = cell.a
    if q_list is None:
        q_list = [np.array([0.25 * 2 * math.pi / a, 0.0, 0.0])]
    return Workload(
        name="c4_si_allelectron_ng749", cell=cell, basis=basis, lattice_range=1, n_occ=9, n_bands=37,
        k_frac=gamma_grid(kgrid), G_int=g_shells(cell.lat, 749), w_eV=np.linspace(0.0, 100.0, n_w),
        eta_eV=0.1, q_list=q_list, seed=seed,
        energy_ranges=[(5, -1800.0, -100.0), (4, -12.0, 0.0), (28, 1.1, 100.0)])


def make_tiny(a: float = 4.0, kgrid: int = 2, n_g: int = 9, n_w: int = 16, with_d: bool = True,
              q_frac: float = 0.15, seed_off: int = 0, smooth: bool = True) -> Workload:
    """A small cell with s, p and d shells (exponents >= 1) for brute-force checks."""
    seed = BASE_SEED + 900 + seed_off
    cell = fcc_cell(a, "tiny")
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    spec = [(0, 2, 1.0, 4.0), (1, 1, 1.0, 3.0)] + ([(2, 1, 1.0, 3.0)] if with_d else [])
    basis = _basis_ranges(rng, 2, cell.species, spec)
    n_ao = basis.n_ao
    n_occ = 2
    n_bands = n_ao
    return Workload(
        name="tiny", cell=cell, basis=basis, lattice_range=1, n_occ=n_occ, n_bands=n_bands,
        k_frac=gamma_grid(kgrid), G_int=g_shells(cell.lat, n_g), w_eV=np.linspace(0.0, 40.0, n_w),
        eta_eV=0.3, q_list=[np.array([q_frac * 2 * math.pi / a, 0.05, 0.0])], seed=seed,
        energy_ranges=[(n_occ, -12.0, 0.0), (n_bands - n_occ, 1.1, 30.0)], smooth=smooth)
