"""Gaussian basis and lattice-summed Fourier integrals (oracle, FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The matrix elements that enter Eq. (RPA), <i k| e^{-i(q+G).r} |j k'> and its
partner, are overlaps of Bloch states with a plane wave.  For states built
from Gaussian-type orbitals (Sec. III: PySCF Gaussian basis sets) they reduce
to the AO matrix

    M_mu,nu(k; Q) = sum_T e^{i k.T} int chi_mu(r - A_mu) e^{i Q.r} chi_nu(r - A_nu - T) d^3r

with the bra at k+q, the ket at k and Q = q + G (translate the bra cell to
the origin; e^{iG.T} = 1).  The Bloch phase is e^{ik.T}, not e^{ik.(T+A)},
and the lattice sum runs over n in {-L..L}^3 primitive cells (L = 1 gives
the 27 cells of the workloads); the truncation defines the model.

Each primitive integral factorises over x, y, z.  Per axis the product of
two Gaussians is K_x e^{-p (x-P_x)^2}; the polynomial prefactor is expanded
binomially about P_x, and the remaining moments

    I_n = int y^n e^{-p y^2 + i Q_x y} dy
    I_0 = sqrt(pi/p) e^{-Q_x^2/(4p)},  I_1 = (i Q_x / 2p) I_0,
    I_{n+1} = (i Q_x I_n + n I_{n-1}) / (2p)

follow from integrating the derivative of the Gaussian by parts.

Parity pins (tests/test_oracle_gto.py): s-s closed form; brute-force
real-space quadrature of M on a tiny cell with s, p and d shells; unit
self-overlap of every AO; Bloch periodicity M(k + b) = M(k); S(k)
Hermitian positive-definite.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

# --------------------------------------------------------------------------
# AO definitions: real solid harmonics, primitive normalised to unit norm.
#   s: (2a/pi)^{3/4} e^{-a r^2}
#   p: (2a/pi)^{3/4} (4a)^{1/2} {x, y, z} e^{-a r^2}
#   d: N_d {xy, yz, (2z^2-x^2-y^2)/(2 sqrt 3), xz, (x^2-y^2)/2} e^{-a r^2},
#      N_d = 4a (2a/pi)^{3/4}
# --------------------------------------------------------------------------


def ao_cartesian_terms(l: int, a: float) -> List[List[Tuple[float, Tuple[int, int, int]]]]:
    """For one shell: a list (one entry per AO) of (coefficient, (i, j, k)) monomials."""
    g = (2.0 * a / math.pi) ** 0.75
    if l == 0:
        return [[(g, (0, 0, 0))]]
    if l == 1:
        c = g * math.sqrt(4.0 * a)
        return [[(c, (1, 0, 0))], [(c, (0, 1, 0))], [(c, (0, 0, 1))]]
    if l == 2:
        nd = 4.0 * a * g
        h = nd / (2.0 * math.sqrt(3.0))
        return [
            [(nd, (1, 1, 0))],
            [(nd, (0, 1, 1))],
            [(-h, (2, 0, 0)), (-h, (0, 2, 0)), (2.0 * h, (0, 0, 2))],
            [(nd, (1, 0, 1))],
            [(0.5 * nd, (2, 0, 0)), (-0.5 * nd, (0, 2, 0))],
        ]
    raise ValueError("only l <= 2")


def n_ao_of(shell_l) -> int:
    return int(sum(2 * int(l) + 1 for l in shell_l))


def ao_offsets(shell_l) -> np.ndarray:
    off = np.zeros(len(shell_l) + 1, dtype=np.int64)
    for i, l in enumerate(shell_l):
        off[i + 1] = off[i] + 2 * int(l) + 1
    return off


def lattice_cells(lattice_range: int) -> np.ndarray:
    """Integer triples n in {-L..L}^3, lexicographic."""
    r = np.arange(-lattice_range, lattice_range + 1)
    return np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)


def reciprocal_basis(lat: np.ndarray) -> np.ndarray:
    """Rows b_j with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(np.asarray(lat, np.float64)).T


# --------------------------------------------------------------------------
# 1D Fourier moments and the per-axis integral
# --------------------------------------------------------------------------


def gaussian_moments(p: float, qx: np.ndarray, nmax: int) -> np.ndarray:
    """I_n(Q) = int y^n exp(-p y^2 + i Q y) dy for n = 0..nmax; shape [nmax+1, len(qx)]."""
    qx = np.asarray(qx, np.float64)
    out = np.zeros((nmax + 1,) + qx.shape, np.complex128)
    out[0] = math.sqrt(math.pi / p) * np.exp(-qx * qx / (4.0 * p))
    if nmax >= 1:
        out[1] = (1j * qx / (2.0 * p)) * out[0]
    for n in range(1, nmax):
        out[n + 1] = (1j * qx * out[n] + n * out[n - 1]) / (2.0 * p)
    return out


def axis_integrals(a: float, b: float, xa, xb, qx: np.ndarray, imax: int, jmax: int) -> np.ndarray:
    """J[i][j] = int (x-xa)^i (x-xb)^j e^{-a(x-xa)^2 - b(x-xb)^2} e^{i qx x} dx.

    xb may be an array (one entry per lattice cell); result shape
    [imax+1, jmax+1, len(xb), len(qx)].
    """
    xb = np.atleast_1d(np.asarray(xb, np.float64))
    qx = np.atleast_1d(np.asarray(qx, np.float64))
    p = a + b
    px = (a * xa + b * xb) / p                            # [nT]
    kx = np.exp(-a * b / p * (xa - xb) ** 2)               # [nT]
    mom = gaussian_moments(p, qx, imax + jmax)             # [n][nQ]
    pa = (px - xa)[:, None]
    pb = (px - xb)[:, None]
    phase = np.exp(1j * px[:, None] * qx[None, :]) * kx[:, None]   # [nT][nQ]
    out = np.zeros((imax + 1, jmax + 1, len(xb), len(qx)), np.complex128)
    for i in range(imax + 1):
        for j in range(jmax + 1):
            acc = np.zeros((len(xb), len(qx)), np.complex128)
            for u in range(i + 1):
                for w in range(j + 1):
                    coef = math.comb(i, u) * math.comb(j, w) * pa ** (i - u) * pb ** (j - w)
                    acc = acc + coef * mom[u + w][None, :]
            out[i, j] = phase * acc
    return out


# --------------------------------------------------------------------------
# lattice-resolved AO Fourier integrals and the Bloch sum
# --------------------------------------------------------------------------


def cell_ft(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range: int, Q: np.ndarray) -> np.ndarray:
    """F[T][g][mu][nu] = int chi_mu(r - A_mu) e^{i Q_g.r} chi_nu(r - A_nu - T) d^3r."""
    lat = np.asarray(lat, np.float64)
    xyz = np.asarray(xyz, np.float64)
    Q = np.atleast_2d(np.asarray(Q, np.float64))
    cells = lattice_cells(lattice_range)
    tvec = cells @ lat
    off = ao_offsets(shell_l)
    nao = int(off[-1])
    out = np.zeros((len(cells), len(Q), nao, nao), np.complex128)
    for sa in range(len(shell_l)):
        la, ea = int(shell_l[sa]), float(shell_exp[sa])
        A = xyz[shell_atom[sa]]
        terms_a = ao_cartesian_terms(la, ea)
        for sb in range(len(shell_l)):
            lb, eb = int(shell_l[sb]), float(shell_exp[sb])
            B = xyz[shell_atom[sb]][None, :] + tvec               # [nT][3]
            terms_b = ao_cartesian_terms(lb, eb)
            J = [axis_integrals(ea, eb, A[x], B[:, x], Q[:, x], la, lb) for x in range(3)]
            for ia, ta in enumerate(terms_a):
                for ib, tb in enumerate(terms_b):
                    acc = 0.0
                    for ca, (px, py, pz) in ta:
                        for cb, (qx_, qy_, qz_) in tb:
                            acc = acc + ca * cb * J[0][px, qx_] * J[1][py, qy_] * J[2][pz, qz_]
                    out[:, :, off[sa] + ia, off[sb] + ib] = acc
    return out


def bloch_phases(k_frac: np.ndarray, lattice_range: int) -> np.ndarray:
    """e^{i k.T} for k = kf.b and T = n.a, i.e. e^{2 pi i kf.n}; shape [nk][nT]."""
    cells = lattice_cells(lattice_range)
    return np.exp(2j * math.pi * (np.asarray(k_frac, np.float64) @ cells.T))


def ao_matrix(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range, k_frac, Q) -> np.ndarray:
    """M[k][g][mu][nu] (Bloch bra at k+q, ket at k; Q = q + G).  Parity: pinned by
    quadrature, closed form and periodicity tests."""
    F = cell_ft(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range, Q)
    ph = bloch_phases(k_frac, lattice_range)
    nT, nG, n, _ = F.shape
    return (ph @ F.reshape(nT, -1)).reshape(len(ph), nG, n, n)


def overlap_matrix(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range, k_frac) -> np.ndarray:
    """S(k) = M(k; Q = 0) (q = 0, G = 0)."""
    M = ao_matrix(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range, k_frac, np.zeros((1, 3)))
    return M[:, 0]


def grad_cell(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range: int) -> np.ndarray:
    """D[T][c][mu][nu] = int chi_mu(r - A_mu) d/dr_c chi_nu(r - A_nu - T) d^3r
    (App. C's <i k| grad |j k> in the AO basis, before the Bloch sum).

    Per axis the ket's derivative is d/dx (x-B)^j e^{-b(x-B)^2} = j (x-B)^{j-1}
    e^{...} - 2b (x-B)^{j+1} e^{...}, so the axis factor of component c is
    j J[i][j-1] - 2 b J[i][j+1] with J the Q = 0 axis integrals; the other
    two axes keep their overlaps."""
    lat = np.asarray(lat, np.float64)
    xyz = np.asarray(xyz, np.float64)
    cells = lattice_cells(lattice_range)
    tvec = cells @ lat
    off = ao_offsets(shell_l)
    nao = int(off[-1])
    out = np.zeros((len(cells), 3, nao, nao))
    for sa in range(len(shell_l)):
        la, ea = int(shell_l[sa]), float(shell_exp[sa])
        A = xyz[shell_atom[sa]]
        terms_a = ao_cartesian_terms(la, ea)
        for sb in range(len(shell_l)):
            lb, eb = int(shell_l[sb]), float(shell_exp[sb])
            B = xyz[shell_atom[sb]][None, :] + tvec
            terms_b = ao_cartesian_terms(lb, eb)
            S1 = [np.real(axis_integrals(ea, eb, A[x], B[:, x], [0.0], la, lb + 1)[..., 0])
                  for x in range(3)]                                  # [i][j][nT]
            D1 = []
            for x in range(3):
                d = np.zeros((la + 1, lb + 1, len(cells)))
                for j in range(lb + 1):
                    d[:, j] = -2.0 * eb * S1[x][:, j + 1]
                    if j > 0:
                        d[:, j] += j * S1[x][:, j - 1]
                D1.append(d)
            for ia, ta in enumerate(terms_a):
                for ib, tb in enumerate(terms_b):
                    for c in range(3):
                        acc = 0.0
                        for ca, pa in ta:
                            for cb, pb in tb:
                                f = ca * cb
                                for x in range(3):
                                    f = f * (D1[x] if x == c else S1[x])[pa[x], pb[x]]
                                acc = acc + f
                        out[:, c, off[sa] + ia, off[sb] + ib] = acc
    return out


def grad_matrix(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range, k_frac) -> np.ndarray:
    """D(k)[k][c][mu][nu] = sum_T e^{ik.T} D[T][c][mu][nu] (anti-Hermitian per k, c)."""
    D = grad_cell(lat, xyz, shell_atom, shell_l, shell_exp, lattice_range)
    ph = bloch_phases(k_frac, lattice_range)
    nT, _, n, _ = D.shape
    return (ph @ D.reshape(nT, -1)).reshape(len(ph), 3, n, n)


def eval_ao(lat, xyz, shell_atom, shell_l, shell_exp, r: np.ndarray, shift=None) -> np.ndarray:
    """Values of every AO chi_mu(r - A_mu - shift) on points r [npts][3]; shape [nao][npts]."""
    r = np.asarray(r, np.float64)
    shift = np.zeros(3) if shift is None else np.asarray(shift, np.float64)
    off = ao_offsets(shell_l)
    out = np.zeros((int(off[-1]), len(r)))
    for s in range(len(shell_l)):
        d = r - (np.asarray(xyz, np.float64)[shell_atom[s]] + shift)[None, :]
        e = np.exp(-float(shell_exp[s]) * np.sum(d * d, axis=1))
        for i, terms in enumerate(ao_cartesian_terms(int(shell_l[s]), float(shell_exp[s]))):
            v = np.zeros(len(r))
            for c, (px, py, pz) in terms:
                v += c * d[:, 0] ** px * d[:, 1] ** py * d[:, 2] ** pz
            out[off[s] + i] = v * e
    return out
