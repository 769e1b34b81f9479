"""Pins for the oracle's Gaussian Fourier integrals and AO matrix (CPU only).

Each test checks the oracle against something other than itself: a closed
form, brute-force real-space quadrature, the generator's independent
real-space overlap recursion, or a symmetry the definition implies.
"""
import math

import numpy as np
import pytest

from oracle import gto
from synth.generator import bloch_overlap, fcc_cell, real_space_overlaps, Basis


def test_moments_against_quadrature():
    # I_n = int y^n exp(-p y^2 + i Q y) dy by dense trapezoid quadrature
    p, q = 1.7, 2.3
    y = np.linspace(-12, 12, 24001)
    h = y[1] - y[0]
    mom = gto.gaussian_moments(p, np.array([q]), 6)[:, 0]
    for n in range(7):
        ref = np.sum(y ** n * np.exp(-p * y * y + 1j * q * y)) * h
        assert abs(mom[n] - ref) < 1e-12 * max(1.0, abs(ref))


def test_ss_closed_form():
    # two s primitives: N^2 (pi/p)^{3/2} K e^{-Q^2/4p} e^{iQ.P}
    lat = np.eye(3) * 50.0
    xyz = np.array([[0.1, -0.2, 0.3], [0.9, 0.4, -0.5]])
    a, b = 0.7, 1.9
    Q = np.array([[0.0, 0.0, 0.0], [0.8, -1.1, 0.4], [2.5, 0.3, 1.7]])
    F = gto.cell_ft(lat, xyz, [0, 1], [0, 0], [a, b], 0, Q)
    A, B = xyz[0], xyz[1]
    p = a + b
    P = (a * A + b * B) / p
    K = math.exp(-a * b / p * np.sum((A - B) ** 2))
    na = (2 * a / math.pi) ** 0.75
    nb = (2 * b / math.pi) ** 0.75
    for g in range(3):
        ref = na * nb * (math.pi / p) ** 1.5 * K * np.exp(-Q[g] @ Q[g] / (4 * p)) * np.exp(1j * Q[g] @ P)
        assert abs(F[0, g, 0, 1] - ref) < 1e-14


def test_single_centre_orthonormal_and_traceless():
    # one atom, one shell of each l: the AOs are orthonormal; d functions are
    # orthogonal to the r^2 Gaussian (traceless, i.e. pure l = 2)
    lat = np.eye(3) * 60.0
    xyz = np.zeros((1, 3))
    for l, e in [(0, 0.9), (1, 1.3), (2, 0.6)]:
        S = gto.cell_ft(lat, xyz, [0], [l], [e], 0, np.zeros((1, 3)))[0, 0]
        assert np.max(np.abs(S - np.eye(2 * l + 1))) < 1e-13
    # r^2 e^{-a r^2} (unnormalised) against the 5 d functions by quadrature
    a = 0.6
    x = np.linspace(-8, 8, 161)
    h = x[1] - x[0]
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    d = gto.eval_ao(lat, xyz, [0], [2], [a], r)
    r2g = np.sum(r * r, axis=1) * np.exp(-a * np.sum(r * r, axis=1))
    assert np.max(np.abs(d @ r2g) * h ** 3) < 1e-10


def test_overlap_matches_generator_recursion():
    # the oracle's S(k) = M(k; 0) against the generator's Obara-Saika route
    cell = fcc_cell(10.26)
    basis = Basis(np.array([0, 0, 0, 1, 1, 1], np.int32), np.array([0, 1, 2, 0, 1, 2], np.int32),
                  np.array([0.45, 0.8, 0.6, 1.7, 0.35, 2.2]))
    kf = np.array([[0.0, 0.0, 0.0], [0.25, -0.125, 0.5], [0.31, 0.77, 0.12]])
    S_or = gto.overlap_matrix(cell.lat, cell.xyz, basis.shell_atom, basis.shell_l, basis.shell_exp, 1, kf)
    tn, s_t = real_space_overlaps(cell, basis, 1)
    S_gen = bloch_overlap(s_t, tn, kf)
    assert np.max(np.abs(S_or - S_gen)) < 1e-12
    for S in S_or:
        assert np.max(np.abs(S - S.conj().T)) < 1e-13
        assert np.linalg.eigvalsh(0.5 * (S + S.conj().T)).min() > 0


def test_bloch_periodicity(tiny):
    b = gto.reciprocal_basis(tiny.cell.lat)
    Q = np.array([[0.3, -0.2, 0.5], [1.1, 0.4, -0.9]])
    kf = np.array([[0.1, 0.2, -0.3]])
    bs = tiny.basis
    M0 = gto.ao_matrix(tiny.cell.lat, tiny.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1, kf, Q)
    M1 = gto.ao_matrix(tiny.cell.lat, tiny.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1,
                       kf + np.array([[1.0, -2.0, 1.0]]), Q)
    assert np.max(np.abs(M0 - M1)) < 1e-12
    assert b.shape == (3, 3)


@pytest.mark.slow
def test_ao_matrix_bruteforce_quadrature(tiny):
    """M(k; Q) against a 3D trapezoid sum of the defining integral over all 27 cells.

    Tiny fcc cell (a = 4 bohr), s, p and d shells with exponents >= 1, |Q| <= 3.
    The trapezoid rule is spectrally accurate for these smooth, decaying
    integrands, so the two must agree to ~1e-10.
    """
    cell, bs = tiny.cell, tiny.basis
    Q = np.array([[0.0, 0.0, 0.0], [0.9, -0.4, 0.3], [1.2, 2.1, -1.5]])
    kf = np.array([[0.0, 0.0, 0.0], [0.2, -0.35, 0.1]])
    M = gto.ao_matrix(cell.lat, cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1, kf, Q)
    h = 0.16
    x = np.arange(-4.8, 5.8 + 1e-9, h)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    bra = gto.eval_ao(cell.lat, cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, r)   # [nao][npts]
    cells = gto.lattice_cells(1)
    tvec = cells @ cell.lat
    pw = np.exp(1j * r @ Q.T)                                                        # [npts][nQ]
    ref = np.zeros_like(M)
    for it, t in enumerate(tvec):
        ket = gto.eval_ao(cell.lat, cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, r, shift=t)
        ph = np.exp(2j * math.pi * kf @ cells[it])
        for g in range(len(Q)):
            blk = (bra * pw[:, g][None, :]) @ ket.T * h ** 3
            ref[:, g] += ph[:, None, None] * blk[None]
    err = np.max(np.abs(M - ref))
    assert err < 1e-10, err
