"""Pins of the oracle's optical limit (App. C): gradient integrals, the k.p
row of the pair densities and the head and wings of eps as q -> 0."""
import math

import numpy as np
import pytest

from oracle import gto, rpa
from synth.generator import Basis


def _single_atom(shells):
    lat = np.eye(3) * 30.0
    xyz = np.zeros((1, 3))
    l = np.array([s[0] for s in shells])
    e = np.array([s[1] for s in shells])
    return lat, xyz, np.zeros(len(shells), int), l, e


def test_grad_single_centre_closed_form():
    """Same centre: <s_a| d/dx |p_x,b> = N_s N_p (pi/p)^{3/2} a/p and
    <p_x,a| d/dx |s_b> = -N_p N_s (pi/p)^{3/2} b/p (p = a + b)."""
    a, b = 0.7, 1.9
    lat, xyz, at, l, e = _single_atom([(0, a), (1, b), (1, a), (0, b)])
    D = gto.grad_cell(lat, xyz, at, l, e, 0)[0]          # [c][mu][nu], one cell
    p = a + b
    Ns = lambda x: (2 * x / math.pi) ** 0.75
    Np = lambda x: (2 * x / math.pi) ** 0.75 * math.sqrt(4 * x)
    ref1 = Ns(a) * Np(b) * (math.pi / p) ** 1.5 * a / p
    ref2 = -Np(a) * Ns(b) * (math.pi / p) ** 1.5 * b / p
    # AO order: s_a (0), p_b x,y,z (1..3), p_a x,y,z (4..6), s_b (7)
    assert abs(D[0, 0, 1] - ref1) < 1e-14 * abs(ref1)
    assert abs(D[0, 4, 7] - ref2) < 1e-14 * abs(ref2)
    assert abs(D[1, 0, 2] - ref1) < 1e-14 * abs(ref1) and abs(D[0, 0, 2]) < 1e-15


def test_grad_translation_identity():
    """d/dx_B of <mu_A | nu_B> (Bloch sums at k) is -<mu_A | d/dx nu_B>: the
    gradient integrals against central differences of the overlap when atom
    B moves (mu on atom A, nu on atom B), s, p and d shells, two k points."""
    a0 = 6.0
    lat = 0.5 * a0 * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    xyz = np.array([[0.0, 0.0, 0.0], [0.25 * a0, 0.27 * a0, 0.23 * a0]])
    l = np.array([0, 1, 2, 0, 1, 2])
    e = np.array([0.6, 0.9, 1.2, 0.8, 0.7, 1.1])
    at = np.array([0, 0, 0, 1, 1, 1])
    kf = np.array([[0.0, 0.0, 0.0], [0.2, -0.1, 0.35]])
    D = gto.grad_matrix(lat, xyz, at, l, e, 1, kf)        # [k][c][mu][nu]
    off = gto.ao_offsets(l)
    A = slice(0, off[3])
    B = slice(off[3], off[6])
    h = 1e-4
    for c in range(3):
        xp, xm = xyz.copy(), xyz.copy()
        xp[1, c] += h
        xm[1, c] -= h
        Sp = gto.overlap_matrix(lat, xp, at, l, e, 1, kf)
        Sm = gto.overlap_matrix(lat, xm, at, l, e, 1, kf)
        fd = -(Sp - Sm) / (2 * h)
        err = np.max(np.abs(fd[:, A, B] - D[:, c, A, B]))
        assert err < 1e-7 * np.max(np.abs(D[:, c, A, B])), (c, err)


def test_grad_bloch_anti_hermitian(tiny):
    bs = tiny.basis
    D = gto.grad_matrix(tiny.cell.lat, tiny.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1,
                        tiny.k_frac)
    assert np.max(np.abs(D + np.conj(np.transpose(D, (0, 1, 3, 2))))) < 1e-13 * np.max(np.abs(D))


def _optical(wl, w, eta, qhat):
    st = wl.states(0)
    bs = wl.basis
    R = rpa.pair_densities_optical(wl.cell, bs, wl.lattice_range, wl.k_frac, wl.G_int, st.C_k,
                                   st.E_k, wl.n_occ, qhat)
    vol = abs(float(np.linalg.det(np.asarray(wl.cell.lat))))
    W = rpa.transition_weights(st.E_k, st.E_k, wl.n_occ, w, eta, vol)
    chi = rpa.chi0(R, W)
    eps = rpa.epsilon_optical(chi, wl.cell.lat, wl.G_int)
    return st, R, vol, eps


@pytest.mark.parametrize("qhat", [(1.0, 0.0, 0.0), (0.3, -0.5, 0.81)])
def test_optical_head_wings_explicit(tiny, qhat):
    """The k.p row inside Eq. (RPA) gives App. C's explicit head and wings."""
    w = np.linspace(0.0, 30.0, 13)
    st, R, vol, eps = _optical(tiny, w, 0.3, qhat)
    bs = tiny.basis
    P = rpa.momentum_bands(tiny.cell, bs, tiny.lattice_range, tiny.k_frac, st.C_k)
    gnorm = np.linalg.norm(rpa.q_plus_g(tiny.cell.lat, np.zeros(3), tiny.G_int), axis=1)[1:]
    head, w0G, wG0 = rpa.optical_head_wings(P, st.E_k, tiny.n_occ, w, 0.3, qhat, vol,
                                            R[..., 1:], gnorm)
    scale = np.max(np.abs(eps[:, 0, 1:]))
    assert np.max(np.abs(eps[:, 0, 0] - head)) < 1e-12 * np.max(np.abs(head))
    assert np.max(np.abs(eps[:, 0, 1:] - w0G)) < 1e-12 * scale
    assert np.max(np.abs(eps[:, 1:, 0] - wG0)) < 1e-12 * scale


def test_optical_head_absorbs(tiny):
    """Im eps_00 >= 0 for w > 0 (absorption), Re eps_00(0) > 1 (screening), and
    the head is even in qhat."""
    w = np.linspace(0.01, 40.0, 60)
    _, _, _, e1 = _optical(tiny, w, 0.2, (0.0, 0.6, 0.8))
    _, _, _, e2 = _optical(tiny, w, 0.2, (0.0, -0.6, -0.8))
    assert np.all(e1[:, 0, 0].imag >= 0.0)
    assert e1[0, 0, 0].real > 1.0
    assert np.max(np.abs(e1[:, 0, 0] - e2[:, 0, 0])) < 1e-13 * np.max(np.abs(e1[:, 0, 0]))
