"""Kramers-Kronig route (qcx_chi0_kk) against the oracle's binned route.

Both sides compute the same quantity in FP64: hat-function bins of the
spectral part, then the exact transform of each hat through the energy
denominator.  The GPU sums each bin over energy-sorted transitions and
transforms on FP64 MFMA; the oracle forms every bin from the dense hat
weights.  Bars: chi0 to 1e-11 of its largest element, the loss to 1e-10
per G curve (the FP64 bars of the direct route).  Cases: the smallest
workload at eta = 0.2 eV and at eta = 0 (pure spectral part + its
Kramers-Kronig transform), one bin wider than every transition energy,
chunk boundaries (very fine bins with empty intervals, intervals above the
chunk budget), the
tiny s/p/d cell (9 G, one 64 x 64 tile, ragged), 137 G (3 x 3 tiles, the
last ragged), repeatability, and second
order convergence to the direct FP64 route on the GPU itself.
"""
import numpy as np
import pytest

from oracle import rpa
from tests.gpu_helpers import normwise, relmax, set_inputs

pytestmark = pytest.mark.gpu

TOL_CHI, TOL_LOSS = 1e-11, 1e-10


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2603_12326_amd import Context

    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def _vol(wl):
    return abs(float(np.linalg.det(np.asarray(wl.cell.lat, np.float64))))


def _gpu_kk(ctx, wl, w, eta, b):
    import torch

    set_inputs(ctx, wl)
    ctx.pair_density(wl.G_int)
    n = len(wl.G_int)
    chi = torch.empty((len(w), n, n), dtype=torch.complex128, device="cuda")
    ctx.chi0_kk(w, eta, b, chi)
    ctx.eps_inv(True)
    return chi.cpu().numpy(), ctx.loss()


def _oracle_kk(wl, w, eta, b, R=None):
    st = wl.states(0)
    if R is None:
        R = rpa.pair_densities_from_workload(wl.cell, wl.basis, wl.lattice_range, wl.k_frac,
                                             st.q_cart, wl.G_int, st.C_k, st.C_kq, wl.n_occ)
    chi = rpa.chi0_kk(R, st.E_k, st.E_kq, wl.n_occ, w, eta, b, _vol(wl))
    Q = rpa.q_plus_g(wl.cell.lat, st.q_cart, wl.G_int)
    return chi, rpa.loss_lfe(rpa.epsilon(chi, Q))


@pytest.mark.parametrize("eta", [0.2, 0.0])
def test_kk_matches_oracle(ctx, small_wl, small_oracle, eta):
    w = small_wl.w_eV[::2]
    chi, L = _gpu_kk(ctx, small_wl, w, eta, 0.05)
    cref, Lref = _oracle_kk(small_wl, w, eta, 0.05, small_oracle["R"])
    ec, el = relmax(chi, cref), normwise(L, Lref)
    print("eta", eta, "chi0", ec, "loss", el)
    assert ec < TOL_CHI and el < TOL_LOSS


def test_kk_multi_tile(ctx, small_wl):
    """137 G: a 3 x 3 grid of 64 x 64 tiles of the (G, G') plane (diagonal and
    off-diagonal tiles, a last tile with 9 real G) against the oracle."""
    import dataclasses

    from synth.generator import g_shells

    wl = dataclasses.replace(small_wl, G_int=g_shells(small_wl.cell.lat, 137))
    w = small_wl.w_eV[::8]
    chi, L = _gpu_kk(ctx, wl, w, 0.2, 0.05)
    cref, Lref = _oracle_kk(wl, w, 0.2, 0.05)
    ec, el = relmax(chi, cref), normwise(L, Lref)
    print("137 G chi0", ec, "loss", el)
    assert ec < TOL_CHI and el < TOL_LOSS


def test_kk_one_wide_bin(ctx, small_wl, small_oracle):
    """bin_eV above every transition energy: one or two intervals per side."""
    w = small_wl.w_eV[::8]
    chi, L = _gpu_kk(ctx, small_wl, w, 0.2, 60.0)
    cref, Lref = _oracle_kk(small_wl, w, 0.2, 60.0, small_oracle["R"])
    assert relmax(chi, cref) < TOL_CHI and normwise(L, Lref) < TOL_LOSS


@pytest.mark.parametrize("bin_eV", [0.004, 5.0])
def test_kk_chunk_boundaries(ctx, small_wl, small_oracle, bin_eV):
    """The binning walks chunks of whole energy intervals (at most 256
    transitions unless one interval holds more) and adds the share of each
    chunk's last interval in the next bin in a pass of its own.  0.004 eV:
    about 6,200 intervals per side of at most 5 transitions, several chunks
    ending on empty intervals (a zero tail); 5 eV: intervals of 328, 518 and
    428 transitions, each a chunk above the 256 budget.  Against the oracle."""
    w = small_wl.w_eV[::8]
    chi, L = _gpu_kk(ctx, small_wl, w, 0.2, bin_eV)
    cref, Lref = _oracle_kk(small_wl, w, 0.2, bin_eV, small_oracle["R"])
    ec, el = relmax(chi, cref), normwise(L, Lref)
    print(bin_eV, "eV bins: chi0", ec, "loss", el)
    assert ec < TOL_CHI and el < TOL_LOSS


def test_kk_tiny_ragged(ctx, tiny):
    w = np.linspace(0.0, 30.0, 37)
    chi, L = _gpu_kk(ctx, tiny, w, 0.3, 0.1)
    cref, Lref = _oracle_kk(tiny, w, 0.3, 0.1)
    ec, el = relmax(chi, cref), normwise(L, Lref)
    print("tiny chi0", ec, "loss", el)
    assert ec < TOL_CHI and el < TOL_LOSS


def test_kk_repeatable(ctx, small_wl):
    """No atomics: two calls give the same bits."""
    w = small_wl.w_eV[::4]
    a, La = _gpu_kk(ctx, small_wl, w, 0.1, 0.03)
    b, Lb = _gpu_kk(ctx, small_wl, w, 0.1, 0.03)
    assert np.array_equal(a, b) and np.array_equal(La, Lb)


def test_kk_converges_to_direct_on_gpu(ctx, small_wl):
    """Halving the bin divides the difference to the direct FP64 route
    (qcx_chi0 at the same eta) by about four."""
    import torch

    w = small_wl.w_eV[::8]
    n = len(small_wl.G_int)
    set_inputs(ctx, small_wl)
    ctx.pair_density(small_wl.G_int)
    ref = torch.empty((len(w), n, n), dtype=torch.complex128, device="cuda")
    ctx.chi0(w, small_wl.eta_eV, "fp64", True, ref)
    ref = ref.cpu().numpy()
    errs = []
    for b in (0.08, 0.04, 0.02):
        chi = torch.empty((len(w), n, n), dtype=torch.complex128, device="cuda")
        ctx.chi0_kk(w, small_wl.eta_eV, b, chi)
        errs.append(relmax(chi.cpu().numpy(), ref))
    print("kk vs direct", errs)
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def test_kk_errors(ctx, small_wl):
    from paper_2603_12326_amd import Context, QcxError
    from paper_2603_12326_amd import qcx as q

    set_inputs(ctx, small_wl)
    ctx.pair_density(small_wl.G_int)
    for eta, b in ((0.2, 0.0), (-0.1, 0.05), (0.2, float("nan")), (0.2, 1e-9)):
        with pytest.raises(QcxError) as e:
            ctx.chi0_kk(small_wl.w_eV, eta, b)
        assert e.value.code == q.EINVAL
    c = Context(0)
    bs = small_wl.basis
    c.set_cell_basis(small_wl.cell.lat, small_wl.cell.xyz, bs.shell_atom, bs.shell_l, bs.shell_exp, 1, 1)
    with pytest.raises(QcxError) as e:
        c.chi0_kk(small_wl.w_eV, 0.2, 0.05)
    assert e.value.code == q.ESTATE
    c.close()


def test_kk_benchmark_size(ctx):
    """The benchmark workload at full size (28 AO, 4 + 16 bands, 8^3 k,
    N_G = 113, first q) through the Kramers-Kronig route with bins of
    0.1 eV (about 600 per side), six frequencies across 0-60 eV, against the
    oracle's binned route: chi0 and the loss at the FP64 bars."""
    from synth import make_si_ng113

    wl = make_si_ng113()
    w = wl.w_eV[[20, 60, 100, 160, 240, 399]]
    print("Kramers-Kronig route, benchmark size", flush=True)
    chi, L = _gpu_kk(ctx, wl, w, wl.eta_eV, 0.1)
    cref, Lref = _oracle_kk(wl, w, wl.eta_eV, 0.1)
    ec, el = relmax(chi, cref), normwise(L, Lref)
    print("benchmark size: chi0", ec, "loss", el)
    assert ec < TOL_CHI and el < TOL_LOSS
