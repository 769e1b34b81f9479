"""The loss surrogate end to end on the GPU: sample the method, train the
ensemble with the library's own kernels, calibrate its error estimate on
held-out samples, and answer a ~1e6-point query grid with fallback to the
method, compared point by point with the method alone.

Workload: the Si-like cell of the mixed batch with smooth bands (the loss
must be a function of Q = q + G), 9^3 k, N_G = 259, eta = 0.1 eV.
Training: N_TRAIN_Q random q x 16 random w x 259 G samples, 10% held out.
Query grid: 40 other random q x 97 w x 259 G = 1,004,920 points.

The expensive part runs once (module fixture); the tests below read its
numbers.  Met, and asserted:
  * training lowers every member's loss by 10x;
  * the networks answer the grid far faster than the method;
  * every (q, w) row the estimate rejects is recomputed and carries the
    method's own values; points the estimate accepts are mostly within the
    tolerance.
The bar of the surrogate (tolerance 2e-2) is asserted but not met yet, so
those tests are marked xfail with the measured values: the networks alone
reach a median relative error of a few per cent on new momenta, not 2e-2,
and at 2e-2 nearly every row falls back, so surrogate plus fallback is
slower than the method alone.
"""
import time

import numpy as np
import pytest

from synth.surrogate import (SURR_SEED, batch_order, holdout_split, make_surrogate_workload, mlp_init, q_max,
                             random_q, random_w)

pytestmark = pytest.mark.gpu

N_TRAIN_Q = 768
EPOCHS = 20
BATCH = 4096
TOLS = (2e-2, 1e-1, 3e-1)


@pytest.fixture(scope="module")
def run():
    import torch

    from paper_2603_12326_amd import Context
    from paper_2603_12326_amd import surrogate as S

    base = make_surrogate_workload([])
    tq = random_q(SURR_SEED + 10, base.cell.lat, N_TRAIN_Q)
    qq = random_q(SURR_SEED + 20, base.cell.lat, 40)
    wl = make_surrogate_workload(list(tq) + list(qq))
    tw = random_w(SURR_SEED + 11, len(tq), 16)
    wq = [np.linspace(0.0, 60.0, 97)] * len(qq)
    ctx = Context(0)
    b = wl.basis
    ctx.set_cell_basis(wl.cell.lat, wl.cell.xyz, b.shell_atom, b.shell_l, b.shell_exp, 1, 1)
    qstates = [wl.states(len(tq) + i) for i in range(len(qq))]    # host generator, untimed

    def set_train(iq):
        st = wl.states(iq)
        ctx.set_states(st.q_cart, wl.k_frac, wl.n_occ, st.C_k, st.E_k, st.C_kq, st.E_kq)

    def set_query(iq):
        st = qstates[iq]
        ctx.set_states(st.q_cart, wl.k_frac, wl.n_occ, st.C_k, st.E_k, st.C_kq, st.E_kq)

    print(f"surrogate: sampling {N_TRAIN_Q} training momenta", flush=True)
    smp = S.sample(ctx, set_train, tq, wl.G_int, wl.cell.lat, tw, wl.eta_eV)
    n = smp.qw.shape[0]
    assert n == N_TRAIN_Q * 16 * 259
    tr, ho = holdout_split(SURR_SEED + 12, n)
    sur = S.Surrogate(ctx, 4)
    hists = sur.fit(smp, tr, q_max(wl), 60.0, wl.cell.lat, lambda k: mlp_init(SURR_SEED + 100 + k),
                    lambda k, nn, bs: batch_order(SURR_SEED + 200 + k, nn, bs, EPOCHS),
                    batch=BATCH, epochs=EPOCHS, lr0=3e-3, lr1=1e-5)
    cal = sur.calibrate(smp, ho)
    print(f"trained 4 members in {sur.train_seconds:.1f} s; held-out relative error "
          f"q50 {np.quantile(cal['rel_err'], .5):.3g} q90 {np.quantile(cal['rel_err'], .9):.3g}; "
          f"calibration factor {cal['calib']:.3g}", flush=True)

    # the method alone on the query grid
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = [S.method_loss(ctx, set_query, i, wl.G_int, wq[i], wl.eta_eV) for i in range(len(qq))]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    refh = np.stack([r.cpu().numpy() for r in ref])

    # the networks alone
    Gc = S.g_cart(wl.G_int, wl.cell.lat)
    grid = torch.cat([torch.from_numpy(S.query_points(q, Gc, w)).cuda() for q, w in zip(qq, wq)])
    sur.query(grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ls, Es, _, _ = sur.query(grid)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    net = Ls.cpu().numpy().reshape(refh.shape)
    rel_net = np.abs(net / refh - 1)
    est = Es.cpu().numpy().reshape(refh.shape)
    print(f"{grid.shape[0]} queries: method {t_plain:.3f} s, networks {1e3 * t_net:.2f} ms "
          f"({t_plain / t_net:.0f}x); networks alone: median {np.median(rel_net):.3g}, "
          f"within 2e-2 {np.mean(rel_net <= 2e-2):.3f}", flush=True)

    fb = {}
    for tol in TOLS:
        out, st = S.query_with_fallback(sur, ctx, set_query, len(qq), wl.G_int, wq, wl.eta_eV, tol)
        got = np.stack([o.cpu().numpy() for o in out])
        E = st.pop("err").cpu().numpy().reshape(refh.shape)
        acc = E <= tol
        fb[tol] = dict(got=got, E=E, st=st, gain=t_plain / st["t_total"],
                       accepted=float(acc.mean()),
                       accepted_within=float(np.mean(rel_net[acc] <= tol)) if acc.any() else 1.0)
        print(f"tol {tol}: accepted points {fb[tol]['accepted']:.4f} "
              f"(of them within tol {fb[tol]['accepted_within']:.4f}), "
              f"fallback rows {st['fallback_points']}/{refh.shape[0] * refh.shape[1]}, "
              f"time {st['t_total']:.3f} s, gain {fb[tol]['gain']:.2f}x", flush=True)
    yield dict(hists=hists, cal=cal, refh=refh, net=net, rel_net=rel_net, est=est, t_plain=t_plain,
               t_net=t_net, fb=fb)
    sur.close()
    ctx.close()


def test_training_and_speed(run):
    for h in run["hists"]:
        assert np.mean(h[-50:]) < 0.1 * np.mean(h[:5])
    assert run["t_net"] < run["t_plain"] / 20


@pytest.mark.parametrize("tol", TOLS)
def test_fallback_rows_carry_the_method(run, tol):
    f = run["fb"][tol]
    rejected_rows = (f["E"] > tol).any(axis=2)               # [q][w] rows recomputed
    # the same method on a subset of the frequencies: other K splits, so
    # agreement to FP32 accumulation order
    assert np.allclose(f["got"][rejected_rows], run["refh"][rejected_rows], rtol=1e-5, atol=0)
    kept = ~rejected_rows                                    # the networks' own answers
    assert np.array_equal(f["got"][kept], run["net"][kept])


def test_accepted_points_within_tolerance(run):
    """The calibrated estimate at tolerance 0.3: of the points it accepts,
    at least 90% are within the tolerance (the factor is set at the 95th
    percentile on held-out samples of the training momenta; the query
    momenta are new, so it holds less tightly there)."""
    f = run["fb"][3e-1]
    assert f["accepted"] > 0.05
    assert f["accepted_within"] >= 0.9


@pytest.mark.xfail(reason="not met: the networks reach a held-out median relative error of "
                          "about 4e-2 and about 5e-2 on new momenta, not 2e-2", strict=False)
def test_network_alone_meets_2e2(run):
    assert np.median(run["cal"]["rel_err"]) <= 2e-2
    assert np.median(run["rel_net"]) <= 2e-2


@pytest.mark.xfail(reason="not met: at tolerance 2e-2 nearly every (q, w) row falls back, so "
                          "surrogate plus fallback is slower than the method alone", strict=False)
def test_gain_at_2e2(run):
    f = run["fb"][2e-2]
    assert f["accepted_within"] >= 0.95
    assert f["gain"] > 1.0
