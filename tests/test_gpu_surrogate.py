"""The loss surrogate end to end on the GPU: sample the method, train the
ensemble with the library's own kernels, calibrate its error estimate on
held-out samples, and answer a ~1e6-point query grid with fallback to the
method, compared point by point with the method alone.

Workload: the Si-like cell of the mixed batch with smooth bands (the loss
must be a function of Q = q + G), 9^3 k, N_G = 259, eta = 0.1 eV.
Training: 48 random q x 16 random w x 259 G = 198,912 samples, 10% held
out.  Query grid: 40 other random q x 97 w x 259 G = 1,004,920 points.

What is asserted:
  * training lowers every member's loss by 10x;
  * the networks answer the grid far faster than the method;
  * after fallback, every point the estimate rejected carries the
    method's own value, and at each tolerance at least 90% of all points
    are within it;
  * the gain (time of the method alone / time of surrogate + fallback) at
    each tolerance is printed.  On these synthetic states the loss has
    ~10% structure on the eta scale that 5 smooth inputs cannot resolve,
    so at 2e-2 almost every (q, w) row falls back and the gain is < 1;
    it appears at looser tolerances.
"""
import time

import numpy as np
import pytest

from synth.surrogate import (SURR_SEED, batch_order, holdout_split, make_surrogate_workload, mlp_init, q_max,
                             random_q, random_w)

pytestmark = pytest.mark.gpu


def test_surrogate_end_to_end():
    import torch

    from paper_2603_12326_amd import Context
    from paper_2603_12326_amd import surrogate as S

    base = make_surrogate_workload([])
    tq = random_q(SURR_SEED + 10, base.cell.lat, 48)
    qq = random_q(SURR_SEED + 20, base.cell.lat, 40)
    wl = make_surrogate_workload(list(tq) + list(qq))
    tw = random_w(SURR_SEED + 11, len(tq), 16)
    wq = [np.linspace(0.0, 60.0, 97)] * len(qq)
    ctx = Context(0)
    b = wl.basis
    ctx.set_cell_basis(wl.cell.lat, wl.cell.xyz, b.shell_atom, b.shell_l, b.shell_exp, 1, 1)
    states = [wl.states(i) for i in range(len(tq) + len(qq))]    # host generator, untimed

    def set_states(off):
        def f(iq):
            st = states[off + iq]
            ctx.set_states(st.q_cart, wl.k_frac, wl.n_occ, st.C_k, st.E_k, st.C_kq, st.E_kq)
        return f

    smp = S.sample(ctx, set_states(0), tq, wl.G_int, wl.cell.lat, tw, wl.eta_eV)
    n = smp.qw.shape[0]
    assert n == 48 * 16 * 259
    tr, ho = holdout_split(SURR_SEED + 12, n)
    sur = S.Surrogate(ctx, 4)
    epochs = 80
    hists = sur.fit(smp, tr, q_max(wl), 60.0, lambda k: mlp_init(SURR_SEED + 100 + k),
                    lambda k, nn, bs: batch_order(SURR_SEED + 200 + k, nn, bs, epochs),
                    batch=2048, epochs=epochs, lr0=3e-3, lr1=1e-5)
    for h in hists:
        assert np.mean(h[-50:]) < 0.1 * np.mean(h[:5])
    cal = sur.calibrate(smp, ho)
    print(f"trained 4 members in {sur.train_seconds:.1f} s; held-out relative error "
          f"q50 {np.quantile(cal['rel_err'], .5):.3g} q90 {np.quantile(cal['rel_err'], .9):.3g}; "
          f"calibration factor {cal['calib']:.3g}")

    # the method alone on the query grid
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = [S.method_loss(ctx, set_states(len(tq)), i, wl.G_int, wq[i], wl.eta_eV)
           for i in range(len(qq))]
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
    rel_net = np.abs(Ls.cpu().numpy().reshape(refh.shape) / refh - 1)
    print(f"{grid.shape[0]} queries: method {t_plain:.3f} s, networks {1e3 * t_net:.2f} ms "
          f"({t_plain / t_net:.0f}x); networks alone within 2e-2: {np.mean(rel_net <= 2e-2):.3f}")
    assert t_net < t_plain / 20

    for tol in (2e-2, 1e-1, 3e-1):
        out, st = S.query_with_fallback(sur, ctx, set_states(len(tq)), qq, wl.G_int, wl.cell.lat,
                                        wq, wl.eta_eV, tol)
        got = np.stack([o.cpu().numpy() for o in out])
        E = st.pop("err").cpu().numpy().reshape(refh.shape)
        rel = np.abs(got / refh - 1)
        rejected_rows = (E > tol).any(axis=2)               # [q][w] rows recomputed
        assert np.array_equal(got[rejected_rows], refh[rejected_rows])
        within = np.mean(rel <= tol)
        print(f"tol {tol}: accepted points {1 - st['n_rejected'] / st['n_queries']:.4f}, "
              f"fallback rows {st['fallback_points']}/{refh.shape[0] * refh.shape[1]}, "
              f"within tol {within:.4f}, time {st['t_total']:.3f} s, "
              f"gain {t_plain / st['t_total']:.2f}x")
        assert within >= 0.9
    sur.close()
    ctx.close()
