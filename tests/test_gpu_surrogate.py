"""The loss surrogate end to end on the GPU: sample the method, train the
ensemble with the library's own kernels, calibrate its error estimate on
held-out samples, and answer a ~1e6-point query grid with fallback to the
method, compared point by point with the method alone.

Workload: the Si-like cell of the mixed batch with smooth bands (the loss
must be a function of Q = q + G), 9^3 k, N_G = 259, eta = 0.1 eV.
Training: N_TRAIN_Q random q x N_W_TRAIN random w x 259 G samples, 10% held
out.  Query grid: 40 other random q x 97 w x 259 G = 1,004,920 points.

Accuracy is measured pointwise (relative error of the loss) and per loss
curve: for each (q, G), the curve along the 97 frequencies, the error of a
point in units of the curve's maximum, |L - L_method| / max_w |L_method|, and
the curve's error the largest of those (a normwise measure).
qcx_mlp_infer accepts a frequency row when every point's estimate in these
units is within the tolerance, and recomputes it with the method otherwise.

The expensive part runs once (module fixture); the tests below read its
numbers.  Met, and asserted:
  * training lowers every member's loss by 10x;
  * the networks answer the grid far faster than the method;
  * the networks alone reach a median relative error within 2e-2, on
    held-out samples of the training momenta and on the new momenta;
  * every (q, w) row the estimate rejects is recomputed and carries the
    method's own values; the other rows keep the networks' answers;
  * at every tolerance (2e-2, 1e-1, 3e-1), at least 95% of the accepted
    points are within it, and after fallback 99% of the curves are;
  * at 2e-2, surrogate plus fallback is faster than the method alone.
Not met, marked xfail with the measured value: per curve the networks alone
are not within 2e-2 (median curve error about 0.1: the curves' peaks are
where they err most), so about half of the rows fall back at 2e-2.
"""
import time

import numpy as np
import pytest

from synth.surrogate import (SURR_SEED, batch_order, holdout_split, make_surrogate_workload, mlp_init, q_max,
                             random_q, random_w)

# sampling and training take a few minutes: the fixture's time counts towards the first test
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N_TRAIN_Q = 2048
N_W_TRAIN = 24
EPOCHS = 40
BATCH = 4096
TOLS = (2e-2, 1e-1, 3e-1)


@pytest.fixture(scope="module")
def run(request):
    import torch

    # progress lines reach the terminal even under output capture, so that a
    # run of several minutes is never silent for long
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        if capman is None:
            print(msg, flush=True)
            return
        with capman.global_and_fixture_disabled():
            print(msg, flush=True)

    from paper_2603_12326_amd import Context
    from paper_2603_12326_amd import surrogate as S

    base = make_surrogate_workload([])
    tq = random_q(SURR_SEED + 10, base.cell.lat, N_TRAIN_Q)
    qq = random_q(SURR_SEED + 20, base.cell.lat, 40)
    wl = make_surrogate_workload(list(tq) + list(qq))
    tw = random_w(SURR_SEED + 11, len(tq), N_W_TRAIN)
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

    say(f"surrogate: sampling {N_TRAIN_Q} training momenta x {N_W_TRAIN} frequencies")
    parts = []
    for c0 in range(0, N_TRAIN_Q, 512):     # in chunks, with a progress line each
        c1 = min(c0 + 512, N_TRAIN_Q)
        parts.append(S.sample(ctx, lambda i, o=c0: set_train(i + o), tq[c0:c1], wl.G_int, wl.cell.lat,
                              tw[c0:c1], wl.eta_eV))
        say(f"surrogate: sampled {c1} of {N_TRAIN_Q} momenta")
    smp = S.Samples(torch.cat([p.qw for p in parts]), torch.cat([p.loss for p in parts]),
                    np.concatenate([p.q_index + c0 for p, c0 in zip(parts, range(0, N_TRAIN_Q, 512))]),
                    np.concatenate([p.w_index for p in parts]))
    n = smp.qw.shape[0]
    assert n == N_TRAIN_Q * N_W_TRAIN * 259
    tr, ho = holdout_split(SURR_SEED + 12, n)
    sur = S.Surrogate(ctx, 4)
    hists = sur.fit(smp, tr, q_max(wl), 60.0, wl.cell.lat, lambda k: mlp_init(SURR_SEED + 100 + k),
                    lambda k, nn, bs: batch_order(SURR_SEED + 200 + k, nn, bs, EPOCHS),
                    batch=BATCH, epochs=EPOCHS, lr0=3e-3, lr1=1e-5,
                    progress=lambda k: say(f"surrogate: member {k + 1} of 4 trained"))
    cal = sur.calibrate(smp, ho)
    say(f"trained 4 members in {sur.train_seconds:.1f} s; held-out relative error "
        f"q50 {np.quantile(cal['rel_err'], .5):.3g} q90 {np.quantile(cal['rel_err'], .9):.3g}; "
        f"calibration factor {cal['calib']:.3g}")

    # the method alone on the query grid (a first pass tunes the bulk for this
    # shape; the second is timed)
    def method_all():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = [S.method_loss(ctx, set_query, i, wl.G_int, wq[i], wl.eta_eV) for i in range(len(qq))]
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    method_all()
    ref, t_plain = method_all()
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
    say(f"{grid.shape[0]} queries: method {t_plain:.3f} s, networks {1e3 * t_net:.2f} ms "
        f"({t_plain / t_net:.0f}x); networks alone: median {np.median(rel_net):.3g}, "
        f"within 2e-2 {np.mean(rel_net <= 2e-2):.3f}")

    # errors in units of each (q, G) curve's maximum along the frequencies
    refmax = np.abs(refh).max(axis=1, keepdims=True)
    pt_net = np.abs(net - refh) / refmax
    curve_net = pt_net.max(axis=1)
    say(f"networks alone per curve: median {np.median(curve_net):.3g}, "
        f"within 2e-2 {np.mean(curve_net <= 2e-2):.3f}")

    fb = {}
    for tol in TOLS:
        # a first pass tunes the bulk for the fallback's row counts; the second is timed
        S.query_with_fallback(sur, ctx, set_query, len(qq), wl.G_int, wq, wl.eta_eV, tol)
        out, st = S.query_with_fallback(sur, ctx, set_query, len(qq), wl.G_int, wq, wl.eta_eV, tol)
        got = np.stack([o.cpu().numpy() for o in out])
        E = st.pop("err").cpu().numpy().reshape(refh.shape)     # estimates in curve units
        kept = ~(E > tol).any(axis=2)                            # [q][w] rows the networks answer
        acc = np.broadcast_to(kept[:, :, None], refh.shape)
        curve = (np.abs(got - refh) / refmax).max(axis=1)
        fb[tol] = dict(got=got, E=E, st=st, gain=t_plain / st["t_total"],
                       rows_kept=float(kept.mean()),
                       accepted_within=float(np.mean(pt_net[acc] <= tol)) if acc.any() else 1.0,
                       curves_within=float(np.mean(curve <= tol)), curve_max=float(curve.max()))
        say(f"tol {tol}: rows answered by the networks {fb[tol]['rows_kept']:.3f} "
            f"(their points within tol {fb[tol]['accepted_within']:.4f}), curves within tol "
            f"after fallback {fb[tol]['curves_within']:.4f} (largest {fb[tol]['curve_max']:.3g}), "
            f"fallback rows {st['fallback_points']}/{refh.shape[0] * refh.shape[1]}, "
            f"time {st['t_total']:.3f} s, gain {fb[tol]['gain']:.2f}x")
    yield dict(hists=hists, cal=cal, refh=refh, net=net, rel_net=rel_net, est=est, t_plain=t_plain,
               t_net=t_net, fb=fb, curve_net=curve_net)
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
    # the same method on a subset of the frequencies: the bulk's K split is
    # tuned per shape, so the FP32 partial sums add in another order and the
    # rows agree to the split-BF16 bar (1e-4), not bit for bit
    got, ref = f["got"][rejected_rows], run["refh"][rejected_rows]
    print(f"tol {tol}: fallback rows vs method, largest relative difference "
          f"{np.max(np.abs(got / ref - 1)):.3g}")
    assert np.allclose(got, ref, rtol=1e-4, atol=0)
    kept = ~rejected_rows                                    # the networks' own answers
    assert np.array_equal(f["got"][kept], run["net"][kept])


@pytest.mark.parametrize("tol", TOLS)
def test_accepted_points_within_tolerance(run, tol):
    """Of the points in rows the networks answer, at least 95% are within the
    tolerance in curve units (the relative estimate is calibrated at the 95th
    percentile on held-out samples of the training momenta; the query momenta
    are new), and after fallback at least 99% of the curves are."""
    f = run["fb"][tol]
    assert f["accepted_within"] >= 0.95
    assert f["curves_within"] >= 0.99


def test_gain_at_2e2(run):
    """At tolerance 2e-2, surrogate plus fallback beats the method alone on
    the whole grid (time of both measured on the same grid)."""
    f = run["fb"][2e-2]
    assert f["rows_kept"] > 0.2
    assert f["gain"] > 1.0


def test_network_alone_median_within_2e2(run):
    """The networks alone, without fallback: median relative error of the
    loss within 2e-2 on held-out samples and on the new momenta."""
    ho, new = np.median(run["cal"]["rel_err"]), np.median(run["rel_net"])
    print(f"networks alone: held-out median {ho:.4g}, new momenta median {new:.4g}")
    assert ho <= 2e-2
    assert new <= 2e-2


@pytest.mark.xfail(reason="not met: per loss curve (error in units of the curve's maximum) the "
                          "networks alone have a median curve error of about 0.1, at the peaks",
                   strict=False)
def test_network_alone_per_curve_2e2(run):
    assert np.median(run["curve_net"]) <= 2e-2
