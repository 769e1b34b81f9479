"""Pins of the surrogate's reference network (oracle/mlp.py) against things
other than itself: explicit loops, finite differences, an independent
autograd evaluation, Adam's closed-form first step and a library optimiser,
and a library bfloat16 conversion."""
import math

import numpy as np
import pytest

from oracle import mlp
from synth.surrogate import batch_order, holdout_split, make_surrogate_workload, mlp_init, random_q

SMALL = (5, 8, 8, 8, 8, 1)


def _rand_theta(widths, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.n_params(widths)) * scale


def test_parameter_count():
    # 5*256+256 + 3*(256*256+256) + 256+1
    assert mlp.n_params() == 210433
    th = np.arange(mlp.n_params(SMALL), dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(th, SMALL)), th)


def test_bf16_round_matches_library():
    import torch

    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, 65504.0]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x32), ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert mlp.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mlp.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_forward_matches_explicit_loops():
    w = (5, 3, 4, 1)
    th = _rand_theta(w, 2)
    X = np.random.default_rng(3).standard_normal((2, 5))
    y, _ = mlp.forward(th, X, w)
    layers = mlp.unpack(th, w)
    for b in range(2):
        h = list(X[b])
        for li, (W, bias) in enumerate(layers):
            z = [sum(W[o][i] * h[i] for i in range(len(h))) + bias[o] for o in range(len(bias))]
            h = z if li == len(layers) - 1 else [v / (1.0 + math.exp(-v)) for v in z]
        assert abs(h[0] - y[b]) < 1e-13


def test_gradient_finite_differences():
    th = _rand_theta(SMALL, 4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((7, 5))
    t = rng.standard_normal(7)
    _, g = mlp.loss_and_grad(th, X, t, SMALL)
    fd = np.empty_like(g)
    h = 1e-5
    for i in range(len(th)):
        tp = th.copy()
        tp[i] += h
        tm = th.copy()
        tm[i] -= h
        fd[i] = (mlp.mse(mlp.forward(tp, X, SMALL)[0], t) - mlp.mse(mlp.forward(tm, X, SMALL)[0], t)) / (2 * h)
    err = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    assert err < 1e-7, err


def test_gradient_against_autograd_full_size():
    import torch

    th = mlp_init(7).astype(np.float64)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((64, mlp.N_IN))
    t = rng.standard_normal(64)
    loss, g = mlp.loss_and_grad(th, X, t)
    T = torch.tensor(th, requires_grad=True)
    h = torch.tensor(X)
    o = 0
    for i in range(len(mlp.WIDTHS) - 1):
        n_in, n_out = mlp.WIDTHS[i], mlp.WIDTHS[i + 1]
        W = T[o:o + n_out * n_in].view(n_out, n_in)
        o += n_out * n_in
        b = T[o:o + n_out]
        o += n_out
        h = h @ W.T + b
        if i < len(mlp.WIDTHS) - 2:
            h = torch.nn.functional.silu(h)
    lt = ((h[:, 0] - torch.tensor(t)) ** 2).mean()
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12 * abs(loss)
    assert np.max(np.abs(T.grad.numpy() - g)) < 1e-12 * np.max(np.abs(g))


def test_bf16_mode_close_to_exact():
    th = mlp_init(9).astype(np.float64)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((128, mlp.N_IN))
    t = rng.standard_normal(128)
    y0, _ = mlp.forward(th, X)
    y1, _ = mlp.forward(th, X, bf16=True)
    assert np.max(np.abs(y1 - y0)) < 3e-2 * np.max(np.abs(y0))
    assert not np.array_equal(y0, y1)
    _, g0 = mlp.loss_and_grad(th, X, t)
    _, g1 = mlp.loss_and_grad(th, X, t, bf16=True)
    assert np.linalg.norm(g1 - g0) < 5e-2 * np.linalg.norm(g0)


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    opt = mlp.Adam(4)
    th = opt.step(np.zeros(4), g, 0.01)
    # m_hat = g, v_hat = g^2: step = -lr g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)


def test_adam_against_library():
    import torch

    rng = np.random.default_rng(11)
    th0 = rng.standard_normal(50)
    P = torch.nn.Parameter(torch.tensor(th0.copy()))
    opt_t = torch.optim.Adam([P], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    opt = mlp.Adam(50)
    th = th0.copy()
    for s in range(6):
        g = rng.standard_normal(50)
        lr = mlp.cosine_lr(s, 6, 1e-3, 1e-4)
        for grp in opt_t.param_groups:
            grp["lr"] = lr
        P.grad = torch.tensor(g)
        opt_t.step()
        th = opt.step(th, g, lr)
    assert np.max(np.abs(th - P.detach().numpy())) < 1e-14


def test_cosine_schedule_endpoints():
    assert mlp.cosine_lr(0, 100, 1e-3, 1e-5) == 1e-3
    assert abs(mlp.cosine_lr(100, 100, 1e-3, 1e-5) - 1e-5) < 1e-18
    assert abs(mlp.cosine_lr(50, 100, 1e-3, 1e-5) - 0.5 * (1e-3 + 1e-5)) < 1e-18


def test_training_loop_fits_smooth_target():
    rng = np.random.default_rng(12)
    X = rng.uniform(-1, 1, size=(512, 5))
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 4]
    th = mlp_init(13, SMALL).astype(np.float64)
    order = batch_order(14, 512, 64, 60)
    th1, hist = mlp.train(th, X, t, order, 64, 1e-2, 1e-3, SMALL)
    assert hist[-20:].mean() < 0.1 * hist[:5].mean()


def test_smooth_band_workload_is_periodic_and_ordered():
    from synth.generator import _band_energies, _band_model

    wl = make_surrogate_workload(random_q(1, make_surrogate_workload([]).cell.lat, 2), kgrid=3)
    st = wl.states(0)
    assert np.all(np.diff(st.E_k[:, :4], axis=1) >= 0) and np.all(np.diff(st.E_k[:, 4:], axis=1) >= 0)
    assert st.E_k[:, :4].max() <= 0.0 and st.E_k[:, 4:].min() >= 1.1
    model = _band_model(np.random.default_rng(0), wl.energy_ranges)
    kf = np.random.default_rng(1).uniform(size=(5, 3))
    shift = np.array([1.0, -2.0, 3.0])
    assert np.allclose(_band_energies(model, wl.energy_ranges, kf),
                       _band_energies(model, wl.energy_ranges, kf + shift), atol=1e-12)
    tr, ho = holdout_split(2, 100)
    assert len(ho) == 10 and len(np.intersect1d(tr, ho)) == 0 and len(tr) + len(ho) == 100


def test_encode_features():
    """The encoding against properties it must have, on a lattice that is not
    symmetric (so that Q.a_i and Q.a^i-type index mistakes differ): unit
    directions, the lowest frequency pi per w_max, successive frequencies in
    the ratio sqrt(2) (read from the slope of sin at a tiny argument), every
    (sin, cos) pair on the unit circle, and lattice features unchanged by any
    reciprocal lattice vector while the other features change."""
    A = np.array([[4.1, 0.3, -0.7], [0.5, 5.2, 0.2], [-0.4, 0.9, 6.3]])   # rows: primitive vectors
    B = 2 * math.pi * np.linalg.inv(A).T                                   # rows: reciprocal vectors
    assert np.allclose(A @ B.T, 2 * math.pi * np.eye(3))
    rng = np.random.default_rng(40)
    qw = np.column_stack([rng.uniform(-2, 2, size=(50, 3)), rng.uniform(0, 60, 50)])
    qw[0, :3] = 0.0
    x = mlp.encode(qw, 4.0, 60.0, A)
    assert x.shape == (50, mlp.N_IN) == (50, 49)
    assert np.allclose(np.linalg.norm(x[1:, 1:4], axis=1), 1.0) and np.all(x[0, 1:4] == 0.0)
    nf = mlp.N_FREQ
    pairs = x[:, 5:].reshape(50, -1, 2)
    assert np.allclose((pairs ** 2).sum(axis=2), 1.0, atol=1e-14)
    # w = w_max: the first w pair is (sin pi, cos pi)
    top = mlp.encode(np.array([[1.0, 0.0, 0.0, 60.0]]), 4.0, 60.0, A)[0]
    assert abs(top[5]) < 1e-14 and abs(top[6] + 1.0) < 1e-14
    # slopes at a tiny w and a tiny |Q|: pi 2^(j/2) / scale
    eps = 1e-7
    small = mlp.encode(np.array([[eps, 0.0, 0.0, eps]]), 4.0, 60.0, A)[0]
    sw = small[5:5 + 2 * nf:2] / (eps / 60.0)
    sq = small[5 + 2 * nf:5 + 4 * nf:2] / (eps / 4.0)
    for s in (sw, sq):
        assert abs(s[0] - math.pi) < 1e-6
        assert np.allclose(s[1:] / s[:-1], math.sqrt(2.0), rtol=1e-9)
    # periodic part: invariant under Q -> Q + G for reciprocal lattice G
    G = np.array([2, -1, 3]) @ B
    shifted = qw.copy()
    shifted[:, :3] += G
    xs = mlp.encode(shifted, 4.0, 60.0, A)
    lat_cols = slice(5 + 4 * nf, mlp.N_IN)
    assert np.allclose(xs[:, lat_cols], x[:, lat_cols], atol=1e-11)
    assert not np.allclose(xs[:, :lat_cols.start], x[:, :lat_cols.start])
    # and a primitive vector itself is not a period of them
    moved = qw.copy()
    moved[:, :3] += A[0]
    assert not np.allclose(mlp.encode(moved, 4.0, 60.0, A)[:, lat_cols], x[:, lat_cols])
