"""Surrogate network kernels against the FP64 reference network, through the
C ABI.

The GPU computes with bf16 weights and activations in its products and FP32
sums; the reference applies the same bf16 roundings to FP64 values
(oracle.mlp, bf16 mode).  What remains is FP32 accumulation order (~1e-6)
and the occasional activation whose FP32 and FP64 values (they differ by
~1e-6 relative through exp) fall on either side of a bf16 rounding
boundary: each such flip moves that activation by 2^-8 relative.  With
the 49 features of the encoding summed in FP32 by the first layer, a batch
of 1000 rows holds a few such flips, which move outputs and gradient
blocks by up to ~1.3e-3 relative (measured; ~4e-4 with 5 inputs), hence
the bars of 2e-3.
"""
import numpy as np
import pytest

from oracle import mlp as ref
from synth.surrogate import batch_order, mlp_init

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    import torch

    from paper_2603_12326_amd import Context, Mlp

    assert torch.cuda.is_available()
    c = Context(0)
    m = Mlp(c, 2)
    yield c, m
    m.close()
    c.close()


def _dev(a, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _blocks(theta):
    """(name, slice) of every parameter block of the flat vector."""
    out, o = [], 0
    for i in range(len(ref.WIDTHS) - 1):
        n_in, n_out = ref.WIDTHS[i], ref.WIDTHS[i + 1]
        out.append((f"W{i + 1}", slice(o, o + n_in * n_out)))
        o += n_in * n_out
        out.append((f"b{i + 1}", slice(o, o + n_out)))
        o += n_out
    return out


@pytest.mark.parametrize("n", [1, 63, 1000])
def test_forward_matches_reference(net, n):
    import torch

    c, m = net
    th = mlp_init(21)
    m.set_params(0, th)
    x = np.random.default_rng(22).uniform(-1, 1, size=(n, ref.N_IN)).astype(np.float32)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(0, _dev(x, torch.float32), y)
    got = y.cpu().numpy().astype(np.float64)
    want, _ = ref.forward(th.astype(np.float64), x.astype(np.float64), bf16=True)
    exact, _ = ref.forward(th.astype(np.float64), x.astype(np.float64))
    scale = np.max(np.abs(want))
    e = np.max(np.abs(got - want)) / scale
    print("n", n, "forward vs bf16 reference", e, "vs exact", np.max(np.abs(got - exact)) / scale)
    assert e < 2e-3
    assert np.max(np.abs(got - exact)) < 3e-2 * scale


@pytest.mark.parametrize("n", [64, 300])
def test_gradient_matches_reference(net, n):
    c, m = net
    import torch

    th = mlp_init(23)
    m.set_params(1, th)
    rng = np.random.default_rng(24)
    x = rng.uniform(-1, 1, size=(n, ref.N_IN)).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    g, loss = m.grad(1, _dev(x, torch.float32), _dev(t, torch.float32))
    lref, gref = ref.loss_and_grad(th.astype(np.float64), x.astype(np.float64),
                                   t.astype(np.float64), bf16=True)
    assert abs(loss - lref) < 1e-4 * lref
    for name, sl in _blocks(th):
        e = np.linalg.norm(g[sl] - gref[sl]) / max(np.linalg.norm(gref[sl]), 1e-30)
        print(name, "grad rel err", e)
        assert e < 2e-3, name


def test_training_steps_match_reference(net):
    import torch

    c, m = net
    th = mlp_init(25)
    m.set_params(0, th)
    rng = np.random.default_rng(26)
    n, batch = 512, 128
    x = rng.uniform(-1, 1, size=(n, ref.N_IN)).astype(np.float32)
    t = (np.sin(3 * x[:, 0]) * x[:, 4]).astype(np.float32)
    order = batch_order(27, n, batch, 2)             # 8 steps
    hist = m.train(0, _dev(x, torch.float32), _dev(t, torch.float32), batch,
                   _dev(order, torch.int32), 1e-3, 1e-4)
    th1 = m.get_params(0).astype(np.float64)
    th1_ref, hist_ref = ref.train(th.astype(np.float64), x.astype(np.float64),
                                  t.astype(np.float64), order, batch, 1e-3, 1e-4, bf16=True)
    print("loss hist", hist, hist_ref)
    assert np.max(np.abs(hist - hist_ref) / hist_ref) < 1e-3
    d, dref = th1 - th, th1_ref - th
    e = np.linalg.norm(d - dref) / np.linalg.norm(dref)
    print("update rel err", e)
    assert e < 1e-2


def test_query_encode_decode_select(net):
    import torch

    c, m = net
    m.set_params(0, mlp_init(31))
    m.set_params(1, mlp_init(32))
    q_max, w_max, mu, sigma, calib = 4.0, 60.0, -3.0, 2.0, 1.5
    lat = np.array([[0.0, 5.13, 5.13], [5.13, 0.0, 5.13], [5.13, 5.13, 0.0]])
    m.set_encoding(q_max, w_max, lat, mu, sigma, calib)
    rng = np.random.default_rng(33)
    n = 70001
    qw = np.column_stack([rng.uniform(-2, 2, size=(n, 3)), rng.uniform(0, 60, n)])
    qw[5, :3] = 0.0                                  # Q = 0
    qd = _dev(qw, torch.float64)
    x = torch.empty((n, ref.N_IN), dtype=torch.float32, device="cuda")
    m.encode(qd, x=x)
    xe = ref.encode(qw, q_max, w_max, lat)
    assert np.max(np.abs(x.cpu().numpy() - xe)) < 1e-6
    ys = torch.empty((2, n), dtype=torch.float32, device="cuda")
    m.forward(0, x, ys[0])
    m.forward(1, x, ys[1])
    loss = torch.empty(n, dtype=torch.float64, device="cuda")
    err = torch.empty(n, dtype=torch.float64, device="cuda")
    idx = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    tol = float(np.median(ref.decode(ys.cpu().numpy(), mu, sigma, calib)[1]))
    nrej = m.query(qd, loss, err, tol, idx)
    lw, ew = ref.decode(ys.cpu().numpy(), mu, sigma, calib)
    assert np.max(np.abs(loss.cpu().numpy() / lw - 1)) < 1e-12
    assert np.max(np.abs(err.cpu().numpy() - ew)) < 1e-12 * max(ew.max(), 1e-300)
    want = np.nonzero(err.cpu().numpy() > tol)[0]
    assert nrej == len(want) and 0 < nrej < n
    assert np.array_equal(idx.cpu().numpy()[:nrej], want)


def test_errors(net):
    import torch

    from paper_2603_12326_amd import QcxError
    from paper_2603_12326_amd import qcx as q

    c, m = net
    x = torch.zeros((10, ref.N_IN), dtype=torch.float32, device="cuda")
    t = torch.zeros(10, dtype=torch.float32, device="cuda")
    bad = torch.tensor([0, 1, 2, 10], dtype=torch.int32, device="cuda")
    with pytest.raises(QcxError) as e:
        m.train(0, x, t, 2, bad, 1e-3, 1e-4)
    assert e.value.code == q.EINVAL
    with pytest.raises(QcxError) as e:
        m.set_params(5, np.zeros(q.MLP_NPARAM, np.float32))
    assert e.value.code == q.EINVAL


def test_infer_with_fallback(net):
    """qcx_mlp_infer on the smallest workload: with an infinite tolerance the
    networks' answers (the grid q + G built on the host here) and their
    estimates in units of each G's curve maximum, with tolerance 0 the method
    itself bit for bit, and in between each rejected frequency row equals the
    method run on exactly those frequencies while the other rows keep the
    networks' answers."""
    import torch

    from synth import make_smallest

    c, m = net
    wl = make_smallest()
    st = wl.states(0)
    b = wl.basis
    c.set_cell_basis(wl.cell.lat, wl.cell.xyz, b.shell_atom, b.shell_l, b.shell_exp, 1, 1)
    c.set_states(st.q_cart, wl.k_frac, wl.n_occ, st.C_k, st.E_k, st.C_kq, st.E_kq)
    m.set_params(0, mlp_init(41))
    m.set_params(1, mlp_init(42))
    lat = np.asarray(wl.cell.lat, np.float64)
    m.set_encoding(4.0, 40.0, lat, -3.0, 2.0, 1.0)
    G = np.asarray(wl.G_int, np.int32)
    w = np.asarray(wl.w_eV, np.float64)
    n_w, n_g = len(w), len(G)
    rec = 2 * np.pi * np.linalg.inv(lat).T
    Q = np.asarray(st.q_cart)[None, :] + G @ rec
    qw = np.concatenate([np.column_stack([Q, np.full(n_g, wv)]) for wv in w])
    Lq = torch.empty(n_w * n_g, dtype=torch.float64, device="cuda")
    Eq = torch.empty(n_w * n_g, dtype=torch.float64, device="cuda")
    m.query(_dev(qw, torch.float64), Lq, Eq)
    Lq, Eq = Lq.cpu().numpy().reshape(n_w, n_g), Eq.cpu().numpy().reshape(n_w, n_g)

    def method(ws):
        c.pair_density(G)
        c.chi0(ws, wl.eta_eV, "split_bf16", True)
        c.eps_inv(True)
        return c.loss(torch.empty((len(ws), n_g), dtype=torch.float64, device="cuda")).cpu().numpy()

    # qcx_mlp_infer reports each estimate in units of its curve's maximum (one
    # curve per G along the call's frequencies)
    Eq = Eq * np.abs(Lq) / np.abs(Lq).max(axis=0, keepdims=True)
    L, E, nfb = m.infer(c, G, w, wl.eta_eV, 1e300, "split_bf16",
                        err_out=torch.empty((n_w, n_g), dtype=torch.float64, device="cuda"))
    assert nfb == 0
    assert np.allclose(L.cpu().numpy(), Lq, rtol=1e-12, atol=0)
    assert np.allclose(E.cpu().numpy(), Eq, rtol=1e-12, atol=0)
    L0, _, nfb = m.infer(c, G, w, wl.eta_eV, 0.0, "split_bf16")
    assert nfb == n_w
    assert np.array_equal(L0.cpu().numpy(), method(w))
    tol = float(np.quantile(Eq.max(axis=1), 0.5))
    rows = np.nonzero((Eq > tol).any(axis=1))[0]
    assert 0 < len(rows) < n_w
    Lm, _, nfb = m.infer(c, G, w, wl.eta_eV, tol, "split_bf16")
    Lm = Lm.cpu().numpy()
    assert nfb == len(rows)
    assert np.array_equal(Lm[rows], method(w[rows]))
    keep = np.setdiff1d(np.arange(n_w), rows)
    assert np.allclose(Lm[keep], Lq[keep], rtol=1e-12, atol=0)
