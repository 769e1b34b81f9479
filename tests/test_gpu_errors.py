"""Error paths of the C ABI on the GPU, each reached without faulting a
kernel: a singular or non-finite eps in every Gauss-Jordan kernel class
(QCX_ESINGULAR with the frequency index), a device-memory cap (QCX_ENOMEM),
graph capture of a call that stages host data (QCX_EINVAL), and a batch whose
second context holds states that fail their deferred check (QCX_ENONORTH from
qcx_batch_sync), with contexts on different streams."""
import numpy as np
import pytest

from synth import make_mixed_batch_items
from tests.gpu_helpers import normwise, set_inputs

pytestmark = pytest.mark.gpu


def _eps_batch(n_w, n_g, seed):
    """Well-conditioned complex matrices near the identity (diagonally dominant)."""
    rng = np.random.default_rng(seed)
    a = (rng.normal(size=(n_w, n_g, n_g)) + 1j * rng.normal(size=(n_w, n_g, n_g))) / (4.0 * np.sqrt(n_g))
    return a + np.eye(n_g)[None] * (1.5 + 0.3j)


def _diag_inv(e):
    return np.stack([np.diag(np.linalg.inv(m)) for m in e])


# register-resident kernel (both shapes) and the panel kernel at its
# smallest and largest register tiling
@pytest.mark.parametrize("n_g", [40, 113, 300, 1024])
def test_singular_eps_each_kernel_class(n_g):
    import torch

    from paper_2603_12326_amd import Context, QcxError
    from paper_2603_12326_amd import qcx as q

    n_w = 3
    e = _eps_batch(n_w, n_g, 11 + n_g)
    e[1, n_g // 3, :] = 0.0                     # an exactly zero row: no pivot at the last step
    c = Context(0)
    print("singular eps, n_G", n_g, flush=True)
    dev = torch.from_numpy(e).cuda()
    diag = torch.empty((n_w, n_g), dtype=torch.complex128, device="cuda")
    loss = c.eps_inv_given(dev, True, diag_out=diag)
    with pytest.raises(QcxError) as ei:
        c.sync()
    assert ei.value.code == q.ESINGULAR and "frequency index 1" in str(ei.value), str(ei.value)
    c.sync()                                    # reported once
    ref = _diag_inv(e[[0, 2]])
    got = diag.cpu().numpy()[[0, 2]]
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))
    assert np.allclose(loss.cpu().numpy()[[0, 2]], -ref.imag, rtol=0, atol=1e-11)
    # a NaN entry makes the pivot of its column non-finite
    e2 = _eps_batch(n_w, n_g, 5)
    e2[2, 0, n_g - 1] = np.nan
    c.eps_inv_given(torch.from_numpy(e2).cuda(), True)
    with pytest.raises(QcxError) as ei:
        c.sync()
    assert ei.value.code == q.ESINGULAR and "frequency index 2" in str(ei.value)
    # a regular batch passes
    c.eps_inv_given(torch.from_numpy(_eps_batch(n_w, n_g, 6)).cuda(), True)
    c.sync()
    # beyond the inversion kernels
    with pytest.raises(QcxError) as ei:
        c.eps_inv_given(torch.zeros((1, 1025, 1025), dtype=torch.complex128, device="cuda"), True)
    assert ei.value.code == q.EINVAL
    c.close()


def test_singular_nolfe_diagonal():
    import torch

    from paper_2603_12326_amd import Context, QcxError
    from paper_2603_12326_amd import qcx as q

    e = _eps_batch(4, 9, 3)
    e[3, 4, 4] = 0.0
    c = Context(0)
    loss = c.eps_inv_given(torch.from_numpy(e).cuda(), False)
    with pytest.raises(QcxError) as ei:
        c.sync()
    assert ei.value.code == q.ESINGULAR and "frequency index 3" in str(ei.value)
    ref = -np.imag(1.0 / np.einsum("wii->wi", e[:3]))
    assert np.allclose(loss.cpu().numpy()[:3], ref, rtol=0, atol=1e-14)
    c.close()


def test_memory_limit_enomem(small_wl):
    from oracle import rpa
    from paper_2603_12326_amd import Context, QcxError
    from paper_2603_12326_amd import qcx as q

    c = Context(0)
    set_inputs(c, small_wl)
    used = c.memory_used()
    assert used > 0
    c.set_memory_limit(used + 64 * 1024)
    with pytest.raises(QcxError) as ei:
        c.pair_density(small_wl.G_int)
    assert ei.value.code == q.ENOMEM
    assert c.memory_used() <= used + 64 * 1024
    c.set_memory_limit(0)
    c.pair_density(small_wl.G_int)
    c.chi0(small_wl.w_eV, small_wl.eta_eV, "fp64")
    c.eps_inv()
    ref = rpa.solve_workload(small_wl, 0)
    assert normwise(c.loss(), ref) < 1e-10
    c.close()


def test_capture_rejected(small_wl):
    """A call that stages host data, issued while its stream is capturing,
    returns QCX_EINVAL and records nothing."""
    import torch

    from paper_2603_12326_amd import Context, QcxError
    from paper_2603_12326_amd import qcx as q

    s = torch.cuda.Stream()
    c = Context(0, stream=s.cuda_stream)
    set_inputs(c, small_wl)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    st = small_wl.states(0)
    codes = []
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            for call in (lambda: c.pair_density(small_wl.G_int),
                         lambda: c.set_states(st.q_cart, small_wl.k_frac, small_wl.n_occ, st.C_k, st.E_k,
                                              st.C_kq, st.E_kq)):
                try:
                    call()
                    codes.append((0, ""))
                except QcxError as ex:
                    codes.append((ex.code, str(ex)))
        finally:
            g.capture_end()
    assert [x[0] for x in codes] == [q.EINVAL, q.EINVAL], codes
    assert all("captured" in x[1] for x in codes), codes
    # the context is unaffected
    c.pair_density(small_wl.G_int)
    c.close()


def test_batch_other_streams_and_deferred_checks():
    """Contexts on their own streams: the batch orders itself after their
    pair densities (results equal the one-stream batch bit for bit), and a
    context whose device-resident states fail the orthonormality check is
    reported by qcx_batch_sync of the first context."""
    import torch

    from paper_2603_12326_amd import Context, QcxError, batch_sync, run_batch
    from paper_2603_12326_amd import qcx as q

    items = make_mixed_batch_items()[:3]
    streams = [torch.cuda.Stream() for _ in items]

    def build(per_stream):
        ctxs = []
        for i, wl in enumerate(items):
            c = Context(0, stream=streams[i].cuda_stream) if per_stream else Context(0)
            set_inputs(c, wl)
            c.pair_density(wl.G_int)
            ctxs.append(c)
        ctxs[0].set_autotune(0)     # one fixed plan, so the two batches compare bit for bit
        return ctxs

    def run(ctxs):
        outs = [torch.full((len(wl.w_eV), len(wl.G_int)), np.nan, dtype=torch.float64, device="cuda")
                for wl in items]
        torch.cuda.synchronize()
        run_batch(ctxs, [dict(ctx=i, w_eV=wl.w_eV, eta_eV=wl.eta_eV, loss_out=outs[i])
                         for i, wl in enumerate(items)], precision="split_bf16")
        batch_sync(ctxs[0])
        torch.cuda.synchronize()
        return [o.cpu().numpy() for o in outs]

    a = build(False)
    ref = run(a)
    b = build(True)
    got = run(b)
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
    # context 1: device states with one bad coefficient matrix at k+q 2
    wl = items[1]
    st = wl.states(0)
    dev = lambda v, t: torch.from_numpy(np.ascontiguousarray(v)).to(t).cuda()  # noqa: E731
    bad = st.C_kq.copy()
    bad[2] *= 1.001
    b[1].set_states(st.q_cart, dev(wl.k_frac, torch.float64), wl.n_occ, dev(st.C_k, torch.complex128),
                    dev(st.E_k, torch.float64), dev(bad, torch.complex128), dev(st.E_kq, torch.float64))
    b[1].pair_density(wl.G_int)
    with pytest.raises(QcxError) as ei:
        run(b)
    assert ei.value.code == q.ENONORTH and "context 1" in str(ei.value) and "k+q 2" in str(ei.value)
    for c in a + b:
        c.close()
