"""Loss surrogate driver: sampling, training and querying with fallback.

A composition of C-ABI calls (qcx.Context for the method, qcx.Mlp for the
networks); every number is computed by the library's kernels.  The host
side only lays out inputs (momenta Q = q + G, frequency lists, sample
orders) and collects the one-off scaling constants of the network (mean
and spread of the training targets, the calibration of the error
estimate).

Sampling: for a momentum q and frequencies w_1..w_m, one pass of the method
(set_states, pair_density, chi0, eps_inv, loss) gives the loss at every
Q = q + G of the G set (Eq. eps_LFE: [eps^-1]_GG is the response at q + G),
so each pass yields m * N_G samples ((Qx, Qy, Qz, w), L).

Query with fallback (qcx_mlp_infer, one call per momentum q): the networks
answer every (Q, w); accuracy is measured per loss curve along frequency
(one per G), as the error in units of the curve's maximum, and each
frequency with a point whose estimate in those units exceeds the tolerance
is recomputed by the method inside the library (one pass per q over the
rejected frequencies), since the inverse of eps gives all G of a frequency
at once.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import qcx


def g_cart(G_int, lat) -> np.ndarray:
    """Cartesian reciprocal vectors G = n . b with b_i . a_j = 2 pi delta_ij."""
    b = 2.0 * np.pi * np.linalg.inv(np.asarray(lat, np.float64)).T
    return np.asarray(G_int, np.float64) @ b


def query_points(q, Gc, w) -> np.ndarray:
    """qw[(iw, iG)] = (q + G[iG], w[iw]) for one q: [n_w * n_G][4], w-major."""
    n_w, n_g = len(w), len(Gc)
    Q = np.asarray(q, np.float64)[None, :] + Gc
    out = np.empty((n_w, n_g, 4))
    out[:, :, :3] = Q[None, :, :]
    out[:, :, 3] = np.asarray(w, np.float64)[:, None]
    return out.reshape(-1, 4)


def method_loss(ctx: "qcx.Context", set_states: Callable[[int], None], iq: int, G_int, w,
                eta_eV: float, precision="split_bf16"):
    """One pass of the method for momentum iq: device loss [n_w][n_G]."""
    import torch

    set_states(iq)
    ctx.pair_density(G_int)
    ctx.chi0(w, eta_eV, precision, True)
    ctx.eps_inv(True)
    out = torch.empty((len(w), len(G_int)), dtype=torch.float64, device="cuda")
    return ctx.loss(out)


@dataclass
class Samples:
    qw: "object"          # device float64 [n][4]
    loss: "object"        # device float64 [n]
    q_index: np.ndarray   # which momentum each sample came from
    w_index: np.ndarray   # index into that momentum's frequency list


def sample(ctx, set_states, q_list, G_int, lat, w_lists: Sequence[np.ndarray], eta_eV,
           precision="split_bf16") -> Samples:
    """Loss samples at Q = q + G for every q of q_list and its frequencies."""
    import torch

    Gc = g_cart(G_int, lat)
    qws, losses, qi, wi = [], [], [], []
    for iq, (q, w) in enumerate(zip(q_list, w_lists)):
        L = method_loss(ctx, set_states, iq, G_int, w, eta_eV, precision)
        qws.append(torch.from_numpy(query_points(q, Gc, w)).cuda())
        losses.append(L.reshape(-1))
        qi.append(np.full(len(w) * len(Gc), iq, np.int32))
        wi.append(np.repeat(np.arange(len(w), dtype=np.int32), len(Gc)))
    return Samples(torch.cat(qws), torch.cat(losses), np.concatenate(qi), np.concatenate(wi))


class Surrogate:
    """An ensemble of networks with the scaling that maps (Q, w) to the loss."""

    def __init__(self, ctx: "qcx.Context", n_members: int = 4):
        self.ctx = ctx
        self.net = qcx.Mlp(ctx, n_members)
        self.K = n_members
        self.q_max = self.w_max = self.mu = self.sigma = None
        self.lattice = None
        self.calib = 1.0

    def fit(self, s: Samples, train_idx: np.ndarray, q_max: float, w_max: float, lattice,
            init_params: Callable[[int], np.ndarray], orders: Callable[[int, int, int], np.ndarray],
            batch: int = 1024, epochs: int = 40, lr0: float = 2e-3, lr1: float = 2e-5,
            progress: Optional[Callable[[int], None]] = None):
        """Train every member on the samples train_idx; lattice (3 x 3, rows
        the primitive vectors, bohr) sets the periodic features of the
        encoding; init_params(k) gives member k's initial parameters and
        orders(k, n, batch) its sample order (indices into train_idx);
        progress(k), if given, is called once member k has trained."""
        import torch

        tl = np.log(np.maximum(s.loss.cpu().numpy()[train_idx], 1e-30))
        self.q_max, self.w_max = float(q_max), float(w_max)
        self.mu, self.sigma = float(tl.mean()), float(tl.std())
        self.lattice = np.asarray(lattice, np.float64).reshape(3, 3)
        self._encoding(self.calib)
        ti = torch.from_numpy(np.ascontiguousarray(train_idx)).cuda()
        qw = s.qw[ti].contiguous()
        loss = s.loss[ti].contiguous()
        n = len(train_idx)
        x = torch.empty((n, qcx.MLP_NIN), dtype=torch.float32, device="cuda")
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        self.net.encode(qw, loss, x, t)
        hists = []
        t0 = time.perf_counter()
        for k in range(self.K):
            self.net.set_params(k, init_params(k))
            order = torch.from_numpy(orders(k, n, batch)).cuda()
            hists.append(self.net.train(k, x, t, batch, order, lr0, lr1))
            if progress is not None:
                torch.cuda.synchronize()
                progress(k)
        torch.cuda.synchronize()
        self.train_seconds = time.perf_counter() - t0
        return hists

    def calibrate(self, s: Samples, idx: np.ndarray, quantile: float = 0.95):
        """Scale the ensemble spread so that it bounds the relative error of
        the held-out points idx at the given quantile."""
        import torch

        self._encoding(1.0)
        ii = torch.from_numpy(np.ascontiguousarray(idx)).cuda()
        qw = s.qw[ii].contiguous()
        L = torch.empty(len(idx), dtype=torch.float64, device="cuda")
        E = torch.empty(len(idx), dtype=torch.float64, device="cuda")
        self.net.query(qw, L, E)
        ref = s.loss[ii].cpu().numpy()
        got, spread = L.cpu().numpy(), E.cpu().numpy()
        rel = np.abs(got / np.maximum(ref, 1e-300) - 1.0)
        ratio = rel / np.maximum(spread, 1e-12)
        self.calib = float(np.quantile(ratio, quantile))
        self._encoding(self.calib)
        return dict(rel_err=rel, spread=spread, calib=self.calib)

    def _encoding(self, calib: float):
        self.net.set_encoding(self.q_max, self.w_max, self.lattice, self.mu, self.sigma, calib)

    def query(self, qw, tol: Optional[float] = None):
        """Device (loss, err, reject indices or None, number rejected)."""
        import torch

        n = qw.shape[0]
        L = torch.empty(n, dtype=torch.float64, device="cuda")
        E = torch.empty(n, dtype=torch.float64, device="cuda")
        if tol is None:
            self.net.query(qw, L, E)
            return L, E, None, 0
        idx = torch.empty(n, dtype=torch.int32, device="cuda")
        nrej = self.net.query(qw, L, E, tol, idx)
        return L, E, idx[:nrej], nrej

    def infer(self, ctx, G_int, w, eta_eV: float, tol: float, precision="split_bf16", err_out=None):
        """qcx_mlp_infer for the momentum of ctx's states: (loss [n_w][n_G],
        err, number of frequencies the method recomputed)."""
        return self.net.infer(ctx, G_int, w, eta_eV, tol, precision, err_out=err_out)

    def close(self):
        self.net.close()


def query_with_fallback(sur: Surrogate, ctx, set_states, n_q: int, G_int, w_lists, eta_eV,
                        tol: float, precision="split_bf16"):
    """Answer every (q + G, w) of the grid (n_q momenta x w_lists x G) with
    the surrogate and the method as fallback: for each momentum, set its
    states (set_states(iq)) and call qcx_mlp_infer, which recomputes every
    frequency row holding a rejected point (enqueued without waiting, so the
    host moves on to the next momentum while the device runs them).  Returns
    (loss per q as device [n_w][n_G] tensors, statistics)."""
    import torch

    n_g = len(G_int)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, errs = [], []
    n_rows = n_pass = 0
    for iq in range(n_q):
        set_states(iq)
        E = torch.empty((len(w_lists[iq]), n_g), dtype=torch.float64, device="cuda")
        L, _, nfb = sur.infer(ctx, G_int, w_lists[iq], eta_eV, tol, precision, err_out=E)
        out.append(L)
        errs.append(E.reshape(-1))
        n_rows += nfb
        n_pass += nfb > 0
    ctx.sync()  # the last fallback rows, and the checks of every fallback pass
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    err = torch.cat(errs)
    return out, dict(n_queries=int(err.numel()), n_rejected=int((err > tol).sum().item()),
                     fallback_passes=n_pass, fallback_points=n_rows, t_total=t1 - t0, err=err)
