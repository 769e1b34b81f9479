"""Composite dielectric function of Sec. III: local field effects inside a
momentum cutoff, the diagonal alone beyond it.

For one q: the G with |q + G| <= q_lfe form the LFE block (Eq. eps_LFE:
pair densities, chi0, the inverse of eps, its diagonal); every other G gets
the noLFE loss of Eq. (eps_noLFE) from qcx_loss_diag.  A composition of C-ABI
calls; the host only splits the G list by |q + G| (argument preparation).
"""
from __future__ import annotations

import numpy as np


def split(lat, q_cart, G_int, q_lfe: float):
    """Indices of the LFE block (|q + G| <= q_lfe, must start with G = 0) and
    of the remaining G."""
    G = np.asarray(G_int, np.int64).reshape(-1, 3)
    b = 2.0 * np.pi * np.linalg.inv(np.asarray(lat, np.float64)).T
    qn = np.linalg.norm(np.asarray(q_cart, np.float64)[None, :] + G @ b, axis=1)
    inner = np.nonzero(qn <= q_lfe)[0]
    outer = np.nonzero(qn > q_lfe)[0]
    if len(inner) == 0 or inner[0] != 0 or np.any(G[0] != 0):
        raise ValueError("the LFE block must start with G = 0")
    return inner, outer


def composite_loss(ctx, lat, q_cart, G_int, w_eV, eta_eV: float, q_lfe: float,
                   precision="split_bf16", with_inv: bool = False):
    """Loss on the context's current states: returns (inner, L_inner, outer,
    L_outer) with L_* CUDA float64 tensors [n_w][len(*)] for the G indices
    inner / outer of G_int; with_inv adds (D_inner, D_outer), CUDA complex128
    [n_w][len(*)] holding 1/eps(w, q+G) (the diagonal of eps^-1 inside the
    block, 1/eps_GG beyond).  Leaves the context's pair densities replaced."""
    import torch

    G = np.asarray(G_int, np.int32).reshape(-1, 3)
    inner, outer = split(lat, q_cart, G, q_lfe)
    w = np.asarray(w_eV, np.float64)
    ctx.pair_density(G[inner])
    ctx.chi0(w, eta_eV, precision, True)
    D_in = D_out = None
    if with_inv:
        D_in = torch.empty((len(w), len(inner)), dtype=torch.complex128, device="cuda")
    ctx.eps_inv(True, diag_out=D_in)
    L_in = torch.empty((len(w), len(inner)), dtype=torch.float64, device="cuda")
    ctx.loss(L_in)
    L_out = None
    if len(outer):
        if with_inv:
            D_out = torch.empty((len(w), len(outer)), dtype=torch.complex128, device="cuda")
        L_out = ctx.loss_diag(G[outer], w, eta_eV, precision, inv_out=D_out)
    if with_inv:
        return inner, L_in, outer, L_out, D_in, D_out
    return inner, L_in, outer, L_out


def assemble(n_g: int, inner, L_in, outer, L_out) -> np.ndarray:
    """Host array [n_w][n_g] in the order of the G list (synchronising copy)."""
    Li = L_in.cpu().numpy()
    out = np.empty((Li.shape[0], n_g))
    out[:, inner] = Li
    if L_out is not None:
        out[:, outer] = L_out.cpu().numpy()
    return out
