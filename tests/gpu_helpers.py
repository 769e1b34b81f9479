"""Drive the HIP library through its C ABI for a synthetic workload (tests only)."""
import numpy as np


def set_inputs(ctx, wl, iq=0, states=None):
    st = wl.states(iq) if states is None else states
    b = wl.basis
    ctx.set_cell_basis(wl.cell.lat, wl.cell.xyz, b.shell_atom, b.shell_l, b.shell_exp, 1,
                       wl.lattice_range)
    ctx.set_states(st.q_cart, wl.k_frac, wl.n_occ, st.C_k, st.E_k, st.C_kq, st.E_kq)
    return st


def gpu_solve(ctx, wl, iq=0, precision="fp64", w_eV=None, hw64=True, lfe=True, G_int=None,
              want_rho=False, want_chi0=False):
    import torch

    set_inputs(ctx, wl, iq)
    G = wl.G_int if G_int is None else G_int
    w = wl.w_eV if w_eV is None else np.asarray(w_eV)
    out = {}
    rho = None
    if want_rho:
        rho = torch.empty((2, wl.n_k, wl.n_occ, wl.n_cond, len(G)), dtype=torch.complex128,
                          device="cuda")
    ctx.pair_density(G, rho)
    chi = None
    if want_chi0:
        chi = torch.empty((len(w), len(G), len(G)), dtype=torch.complex128, device="cuda")
    ctx.chi0(w, wl.eta_eV, precision, hw64, chi)
    ctx.eps_inv(lfe)
    out["loss"] = ctx.loss()
    if rho is not None:
        out["rho"] = rho.cpu().numpy()
    if chi is not None:
        out["chi0"] = chi.cpu().numpy()
    return out


def normwise(L, Lref):
    """max over G of max_w |L - Lref| / max_w |Lref| (one curve per G)."""
    num = np.max(np.abs(L - Lref), axis=0)
    den = np.max(np.abs(Lref), axis=0)
    return float(np.max(num / np.where(den == 0, 1.0, den)))


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
