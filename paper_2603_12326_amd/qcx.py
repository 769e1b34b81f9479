"""Thin Python binding of libqcx (include/qcx.h): argument marshalling only.

Every step of the path runs in the HIP library; this module converts numpy
arrays (host) and torch CUDA tensors (device) to plain pointers, passes the
caller's torch stream, and raises QcxError on a non-zero status.  There is no
CPU fallback: if libqcx.so is missing or the device is not gfx950, creating a
Context fails loudly.

Method names follow the C entry points without their `qcx_` prefix:
set_cell_basis, set_states, pair_density, chi0, eps_inv, loss, sync,
stage_times, set_timing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcx.so")

OK, EINVAL, ESTATE, ENONORTH, ESINGULAR, EDEVICE, ENOMEM = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32, SPLIT_BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "split_bf16": SPLIT_BF16}

_ERRNAMES = {EINVAL: "QCX_EINVAL", ESTATE: "QCX_ESTATE", ENONORTH: "QCX_ENONORTH",
             ESINGULAR: "QCX_ESINGULAR", EDEVICE: "QCX_EDEVICE", ENOMEM: "QCX_ENOMEM"}


class QcxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double

_SIGS = {
    "qcx_create": [ctypes.POINTER(_P), _I, _P],
    "qcx_destroy": [_P],
    "qcx_last_error": [_P],
    "qcx_sync": [_P],
    "qcx_set_cell_basis": [_P, _P, _I, _P, _I, _P, _P, _P, _I, _I],
    "qcx_set_states": [_P, _P, _I, _P, _I, _I, _P, _P, _P, _P, _I],
    "qcx_pair_density": [_P, _I, _P, _P],
    "qcx_pair_density_optical": [_P, _I, _P, _P, _P],
    "qcx_chi0": [_P, _I, _P, _D, _I, _I, _P],
    "qcx_eps_inv": [_P, _I, _P, _P],
    "qcx_eps_inv_given": [_P, _I, _I, _P, _I, _P, _P, _P],
    "qcx_eps_inv_given_noalloc": [_P, _I, _I, _P, _I, _P, _P, _P, _P],
    "qcx_set_memory_limit": [_P, ctypes.c_size_t],
    "qcx_memory_used": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "qcx_loss": [_P, _P, _I],
    "qcx_stage_times": [_P, _P],
    "qcx_set_timing": [_P, _I],
    "qcx_build_info": [],
    "qcx_set_autotune": [_P, _I],
    "qcx_bulk_config": [_P, _P, _P],
    "qcx_set_bulk_pipeline": [_P, _I],
    "qcx_run_batch": [_P, _I, _P, _I, _I, _I, _I],
    "qcx_run_batch_rho": [_P, _I, _P, _P, _P, _I, _I, _I, _I],
    "qcx_batch_sync": [_P],
    "qcx_batch_config": [_P, _P, _P],
    "qcx_loss_diag": [_P, _I, _P, _I, _P, _D, _I, _P, _P],
    "qcx_chi0_kk": [_P, _I, _P, _D, _D, _P],
    "qcx_mlp_create": [ctypes.POINTER(_P), _P, _I],
    "qcx_mlp_destroy": [_P],
    "qcx_mlp_set_params": [_P, _I, _P],
    "qcx_mlp_get_params": [_P, _I, _P],
    "qcx_mlp_forward": [_P, _I, _I, _P, _P],
    "qcx_mlp_grad": [_P, _I, _I, _P, _P, _P, _P],
    "qcx_mlp_train": [_P, _I, _I, _P, _P, _I, _I, _P, ctypes.c_float, ctypes.c_float, _P],
    "qcx_mlp_set_encoding": [_P, _D, _D, _P, _D, _D, _D],
    "qcx_mlp_encode": [_P, _I, _P, _P, _P, _P],
    "qcx_mlp_query": [_P, _I, _P, _P, _P, _D, _P, _P],
    "qcx_mlp_infer": [_P, _P, _I, _P, _I, _P, _D, _D, _I, _P, _P, _P],
    "qcx_qbin_create": [ctypes.POINTER(_P), _P, _I, _I, _D, _I, _I],
    "qcx_qbin_destroy": [_P],
    "qcx_qbin_reset": [_P],
    "qcx_qbin_add": [_P, _I, _P, _P, _I, _I],
    "qcx_qbin_finish": [_P, _P, _P, _P],
    "qcx_qbin_rate_halo": [_P, _P, _P, _P, _P],
}
QBIN_EPS, QBIN_INV = 0, 1
MLP_NIN = 49
MLP_NPARAM = 210433


class QcxHalo(ctypes.Structure):
    _fields_ = [("m_chi_eV", _D), ("m_med_eV", _D), ("sigma_e_cm2", _D), ("rho_T_g_cm3", _D),
                ("rho_chi_GeV_cm3", _D), ("v0_kms", _D), ("vE_kms", _D), ("vesc_kms", _D)]


class QcxItem(ctypes.Structure):
    """struct qcx_item of include/qcx.h."""
    _fields_ = [("ctx", _I), ("n_w", _I), ("w_eV", _P), ("eta_eV", _D), ("loss_out", _P)]


def load_library(path: str = LIB_PATH):
    """Load libqcx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own libamdhip64.so.7 and HSA runtime; load them first so
    # that libqcx's dependency resolves to the same copy (a second HIP runtime
    # in the process cannot open the device).
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2603_12326_amd.build`")
    lib = ctypes.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("qcx_last_error", "qcx_build_info") else _I
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr_host(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _is_torch_cuda(x) -> bool:
    return hasattr(x, "is_cuda") and hasattr(x, "data_ptr") and bool(x.is_cuda)


def _dev_ptr(t, dtype_name: str, numel: int, what: str):
    import torch

    want = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128,
            "i32": torch.int32}[dtype_name]
    if not _is_torch_cuda(t):
        raise TypeError(f"{what}: expected a CUDA tensor")
    if t.dtype != want or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{what}: need contiguous {want} with {numel} elements, got "
                         f"{t.dtype} {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context on one device and stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self.lib = load_library()
        if stream is None:
            import torch

            torch.cuda.set_device(device)
            stream = torch.cuda.current_stream(device).cuda_stream
        self._stream = int(stream)
        h = ctypes.c_void_p()
        rc = self.lib.qcx_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream))
        if rc != OK:
            raise QcxError(rc, self.lib.qcx_last_error(None).decode())
        self._h = h
        self.n_g = self.n_w = self.n_k = self.n_occ = self.n_bands = None

    # -- plumbing
    def _check(self, rc: int):
        if rc != OK:
            raise QcxError(rc, self.lib.qcx_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.qcx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- the C entry points
    def set_cell_basis(self, lat, xyz, shell_atom, shell_l, shell_exp, pure_d: int = 1,
                       lattice_range: int = 1):
        lat = _host(lat, np.float64).reshape(9)
        xyz = _host(xyz, np.float64).reshape(-1, 3)
        sa = _host(shell_atom, np.int32)
        sl = _host(shell_l, np.int32)
        se = _host(shell_exp, np.float64)
        self._check(self.lib.qcx_set_cell_basis(self._h, _ptr_host(lat), len(xyz), _ptr_host(xyz),
                                                len(sl), _ptr_host(sa), _ptr_host(sl),
                                                _ptr_host(se), pure_d, lattice_range))

    def set_states(self, q_cart, k_frac, n_occ: int, C_k, E_k, C_kq, E_kq):
        """Host numpy arrays, or CUDA tensors (complex128 C, float64 k and E)."""
        q = _host(q_cart, np.float64).reshape(3)
        if _is_torch_cuda(C_k):
            n_k, n_ao, n_b = C_k.shape
            kf = _dev_ptr(k_frac, "f64", n_k * 3, "k_frac")
            ptrs = [_dev_ptr(C_k, "c128", n_k * n_ao * n_b, "C_k"),
                    _dev_ptr(E_k, "f64", n_k * n_b, "E_k"),
                    _dev_ptr(C_kq, "c128", n_k * n_ao * n_b, "C_kq"),
                    _dev_ptr(E_kq, "f64", n_k * n_b, "E_kq")]
            mem = MEM_DEVICE
            keep = None
        else:
            kf_a = _host(k_frac, np.float64)
            arrs = [_host(C_k, np.complex128), _host(E_k, np.float64),
                    _host(C_kq, np.complex128), _host(E_kq, np.float64)]
            n_k, n_ao, n_b = arrs[0].shape
            kf = _ptr_host(kf_a)
            ptrs = [_ptr_host(a) for a in arrs]
            mem = MEM_HOST
            keep = (kf_a, arrs)
        self._check(self.lib.qcx_set_states(self._h, _ptr_host(q), n_k, kf, n_occ, n_b, ptrs[0],
                                            ptrs[1], ptrs[2], ptrs[3], mem))
        del keep
        self.n_k, self.n_occ, self.n_bands = n_k, n_occ, n_b

    def pair_density(self, G_int, rho_out=None):
        G = _host(G_int, np.int32).reshape(-1, 3)
        out = None
        if rho_out is not None:
            n_c = self.n_bands - self.n_occ
            out = _dev_ptr(rho_out, "c128", 2 * self.n_k * self.n_occ * n_c * len(G), "rho_out")
        self._check(self.lib.qcx_pair_density(self._h, len(G), _ptr_host(G), out))
        self.n_g = len(G)

    def pair_density_optical(self, G_int, qhat, rho_out=None):
        """Pair densities as q -> 0 along qhat (qcx_pair_density_optical); the
        states must have been set with q = 0."""
        G = _host(G_int, np.int32).reshape(-1, 3)
        qh = _host(qhat, np.float64).reshape(3)
        out = None
        if rho_out is not None:
            n_c = self.n_bands - self.n_occ
            out = _dev_ptr(rho_out, "c128", 2 * self.n_k * self.n_occ * n_c * len(G), "rho_out")
        self._check(self.lib.qcx_pair_density_optical(self._h, len(G), _ptr_host(G), _ptr_host(qh),
                                                      out))
        self.n_g = len(G)

    def chi0(self, w_eV, eta_eV: float, precision=FP64, headwings_fp64: bool = True,
             chi0_out=None):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        w = _host(w_eV, np.float64).reshape(-1)
        out = None
        if chi0_out is not None:
            out = _dev_ptr(chi0_out, "c128", len(w) * self.n_g * self.n_g, "chi0_out")
        self._check(self.lib.qcx_chi0(self._h, len(w), _ptr_host(w), float(eta_eV), int(precision),
                                      1 if headwings_fp64 else 0, out))
        self.n_w = len(w)

    def chi0_kk(self, w_eV, eta_eV: float, bin_eV: float, chi0_out=None):
        """chi0 from the binned spectral part, all FP64 (qcx_chi0_kk)."""
        w = _host(w_eV, np.float64).reshape(-1)
        out = None
        if chi0_out is not None:
            out = _dev_ptr(chi0_out, "c128", len(w) * self.n_g * self.n_g, "chi0_out")
        self._check(self.lib.qcx_chi0_kk(self._h, len(w), _ptr_host(w), float(eta_eV),
                                         float(bin_eV), out))
        self.n_w = len(w)

    def eps_inv(self, lfe: bool = True, diag_out=None, epsM_out=None):
        d = None if diag_out is None else _dev_ptr(diag_out, "c128", self.n_w * self.n_g, "diag_out")
        e = None if epsM_out is None else _dev_ptr(epsM_out, "c128", self.n_w, "epsM_out")
        self._check(self.lib.qcx_eps_inv(self._h, 1 if lfe else 0, d, e))

    def eps_inv_given(self, eps, lfe: bool = True, loss_out=None, diag_out=None, epsM_out=None):
        """diag(eps^-1) and the loss of caller-supplied matrices (qcx_eps_inv_given):
        eps a CUDA complex128 tensor [n_w][n_G][n_G]; returns loss_out (CUDA
        float64 [n_w][n_G], allocated when None)."""
        import torch

        n_w, n_g, n_g2 = eps.shape
        if n_g != n_g2:
            raise ValueError("eps must be [n_w][n_G][n_G]")
        if loss_out is None:
            loss_out = torch.empty((n_w, n_g), dtype=torch.float64, device=eps.device)
        self._check(self.lib.qcx_eps_inv_given(
            self._h, n_w, n_g, _dev_ptr(eps, "c128", n_w * n_g * n_g, "eps"), 1 if lfe else 0,
            _dev_ptr(loss_out, "f64", n_w * n_g, "loss_out"),
            None if diag_out is None else _dev_ptr(diag_out, "c128", n_w * n_g, "diag_out"),
            None if epsM_out is None else _dev_ptr(epsM_out, "c128", n_w, "epsM_out")))
        return loss_out

    def eps_inv_given_noalloc(self, eps, lfe: bool, loss_out, status_out, diag_out=None,
                              epsM_out=None):
        """qcx_eps_inv_given_noalloc: the caller passes every output (CUDA
        tensors: loss_out float64 [n_w][n_G], status_out int32 [1])."""
        n_w, n_g, _ = eps.shape
        self._check(self.lib.qcx_eps_inv_given_noalloc(
            self._h, n_w, n_g, _dev_ptr(eps, "c128", n_w * n_g * n_g, "eps"), 1 if lfe else 0,
            _dev_ptr(loss_out, "f64", n_w * n_g, "loss_out"),
            None if diag_out is None else _dev_ptr(diag_out, "c128", n_w * n_g, "diag_out"),
            None if epsM_out is None else _dev_ptr(epsM_out, "c128", n_w, "epsM_out"),
            _dev_ptr(status_out, "i32", 1, "status_out")))

    def set_memory_limit(self, nbytes: int):
        """Cap the context's own device buffers (0: no cap)."""
        self._check(self.lib.qcx_set_memory_limit(self._h, int(nbytes)))

    def memory_used(self) -> int:
        v = ctypes.c_size_t(0)
        self._check(self.lib.qcx_memory_used(self._h, ctypes.byref(v)))
        return int(v.value)

    def loss(self, out=None):
        """Host numpy [n_w][n_G] (synchronising) when out is None, else a CUDA tensor."""
        if out is None:
            arr = np.empty((self.n_w, self.n_g), np.float64)
            self._check(self.lib.qcx_loss(self._h, _ptr_host(arr), MEM_HOST))
            return arr
        self._check(self.lib.qcx_loss(self._h, _dev_ptr(out, "f64", self.n_w * self.n_g, "out"),
                                      MEM_DEVICE))
        return out

    def loss_diag(self, G_int, w_eV, eta_eV: float, precision="split_bf16", out=None,
                  inv_out=None):
        """noLFE loss for any number of G (qcx_loss_diag): CUDA float64 tensor
        [n_w][n_G] (allocated when out is None); inv_out (CUDA complex128
        [n_w][n_G]) receives 1/eps_GG.  Replaces the pair densities."""
        import torch

        G = _host(G_int, np.int32).reshape(-1, 3)
        w = _host(w_eV, np.float64).reshape(-1)
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        if out is None:
            out = torch.empty((len(w), len(G)), dtype=torch.float64, device="cuda")
        self._check(self.lib.qcx_loss_diag(self._h, len(G), _ptr_host(G), len(w), _ptr_host(w),
                                           float(eta_eV), int(precision),
                                           _dev_ptr(out, "f64", len(w) * len(G), "out"),
                                           None if inv_out is None else
                                           _dev_ptr(inv_out, "c128", len(w) * len(G), "inv_out")))
        return out

    def sync(self):
        self._check(self.lib.qcx_sync(self._h))

    def set_timing(self, enable: bool = True):
        self._check(self.lib.qcx_set_timing(self._h, 1 if enable else 0))

    def set_autotune(self, mode: int = 1):
        self._check(self.lib.qcx_set_autotune(self._h, int(mode)))

    def bulk_config(self) -> dict:
        cfg = np.zeros(3, np.int32)
        ms = ctypes.c_double(0.0)
        self._check(self.lib.qcx_bulk_config(self._h, _ptr_host(cfg), ctypes.byref(ms)))
        return dict(ksplit=int(cfg[0]), stages=int(cfg[1]), row_frags=int(cfg[2]),
                    tune_ms=ms.value)

    def set_bulk_pipeline(self, nst: int):
        """Force the bulk kernel's LDS pipeline (2, 3, 4) or restore the tuned choice (0)."""
        self._check(self.lib.qcx_set_bulk_pipeline(self._h, int(nst)))

    def batch_config(self) -> dict:
        """Plan of the last batch whose first context is this one."""
        cfg = np.zeros(3, np.int32)
        ms = ctypes.c_double(0.0)
        self._check(self.lib.qcx_batch_config(self._h, _ptr_host(cfg), ctypes.byref(ms)))
        return dict(target_steps=int(cfg[0]), tiles=int(cfg[1]), blocks=int(cfg[2]),
                    tune_ms=ms.value)

    def stage_times(self) -> dict:
        t = np.zeros(7, np.float64)
        self._check(self.lib.qcx_stage_times(self._h, _ptr_host(t)))
        return dict(pair_density_ms=t[0], chi0_bulk_ms=t[1], chi0_headwings_ms=t[2],
                    chi0_total_ms=t[3], eps_inv_ms=t[4], bulk_launches=int(t[5]),
                    kk_transform_ms=t[6])


def run_batch(contexts, items, precision=SPLIT_BF16, headwings_fp64: bool = True,
              lfe: bool = True, G_lists=None):
    """Batched chi0 -> eps -> loss (qcx_run_batch, or qcx_run_batch_rho).

    contexts: list of Context with pair densities, or with states only when
    G_lists (one int array [n_G][3] per context, G = 0 first) is given: the
    pair densities are then computed inside the batch.  items: list of dicts
    with keys ctx (index), w_eV, eta_eV, loss_out (CUDA float64 tensor
    [n_w][n_G]).  Asynchronous; call batch_sync(contexts[0]) to wait and
    check errors.
    """
    lib = load_library()
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    handles = (ctypes.c_void_p * len(contexts))(*[c._h.value for c in contexts])
    keep = []
    if G_lists is not None:
        if len(G_lists) != len(contexts):
            raise ValueError("one G list per context")
        gl = [_host(g, np.int32).reshape(-1, 3) for g in G_lists]
        keep += gl
        n_g = np.array([len(g) for g in gl], np.int32)
        gptr = (ctypes.c_void_p * len(gl))(*[g.ctypes.data for g in gl])
    arr = (QcxItem * len(items))()
    for i, it in enumerate(items):
        w = _host(it["w_eV"], np.float64).reshape(-1)
        keep.append(w)
        ng = len(gl[it["ctx"]]) if G_lists is not None else contexts[it["ctx"]].n_g
        out = _dev_ptr(it["loss_out"], "f64", len(w) * ng, "loss_out")
        arr[i] = QcxItem(int(it["ctx"]), len(w), w.ctypes.data, float(it["eta_eV"]), out.value)
    flags = (int(precision), 1 if headwings_fp64 else 0, 1 if lfe else 0)
    if G_lists is None:
        rc = lib.qcx_run_batch(handles, len(contexts), ctypes.cast(arr, ctypes.c_void_p), len(items),
                               *flags)
    else:
        rc = lib.qcx_run_batch_rho(handles, len(contexts), _ptr_host(n_g), ctypes.cast(gptr, ctypes.c_void_p),
                                   ctypes.cast(arr, ctypes.c_void_p), len(items), *flags)
    del keep
    if rc != OK:
        raise QcxError(rc, lib.qcx_last_error(contexts[0]._h).decode())
    if G_lists is not None:
        for c, g in zip(contexts, gl):
            c.n_g = len(g)


def batch_sync(ctx0):
    ctx0._check(ctx0.lib.qcx_batch_sync(ctx0._h))


class Mlp:
    """Surrogate ensemble (qcx_mlp_*) on a Context's device and stream."""

    def __init__(self, ctx: Context, n_members: int = 4):
        self.ctx = ctx
        self.lib = ctx.lib
        self.n_members = n_members
        h = ctypes.c_void_p()
        ctx._check(self.lib.qcx_mlp_create(ctypes.byref(h), ctx._h, n_members))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.qcx_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, member: int, params):
        p = _host(params, np.float32).reshape(-1)
        if len(p) != MLP_NPARAM:
            raise ValueError(f"need {MLP_NPARAM} parameters")
        self.ctx._check(self.lib.qcx_mlp_set_params(self._h, member, _ptr_host(p)))

    def get_params(self, member: int) -> np.ndarray:
        p = np.empty(MLP_NPARAM, np.float32)
        self.ctx._check(self.lib.qcx_mlp_get_params(self._h, member, _ptr_host(p)))
        return p

    def forward(self, member: int, x, y):
        n = x.shape[0]
        self.ctx._check(self.lib.qcx_mlp_forward(self._h, member, n, _dev_ptr(x, "f32", n * MLP_NIN, "x"),
                                                 _dev_ptr(y, "f32", n, "y")))
        return y

    def grad(self, member: int, x, t):
        n = x.shape[0]
        g = np.empty(MLP_NPARAM, np.float32)
        loss = ctypes.c_float()
        self.ctx._check(self.lib.qcx_mlp_grad(self._h, member, n, _dev_ptr(x, "f32", n * MLP_NIN, "x"),
                                              _dev_ptr(t, "f32", n, "t"), _ptr_host(g),
                                              ctypes.byref(loss)))
        return g, loss.value

    def train(self, member: int, x, t, batch: int, order, lr0: float, lr1: float,
              want_hist: bool = True):
        n = x.shape[0]
        n_steps = order.numel() // batch
        hist = np.empty(n_steps, np.float32) if want_hist else None
        self.ctx._check(self.lib.qcx_mlp_train(
            self._h, member, n, _dev_ptr(x, "f32", n * MLP_NIN, "x"), _dev_ptr(t, "f32", n, "t"), batch,
            n_steps, _dev_ptr(order, "i32", order.numel(), "order"), float(lr0), float(lr1),
            _ptr_host(hist) if want_hist else None))
        return hist

    def set_encoding(self, q_max, w_max_eV, lattice, mu, sigma, calib=1.0):
        lat = _host(lattice, np.float64).reshape(-1)
        if lat.size != 9:
            raise ValueError("lattice: three primitive vectors (3 x 3)")
        self.ctx._check(self.lib.qcx_mlp_set_encoding(self._h, q_max, w_max_eV, _ptr_host(lat), mu,
                                                      sigma, calib))

    def encode(self, qw, loss=None, x=None, t=None):
        n = qw.shape[0]
        self.ctx._check(self.lib.qcx_mlp_encode(
            self._h, n, _dev_ptr(qw, "f64", n * 4, "qw"),
            None if loss is None else _dev_ptr(loss, "f64", n, "loss"),
            _dev_ptr(x, "f32", n * MLP_NIN, "x"), None if t is None else _dev_ptr(t, "f32", n, "t")))

    def query(self, qw, loss, err=None, tol=None, reject_idx=None):
        """Returns the number of rejected points when reject_idx is given."""
        n = qw.shape[0]
        nrej = ctypes.c_int(0)
        rej = reject_idx is not None
        self.ctx._check(self.lib.qcx_mlp_query(
            self._h, n, _dev_ptr(qw, "f64", n * 4, "qw"), _dev_ptr(loss, "f64", n, "loss"),
            None if err is None else _dev_ptr(err, "f64", n, "err"),
            float(tol) if tol is not None else 0.0,
            _dev_ptr(reject_idx, "i32", n, "reject_idx") if rej else None,
            ctypes.byref(nrej) if rej else None))
        return nrej.value if rej else None

    def infer(self, ctx: "Context", G_int, w_eV, eta_eV: float, tol: float, precision="split_bf16",
              loss_out=None, err_out=None):
        """Loss at (q + G, w) for the momentum of ctx's states with fallback
        to the method (qcx_mlp_infer): (loss [n_w][n_G], err or None, number
        of recomputed frequencies)."""
        import torch

        G = _host(G_int, np.int32).reshape(-1, 3)
        w = _host(w_eV, np.float64).reshape(-1)
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        if loss_out is None:
            loss_out = torch.empty((len(w), len(G)), dtype=torch.float64, device="cuda")
        nfb = ctypes.c_int(0)
        n = len(w) * len(G)
        ctx._check(self.lib.qcx_mlp_infer(
            self._h, ctx._h, len(G), _ptr_host(G), len(w), _ptr_host(w), float(eta_eV), float(tol),
            int(precision), _dev_ptr(loss_out, "f64", n, "loss_out"),
            None if err_out is None else _dev_ptr(err_out, "f64", n, "err_out"), ctypes.byref(nfb)))
        return loss_out, err_out, nfb.value


class QBins:
    """Momentum binning of eps(w, q+G), isotropic S(w, q) and the halo rate
    (qcx_qbin_*) on a Context's device and stream.  Momenta in bohr^-1
    (= alpha m_e); paper defaults n_theta = 9, n_phi = 16, dq = 0.02."""

    def __init__(self, ctx: Context, n_w: int, n_shell: int, dq: float = 0.02,
                 n_theta: int = 9, n_phi: int = 16):
        self.ctx, self.lib = ctx, ctx.lib
        self.n_w, self.n_shell, self.dq = n_w, n_shell, dq
        self.n_bins = n_shell * n_theta * n_phi
        h = ctypes.c_void_p()
        ctx._check(self.lib.qcx_qbin_create(ctypes.byref(h), ctx._h, n_w, n_shell, float(dq),
                                            n_theta, n_phi))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.qcx_qbin_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        self.ctx._check(self.lib.qcx_qbin_reset(self._h))

    def add(self, qvec, vals, kind: str = "inv"):
        """qvec: host [n][3]; vals: CUDA complex128 [n_w][n] (eps, or 1/eps for kind "inv")."""
        q = _host(qvec, np.float64).reshape(-1, 3)
        n = len(q)
        ld = vals.shape[-1] if hasattr(vals, "shape") else n
        self.ctx._check(self.lib.qcx_qbin_add(self._h, n, _ptr_host(q),
                                              _dev_ptr(vals, "c128", self.n_w * ld, "vals"), ld,
                                              QBIN_INV if kind == "inv" else QBIN_EPS))

    def finish(self, want_eps: bool = False):
        """(S_iso CUDA float64 [n_w][n_shell], state numpy [bins], eps CUDA or None)."""
        import torch

        S = torch.empty((self.n_w, self.n_shell), dtype=torch.float64, device="cuda")
        eps = (torch.empty((self.n_w, self.n_bins), dtype=torch.complex128, device="cuda")
               if want_eps else None)
        state = np.zeros(self.n_bins, np.int32)
        self.ctx._check(self.lib.qcx_qbin_finish(
            self._h, None if eps is None else _dev_ptr(eps, "c128", eps.numel(), "eps"),
            _dev_ptr(S, "f64", S.numel(), "S"), _ptr_host(state)))
        return S, state, eps

    def rate_halo(self, w_eV, S_iso, m_chi_eV: float, m_med_eV: float = float("inf"),
                  sigma_e_cm2: float = 1e-39, rho_T_g_cm3: float = 2.33,
                  rho_chi_GeV_cm3: float = 0.3, v0_kms: float = 238.0, vE_kms: float = 250.2,
                  vesc_kms: float = 544.0):
        """dR/dw (events / kg / year / eV), CUDA float64 [n_w]."""
        import torch

        w = _host(w_eV, np.float64).reshape(-1)
        h = QcxHalo(m_chi_eV, m_med_eV, sigma_e_cm2, rho_T_g_cm3, rho_chi_GeV_cm3, v0_kms, vE_kms,
                    vesc_kms)
        out = torch.empty(self.n_w, dtype=torch.float64, device="cuda")
        self.ctx._check(self.lib.qcx_qbin_rate_halo(self._h, _ptr_host(w),
                                                    _dev_ptr(S_iso, "f64", self.n_w * self.n_shell, "S_iso"),
                                                    ctypes.byref(h), _dev_ptr(out, "f64", self.n_w, "out")))
        return out


def build_info() -> str:
    return load_library().qcx_build_info().decode()
