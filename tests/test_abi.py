"""The C-ABI library loads and exports every symbol include/qcx.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qcx.h")
LIB = os.path.join(ROOT, "paper_2603_12326_amd", "libqcx.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qcx_\w+)\s*\(", text)))


def test_header_declares_the_path_calls():
    syms = declared_symbols()
    for name in ("qcx_create", "qcx_destroy", "qcx_set_cell_basis", "qcx_set_states",
                 "qcx_pair_density", "qcx_chi0", "qcx_eps_inv", "qcx_loss", "qcx_last_error"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcx.so not built")
def test_binding_covers_every_declared_symbol():
    from paper_2603_12326_amd import qcx

    assert sorted(qcx.exported_symbols()) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcx.so not built")
def test_create_without_gpu_fails_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2603_12326_amd import qcx

    lib = qcx.load_library()
    h = ctypes.c_void_p()
    rc = lib.qcx_create(ctypes.byref(h), 0, None)
    assert rc in (qcx.EINVAL, qcx.EDEVICE)
    assert lib.qcx_last_error(None)
