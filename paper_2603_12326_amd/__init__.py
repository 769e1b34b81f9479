"""MI355X (gfx950) library for the hot path of all-electron RPA screening with
local field effects: Gaussian-orbital pair densities -> chi0 on MFMA (FP32 or
split-BF16, FP64 head and wings) -> FP64 inversion of eps -> loss Im[-1/eps].

The compute runs in libqcx.so (HIP, built by `python -m
paper_2603_12326_amd.build`); `qcx.Context` is a thin ctypes binding over its C
ABI (include/qcx.h).
"""
from .qcx import (  # noqa: F401
    FP32,
    FP64,
    SPLIT_BF16,
    Context,
    Mlp,
    QBins,
    QcxError,
    batch_sync,
    run_batch,
    build_info,
    exported_symbols,
    load_library,
)
