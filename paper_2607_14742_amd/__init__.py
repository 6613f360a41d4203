"""MI355X (gfx950) mixed-precision Newton refinement for large sparse CAREs.

The computation lives in the HIP library libmpcare.so (C ABI in
include/mpcare.h); this package only marshals arguments.  Importing it does
not load the library; the first call does, and fails loudly when the library
has not been built.
"""
from ._lib import (CARE_AUTO, CARE_BF16_SPMM, CARE_FP16_SPMM, CARE_ERR_ARG, CARE_ERR_BREAKDOWN, CARE_ERR_CAPACITY,  # noqa: F401
                   CARE_ERR_NONFINITE, CARE_ERR_UNSTABLE, CARE_FP32, CARE_FP64, LIB_PATH, SIGNATURES, STATUS_NAMES,
                   load)

__all__ = ["load", "LIB_PATH", "SIGNATURES", "STATUS_NAMES", "CARE_FP64", "CARE_FP32", "CARE_BF16_SPMM", "CARE_FP16_SPMM", "CARE_AUTO",
           "CARE_ERR_ARG", "CARE_ERR_CAPACITY", "CARE_ERR_UNSTABLE", "CARE_ERR_BREAKDOWN", "CARE_ERR_NONFINITE"]


def __getattr__(name):
    # the torch-based API is imported lazily so that the CPU-only checks
    # (library loads, symbols exported) do not need torch
    import importlib
    if name in ("api", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    if name.startswith("__"):
        raise AttributeError(name)
    api = importlib.import_module(f"{__name__}.api")
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)
