"""MI355X (gfx950) implementation of the hot path of the sixth-order Hermite,
block-time-step, direct-summation N-body method of arXiv:1207.2367.

The work runs in the HIP kernels of ``libnbody.so`` behind the C ABI of
``include/nbody.h``; :mod:`paper_1207_2367_amd.nbody` is a thin ctypes
binding of that ABI (argument marshalling only) that takes torch device
tensors.  There is no CPU path: without the built library every call fails.
"""
from .nbody import (  # noqa: F401
    NBodyError, System, default_config, lib_path, load, workspace_bytes,
    PREC_MIXED, PREC_FP64, PREC_FP32PAIR,
)
