"""ctypes loader for libqhvp.so (the gfx950 HIP library behind include/qhvp.h).

Argument marshalling only; every step of the computation runs in the
library.  There is no fallback: if the library is missing, importing this
module raises.
"""
from __future__ import annotations

import ctypes as C
import os

# PyTorch-ROCm ships its own HIP and HSA runtimes under the same sonames as the system ROCm ones
# that libqhvp.so links.  Loading torch first makes the library bind to torch's runtime, so the
# process holds one HIP runtime and device memory is shared freely; loaded the other way round the
# process would hold two, and whichever initialised second would find no device.
import torch  # noqa: F401  (load order only)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QHVP_LIB", os.path.join(_HERE, "libqhvp.so"))

QHVP_OK, QHVP_ERR_INVALID, QHVP_ERR_NOMEM, QHVP_ERR_DEVICE, QHVP_ERR_UNSUPPORTED = range(5)
QHVP_C128, QHVP_C64_ACC64 = 0, 1
QHVP_CKPT_REBUILD = -(1 << 30)
QHVP_DEV_NONFINITE, QHVP_DEV_NOT_UNITARY, QHVP_DEV_NOT_INVERTIBLE = 1, 2, 4
QHVP_EUCLIDEAN, QHVP_RIEMANNIAN = 0, 1

_STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "UNSUPPORTED"}


class QhvpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qhvp {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libqhvp.so not found at {LIB_PATH}; build it with "
                      f"`python -c 'import __graft_entry__ as g; g.build()'`")

lib = C.CDLL(LIB_PATH)

_dp = C.POINTER(C.c_double)
_vp = C.c_void_p
_ip = C.POINTER(C.c_int)
_szp = C.POINTER(C.c_size_t)

_SIGS = {
    "qhvp_version": (C.c_int, []),
    "qhvp_last_error": (C.c_char_p, []),
    "qhvp_num_gates": (C.c_int, [C.c_int, C.c_int]),
    "qhvp_plan": (C.c_int, [C.c_int, C.c_int, C.c_int, _ip, _ip]),
    "qhvp_ctx_create": (C.c_int, [C.c_int, C.POINTER(_vp)]),
    "qhvp_ctx_destroy": (None, [_vp]),
    "qhvp_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "qhvp_problem_create": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _dp, _dp, C.c_int, C.c_int, C.c_int,
                                      C.c_int, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "qhvp_problem_destroy": (None, [_vp]),
    "qhvp_cost": (C.c_int, [_vp, _dp, _dp, _dp]),
    "qhvp_grad": (C.c_int, [_vp, _dp, C.c_int, _dp, _dp, _dp]),
    "qhvp_hvp": (C.c_int, [_vp, _dp, _dp, C.c_int, _dp, _dp, _dp, _dp]),
    "qhvp_cost_dev": (C.c_int, [_vp, _vp, _vp, _vp]),
    "qhvp_grad_dev": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, _vp]),
    "qhvp_hvp_dev": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp, _vp, _vp, _vp]),
    "qhvp_forward_dev": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp, _vp]),
    "qhvp_backward_dev": (C.c_int, [_vp, _vp, _vp]),
    "qhvp_device_status": (C.c_int, [_vp, _ip]),
    "qhvp_hvp_noalloc": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int, C.c_int, _vp, _vp, C.c_int,
                                   _vp, _vp, _vp, _vp, _vp]),
    "qhvp_hvp_batch": (C.c_int, [_vp, _dp, C.c_int, _dp, C.c_int, _dp, _dp, _dp]),
    "qhvp_states_kept_for": (C.c_int, [_vp, _dp]),
    "qhvp_forward": (C.c_int, [_vp, _dp, _dp, C.c_int, _dp, _dp]),
    "qhvp_backward": (C.c_int, [_vp, _dp, _dp]),
    "qhvp_grad_ti": (C.c_int, [_vp, _dp, C.c_int, _dp, _dp, _dp]),
    "qhvp_hvp_ti": (C.c_int, [_vp, _dp, _dp, C.c_int, _dp, _dp, _dp, _dp]),
    "qhvp_grad_ti_dev": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, _vp]),
    "qhvp_hvp_ti_dev": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp, _vp, _vp, _vp]),
    "qhvp_overlaps": (C.c_int, [_vp, _dp, _dp]),
    "qhvp_problem_info": (C.c_int, [_vp, _ip, _ip, _szp, _ip]),
    "qhvp_last_device_ms": (C.c_double, [_vp]),
    "qhvp_backward_from_outputs": (C.c_int, [_vp]),
    "qhvp_set_profiling": (C.c_int, [_vp, C.c_int]),
    "qhvp_kernel_stats": (C.c_int, [_vp, C.c_int, _dp, C.POINTER(C.c_longlong), _dp, _dp]),
    "qhvp_project": (C.c_int, [C.c_int, _dp, _dp, _dp]),
    "qhvp_riemannian_hvp": (C.c_int, [C.c_int, _dp, _dp, _dp, _dp, _dp]),
    "qhvp_retract": (C.c_int, [C.c_int, _dp, _dp, _dp]),
    "qhvp_unitarity_error": (C.c_double, [C.c_int, _dp]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def check(status: int) -> None:
    if status != QHVP_OK:
        raise QhvpError(status, lib.qhvp_last_error().decode())


def dptr(a):
    """double* of a C-contiguous float64 numpy array (or None)."""
    if a is None:
        return None
    return a.ctypes.data_as(_dp)
