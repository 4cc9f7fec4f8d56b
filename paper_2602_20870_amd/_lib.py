"""ctypes declarations for libfgfrft.so (the C ABI in include/fgfrft.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgfrft.so")

c_int, c_double, c_size_t, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
P_double = ctypes.POINTER(ctypes.c_double)
P_int = ctypes.POINTER(ctypes.c_int)
P_size_t = ctypes.POINTER(ctypes.c_size_t)

# name -> (restype, argtypes); every symbol declared in include/fgfrft.h
SIGNATURES = {
    "fgfrft_plan_bytes": (c_int, [c_int, c_int, c_int, c_int, P_size_t, P_size_t]),
    "fgfrft_plan": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_double, c_void_p, c_size_t, c_void_p,
                            c_size_t, c_void_p, ctypes.POINTER(c_void_p)]),
    "fgfrft_plan_info": (c_int, [c_void_p, P_int, P_double, P_double, P_double, P_double, P_double]),
    "fgfrft_plan_buffers": (c_int, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    "fgfrft_destroy": (None, [c_void_p]),
    "fgfrft_update_workspace_bytes": (c_size_t, [c_void_p, c_int]),
    "fgfrft_update": (c_int, [c_void_p, P_double, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "fgfrft_update_dev": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "fgfrft_update_dev_static": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "fgfrft_apply_operator_workspace_bytes": (c_size_t, [c_int, c_int, c_int, c_int]),
    "fgfrft_apply_operator": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_int, c_int, c_void_p,
                                      c_int, c_void_p, c_size_t, c_void_p]),
    "fgfrft_apply_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "fgfrft_apply": (c_int, [c_void_p, P_double, c_int, c_void_p, c_int, c_int, c_int, c_void_p, c_int,
                             c_void_p, c_size_t, c_void_p]),
    "fgfrft_apply_direct_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int]),
    "fgfrft_apply_direct": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p,
                                    c_int, c_void_p, c_size_t, c_void_p]),
    "fgfrft_apply_batched_workspace_bytes": (c_size_t, [c_void_p, c_int, P_int, c_int]),
    "fgfrft_apply_batched": (c_int, [c_void_p, P_double, c_int, P_int, ctypes.POINTER(c_void_p), c_int,
                                     ctypes.POINTER(c_void_p), c_void_p, c_size_t, c_void_p]),
    "fgfrft_grad_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int]),
    "fgfrft_grad": (c_int, [c_void_p, P_double, c_int, c_void_p, c_int, c_int, c_int, c_void_p, P_double,
                            c_void_p, c_void_p, c_size_t, c_void_p]),
    "fgfrft_gfrft_exact_workspace_bytes": (c_size_t, [c_int]),
    "fgfrft_gfrft_exact": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
    "fgfrft_apply_dev_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int, c_int]),
    "fgfrft_apply_dev": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p,
                                 c_size_t, c_void_p]),
    "fgfrft_probe_write": (c_int, [c_void_p, c_size_t, c_void_p]),
    "fgfrft_probe_update_traffic": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p]),
    "fgfrft_strerror": (ctypes.c_char_p, [c_int]),
    "fgfrft_last_error": (ctypes.c_char_p, []),
}

STATUS = {0: "FGFRFT_OK", -1: "FGFRFT_EINVAL", -2: "FGFRFT_ENOTUNITARY", -3: "FGFRFT_EALPHA",
          -4: "FGFRFT_ENOMEM", -5: "FGFRFT_EHIP", -6: "FGFRFT_EDRIFT", -7: "FGFRFT_EUNSUPPORTED"}

_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2602_20870_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class FGFRFTError(RuntimeError):
    def __init__(self, status: int, where: str):
        detail = lib().fgfrft_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)} ({detail})")
        self.status = status
        self.name = STATUS.get(status, str(status))


def check(status: int, where: str) -> None:
    if status != 0:
        raise FGFRFTError(status, where)
