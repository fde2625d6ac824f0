"""Raw HIP events through the HIP runtime (timing plumbing for cmc_step_timed)."""
from __future__ import annotations

import ctypes as C
import ctypes.util
import os

_hip = None


def hip() -> C.CDLL:
    global _hip
    if _hip is None:
        # the soname first, so the runtime torch already loaded is reused
        cands = ["libamdhip64.so.7",
                 os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "libamdhip64.so"),
                 ctypes.util.find_library("amdhip64") or "libamdhip64.so"]
        err = None
        for c in cands:
            try:
                _hip = C.CDLL(c)
                break
            except OSError as e:  # try the next location
                err = e
        if _hip is None:
            raise OSError(f"HIP runtime not found: {err}")
        _hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        _hip.hipEventDestroy.argtypes = [C.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        _hip.hipEventSynchronize.argtypes = [C.c_void_p]
    return _hip


class EventSet:
    """``count`` HIP events; elapsed(i, j) in milliseconds."""

    def __init__(self, count: int):
        self.h = []
        for _ in range(count):
            e = C.c_void_p()
            if hip().hipEventCreate(C.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.h.append(e.value)

    def elapsed(self, i: int, j: int) -> float:
        ms = C.c_float()
        hip().hipEventSynchronize(self.h[j])
        if hip().hipEventElapsedTime(C.byref(ms), self.h[i], self.h[j]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for e in self.h:
            hip().hipEventDestroy(e)
        self.h = []
