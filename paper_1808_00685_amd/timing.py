"""HIP events through libamdhip64 for kernel timing.

The library records such events on the stream its kernels run on (see
corr2d_set_timing_events); torch's own events only see torch's current
stream.
"""
from __future__ import annotations

import ctypes


class HipEvents:
    """Create, read and destroy hipEvent_t handles."""

    def __init__(self):
        self.h = ctypes.CDLL("libamdhip64.so")
        self.h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.h.hipEventSynchronize.argtypes = [ctypes.c_void_p]

    def create(self, n):
        evs = []
        for _ in range(n):
            e = ctypes.c_void_p()
            if self.h.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            evs.append(e.value)
        return evs

    def elapsed_ms(self, a, b):
        self.h.hipEventSynchronize(b)
        t = ctypes.c_float()
        if self.h.hipEventElapsedTime(ctypes.byref(t), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(t.value)

    def destroy(self, evs):
        for e in evs:
            self.h.hipEventDestroy(e)
