"""Batched RK2 stepping of many particle sets (one persistent launch per
step, optionally replayed from a hipGraph) and its autotuner."""
import ctypes

import numpy as np

from ._lib import check, lib
from .particles import current_stream

PER_SET, PERSISTENT, GRAPH = 0, 1, 2


class Batch:
    def __init__(self, sets):
        self.sets = list(sets)  # keep the sets (and their memory) alive
        arr = (ctypes.c_void_p * len(self.sets))(*[s.handle for s in self.sets])
        h = ctypes.c_void_p()
        check(lib().soax_batch_create(arr, len(self.sets), ctypes.byref(h)), "soax_batch_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().soax_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dt, abc, nsteps, mode=GRAPH):
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        abc = np.ascontiguousarray(abc, dtype=np.float64).reshape(-1)
        assert dt.size == len(self.sets) and abc.size == 3 * len(self.sets)
        check(lib().soax_batch_step(self.handle, dt.ctypes.data, abc.ctypes.data, int(nsteps),
                                    int(mode), current_stream()), "soax_batch_step")

    def config(self, block=0, per_thread=0, blocks_per_cu=0):
        check(lib().soax_batch_config(self.handle, block, per_thread, blocks_per_cu),
              "soax_batch_config")

    def get_config(self):
        v = [ctypes.c_int32() for _ in range(3)]
        check(lib().soax_batch_get_config(self.handle, *[ctypes.byref(x) for x in v]),
              "soax_batch_get_config")
        return tuple(x.value for x in v)

    def tune(self, cache_path=None):
        """Time candidate kernel shapes on this batch (its particles are left
        as they were) with the dt and amplitudes of the most recent step(),
        keep the fastest and return it as (block, per_thread, blocks_per_cu)."""
        check(lib().soax_batch_tune(self.handle, cache_path.encode() if cache_path else None),
              "soax_batch_tune")
        return self.get_config()
