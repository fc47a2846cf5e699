"""Tensor wrapper of the separate-chaining backend kept for the backend
ablation (include/ash_slab.h; Sec. 4.4 and Sec. 5.3 of the paper).  Used by
the ablation benchmark and its tests only; the product map is HashMap."""
import ctypes

import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class SlabMap:
    """int32 keys of key_dim words -> one value row of value_bytes (0: a set)."""

    def __init__(self, capacity, key_dim=3, value_bytes=0):
        self._lib = L.load()
        self.key_dim, self.value_bytes = int(key_dim), int(value_bytes)
        self._m = ctypes.c_void_p()
        L.check(self._lib.ash_slab_create(int(capacity), self.key_dim, self.value_bytes, _stream(),
                                          ctypes.byref(self._m)), "ash_slab_create")
        self.capacity = int(capacity)

    def close(self):
        m = getattr(self, "_m", None)
        if m is not None and m.value:
            self._m = None
            self._lib.ash_slab_destroy(m)

    def __del__(self):
        self.close()

    def insert(self, keys, values=None):
        n = keys.shape[0]
        idx = torch.empty(n, dtype=torch.int32, device="cuda")
        mask = torch.empty(n, dtype=torch.uint8, device="cuda")
        vp = ctypes.c_void_p(values.data_ptr()) if values is not None else None
        st = self._lib.ash_slab_insert(self._m, ctypes.c_void_p(keys.data_ptr()), n, vp,
                                       ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(mask.data_ptr()), _stream())
        return st, idx, mask

    def find(self, keys, gather=False):
        n = keys.shape[0]
        idx = torch.empty(n, dtype=torch.int32, device="cuda")
        mask = torch.empty(n, dtype=torch.uint8, device="cuda")
        out = torch.zeros((n, self.value_bytes), dtype=torch.uint8, device="cuda") if gather else None
        L.check(self._lib.ash_slab_find(self._m, ctypes.c_void_p(keys.data_ptr()), n, ctypes.c_void_p(idx.data_ptr()),
                                        ctypes.c_void_p(mask.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()) if out is not None else None, _stream()),
                "ash_slab_find")
        return idx, mask, out

    def size(self):
        t = ctypes.c_int64()
        L.check(self._lib.ash_slab_size(self._m, ctypes.byref(t), _stream()), "ash_slab_size")
        return t.value

    def buffers(self):
        """Device addresses of k^B ([c, key_dim] int32), v^B ([c, value_bytes],
        0 for a set) and the heap ([c] int32)."""
        kb, vb, hp = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        L.check(self._lib.ash_slab_buffers(self._m, ctypes.byref(kb), ctypes.byref(vb), ctypes.byref(hp)),
                "ash_slab_buffers")
        return kb.value or 0, vb.value or 0, hp.value or 0

    def read(self):
        """Host copies of (k^B, v^B or None, heap): the map owns them (hipMalloc),
        so they are copied out through the runtime torch uses."""
        import numpy as np
        kb, vb, hp = self.buffers()
        c = self.capacity
        lib = ctypes.CDLL("libamdhip64.so")
        lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        torch.cuda.synchronize()

        def copy(ptr, nbytes):
            out = np.empty(nbytes, np.uint8)
            if nbytes:
                assert lib.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0  # device to host
            return out
        k = copy(kb, c * self.key_dim * 4).view(np.int32).reshape(c, self.key_dim)
        v = copy(vb, c * self.value_bytes).reshape(c, self.value_bytes) if self.value_bytes else None
        h = copy(hp, c * 4).view(np.int32)
        return k, v, h
