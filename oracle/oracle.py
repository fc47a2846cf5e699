"""ctypes wrapper of liboracle.so (test infrastructure only; see ash_oracle.h).

Every array crossing the boundary is a C-contiguous numpy array in host
memory.  build_oracle() compiles ash_oracle.cpp with g++ -O2 (no fast-math, so
binary32 division and floor keep their IEEE meaning).
"""
import ctypes
import os
import subprocess

import numpy as np

ORACLE_OK = 0
ORACLE_E_INVALID = 1
ORACLE_E_CAPACITY = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ash_oracle.cpp")
# A test may point the wrapper at a deliberately broken build of the oracle
# (mutation check of the pins) through ASH_ORACLE_LIB.
_LIB = os.environ.get("ASH_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build_oracle(src=_SRC, out=_LIB, extra_flags=()):
    """Compile the oracle into a shared library and return its path."""
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
           *extra_flags, "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


_lib_cache = {}


def _load(path=_LIB):
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        build_oracle(out=path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    lib.oracle_create.argtypes = [i64, i32, i32, P, ctypes.POINTER(P)]
    lib.oracle_create.restype = ctypes.c_int
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_destroy.restype = None
    lib.oracle_insert.argtypes = [P, P, i64, P, P, P, ctypes.c_int]
    lib.oracle_insert.restype = ctypes.c_int
    lib.oracle_activate.argtypes = [P, P, i64, P, P, ctypes.c_int]
    lib.oracle_activate.restype = ctypes.c_int
    lib.oracle_find.argtypes = [P, P, i64, P, P, P]
    lib.oracle_find.restype = ctypes.c_int
    lib.oracle_erase.argtypes = [P, P, i64, P]
    lib.oracle_erase.restype = ctypes.c_int
    lib.oracle_active_indices.argtypes = [P, P]
    lib.oracle_active_indices.restype = i64
    lib.oracle_rehash.argtypes = [P, i64]
    lib.oracle_rehash.restype = ctypes.c_int
    for name in ("oracle_size", "oracle_capacity", "oracle_heap_top"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = i64
    for name in ("oracle_key_buffer", "oracle_heap", "oracle_active_flags"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = P
    lib.oracle_value_buffer.argtypes = [P, i32]
    lib.oracle_value_buffer.restype = P
    lib.oracle_find_offsets.argtypes = [P, P, i64, P, i64, P, P]
    lib.oracle_find_offsets.restype = ctypes.c_int
    lib.oracle_intersect.argtypes = [P, P, i64, P]
    lib.oracle_intersect.restype = i64
    lib.oracle_block_coords.argtypes = [P, i64, ctypes.c_float, i32, P, P, P]
    lib.oracle_block_coords.restype = None
    lib.oracle_voxelize.argtypes = [P, i64, ctypes.c_float, P, P, P]
    lib.oracle_voxelize.restype = i64
    _lib_cache[path] = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _ptr_array(arrs):
    if arrs is None:
        return None, None
    arr = (ctypes.c_void_p * max(len(arrs), 1))(*[a.ctypes.data for a in arrs])
    return arr, ctypes.cast(arr, ctypes.c_void_p)


class OracleMap:
    """Sequential reference hash map: int32 keys of key_dim words, value
    buffers described by (numpy dtype, elements per row)."""

    def __init__(self, capacity, key_dim=3, value_specs=(), lib_path=_LIB):
        self._lib = _load(lib_path)
        self.key_dim = key_dim
        self.value_specs = [(np.dtype(dt), int(e)) for dt, e in value_specs]
        rb = np.array([dt.itemsize * e for dt, e in self.value_specs] or [0], dtype=np.int64)
        self._m = ctypes.c_void_p()
        st = self._lib.oracle_create(int(capacity), key_dim, len(self.value_specs),
                                     rb.ctypes.data, ctypes.byref(self._m))
        if st != ORACLE_OK:
            raise ValueError(f"oracle_create failed with status {st}")

    def __del__(self):
        m = getattr(self, "_m", None)
        if m is not None and m.value:
            self._lib.oracle_destroy(m)
            self._m = None

    def _keys(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, self.key_dim)
        return keys, keys.shape[0]

    def insert(self, keys, values=(), autogrow=False):
        keys, n = self._keys(keys)
        vals = [np.ascontiguousarray(v, dtype=dt).reshape(n, e)
                for v, (dt, e) in zip(values, self.value_specs)]
        if len(vals) != len(self.value_specs):
            raise ValueError("one value array per value buffer is required")
        idx = np.empty(n, np.int32)
        mask = np.empty(n, np.uint8)
        _keep, vp = _ptr_array(vals)
        st = self._lib.oracle_insert(self._m, _ptr(keys), n, vp, _ptr(idx), _ptr(mask), int(autogrow))
        return st, idx, mask

    def activate(self, keys, autogrow=False):
        keys, n = self._keys(keys)
        idx = np.empty(n, np.int32)
        mask = np.empty(n, np.uint8)
        st = self._lib.oracle_activate(self._m, _ptr(keys), n, _ptr(idx), _ptr(mask), int(autogrow))
        return st, idx, mask

    def find(self, keys, gather=False, fill=0):
        keys, n = self._keys(keys)
        idx = np.empty(n, np.int32)
        mask = np.empty(n, np.uint8)
        outs = None
        if gather:
            outs = [np.full((n, e), fill, dtype=dt) for dt, e in self.value_specs]
        _keep, vp = _ptr_array(outs)
        st = self._lib.oracle_find(self._m, _ptr(keys), n, _ptr(idx), _ptr(mask), vp)
        return (st, idx, mask, outs) if gather else (st, idx, mask)

    def erase(self, keys):
        keys, n = self._keys(keys)
        mask = np.empty(n, np.uint8)
        st = self._lib.oracle_erase(self._m, _ptr(keys), n, _ptr(mask))
        return st, mask

    def find_offsets(self, keys, offsets):
        """Finds of keys[q] + offsets[o] (int32 words, wrapping); returns
        (status, idx[n, K], mask[n, K])."""
        keys, n = self._keys(keys)
        offs = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, self.key_dim)
        k = offs.shape[0]
        idx = np.empty((n, k), np.int32)
        mask = np.empty((n, k), np.uint8)
        st = self._lib.oracle_find_offsets(self._m, _ptr(keys), n, _ptr(offs), k, _ptr(idx), _ptr(mask))
        return st, idx, mask

    def intersect(self, keys):
        """The query rows the map holds, in batch order (duplicates kept)."""
        keys, n = self._keys(keys)
        out = np.empty((max(n, 1), self.key_dim), np.int32)
        cnt = self._lib.oracle_intersect(self._m, _ptr(keys), n, _ptr(out))
        if cnt < 0:
            raise ValueError("oracle_intersect rejected its arguments")
        return out[:cnt].copy()

    def active_indices(self):
        out = np.empty(max(self.capacity, 1), np.int32)
        cnt = self._lib.oracle_active_indices(self._m, out.ctypes.data)
        return out[:cnt].copy()

    def rehash(self, new_capacity):
        return self._lib.oracle_rehash(self._m, int(new_capacity))

    @property
    def size(self):
        return int(self._lib.oracle_size(self._m))

    @property
    def capacity(self):
        return int(self._lib.oracle_capacity(self._m))

    @property
    def heap_top(self):
        return int(self._lib.oracle_heap_top(self._m))

    def _view(self, addr, dtype, count):
        if count == 0:
            return np.empty(0, dtype)
        buf = (ctypes.c_char * (count * np.dtype(dtype).itemsize)).from_address(addr)
        return np.frombuffer(buf, dtype=dtype, count=count).copy()

    def key_buffer(self):
        c = self.capacity
        return self._view(self._lib.oracle_key_buffer(self._m), np.int32, c * self.key_dim).reshape(c, self.key_dim)

    def value_buffer(self, j):
        dt, e = self.value_specs[j]
        c = self.capacity
        return self._view(self._lib.oracle_value_buffer(self._m, j), dt, c * e).reshape(c, e)

    def heap(self):
        return self._view(self._lib.oracle_heap(self._m), np.int32, self.capacity)

    def active_flags(self):
        return self._view(self._lib.oracle_active_flags(self._m), np.uint8, self.capacity)


def oracle_voxelize(points, voxel, lib_path=_LIB):
    """Returns (point_voxel[n], voxel_keys[u,3], counts[u])."""
    lib = _load(lib_path)
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    n = pts.shape[0]
    pv = np.empty(n, np.int32)
    vk = np.empty((max(n, 1), 3), np.int32)
    cnt = np.empty(max(n, 1), np.int32)
    u = lib.oracle_voxelize(_ptr(pts), n, ctypes.c_float(np.float32(voxel)), _ptr(pv), _ptr(vk), _ptr(cnt))
    return pv, vk[:u].copy(), cnt[:u].copy()


def oracle_block_coords(points, voxel, res, lib_path=_LIB):
    """Returns (block_keys[n,3], local_coords[n,3], valid[n])."""
    lib = _load(lib_path)
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    n = pts.shape[0]
    bk = np.empty((n, 3), np.int32)
    lc = np.empty((n, 3), np.int32)
    ok = np.empty(n, np.uint8)
    lib.oracle_block_coords(_ptr(pts), n, ctypes.c_float(np.float32(voxel)), int(res), _ptr(bk), _ptr(lc), _ptr(ok))
    return bk, lc, ok
