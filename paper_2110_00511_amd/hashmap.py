"""Tensor interface of the MI355X hash map (ASH, arXiv 2110.00511).

As in the paper's tensor interface (Sec. 3, Fig. 1), every call returns buffer
indices and masks; keys and values are read and modified in place through
the key / value buffers (advanced indexing with the returned indices).
Inputs and outputs are torch tensors on the GPU; all work runs in libash.so.
"""
import atexit
import ctypes
import weakref

import torch

from . import _lib as L

# Maps and servers still alive when the interpreter exits are released by an
# exit hook, while torch and the HIP runtime are still whole (servers first:
# they own a map's stream).  Their __del__ is then a no-op.
_LIVE_SERVERS = weakref.WeakSet()
_LIVE_MAPS = weakref.WeakSet()


@atexit.register
def _release_all():
    for s in list(_LIVE_SERVERS):
        try:
            s.close()
        except Exception:
            pass
    for m in list(_LIVE_MAPS):
        try:
            m.close()
        except Exception:
            pass

_DTYPES = {
    torch.uint8: L.ASH_U8, torch.int32: L.ASH_I32, torch.float32: L.ASH_F32, torch.int64: L.ASH_I64,
    torch.float64: L.ASH_F64, torch.float16: L.ASH_F16, torch.bfloat16: L.ASH_BF16,
}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _keys(keys, key_dim, device):
    if not (keys.is_cuda and keys.dtype == torch.int32):
        raise TypeError("keys must be an int32 tensor on the GPU")
    keys = keys.reshape(-1, key_dim)
    if not keys.is_contiguous():
        keys = keys.contiguous()
    return keys


class HashMap:
    """int32 keys of `key_dim` words -> one or more value buffers.

    value_specs: sequence of (torch dtype, elements per row).  Tuning:
    bucket_width W, probe_group g (lanes per key), max_load, autogrow."""

    def __init__(self, capacity, key_dim=3, value_specs=(), device="cuda", bucket_width=4, probe_group=4,
                 max_load=0.5, autogrow=False, lds_dedup=False):
        self._lib = L.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.key_dim = int(key_dim)
        self.value_specs = [(dt, int(e)) for dt, e in value_specs]
        n = len(self.value_specs)
        dts = (ctypes.c_int * max(n, 1))(*[_DTYPES[dt] for dt, _ in self.value_specs])
        els = (ctypes.c_int64 * max(n, 1))(*[e for _, e in self.value_specs])
        self._alloc = L.TorchAllocator(self.device)
        flags = (L.ASH_F_AUTOGROW if autogrow else 0) | (L.ASH_F_LDS_DEDUP if lds_dedup else 0)
        tun = L.AshTuning(bucket_width, probe_group, max_load, flags)
        self._m = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self._lib.ash_create(int(capacity), self.key_dim, n, ctypes.cast(dts, ctypes.c_void_p),
                                         ctypes.cast(els, ctypes.c_void_p), ctypes.byref(self._alloc.struct),
                                         ctypes.byref(tun), _stream(), ctypes.byref(self._m)), "ash_create")
        _LIVE_MAPS.add(self)

    def save(self, path):
        """Writes the map's state (capacity, heap, live indices, keys, value
        rows) to a file; synchronizes."""
        L.check(self._lib.ash_save(self._m, str(path).encode(), _stream()), "ash_save")

    @classmethod
    def load(cls, path, device="cuda", bucket_width=4, probe_group=4, max_load=0.5, autogrow=False, lds_dedup=False):
        """A map holding exactly the state a file was saved with (same
        indices, heap and rows), with the given table tuning."""
        self = cls.__new__(cls)
        self._lib = L.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._alloc = L.TorchAllocator(self.device)
        flags = (L.ASH_F_AUTOGROW if autogrow else 0) | (L.ASH_F_LDS_DEDUP if lds_dedup else 0)
        tun = L.AshTuning(bucket_width, probe_group, max_load, flags)
        self._m = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self._lib.ash_load(str(path).encode(), ctypes.byref(self._alloc.struct), ctypes.byref(tun),
                                       _stream(), ctypes.byref(self._m)), "ash_load")
        _LIVE_MAPS.add(self)
        kd, nv = ctypes.c_int32(), ctypes.c_int32()
        L.check(self._lib.ash_describe(self._m, ctypes.byref(kd), ctypes.byref(nv), None, None), "ash_describe")
        dts = (ctypes.c_int * max(nv.value, 1))()
        els = (ctypes.c_int64 * max(nv.value, 1))()
        L.check(self._lib.ash_describe(self._m, ctypes.byref(kd), ctypes.byref(nv), ctypes.cast(dts, ctypes.c_void_p),
                                       ctypes.cast(els, ctypes.c_void_p)), "ash_describe")
        codes = {v: k for k, v in _DTYPES.items()}
        self.key_dim = kd.value
        self.value_specs = [(codes[dts[j]], int(els[j])) for j in range(nv.value)]
        return self

    def close(self):
        """Destroys the map now (its buffers return to torch's allocator)."""
        m = getattr(self, "_m", None)
        if m is not None and m.value:
            self._m = None
            self._lib.ash_destroy(m)

    def __del__(self):
        self.close()

    # -- operations ---------------------------------------------------------
    def insert(self, keys, values=()):
        keys = _keys(keys, self.key_dim, self.device)
        n = keys.shape[0]
        if len(values) != len(self.value_specs):
            raise ValueError("one value tensor per value buffer is required")
        vals = []
        for v, (dt, e) in zip(values, self.value_specs):
            if v.dtype != dt or not v.is_cuda:
                raise TypeError(f"value tensor must be {dt} on the GPU")
            vals.append(v.reshape(n, e).contiguous())
        idx = torch.empty(n, dtype=torch.int32, device=self.device)
        mask = torch.empty(n, dtype=torch.uint8, device=self.device)
        arr = (ctypes.c_void_p * max(len(vals), 1))(*[v.data_ptr() for v in vals])
        L.check(self._lib.ash_insert(self._m, _ptr(keys), n, ctypes.cast(arr, ctypes.c_void_p) if vals else None,
                                     _ptr(idx), _ptr(mask), _stream()), "ash_insert")
        return idx, mask.bool()

    def activate(self, keys):
        keys = _keys(keys, self.key_dim, self.device)
        n = keys.shape[0]
        idx = torch.empty(n, dtype=torch.int32, device=self.device)
        mask = torch.empty(n, dtype=torch.uint8, device=self.device)
        L.check(self._lib.ash_activate(self._m, _ptr(keys), n, _ptr(idx), _ptr(mask), _stream()), "ash_activate")
        return idx, mask.bool()

    def find(self, keys, gather=False, out_values=None):
        keys = _keys(keys, self.key_dim, self.device)
        n = keys.shape[0]
        idx = torch.empty(n, dtype=torch.int32, device=self.device)
        mask = torch.empty(n, dtype=torch.uint8, device=self.device)
        outs = None
        if gather:
            outs = out_values if out_values is not None else [
                torch.zeros((n, e), dtype=dt, device=self.device) for dt, e in self.value_specs]
        arr = (ctypes.c_void_p * max(len(outs or []), 1))(*[o.data_ptr() for o in (outs or [])])
        L.check(self._lib.ash_find(self._m, _ptr(keys), n, _ptr(idx), _ptr(mask),
                                   ctypes.cast(arr, ctypes.c_void_p) if outs else None, _stream()), "ash_find")
        return (idx, mask.bool(), outs) if gather else (idx, mask.bool())

    def erase(self, keys):
        keys = _keys(keys, self.key_dim, self.device)
        n = keys.shape[0]
        mask = torch.empty(n, dtype=torch.uint8, device=self.device)
        L.check(self._lib.ash_erase(self._m, _ptr(keys), n, _ptr(mask), _stream()), "ash_erase")
        return mask.bool()

    def find_offsets(self, keys, offsets):
        """Neighbor lookups: finds of keys[q] + offsets[o] (int32, wrapping),
        returned as (idx[n, K], mask[n, K]) (Listing 3, Sec. 6.2.4)."""
        keys = _keys(keys, self.key_dim, self.device)
        offsets = _keys(offsets, self.key_dim, self.device)
        n, k = keys.shape[0], offsets.shape[0]
        idx = torch.empty((n, k), dtype=torch.int32, device=self.device)
        mask = torch.empty((n, k), dtype=torch.uint8, device=self.device)
        L.check(self._lib.ash_find_offsets(self._m, _ptr(keys), n, _ptr(offsets), k, _ptr(idx), _ptr(mask),
                                           _stream()), "ash_find_offsets")
        return idx, mask.bool()

    def intersect(self, keys):
        """The rows of keys that the map holds, in order, duplicates kept
        (Sec. 6.4)."""
        keys = _keys(keys, self.key_dim, self.device)
        n = keys.shape[0]
        out = torch.empty((max(n, 1), self.key_dim), dtype=torch.int32, device=self.device)
        cnt = ctypes.c_int64()
        L.check(self._lib.ash_intersect(self._m, _ptr(keys), n, _ptr(out), ctypes.byref(cnt), _stream()),
                "ash_intersect")
        return out[: cnt.value]

    def active_indices(self):
        out = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.device)
        cnt = ctypes.c_int64()
        L.check(self._lib.ash_active_indices(self._m, _ptr(out), ctypes.byref(cnt), _stream()), "ash_active_indices")
        return out[: cnt.value]

    def rehash(self, new_capacity):
        L.check(self._lib.ash_rehash(self._m, int(new_capacity), _stream()), "ash_rehash")

    def clear(self):
        L.check(self._lib.ash_clear(self._m, _stream()), "ash_clear")

    def device_status(self):
        """Returns and clears the sticky device error as a status code."""
        return self._lib.ash_device_status(self._m, _stream())

    def profile(self, enable=True):
        """Brackets every kernel launch of this map with HIP events."""
        L.check(self._lib.ash_profile_enable(self._m, 1 if enable else 0), "ash_profile_enable")

    def profile_collect(self):
        """{kernel name: (launches, total milliseconds)} since the last collect."""
        buf = (L.AshKernelTime * 32)()
        n = ctypes.c_int32()
        L.check(self._lib.ash_profile_collect(self._m, buf, 32, ctypes.byref(n), _stream()), "ash_profile_collect")
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(n.value)}

    # -- state --------------------------------------------------------------
    def size(self):
        out = ctypes.c_int64()
        L.check(self._lib.ash_size(self._m, ctypes.byref(out), _stream()), "ash_size")
        return out.value

    @property
    def capacity(self):
        out = ctypes.c_int64()
        L.check(self._lib.ash_capacity(self._m, ctypes.byref(out)), "ash_capacity")
        return out.value

    def stats(self):
        s = L.AshStats()
        L.check(self._lib.ash_stats(self._m, ctypes.byref(s), _stream()), "ash_stats")
        return dict(size=s.size, capacity=s.capacity, slots=s.slots, used_slots=s.used_slots, tombstones=s.tombstones)

    def _view(self, ptr, dtype, shape):
        count = 1
        for d in shape:
            count *= d
        base = self._alloc.tensor(ptr)
        return base.view(dtype)[:count].view(*shape)

    def key_buffer(self):
        """k^B as a [capacity, key_dim] int32 tensor sharing the map's memory."""
        p = ctypes.c_void_p()
        L.check(self._lib.ash_key_buffer(self._m, ctypes.byref(p)), "ash_key_buffer")
        return self._view(p.value, torch.int32, (self.capacity, self.key_dim))

    def value_buffer(self, j=0):
        """v^B_j as a [capacity, elems] tensor sharing the map's memory."""
        p = ctypes.c_void_p()
        L.check(self._lib.ash_value_buffer(self._m, j, ctypes.byref(p)), "ash_value_buffer")
        dt, e = self.value_specs[j]
        return self._view(p.value, dt, (self.capacity, e))

    def heap_buffer(self):
        """Index heap h as a [capacity] int32 tensor (t = size())."""
        p = ctypes.c_void_p()
        L.check(self._lib.ash_heap_buffer(self._m, ctypes.byref(p)), "ash_heap_buffer")
        return self._view(p.value, torch.int32, (self.capacity,))


class HashSet(HashMap):
    """Hash map without value buffers (Sec. 4.7)."""

    def __init__(self, capacity, key_dim=3, **kw):
        super().__init__(capacity, key_dim=key_dim, value_specs=(), **kw)


NEIGHBORHOODS = {"radius": L.ASH_NB_RADIUS, "cube": L.ASH_NB_CUBE, "ring": L.ASH_NB_RING}


def neighbor_offsets(kind="radius", radius=1, key_dim=3, device="cuda"):
    """Offset table of a standard neighborhood ("radius": every word in
    [-r, r]; "cube": every word in [0, r]; "ring": nonzero offsets with L1
    norm <= r) as an int32 [K, key_dim] tensor."""
    lib = L.load()
    code = NEIGHBORHOODS[kind]
    cnt = ctypes.c_int64()
    L.check(lib.ash_neighbor_offsets(code, int(radius), int(key_dim), None, ctypes.byref(cnt)), "ash_neighbor_offsets")
    host = (ctypes.c_int32 * max(cnt.value * key_dim, 1))()
    L.check(lib.ash_neighbor_offsets(code, int(radius), int(key_dim), host, ctypes.byref(cnt)), "ash_neighbor_offsets")
    out = torch.tensor(list(host)[: cnt.value * key_dim], dtype=torch.int32).reshape(cnt.value, key_dim)
    return out.to(device) if device is not None else out


def block_coords(points, voxel_size, block_res):
    """(block_keys [n, 3] int32, local [n, 3] int32, valid [n] bool) of
    float32 [n, 3] points on the GPU: the voxel block of res^3 voxels each
    point falls in and its voxel inside that block (Sec. 6.2.2)."""
    if not (points.is_cuda and points.dtype == torch.float32):
        raise TypeError("points must be a float32 tensor on the GPU")
    pts = points.reshape(-1, 3).contiguous()
    n = pts.shape[0]
    bk = torch.empty((n, 3), dtype=torch.int32, device=pts.device)
    lc = torch.empty((n, 3), dtype=torch.int32, device=pts.device)
    ok = torch.empty(n, dtype=torch.uint8, device=pts.device)
    lib = L.load()
    L.check(lib.ash_block_coords(_ptr(pts), n, ctypes.c_float(voxel_size), int(block_res), _ptr(bk), _ptr(lc),
                                 _ptr(ok), _stream()), "ash_block_coords")
    return bk, lc, ok.bool()


def voxelize(points, voxel_size):
    """Point-cloud voxelization (Sec. 6.1): returns (point_voxel [n] int32,
    voxel_keys [u, 3] int32, counts [u] int32), voxels in first-occurrence
    order; rejected points (non-finite or out of int32 range) get -1."""
    lib = L.load()
    if not (points.is_cuda and points.dtype == torch.float32):
        raise TypeError("points must be a float32 tensor on the GPU")
    pts = points.reshape(-1, 3).contiguous()
    n = pts.shape[0]
    dev = pts.device
    pv = torch.empty(n, dtype=torch.int32, device=dev)
    vk = torch.empty((max(n, 1), 3), dtype=torch.int32, device=dev)
    cnt = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    nv = ctypes.c_int64()
    alloc = L.TorchAllocator(dev)
    L.check(lib.ash_voxelize(_ptr(pts), n, ctypes.c_float(float(voxel_size)), _ptr(pv), _ptr(vk), _ptr(cnt),
                             ctypes.byref(nv), ctypes.byref(alloc.struct), _stream()), "ash_voxelize")
    u = nv.value
    return pv, vk[:u], cnt[:u]


def autotune(capacity, n_insert, distinct_ratio, key_dim=3, value_specs=(), device="cuda", batched=False,
             grid=None):
    """Table shape for a map of `capacity` receiving batches of `n_insert`
    keys with the given distinct ratio: times insert + find of a synthetic
    batch for every point of the sweep on this GPU (through the persistent
    batched launch when batched=True).  grid = (widths, groups, loads) sweeps
    that grid instead of the library's default one.  Returns
    (dict(bucket_width, probe_group, max_load), milliseconds)."""
    lib = L.load()
    specs = [(dt, int(e)) for dt, e in value_specs]
    n = len(specs)
    dts = (ctypes.c_int * max(n, 1))(*[_DTYPES[dt] for dt, _ in specs])
    els = (ctypes.c_int64 * max(n, 1))(*[e for _, e in specs])
    alloc = L.TorchAllocator(device)
    out = L.AshTuning()
    ms = ctypes.c_double()
    if grid is not None:
        ws, gs, ls = [list(x) for x in grid]
        wa = (ctypes.c_int32 * len(ws))(*ws)
        ga = (ctypes.c_int32 * len(gs))(*gs)
        la = (ctypes.c_float * len(ls))(*ls)
        L.check(lib.ash_autotune_sweep(int(capacity), int(key_dim), n, ctypes.cast(dts, ctypes.c_void_p),
                                       ctypes.cast(els, ctypes.c_void_p), int(n_insert), float(distinct_ratio),
                                       ctypes.cast(wa, ctypes.c_void_p), len(ws), ctypes.cast(ga, ctypes.c_void_p),
                                       len(gs), ctypes.cast(la, ctypes.c_void_p), len(ls), 1 if batched else 0,
                                       ctypes.byref(alloc.struct), _stream(), ctypes.byref(out), ctypes.byref(ms)),
                "ash_autotune_sweep")
        return dict(bucket_width=out.bucket_width, probe_group=out.probe_group, max_load=out.max_load), ms.value
    fn = lib.ash_autotune_batched if batched else lib.ash_autotune
    L.check(fn(int(capacity), int(key_dim), n, ctypes.cast(dts, ctypes.c_void_p), ctypes.cast(els, ctypes.c_void_p),
               int(n_insert), float(distinct_ratio), ctypes.byref(alloc.struct), _stream(), ctypes.byref(out),
               ctypes.byref(ms)), "ash_autotune")
    return dict(bucket_width=out.bucket_width, probe_group=out.probe_group, max_load=out.max_load), ms.value


def batched(ops, fused=True):
    """Inserts then finds on many maps at once (one persistent launch when
    fused).  ops: list of dicts with keys map, insert_keys, insert_values,
    find_keys, gather (bool).  Returns a list of dicts with insert_idx,
    insert_mask, find_idx, find_mask and find_values."""
    lib = L.load()
    arr = (L.AshBatchOp * max(len(ops), 1))()
    keep = []
    results = []
    for i, op in enumerate(ops):
        m = op["map"]
        ik = _keys(op["insert_keys"], m.key_dim, m.device)
        fk = _keys(op["find_keys"], m.key_dim, m.device)
        ni, nf = ik.shape[0], fk.shape[0]
        vals = [v.reshape(ni, e).contiguous() for v, (dt, e) in zip(op.get("insert_values", ()), m.value_specs)]
        if len(vals) != len(m.value_specs):
            raise ValueError("one value tensor per value buffer is required")
        res = dict(insert_idx=torch.empty(ni, dtype=torch.int32, device=m.device),
                   insert_mask=torch.empty(ni, dtype=torch.uint8, device=m.device),
                   find_idx=torch.empty(nf, dtype=torch.int32, device=m.device),
                   find_mask=torch.empty(nf, dtype=torch.uint8, device=m.device), find_values=None)
        vin = (ctypes.c_void_p * max(len(vals), 1))(*[v.data_ptr() for v in vals])
        vout = None
        if op.get("gather") and m.value_specs:
            res["find_values"] = [torch.zeros((nf, e), dtype=dt, device=m.device) for dt, e in m.value_specs]
            vout = (ctypes.c_void_p * len(m.value_specs))(*[o.data_ptr() for o in res["find_values"]])
        keep.extend([ik, fk, vals, vin, vout])
        arr[i] = L.AshBatchOp(m._m, ik.data_ptr(), ni, ctypes.cast(vin, ctypes.c_void_p) if vals else None,
                              res["insert_idx"].data_ptr(), res["insert_mask"].data_ptr(), fk.data_ptr(), nf,
                              ctypes.cast(vout, ctypes.c_void_p) if vout is not None else None,
                              res["find_idx"].data_ptr(), res["find_mask"].data_ptr())
        results.append(res)
    L.check(lib.ash_batched(arr, len(ops), 1 if fused else 0, _stream()), "ash_batched")
    for r in results:
        r["insert_mask"] = r["insert_mask"].bool()
        r["find_mask"] = r["find_mask"].bool()
    return results


class Server:
    """Served map: continuous batching of insert / find / erase requests on a
    device-resident map (see ash_server_* in include/ash.h).  The map must not
    be used directly while it is served."""

    FIND, INSERT, ERASE = 0, 1, 2

    def __init__(self, hashmap, max_fused=256, max_batch=1 << 22, in_flight=4, fuse=True):
        self._lib = L.load()
        self.map = hashmap
        cfg = L.AshServerConfig(max_fused, max_batch, in_flight, 1 if fuse else 0)
        self._s = ctypes.c_void_p()
        L.check(self._lib.ash_server_create(hashmap._m, ctypes.byref(cfg), ctypes.byref(self._s)),
                "ash_server_create")
        self._keep = {}
        _LIVE_SERVERS.add(self)

    def request(self, kind, keys, values=(), out_idx=None, out_mask=None, out_values=None):
        """Builds an ash_request_t over device tensors (kept alive by the caller)."""
        m = self.map
        keys = _keys(keys, m.key_dim, m.device)
        vin = (ctypes.c_void_p * max(len(values), 1))(*[v.data_ptr() for v in values])
        vout = None
        if out_values is not None:
            vout = (ctypes.c_void_p * max(len(out_values), 1))(*[o.data_ptr() for o in out_values])
        r = L.AshRequest(kind, keys.data_ptr(), keys.shape[0],
                         ctypes.cast(vin, ctypes.c_void_p) if values else None,
                         out_idx.data_ptr() if out_idx is not None else None,
                         out_mask.data_ptr() if out_mask is not None else None,
                         ctypes.cast(vout, ctypes.c_void_p) if vout is not None else None)
        return r, (keys, vin, vout)

    def submit(self, kind, keys, values=(), out_idx=None, out_mask=None, out_values=None):
        r, keep = self.request(kind, keys, values, out_idx, out_mask, out_values)
        # the server's stream does not wait on torch's: the tensors must be ready
        torch.cuda.current_stream(self.map.device).synchronize()
        t = ctypes.c_int64()
        L.check(self._lib.ash_server_submit(self._s, ctypes.byref(r), ctypes.byref(t)), "ash_server_submit")
        self._keep[t.value] = keep
        return t.value

    def wait(self, ticket):
        """(status, latency in seconds) of a submitted request."""
        lat = ctypes.c_double()
        st = self._lib.ash_server_wait(self._s, int(ticket), ctypes.byref(lat))
        self._keep.pop(ticket, None)
        return st, lat.value

    def replay(self, requests, arrivals_s):
        """Submits ctypes requests at their arrival times; returns
        (latencies s, statuses, span s)."""
        import numpy as np
        n = len(requests)
        arr = (L.AshRequest * max(n, 1))(*requests)
        at = np.ascontiguousarray(arrivals_s, dtype=np.float64)
        lat = np.zeros(n, np.float64)
        sts = np.zeros(n, np.int32)
        span = ctypes.c_double()
        torch.cuda.current_stream(self.map.device).synchronize()
        L.check(self._lib.ash_server_replay(self._s, arr, n, at.ctypes.data, lat.ctypes.data, sts.ctypes.data,
                                            ctypes.byref(span)), "ash_server_replay")
        return lat, sts, span.value

    def stats(self):
        b, r, g = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        L.check(self._lib.ash_server_stats(self._s, ctypes.byref(b), ctypes.byref(r), ctypes.byref(g)),
                "ash_server_stats")
        return dict(batches=b.value, requests=r.value, largest=g.value)

    def close(self):
        s = getattr(self, "_s", None)
        if s is not None and s.value:
            self._s = None
            L.check(self._lib.ash_server_destroy(s), "ash_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

