"""ctypes binding of libash.so with the C-ABI names of include/ash.h.

Argument marshalling only: every step runs in the library's HIP kernels.
torch must be imported first so that the library binds to the HIP runtime
torch already loaded (one runtime per process).  Loading fails loudly when
libash.so has not been built; there is no fallback path.
"""
import ctypes
import os
import sys

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libash.so")

ASH_OK = 0
ASH_E_INVALID = 1
ASH_E_CAPACITY = 2
ASH_E_NOMEM = 3
ASH_E_DEVICE = 4
ASH_E_UNSUPPORTED = 5
ASH_F_AUTOGROW = 1
ASH_F_LDS_DEDUP = 2
ASH_NB_RADIUS, ASH_NB_CUBE, ASH_NB_RING = 0, 1, 2
ASH_ACC_READ, ASH_ACC_STORE, ASH_ACC_CAS64, ASH_ACC_MIN32, ASH_ACC_STREAM_READ, ASH_ACC_STREAM_COPY = range(6)

ASH_U8, ASH_I32, ASH_F32, ASH_I64, ASH_F64, ASH_F16, ASH_BF16 = range(7)

# Functions declared in include/ash.h: name -> (restype, argtypes)
P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
ST = ctypes.c_int


class AshAllocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(P, P, ctypes.c_size_t, P)),
                ("free", ctypes.CFUNCTYPE(None, P, P, P)),
                ("ctx", P)]


class AshTuning(ctypes.Structure):
    _fields_ = [("bucket_width", I32), ("probe_group", I32), ("max_load", ctypes.c_float), ("flags", ctypes.c_uint32)]


class AshKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", I64), ("total_ms", ctypes.c_double)]


class AshBatchOp(ctypes.Structure):
    _fields_ = [("map", P), ("insert_keys", P), ("n_insert", I64), ("insert_values", P), ("insert_idx", P),
                ("insert_mask", P), ("find_keys", P), ("n_find", I64), ("find_values", P), ("find_idx", P),
                ("find_mask", P)]


class AshRequest(ctypes.Structure):
    _fields_ = [("kind", I32), ("keys", P), ("n", I64), ("values", P), ("out_idx", P), ("out_mask", P),
                ("out_values", P)]


class AshServerConfig(ctypes.Structure):
    _fields_ = [("max_fused", I32), ("max_batch", I64), ("in_flight", I32), ("fuse", I32)]


class AshStats(ctypes.Structure):
    _fields_ = [("size", I64), ("capacity", I64), ("slots", I64), ("used_slots", I64), ("tombstones", I64)]


SIGNATURES = {
    "ash_create": (ST, [I64, I32, I32, P, P, P, P, P, ctypes.POINTER(P)]),
    "ash_destroy": (ST, [P]),
    "ash_insert": (ST, [P, P, I64, P, P, P, P]),
    "ash_activate": (ST, [P, P, I64, P, P, P]),
    "ash_find": (ST, [P, P, I64, P, P, P, P]),
    "ash_erase": (ST, [P, P, I64, P, P]),
    "ash_find_offsets": (ST, [P, P, I64, P, I32, P, P, P]),
    "ash_neighbor_offsets": (ST, [I32, I32, I32, P, ctypes.POINTER(I64)]),
    "ash_block_coords": (ST, [P, I64, ctypes.c_float, I32, P, P, P, P]),
    "ash_intersect": (ST, [P, P, I64, P, ctypes.POINTER(I64), P]),
    "ash_save": (ST, [P, ctypes.c_char_p, P]),
    "ash_load": (ST, [ctypes.c_char_p, P, P, P, ctypes.POINTER(P)]),
    "ash_describe": (ST, [P, ctypes.POINTER(I32), ctypes.POINTER(I32), P, P]),
    "ash_active_indices": (ST, [P, P, ctypes.POINTER(I64), P]),
    "ash_rehash": (ST, [P, I64, P]),
    "ash_clear": (ST, [P, P]),
    "ash_size": (ST, [P, ctypes.POINTER(I64), P]),
    "ash_capacity": (ST, [P, ctypes.POINTER(I64)]),
    "ash_stats": (ST, [P, ctypes.POINTER(AshStats), P]),
    "ash_key_buffer": (ST, [P, ctypes.POINTER(P)]),
    "ash_value_buffer": (ST, [P, I32, ctypes.POINTER(P)]),
    "ash_heap_buffer": (ST, [P, ctypes.POINTER(P)]),
    "ash_device_status": (ST, [P, P]),
    "ash_voxelize": (ST, [P, I64, ctypes.c_float, P, P, P, ctypes.POINTER(I64), P, P]),
    "ash_voxelize_noalloc": (ST, [P, I64, ctypes.c_float, P, P, P, ctypes.POINTER(I64), P]),
    "ash_batched": (ST, [ctypes.POINTER(AshBatchOp), I32, I32, P]),
    "ash_autotune": (ST, [I64, I32, I32, P, P, I64, ctypes.c_double, P, P, ctypes.POINTER(AshTuning),
                          ctypes.POINTER(ctypes.c_double)]),
    "ash_autotune_batched": (ST, [I64, I32, I32, P, P, I64, ctypes.c_double, P, P, ctypes.POINTER(AshTuning),
                                  ctypes.POINTER(ctypes.c_double)]),
    "ash_autotune_sweep": (ST, [I64, I32, I32, P, P, I64, ctypes.c_double, P, I32, P, I32, P, I32, I32, P, P,
                                ctypes.POINTER(AshTuning), ctypes.POINTER(ctypes.c_double)]),
    "ash_server_create": (ST, [P, P, ctypes.POINTER(P)]),
    "ash_batched_fallbacks": (I64, []),
    "ash_batched_grid": (ST, [I32, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), P]),
    "ash_server_submit": (ST, [P, ctypes.POINTER(AshRequest), ctypes.POINTER(I64)]),
    "ash_server_wait": (ST, [P, I64, ctypes.POINTER(ctypes.c_double)]),
    "ash_server_replay": (ST, [P, ctypes.POINTER(AshRequest), I64, P, P, P, ctypes.POINTER(ctypes.c_double)]),
    "ash_server_stats": (ST, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    "ash_server_destroy": (ST, [P]),
    "ash_profile_enable": (ST, [P, I32]),
    "ash_profile_collect": (ST, [P, ctypes.POINTER(AshKernelTime), I32, ctypes.POINTER(I32), P]),
    "ash_access_bench": (ST, [I32, P, I64, I32, I64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), P]),
    "ash_status_string": (ctypes.c_char_p, [ST]),
    # include/ash_slab.h: the separate-chaining backend of the backend ablation
    "ash_slab_create": (ST, [I64, I32, I64, P, ctypes.POINTER(P)]),
    "ash_slab_destroy": (ST, [P]),
    "ash_slab_clear": (ST, [P, P]),
    "ash_slab_insert": (ST, [P, P, I64, P, P, P, P]),
    "ash_slab_find": (ST, [P, P, I64, P, P, P, P]),
    "ash_slab_size": (ST, [P, ctypes.POINTER(I64), P]),
    "ash_slab_buffers": (ST, [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P)]),
}

_lib = None


def load(path=LIB_PATH):
    """Loads libash.so (raises if it is missing) and declares every symbol."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2110_00511_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AshError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = load().ash_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})")


def check(status, what):
    if status != ASH_OK:
        raise AshError(status, what)


class TorchAllocator:
    """Routes the library's device allocations to torch's caching allocator.

    Each allocation is a uint8 tensor kept alive in `blocks` until the library
    frees it, so map-owned buffers can be viewed as tensors without copies."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.blocks = {}
        self._alloc = AshAllocator._fields_[0][1](self._do_alloc)
        self._free = AshAllocator._fields_[1][1](self._do_free)
        self.struct = AshAllocator(self._alloc, self._free, None)

    def _stream(self, stream):
        if not stream:
            return torch.cuda.current_stream(self.device)
        return torch.cuda.ExternalStream(stream, device=self.device)

    def _do_alloc(self, ctx, nbytes, stream):
        # allocate on the stream the library will use the block on, so that
        # torch only reuses it in that stream's order
        with torch.cuda.stream(self._stream(stream)):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        ptr = t.data_ptr()
        self.blocks[ptr] = t
        return ptr

    def _do_free(self, ctx, ptr, stream):
        t = self.blocks.pop(ptr, None)
        if t is not None and stream and not sys.is_finalizing():
            t.record_stream(self._stream(stream))

    def tensor(self, ptr):
        return self.blocks[ptr]
