"""The C-ABI library loads on a machine without a GPU and exports every
function include/*.h declares; the Python binding declares the same names.
No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2110_00511_amd", "libash.so")


def declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(ash_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2110_00511_amd.build import build
        build()
    import torch  # noqa: F401  (the binding loads torch's HIP runtime first)
    return ctypes.CDLL(LIB)


def test_header_declares_the_operations():
    names = declared()
    for op in ("ash_create", "ash_destroy", "ash_insert", "ash_activate", "ash_find", "ash_erase",
               "ash_active_indices", "ash_rehash", "ash_voxelize", "ash_size", "ash_device_status"):
        assert op in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header(lib):
    from paper_2110_00511_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared()
    _lib.load()


def test_status_strings_and_host_side_errors(lib):
    from paper_2110_00511_amd import _lib
    L = _lib.load()
    assert L.ash_status_string(0) == b"ok"
    assert L.ash_status_string(2) == b"capacity exceeded"
    out = ctypes.c_void_p()
    # rejected before any device work: bad key_dim, bad capacity, NULL output
    assert L.ash_create(10, 0, 0, None, None, None, None, None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    assert L.ash_create(10, 5, 0, None, None, None, None, None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    assert L.ash_create(-1, 3, 0, None, None, None, None, None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    assert L.ash_create(1 << 31, 3, 0, None, None, None, None, None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    assert L.ash_create(10, 3, 0, None, None, None, None, None, None) == _lib.ASH_E_INVALID
    bad = _lib.AshTuning(4, 5, 0.5, 0)
    assert L.ash_create(10, 3, 0, None, None, None, ctypes.byref(bad), None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    bad = _lib.AshTuning(4, 4, 0.95, 0)
    assert L.ash_create(10, 3, 0, None, None, None, ctypes.byref(bad), None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    n = ctypes.c_int64()
    assert L.ash_voxelize(None, 10, ctypes.c_float(0.01), None, None, None, ctypes.byref(n), None, None) == _lib.ASH_E_INVALID
    assert L.ash_voxelize(None, 0, ctypes.c_float(-1.0), None, None, None, ctypes.byref(n), None, None) == _lib.ASH_E_INVALID
    assert L.ash_voxelize(None, 0, ctypes.c_float(0.01), None, None, None, ctypes.byref(n), None, None) == _lib.ASH_OK
    assert n.value == 0
    assert L.ash_insert(None, None, 0, None, None, None, None) == _lib.ASH_E_INVALID
    assert L.ash_destroy(None) == _lib.ASH_E_INVALID


def test_server_and_batched_reject_bad_arguments_on_the_host(lib):
    """Argument checks that return before any HIP call (no device needed)."""
    from paper_2110_00511_amd import _lib
    L = _lib.load()
    out = ctypes.c_void_p()
    assert L.ash_server_create(None, None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    t = ctypes.c_int64()
    req = _lib.AshRequest(0, None, 0, None, None, None, None)
    assert L.ash_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == _lib.ASH_E_INVALID
    assert L.ash_server_wait(None, 0, None) == _lib.ASH_E_INVALID
    assert L.ash_server_stats(None, None, None, None) == _lib.ASH_E_INVALID
    assert L.ash_server_destroy(None) == _lib.ASH_E_INVALID
    assert L.ash_server_replay(None, None, 0, None, None, None, None) == _lib.ASH_E_INVALID
    blocks, reported = ctypes.c_int64(), ctypes.c_int64()
    for kd, narrow in ((0, 0), (5, 0), (3, 2), (3, -1)):  # key width 1-4, build 0 or 1
        assert L.ash_batched_grid(kd, narrow, ctypes.byref(blocks), ctypes.byref(reported), None) == _lib.ASH_E_INVALID
    assert L.ash_batched_grid(3, 1, None, ctypes.byref(reported), None) == _lib.ASH_E_INVALID
    assert L.ash_batched(None, 2, 1, None) == _lib.ASH_E_INVALID
    assert L.ash_batched(None, -1, 1, None) == _lib.ASH_E_INVALID


def _offsets(L, kind, radius, kd):
    cnt = ctypes.c_int64()
    assert L.ash_neighbor_offsets(kind, radius, kd, None, ctypes.byref(cnt)) == 0
    buf = (ctypes.c_int32 * max(cnt.value * kd, 1))()
    assert L.ash_neighbor_offsets(kind, radius, kd, buf, ctypes.byref(cnt)) == 0
    return [tuple(buf[i * kd:(i + 1) * kd]) for i in range(cnt.value)]


@pytest.mark.parametrize("kd", [1, 2, 3, 4])
@pytest.mark.parametrize("radius", [1, 2])
def test_neighbor_offsets_are_the_standard_neighborhoods(lib, kd, radius):
    """Host-only helper: the neighborhoods by their definitions, enumerated
    with itertools (first word slowest)."""
    import itertools
    from paper_2110_00511_amd import _lib
    L = _lib.load()
    full = list(itertools.product(range(-radius, radius + 1), repeat=kd))
    assert _offsets(L, _lib.ASH_NB_RADIUS, radius, kd) == full
    assert _offsets(L, _lib.ASH_NB_CUBE, radius, kd) == list(itertools.product(range(radius + 1), repeat=kd))
    ring = [o for o in full if 0 < sum(map(abs, o)) <= radius]
    assert _offsets(L, _lib.ASH_NB_RING, radius, kd) == ring
    if radius == 1:
        assert len(full) == 3 ** kd and len(ring) == 2 * kd  # 27 and 6 in 3-D


def test_neighbor_and_intersect_argument_errors(lib):
    from paper_2110_00511_amd import _lib
    L = _lib.load()
    cnt = ctypes.c_int64()
    assert L.ash_neighbor_offsets(7, 1, 3, None, ctypes.byref(cnt)) == _lib.ASH_E_INVALID
    assert L.ash_neighbor_offsets(0, 0, 3, None, ctypes.byref(cnt)) == _lib.ASH_E_INVALID
    assert L.ash_neighbor_offsets(0, 1, 5, None, ctypes.byref(cnt)) == _lib.ASH_E_INVALID
    assert L.ash_neighbor_offsets(0, 64, 4, None, ctypes.byref(cnt)) == _lib.ASH_E_INVALID  # 129^4 candidates
    assert L.ash_neighbor_offsets(0, 1, 3, None, None) == _lib.ASH_E_INVALID
    assert L.ash_find_offsets(None, None, 0, None, 0, None, None, None) == _lib.ASH_E_INVALID
    assert L.ash_intersect(None, None, 0, None, ctypes.byref(cnt), None) == _lib.ASH_E_INVALID


def _map_file(kd=2, c=4, live=(1, 3), keys=((1, 2), (3, 4)), heap=None, extra=b"", magic=b"ASHMAP\x00\x01"):
    import struct
    heap = list(heap) if heap is not None else list(live) + [i for i in range(c) if i not in live]
    out = magic + struct.pack("<iiqq", kd, 1, c, len(live)) + struct.pack("<iiq", 2, 0, 1)
    out += struct.pack(f"<{c}i", *heap) + struct.pack(f"<{len(live)}i", *live)
    out += b"".join(struct.pack(f"<{kd}i", *k) for k in keys) + b"\0" * 4 * len(live)
    return out + extra


@pytest.mark.parametrize("case", ["missing", "magic", "truncated", "trailing", "free_index_twice",
                                  "live_index_free", "stale_entry_out_of_range", "live_unsorted",
                                  "duplicate_keys", "bad_dtype"])
def test_load_rejects_bad_files_before_device_work(lib, tmp_path, case):
    """Every check of ash_load runs on the host before a map is created, so a
    bad file fails here without a GPU."""
    from paper_2110_00511_amd import _lib
    L = _lib.load()
    files = {
        "magic": _map_file(magic=b"ASHMAP\x00\x02"),
        "truncated": _map_file()[:-3],
        "trailing": _map_file(extra=b"\0"),
        "free_index_twice": _map_file(heap=[1, 3, 0, 0]),
        "live_index_free": _map_file(heap=[0, 2, 3, 2]),
        "stale_entry_out_of_range": _map_file(heap=[7, 3, 0, 2]),
        "live_unsorted": _map_file(live=(3, 1), heap=[3, 1, 0, 2]),
        "duplicate_keys": _map_file(keys=((1, 2), (1, 2))),
        "bad_dtype": _map_file().replace(b"\x02\x00\x00\x00\x00\x00\x00\x00\x01\x00", b"\x09\x00\x00\x00\x00\x00\x00\x00\x01\x00", 1),
    }
    path = tmp_path / "m.ash"
    if case != "missing":
        path.write_bytes(files[case])
    out = ctypes.c_void_p()
    assert L.ash_load(str(path).encode(), None, None, None, ctypes.byref(out)) == _lib.ASH_E_INVALID
    assert not out.value


def test_missing_library_fails_loudly(tmp_path):
    """There is no fallback: without libash.so the binding raises."""
    import subprocess
    import sys
    code = ("from paper_2110_00511_amd import _lib\n"
            "try:\n"
            f"    _lib.load({str(tmp_path / 'libash.so')!r})\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert "raised:" in r.stdout and "is missing" in r.stdout


def test_block_coords_argument_errors(lib):
    from paper_2110_00511_amd import _lib
    L = _lib.load()
    P = ctypes.c_void_p(16)  # never dereferenced: the host checks fail first
    assert L.ash_block_coords(P, -1, ctypes.c_float(0.1), 8, P, P, P, None) == _lib.ASH_E_INVALID
    assert L.ash_block_coords(P, 10, ctypes.c_float(0.0), 8, P, P, P, None) == _lib.ASH_E_INVALID
    assert L.ash_block_coords(P, 10, ctypes.c_float(float("inf")), 8, P, P, P, None) == _lib.ASH_E_INVALID
    assert L.ash_block_coords(P, 10, ctypes.c_float(0.1), 0, P, P, P, None) == _lib.ASH_E_INVALID
    assert L.ash_block_coords(None, 10, ctypes.c_float(0.1), 8, P, P, P, None) == _lib.ASH_E_INVALID
    assert L.ash_block_coords(None, 0, ctypes.c_float(0.1), 8, None, None, None, None) == _lib.ASH_OK
