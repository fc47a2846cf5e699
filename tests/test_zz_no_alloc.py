"""The allocation-free voxelization entry point against ash_voxelize.

ash_voxelize_noalloc runs the same kernels on a fixed device workspace inside
the library; its outputs must equal ash_voxelize's bit for bit.  Two calls in
a row (the second smaller, so the workspace still holds the first call's
table and counters) check that every call starts from a clean state; the
small call is also checked against the oracle.  A batch above the limit is
refused on the host.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import oracle_voxelize  # noqa: E402

LIMIT = 1 << 20


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_00511_amd import _lib as L
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _run(L, entry, pts, voxel):
    """Calls one entry point through the C ABI; returns (status, pv, keys, counts, n_voxels)."""
    lib = L.load()
    n = pts.shape[0]
    pv = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    vk = torch.full((n, 3), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    nv = ctypes.c_int64(-1)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (_ptr(pts), n, ctypes.c_float(voxel), _ptr(pv), _ptr(vk), _ptr(cnt), ctypes.byref(nv))
    if entry == "noalloc":
        st = lib.ash_voxelize_noalloc(*args, stream)
    else:
        st = lib.ash_voxelize(*args, None, stream)
    torch.cuda.synchronize()
    return st, pv, vk, cnt, nv.value


def _same(a, b):
    sa, pva, vka, ca, ua = a
    sb, pvb, vkb, cb, ub = b
    assert sa == sb == 0
    assert ua == ub
    assert torch.equal(pva, pvb)
    assert torch.equal(vka[:ua], vkb[:ub])
    assert torch.equal(ca[:ua], cb[:ub])


def test_noalloc_matches_voxelize_twice(lib):
    # first call at the workspace limit (C3-like surface points, 5 mm voxels)
    big = synth.points(n=LIMIT, seed=21)
    big_d = torch.from_numpy(big).cuda()
    print(f"noalloc: n={LIMIT} voxel=0.005 seed=21", flush=True)
    a = _run(lib, "noalloc", big_d, 0.005)
    b = _run(lib, "alloc", big_d, 0.005)
    _same(a, b)
    assert a[4] > 100_000
    # second call smaller, ragged and with another voxel size: nothing of
    # the first call's table or counters may leak into it
    small = synth.points(n=100_003, seed=22)
    small[17] = np.nan  # a rejected point
    small_d = torch.from_numpy(small).cuda()
    print("noalloc: n=100003 voxel=0.02 seed=22", flush=True)
    c = _run(lib, "noalloc", small_d, 0.02)
    d = _run(lib, "alloc", small_d, 0.02)
    _same(c, d)
    opv, ovk, ocnt = oracle_voxelize(small, np.float32(0.02))
    assert c[4] == ovk.shape[0]
    assert np.array_equal(c[1].cpu().numpy(), opv)
    assert np.array_equal(c[2][:c[4]].cpu().numpy(), ovk)
    assert np.array_equal(c[3][:c[4]].cpu().numpy(), ocnt)
    assert opv[17] == -1


def test_noalloc_limits(lib):
    L = lib
    lib_ = L.load()
    pts = torch.zeros((LIMIT + 1, 3), dtype=torch.float32, device="cuda")
    out = torch.zeros(LIMIT + 1, dtype=torch.int32, device="cuda")
    keys = torch.zeros((LIMIT + 1, 3), dtype=torch.int32, device="cuda")
    nv = ctypes.c_int64(-1)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib_.ash_voxelize_noalloc(_ptr(pts), LIMIT + 1, ctypes.c_float(0.01), _ptr(out), _ptr(keys), _ptr(out),
                                   ctypes.byref(nv), stream)
    assert st == L.ASH_E_UNSUPPORTED and nv.value == -1
    st = lib_.ash_voxelize_noalloc(_ptr(pts), 0, ctypes.c_float(0.01), _ptr(out), _ptr(keys), _ptr(out),
                                   ctypes.byref(nv), stream)
    assert st == 0 and nv.value == 0
    st = lib_.ash_voxelize_noalloc(_ptr(pts), 10, ctypes.c_float(-1.0), _ptr(out), _ptr(keys), _ptr(out),
                                   ctypes.byref(nv), stream)
    assert st == L.ASH_E_INVALID
