"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Buffer indices are handed out in batch order on both sides, so beyond the
canonical checks (masks, key -> value maps, heap invariant) the GPU's indices,
key buffer, value rows, heap and heap top must equal the oracle's exactly.
Value rows of activated-only entries are excluded (the paper leaves them to
the caller).  Every comparison is bit-exact (values compared as raw bits).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import ORACLE_E_CAPACITY, OracleMap  # noqa: E402


@pytest.fixture(scope="module")
def ash():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash_mod
    return ash_mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint8)


class Pair:
    """A GPU map and an oracle map driven with the same batches."""

    def __init__(self, ash, capacity, key_dim=3, value_specs=(), **tuning):
        self.gpu = ash.HashMap(capacity, key_dim=key_dim,
                               value_specs=[(torch.from_numpy(np.zeros(1, dt)).dtype, e) for dt, e in value_specs],
                               **tuning)
        self.orc = OracleMap(capacity, key_dim, value_specs)
        self.key_dim = key_dim
        self.value_specs = [(np.dtype(dt), e) for dt, e in value_specs]
        self.written = set()  # indices whose value rows were written by insert
        self.overflowed = False  # an insert since the last check returned CAPACITY

    def insert(self, keys, values):
        gi, gm = self.gpu.insert(dev(keys), [dev(v) for v in values])
        st, oi, om = self.orc.insert(keys, values, autogrow=self.gpu_autogrow())
        gi, gm = host(gi), host(gm).astype(np.uint8)
        self.overflowed |= st == ORACLE_E_CAPACITY
        assert np.array_equal(gm, om), "insert masks differ"
        assert np.array_equal(gi, oi), "insert indices differ"
        self.written.update(oi[om == 1].tolist())
        return st, oi, om

    def activate(self, keys):
        gi, gm = self.gpu.activate(dev(keys))
        st, oi, om = self.orc.activate(keys, autogrow=self.gpu_autogrow())
        self.overflowed |= st == ORACLE_E_CAPACITY
        assert np.array_equal(host(gm).astype(np.uint8), om), "activate masks differ"
        assert np.array_equal(host(gi), oi), "activate indices differ"
        self.written.difference_update(oi[om == 1].tolist())
        return st, oi, om

    def find(self, keys, gather=True):
        if gather and self.value_specs:
            gi, gm, gout = self.gpu.find(dev(keys), gather=True)
            st, oi, om, oout = self.orc.find(keys, gather=True, fill=0)
            for j, (g, o) in enumerate(zip(gout, oout)):
                g = host(g)
                hit = om == 1
                ok = np.isin(oi, list(self.written)) & hit
                assert np.array_equal(bits(g[ok]), bits(o[ok])), f"gathered values of buffer {j} differ"
                assert np.array_equal(bits(g[~hit]), bits(np.zeros_like(o[~hit]))), "miss rows were modified"
        else:
            gi, gm = self.gpu.find(dev(keys))
            st, oi, om = self.orc.find(keys)
        assert np.array_equal(host(gm).astype(np.uint8), om), "find masks differ"
        assert np.array_equal(host(gi), oi), "find indices differ"
        return oi, om

    def erase(self, keys):
        gm = self.gpu.erase(dev(keys))
        st, om = self.orc.erase(keys)
        assert np.array_equal(host(gm).astype(np.uint8), om), "erase masks differ"
        return om

    def gpu_autogrow(self):
        return getattr(self, "autogrow", False)

    def check_state(self):
        g = self.gpu
        o = self.orc
        torch.cuda.synchronize()
        assert g.capacity == o.capacity
        assert g.size() == o.size == o.heap_top
        assert np.array_equal(host(g.heap_buffer()), o.heap()), "index heaps differ"
        act = host(g.active_indices())
        assert np.array_equal(act, o.active_indices()), "active indices differ"
        kb = host(g.key_buffer())
        assert np.array_equal(kb[act], o.key_buffer()[act]), "key buffers differ on live indices"
        live_written = np.array(sorted(set(act.tolist()) & self.written), dtype=np.int64)
        for j in range(len(self.value_specs)):
            gv = host(g.value_buffer(j))
            assert np.array_equal(bits(gv[live_written]), bits(o.value_buffer(j)[live_written])), \
                f"value buffer {j} differs on live written indices"
        stats = g.stats()
        assert stats["size"] == o.size
        # exact counts: every occupied slot is a live key or a tombstone (no
        # claim left pending, none lost)
        assert stats["used_slots"] - stats["tombstones"] == o.size
        assert g.device_status() == (2 if self.overflowed else 0), "sticky status differs from the oracle's"
        self.overflowed = False


def plain_small_sequence(pair, d):
    pair.insert(d["keys"], [d["values"]])
    pair.check_state()
    pair.find(d["find_keys"])
    pair.erase(d["erase_keys"])
    pair.check_state()
    pair.find(d["find_keys"])
    pair.find(d["keys"])


def test_plain_small_sequence(ash):
    """65,536-key insert / find / erase / re-find (the CPU-checkable workload)."""
    d = synth.plain_small()
    pair = Pair(ash, d["capacity"], 3, [(np.float32, 1)])
    plain_small_sequence(pair, d)


@pytest.mark.parametrize("g,w,lf,dd", [(1, 2, 0.5, 0), (1, 4, 0.7, 0), (1, 8, 0.9, 0), (4, 4, 0.5, 0),
                                        (8, 8, 0.7, 0), (16, 4, 0.85, 0), (32, 32, 0.5, 0), (64, 16, 0.9, 0),
                                        (4, 4, 0.5, 1), (1, 4, 0.7, 1), (16, 4, 0.85, 1)])
def test_tuning_grid_same_results(ash, g, w, lf, dd):
    d = synth.plain_small(seed=11)
    pair = Pair(ash, d["capacity"], 3, [(np.float32, 1)], probe_group=g, bucket_width=w, max_load=lf,
                lds_dedup=bool(dd))
    plain_small_sequence(pair, d)


@pytest.mark.parametrize("g", [1, 4, 64])
def test_lds_dedup_with_local_duplicates(ash, g):
    """Batches where equal keys sit close together (runs of a key, sorted
    keys): most duplicates are removed inside a block, some straddle block
    boundaries, and keys already in the map recur."""
    rng = np.random.default_rng(19)
    base = rng.integers(-50, 50, size=(20_000, 3), dtype=np.int32)
    runs = np.repeat(base, rng.integers(1, 12, size=len(base)), axis=0)  # runs of equal keys
    srt = runs[np.lexsort(runs.T[::-1])]  # sorted: long runs per key
    pair = Pair(ash, 150_000, 3, [(np.float32, 8)], probe_group=g, bucket_width=4, lds_dedup=True)
    for batch in (runs, srt[: len(srt) // 2], srt):
        pair.insert(batch, [rng.standard_normal((len(batch), 8)).astype(np.float32)])
        pair.find(np.concatenate([batch[::7], rng.integers(60, 90, size=(5000, 3), dtype=np.int32)]))
    pair.erase(srt[::3])
    pair.insert(runs, [rng.standard_normal((len(runs), 8)).astype(np.float32)])
    pair.check_state()


@pytest.mark.parametrize("key_dim", [1, 2, 3, 4])
def test_key_dims_and_value_types(ash, key_dim):
    rng = np.random.default_rng(100 + key_dim)
    n = 30_000
    keys = rng.integers(-20, 20, size=(n, key_dim), dtype=np.int32)
    specs = [(np.float32, 3), (np.uint8, 5), (np.float64, 2), (np.int32, 16)]
    vals = [rng.standard_normal((n, 3)).astype(np.float32), rng.integers(0, 255, (n, 5), dtype=np.uint8),
            rng.standard_normal((n, 2)), rng.integers(-9, 9, (n, 16), dtype=np.int32)]
    pair = Pair(ash, 2 * n, key_dim, specs)
    pair.insert(keys, vals)
    pair.find(np.concatenate([keys[: n // 2], rng.integers(20, 40, size=(n // 2, key_dim), dtype=np.int32)]))
    pair.erase(keys[rng.choice(n, n // 3, replace=False)])
    pair.insert(rng.integers(-25, 25, size=(n // 2, key_dim), dtype=np.int32),
                [v[: n // 2] for v in vals])
    pair.check_state()
    pair.find(keys)


def test_hash_set_and_activate(ash):
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 50, size=(40_000, 3), dtype=np.int32)
    pair = Pair(ash, 80_000, 3, [])
    pair.activate(keys)
    pair.find(keys)
    pair.erase(keys[:10_000])
    pair.activate(keys[5_000:20_000])
    pair.check_state()
    # a map with values: activate leaves value rows alone, insert after activate is a miss
    pv = Pair(ash, 1000, 3, [(np.float32, 4)])
    k = rng.integers(0, 8, size=(600, 3), dtype=np.int32)
    pv.activate(k)
    pv.insert(k, [rng.standard_normal((600, 4)).astype(np.float32)])
    pv.check_state()


def test_edge_cases(ash):
    pair = Pair(ash, 64, 3, [(np.float32, 1)])
    z = np.zeros((0, 3), np.int32)
    pair.insert(z, [np.zeros((0, 1), np.float32)])
    pair.find(z)
    pair.erase(z)
    lo, hi = np.iinfo(np.int32).min, np.iinfo(np.int32).max
    ext = np.array([[lo, lo, lo], [hi, hi, hi], [lo, hi, 0], [-1, -1, -1], [lo, lo, lo], [0, 0, 0]], np.int32)
    pair.insert(ext, [np.arange(6, dtype=np.float32).reshape(6, 1)])
    pair.find(ext)
    # all-identical keys: exactly one winner, the lowest position
    same = np.full((5000, 3), 7, np.int32)
    st, oi, om = pair.insert(same, [np.arange(5000, dtype=np.float32).reshape(-1, 1)])
    assert om.sum() == 1 and om[0] == 1
    pair.erase(same)
    pair.check_state()


@pytest.mark.parametrize("channels", [2, 32])  # rows copied inside the commit / in a pass of their own
def test_capacity_overflow_rolls_back(ash, channels):
    rng = np.random.default_rng(9)
    pair = Pair(ash, 1000, 3, [(np.float32, channels)])
    k1 = rng.integers(0, 100, size=(900, 3), dtype=np.int32)
    pair.insert(k1, [rng.standard_normal((900, channels)).astype(np.float32)])
    before = (host(pair.gpu.heap_buffer()).copy(), host(pair.gpu.key_buffer()).copy(),
              host(pair.gpu.value_buffer(0)).copy())
    k2 = rng.integers(100, 200, size=(300, 3), dtype=np.int32)
    gi, gm = pair.gpu.insert(dev(k2), [dev(rng.standard_normal((300, channels)).astype(np.float32))])
    st, oi, om = pair.orc.insert(k2, [np.zeros((300, channels), np.float32)])
    assert st == ORACLE_E_CAPACITY
    assert np.all(host(gi) == -1) and not host(gm).any()
    assert pair.gpu.device_status() == 2  # ASH_E_CAPACITY, then cleared
    assert np.array_equal(host(pair.gpu.heap_buffer()), before[0])
    # no value row moved, the free rows included
    assert np.array_equal(bits(host(pair.gpu.value_buffer(0))), bits(before[2]))
    pair.check_state()
    pair.find(np.concatenate([k1, k2]))


@pytest.mark.parametrize("channels", [1, 32])  # rows copied inside the commit / in a pass of their own
def test_autogrow(ash, channels):
    rng = np.random.default_rng(13)
    pair = Pair(ash, 100, 3, [(np.float32, channels)], autogrow=True)
    pair.autogrow = True
    for step in range(6):
        k = rng.integers(0, 40, size=(700, 3), dtype=np.int32)
        pair.insert(k, [rng.standard_normal((700, channels)).astype(np.float32)])
        pair.erase(k[:100])
    pair.check_state()
    assert pair.gpu.capacity == pair.orc.capacity


def test_rehash_keeps_indices(ash):
    rng = np.random.default_rng(17)
    keys = rng.integers(0, 60, size=(50_000, 3), dtype=np.int32)
    pair = Pair(ash, 60_000, 3, [(np.float32, 8)])
    pair.insert(keys, [rng.standard_normal((50_000, 8)).astype(np.float32)])
    pair.erase(keys[:20_000])
    for new_c in (60_000, 100_000, 250_000):
        pair.gpu.rehash(new_c)
        assert pair.orc.rehash(new_c) == 0
        pair.check_state()
        pair.find(keys)
    assert pair.gpu.stats()["tombstones"] == 0


@pytest.mark.parametrize("capacity", [27_000, 4096])
def test_erase_insert_churn(ash, capacity):
    """Erases leave tombstones; inserts reuse those they pass before the first
    EMPTY slot, and table rebuilds drop the rest.  Occupancy stays bounded;
    the smaller capacity also overflows on some batches (CAPACITY, claims
    rolled back to tombstones)."""
    rng = np.random.default_rng(21)
    pair = Pair(ash, capacity, 3, [(np.int32, 1)], max_load=0.5)
    consumed = False
    for step in range(40):
        k = rng.integers(0, 30, size=(3000, 3), dtype=np.int32)
        before = pair.gpu.stats()
        pair.insert(k, [rng.integers(0, 1000, (3000, 1), dtype=np.int32)])
        after = pair.gpu.stats()
        consumed |= after["tombstones"] < before["tombstones"]  # reused by the insert, or a rebuild
        pair.erase(rng.integers(0, 30, size=(3000, 3), dtype=np.int32))
        pair.find(k, gather=False)
        s = pair.gpu.stats()
        assert s["used_slots"] <= s["capacity"] + (s["slots"] - s["capacity"]) // 4 + 3000
        assert s["used_slots"] - s["tombstones"] == s["size"]
        if step % 10 == 9:
            pair.check_state()
    assert consumed


@pytest.mark.parametrize("g", [1, 4])
def test_small_table_long_probes(ash, g):
    """Capacity 200 at max_load 0.9: windows wrap the table end, probes are long."""
    rng = np.random.default_rng(23)
    pair = Pair(ash, 200, 2, [(np.float32, 1)], max_load=0.9, probe_group=g, bucket_width=4)
    k = rng.integers(0, 1000, size=(2000, 2), dtype=np.int32)
    pair.insert(k[:400], [rng.standard_normal((400, 1)).astype(np.float32)])
    pair.find(k)
    pair.erase(k[:150])
    pair.insert(k[150:500], [rng.standard_normal((350, 1)).astype(np.float32)])
    pair.check_state()
    pair.find(k)


# ---------------------------------------------------------------------------
# Voxelization
def check_voxelize(ash, pts, voxel):
    from oracle import oracle_voxelize
    gpv, gvk, gcnt = ash.voxelize(dev(pts), voxel)
    opv, ovk, ocnt = oracle_voxelize(pts, voxel)
    assert np.array_equal(host(gpv), opv), "per-point voxel ids differ"
    assert np.array_equal(host(gvk), ovk), "voxel keys differ"
    assert np.array_equal(host(gcnt), ocnt), "voxel counts differ"
    return opv, ovk, ocnt


@pytest.mark.parametrize("voxel", [0.005, 0.01, 0.02, 0.05])
def test_voxelize_surface_points(ash, voxel):
    check_voxelize(ash, synth.points(n=300_000, seed=31), voxel)


@pytest.mark.parametrize("voxel", [0.01, 0.1])
def test_voxelize_ordered_points(ash, voxel):
    """Points in scan order (sorted along x), so many points of a voxel fall
    in the same block: the block-local duplicate removal resolves them through
    their representative's slot."""
    pts = synth.points(n=200_000, seed=32)
    check_voxelize(ash, pts[np.argsort(pts[:, 0], kind="stable")], voxel)


def test_voxelize_full_size(ash):
    """The benchmark's 5M surface points at 5 mm against the oracle, whole."""
    check_voxelize(ash, synth.points(), 0.005)


def test_voxelize_boundaries_and_rejects(ash):
    s = np.float32(0.1)
    k = np.arange(-3000, 3000, dtype=np.float32)
    x = (k * s).astype(np.float32)
    x = np.concatenate([x, np.nextafter(x, np.float32(np.inf)), np.nextafter(x, np.float32(-np.inf))])
    pts = np.stack([x, -x, x * np.float32(0.5)], axis=1)
    check_voxelize(ash, pts, s)
    big = np.float32(3e38)
    tiny = np.float32(1e-40)  # denormal
    rej = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0, 0, -np.inf], [big, 0, 0], [1.0, 1.0, 1.0],
                    [-big, 0, 0], [-tiny, tiny, -0.0], [np.float32(2147483520.0), 0, 0],
                    [np.float32(2.0 ** 31), 0, 0], [np.float32(-2.0 ** 31), 0, 0]], np.float32)
    check_voxelize(ash, rej, 1.0)
    check_voxelize(ash, rej, 0.005)
    check_voxelize(ash, np.array([[0.5, 0.5, 0.5]], np.float32), 0.01)
    pv, vk, cnt = ash.voxelize(dev(np.zeros((0, 3), np.float32)), 0.01)
    assert pv.numel() == 0 and vk.shape[0] == 0


# ---------------------------------------------------------------------------
# Full-size workloads: properties that hold at any size (exact).
def _pack(keys):
    k = keys.astype(np.int64) + (1 << 20)
    return (k[:, 0] << 42) | (k[:, 1] << 21) | k[:, 2]


def _closed_forms(d):
    """numpy closed forms of one 10M-key workload `d` (synth.plain_large) on a
    fresh map: indices are ranks of first occurrences; erase winners are the
    first occurrences in the erase batch, which push their indices in batch
    order."""
    keys, fk, ek = d["keys"], d["find_keys"], d["erase_keys"]
    pk = _pack(keys)
    uniq, first = np.unique(pk, return_index=True)
    rank_sorted = np.empty(len(uniq), np.int64)  # rank (insert order) of sorted distinct key j
    rank_sorted[np.argsort(first)] = np.arange(len(first))
    first = np.sort(first)
    pf = _pack(fk)
    pos = np.searchsorted(uniq, pf)
    hit = (pos < len(uniq)) & (uniq[np.minimum(pos, len(uniq) - 1)] == pf)
    pe = _pack(ek)
    efirst = np.sort(np.unique(pe, return_index=True)[1])
    erank = rank_sorted[np.searchsorted(uniq, pe[efirst])]  # every erase key was inserted
    return dict(first=first, uniq=uniq, rank_sorted=rank_sorted, pos=pos, hit=hit, efirst=efirst, erank=erank,
                erased=np.isin(pf, pe))


@pytest.mark.parametrize("rho", [0.1, 0.5, 0.99])
@pytest.mark.parametrize("channels", [1, 8, 32])
def test_plain_large_properties(ash, rho, channels):
    """The 10M-key workload at every (distinct ratio, channels) pair, in the
    benchmark's launch configuration (the table shape the tuner picks for the
    workload, as the benchmark takes it), checked for every position against
    closed forms: insert masks and indices, k^B and v^B, find masks, indices
    and gathered rows, erase masks, and after the 5M erase the whole heap,
    t, the active indices and re-find masks."""
    d = synth.plain_large(rho=rho, channels=channels)
    tun, _ = ash.autotune(d["capacity"], len(d["keys"]), rho, 3, [(torch.float32, channels)])
    print(f"case: plain 10M rho={rho} C={channels} shape {tun}", flush=True)
    _check_plain_large(ash, d, channels, tun)


@pytest.mark.parametrize("g,w,lf", [(1, 2, 0.85), (1, 4, 0.85), (4, 4, 0.5), (1, 2, 0.7)])
def test_plain_large_shapes(ash, g, w, lf):
    """The benchmark's 10M-key workload (distinct ratio 0.5, f32x8) on the
    shapes the tuner picks between for it, whatever it picks in this run."""
    d = synth.plain_large(rho=0.5, channels=8)
    print(f"case: plain 10M shape g={g} W={w} load={lf}", flush=True)
    _check_plain_large(ash, d, 8, dict(probe_group=g, bucket_width=w, max_load=lf))


def _check_plain_large(ash, d, channels, shape):
    keys, vals = d["keys"], d["values"]
    cf = _closed_forms(d)
    first = cf["first"]
    m = ash.HashMap(d["capacity"], 3, [(torch.float32, channels)], **shape)
    gi, gm = m.insert(dev(keys), [dev(vals)])
    gi, gm = host(gi), host(gm)
    want_mask = np.zeros(len(keys), bool)
    want_mask[first] = True
    assert np.array_equal(gm, want_mask)
    want_idx = np.full(len(keys), -1, np.int32)
    want_idx[first] = np.arange(len(first), dtype=np.int32)  # fresh heap: ranks
    assert np.array_equal(gi, want_idx)
    kb = host(m.key_buffer())
    assert np.array_equal(kb[: len(first)], keys[first])
    vb = host(m.value_buffer(0))
    assert np.array_equal(bits(vb[: len(first)]), bits(vals[first]))
    fk = d["find_keys"]
    fi, fm, (fv,) = m.find(dev(fk), gather=True)
    fi, fm, fv = host(fi), host(fm), host(fv)
    hit, pos = cf["hit"], cf["pos"]
    assert np.array_equal(fm, hit)
    assert np.array_equal(fi[hit], cf["rank_sorted"][pos[hit]].astype(np.int32))
    assert np.all(fi[~hit] == -1)
    assert np.array_equal(bits(fv[hit]), bits(vb[fi[hit]]))
    assert np.all(bits(fv[~hit]) == 0)  # rows of misses untouched (zero-filled)
    ek = d["erase_keys"]
    em = host(m.erase(dev(ek)))
    efirst, erank = cf["efirst"], cf["erank"]
    want = np.zeros(len(ek), bool)
    want[efirst] = True  # every erase key was inserted; its first occurrence wins
    assert np.array_equal(em, want)
    t0 = len(first)
    t1 = t0 - len(efirst)
    assert m.size() == t1
    heap = np.arange(d["capacity"], dtype=np.int32)
    heap[t0 - 1 - np.arange(len(efirst))] = erank  # the r-th winner pushes h[t0 - 1 - r]
    assert np.array_equal(host(m.heap_buffer()), heap)
    live = np.ones(t0, bool)
    live[erank] = False
    assert np.array_equal(host(m.active_indices()), np.flatnonzero(live).astype(np.int32))
    fi2, fm2 = m.find(dev(fk))
    assert np.array_equal(host(fm2), hit & ~cf["erased"])
    assert m.device_status() == 0


def test_misaligned_allocator_is_refused(ash):
    """A provider whose blocks are not 256-byte aligned gets each block back
    and the call fails with ASH_E_NOMEM; nothing is launched on such memory."""
    import ctypes
    from paper_2110_00511_amd import _lib as L

    class Shifted(L.TorchAllocator):
        def _do_alloc(self, ctx, nbytes, stream):
            t = torch.empty(int(nbytes) + 64, dtype=torch.uint8, device=self.device)
            ptr = t.data_ptr() + 16  # 16-byte aligned only
            self.blocks[ptr] = t
            return ptr

    alloc = Shifted("cuda")
    dts = (ctypes.c_int * 1)(L.ASH_F32)
    els = (ctypes.c_int64 * 1)(4)
    out = ctypes.c_void_p()
    lib = L.load()
    st = lib.ash_create(1000, 3, 1, ctypes.cast(dts, ctypes.c_void_p), ctypes.cast(els, ctypes.c_void_p),
                        ctypes.byref(alloc.struct), None, None, ctypes.byref(out))
    assert st == L.ASH_E_NOMEM
    assert not alloc.blocks  # every block was handed back


@pytest.mark.parametrize("g,w", [(4, 4), (1, 4), (16, 4)])
def test_tombstones_are_reused_under_churn(ash, g, w):
    """Erase-heavy churn on a small table: inserts take tombstones seen before
    the first EMPTY slot of their sequence, so occupancy stays near the live
    count, and every result still equals the oracle's (duplicates in the
    batch, keys erased and re-inserted in the same region, rollbacks)."""
    rng = np.random.default_rng(60 + g)
    cap = 3000
    pair = Pair(ash, cap, 3, [(np.float32, 2)], probe_group=g, bucket_width=w, max_load=0.5)
    universe = rng.integers(-40, 40, size=(9000, 3), dtype=np.int32)
    for step in range(12):
        k = universe[rng.integers(0, len(universe), size=2500)]
        pair.insert(k, [rng.standard_normal((len(k), 2)).astype(np.float32)])
        pair.find(universe[rng.integers(0, len(universe), size=3000)])
        pair.erase(k[rng.permutation(len(k))[:1800]])
        pair.check_state()
    st = pair.gpu.stats()
    # without reuse every insert after an erase would take a fresh slot
    assert st["used_slots"] <= st["size"] + st["tombstones"]
    assert st["used_slots"] - st["tombstones"] == st["size"]
    assert st["used_slots"] < 2 * cap


def test_tombstones_and_overflow_rollback(ash):
    """An insert that overflows the heap after tombstones exist rolls its
    claims back to tombstones; the map stays equal to the oracle's."""
    rng = np.random.default_rng(63)
    pair = Pair(ash, 1200, 3, [(np.float32, 1)])
    k1 = rng.integers(0, 30, size=(1500, 3), dtype=np.int32)
    pair.insert(k1, [rng.standard_normal((1500, 1)).astype(np.float32)])
    pair.erase(k1[:600])
    big = rng.integers(30, 60, size=(2000, 3), dtype=np.int32)  # more new keys than free indices
    pair.insert(big, [rng.standard_normal((2000, 1)).astype(np.float32)])
    pair.check_state()
    pair.insert(k1[:700], [rng.standard_normal((700, 1)).astype(np.float32)])
    pair.find(np.concatenate([k1, big]))
    pair.check_state()


@pytest.mark.parametrize("key_dim", [2, 3])
@pytest.mark.parametrize("g,w", [(1, 4), (4, 4), (16, 8)])
def test_claims_that_keep_pending_keys(ash, key_dim, g, w):
    """After an insert whose positions mostly repeat a key, the next claims
    keep pending keys in their slots.  Their batches mix keys whose leading
    words are all -1 (the value an unwritten slot word holds), many keys that
    share their last word (the pending tag), repeats of earlier keys and new
    ones; every result must still equal the oracle's."""
    rng = np.random.default_rng(110 + key_dim * 10 + g)
    pair = Pair(ash, 60_000, key_dim, [(np.float32, 2)], probe_group=g, bucket_width=w)

    def batch(n, distinct):
        base = rng.integers(-20, 20, size=(distinct, key_dim), dtype=np.int32)
        base[: distinct // 8, : key_dim - 1] = -1           # leading words all -1
        base[distinct // 8: distinct // 2, key_dim - 1] = 7  # one shared last word
        keys = base[rng.integers(0, distinct, size=n)]
        return keys, [rng.standard_normal((n, 2)).astype(np.float32)]

    pair.insert(*batch(20_000, 2_000))  # 90% repeats: the next inserts keep pending keys
    pair.check_state()
    for _ in range(3):
        pair.insert(*batch(30_000, 3_000))
        pair.check_state()
    keys, _ = batch(10_000, 4_000)
    pair.find(keys)


@pytest.mark.parametrize("voxel,res", [(0.05, 8), (0.005, 16), (0.1, 3), (1.0, 1)])
def test_block_coords_match_oracle(ash, voxel, res):
    """Block keys, in-block voxel coordinates and the valid flag of surface
    points moved to straddle the origin, of points on voxel boundaries and of
    rejected points, bit-exact against the oracle."""
    from oracle import oracle_block_coords
    pts = synth.points(n=100_001, seed=33) - np.float32(5.0)
    s = np.float32(voxel)
    k = np.arange(-500, 500, dtype=np.float32)
    edge = (k * s).astype(np.float32)
    edge = np.stack([edge, np.nextafter(edge, np.float32(-np.inf)), np.nextafter(edge, np.float32(np.inf))], axis=1)
    rej = np.array([[np.nan, 0, 0], [0, np.inf, 0], [3e38, 0, 0], [-3e38, 1, 1],
                    [np.float32(2.0 ** 31) * s, 0, 0]], np.float32)
    pts = np.concatenate([pts, edge, rej]).astype(np.float32)
    gb, gl, gv = ash.block_coords(dev(pts), float(s), res)
    ob, ol, ov = oracle_block_coords(pts, s, res)
    assert np.array_equal(host(gv).astype(np.uint8), ov)
    assert np.array_equal(host(gb), ob) and np.array_equal(host(gl), ol)
    assert ov[:100_001].all() and not ov[-5:-1].any()
    e = ash.block_coords(dev(np.zeros((0, 3), np.float32)), float(s), res)
    assert e[0].shape == (0, 3)
