"""Batched maps: many independent maps of uneven sizes in one persistent
launch.  Each map's results must equal the oracle's for the same insert and
find batches (and therefore the op-by-op single-map path), bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import ORACLE_E_CAPACITY, OracleMap  # noqa: E402
from tests.test_gpu_parity import bits, dev, host  # noqa: E402

SHAPES = [(4, 4, 0.5), (1, 4, 0.7), (8, 8, 0.85), (64, 16, 0.5), (16, 4, 0.7), (1, 8, 0.5), (32, 32, 0.85),
          (1, 2, 0.5)]


@pytest.fixture(scope="module")
def ash():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash_mod
    return ash_mod


def make_case(rng, u, channels=8):
    side = max(2, int(round((2 * u / 1.5936) ** (1 / 3))))
    keys = rng.integers(0, side, size=(2 * u, 3), dtype=np.int32)
    vals = rng.standard_normal((2 * u, channels)).astype(np.float32)
    present = keys[rng.integers(0, 2 * u, size=u)]
    absent = rng.integers(side, 2 * side, size=(u, 3), dtype=np.int32)
    finds = np.concatenate([present, absent])[rng.permutation(2 * u)]
    return keys, vals, np.ascontiguousarray(finds)


def run_round(ash, maps, oracles, cases, fused):
    ops = [dict(map=m, insert_keys=dev(k), insert_values=[dev(v)], find_keys=dev(f), gather=True)
           for m, (k, v, f) in zip(maps, cases)]
    res = ash.batched(ops, fused=fused)
    statuses = []
    for r, o, (k, v, f) in zip(res, oracles, cases):
        st, oi, om = o.insert(k, [v])
        statuses.append(st)
        assert np.array_equal(host(r["insert_mask"]).astype(np.uint8), om)
        assert np.array_equal(host(r["insert_idx"]), oi)
        st, fi, fm, (fv,) = o.find(f, gather=True, fill=0)
        assert np.array_equal(host(r["find_mask"]).astype(np.uint8), fm)
        assert np.array_equal(host(r["find_idx"]), fi)
        assert np.array_equal(bits(host(r["find_values"][0])), bits(fv))
    return statuses


def check_maps(maps, oracles):
    torch.cuda.synchronize()
    for m, o in zip(maps, oracles):
        assert m.size() == o.size
        assert np.array_equal(host(m.heap_buffer()), o.heap())
        act = host(m.active_indices())
        assert np.array_equal(act, o.active_indices())
        assert np.array_equal(host(m.key_buffer())[act], o.key_buffer()[act])
        assert np.array_equal(bits(host(m.value_buffer(0))[act]), bits(o.value_buffer(0)[act]))


@pytest.mark.parametrize("fused", [True, False])
def test_batched_maps_match_oracle(ash, fused):
    rng = np.random.default_rng(40)
    sizes = [1000, 3000, 20000, 70000, 5000, 150000, 40000, 2000]
    maps, oracles, cases = [], [], []
    for i, (u, (g, w, lf)) in enumerate(zip(sizes, SHAPES)):
        maps.append(ash.HashMap(2 * u, 3, [(torch.float32, 8)], probe_group=g, bucket_width=w, max_load=lf,
                                lds_dedup=i % 2 == 1))
        oracles.append(OracleMap(2 * u, 3, [(np.float32, 8)]))
        cases.append(make_case(rng, u))
    run_round(ash, maps, oracles, cases, fused)
    check_maps(maps, oracles)
    # a second round on the populated maps: re-inserted keys are misses, new
    # keys take the next heap indices
    cases2 = [make_case(rng, max(u // 4, 1)) for u in sizes]
    run_round(ash, maps, oracles, cases2, fused)
    check_maps(maps, oracles)
    for m in maps:
        assert m.device_status() == 0


def test_batched_overflow_is_per_map(ash):
    rng = np.random.default_rng(41)
    sizes = [4000, 6000, 9000]
    caps = [8000, 1000, 18000]  # the middle map cannot take its batch
    maps = [ash.HashMap(c, 3, [(torch.float32, 8)]) for c in caps]
    oracles = [OracleMap(c, 3, [(np.float32, 8)]) for c in caps]
    cases = [make_case(rng, u) for u in sizes]
    statuses = run_round(ash, maps, oracles, cases, True)
    assert statuses[1] == ORACLE_E_CAPACITY and statuses[0] == 0 and statuses[2] == 0
    assert [m.device_status() for m in maps] == [0, 2, 0]
    check_maps(maps, oracles)


def test_batched_empty_ops_and_hash_sets(ash):
    rng = np.random.default_rng(42)
    a = ash.HashSet(5000, 3)
    b = ash.HashSet(5000, 3)
    oa, ob = OracleMap(5000, 3), OracleMap(5000, 3)
    ka = rng.integers(0, 20, size=(3000, 3), dtype=np.int32)
    empty = np.zeros((0, 3), np.int32)
    res = ash.batched([dict(map=a, insert_keys=dev(ka), find_keys=dev(empty)),
                       dict(map=b, insert_keys=dev(empty), find_keys=dev(ka))])
    st, oi, om = oa.insert(ka)
    assert np.array_equal(host(res[0]["insert_idx"]), oi)
    st, fi, fm = ob.find(ka)
    assert np.array_equal(host(res[1]["find_mask"]).astype(np.uint8), fm)
    assert a.size() == oa.size and b.size() == 0


@pytest.mark.parametrize("batched", [False, True])
def test_autotune_picks_a_valid_shape(ash, batched):
    tun, ms = ash.autotune(40_000, 20_000, 0.5, key_dim=3, value_specs=[(torch.float32, 8)], batched=batched)
    if batched:  # the batched sweep keeps one lane per key
        assert tun["probe_group"] == 1 and tun["bucket_width"] in (2, 4)
    else:
        assert tun["probe_group"] in (1, 4, 8, 16, 64)
        assert tun["bucket_width"] in (2, 4, 8, 16, 32)
    assert min(abs(tun["max_load"] - x) for x in (0.5, 0.7, 0.85)) < 1e-6
    assert ms > 0
    # cached: the second call returns the same answer at once
    tun2, ms2 = ash.autotune(40_000, 20_000, 0.5, key_dim=3, value_specs=[(torch.float32, 8)], batched=batched)
    assert tun2 == tun and ms2 == ms
    rng = np.random.default_rng(43)
    m = ash.HashMap(40_000, 3, [(torch.float32, 8)], **tun)
    o = OracleMap(40_000, 3, [(np.float32, 8)])
    k, v, f = make_case(rng, 20_000)
    run_round(ash, [m], [o], [(k, v, f)], True)
    check_maps([m], [o])


@pytest.mark.parametrize("key_dim", [1, 2, 4])
def test_batched_other_key_dims(ash, key_dim):
    """The persistent kernel of each key width (their register use, and so
    the number of blocks that run at once, differ)."""
    rng = np.random.default_rng(44 + key_dim)
    sizes = [3000, 20000, 500]
    maps = [ash.HashMap(2 * u, key_dim, [(torch.float32, 4)]) for u in sizes]
    oracles = [OracleMap(2 * u, key_dim, [(np.float32, 4)]) for u in sizes]
    ops, cases = [], []
    for u in sizes:
        k = rng.integers(-30, 30, size=(2 * u, key_dim), dtype=np.int32)
        v = rng.standard_normal((2 * u, 4)).astype(np.float32)
        f = np.concatenate([k[: u], rng.integers(40, 60, size=(u, key_dim), dtype=np.int32)])
        cases.append((k, v, f))
        ops.append(dict(insert_keys=dev(k), insert_values=[dev(v)], find_keys=dev(f), gather=True))
    res = ash.batched([dict(map=m, **op) for m, op in zip(maps, ops)], fused=True)
    for r, o, (k, v, f) in zip(res, oracles, cases):
        st, oi, om = o.insert(k, [v])
        assert np.array_equal(host(r["insert_idx"]), oi)
        st, fi, fm, (fv,) = o.find(f, gather=True, fill=0)
        assert np.array_equal(host(r["find_idx"]), fi)
        assert np.array_equal(bits(host(r["find_values"][0])), bits(fv))
    check_maps(maps, oracles)
    assert [m.device_status() for m in maps] == [0, 0, 0]


@pytest.mark.parametrize("key_dim", [1, 2, 3, 4])
def test_batched_narrow_build(ash, key_dim):
    """Launches whose maps all probe one lane per key with W = 2 or 4 run the
    build of the persistent kernel that holds only those probes; it needs
    fewer registers, so more of its blocks run at once.  Two rounds against
    the oracle, then the grid of both builds."""
    import ctypes

    from paper_2110_00511_amd import _lib as L
    rng = np.random.default_rng(60 + key_dim)
    sizes = [40000, 700, 9000, 120000, 3000]
    maps, oracles, cases = [], [], []
    for i, u in enumerate(sizes):
        # room for both rounds' distinct keys (up to about 2.5u)
        maps.append(ash.HashMap(3 * u, key_dim, [(torch.float32, 8)], probe_group=1, bucket_width=(2, 4)[i % 2],
                                max_load=(0.5, 0.7, 0.85)[i % 3], lds_dedup=i % 2 == 0))
        oracles.append(OracleMap(3 * u, key_dim, [(np.float32, 8)]))
    for rnd in range(2):
        cases = []
        for u in sizes:
            n = 2 * u if rnd == 0 else max(u // 3, 1)
            side = max(2, int(round(n ** (1 / key_dim))))
            k = rng.integers(-side, side, size=(n, key_dim), dtype=np.int32)
            v = rng.standard_normal((n, 8)).astype(np.float32)
            f = np.concatenate([k[rng.integers(0, n, size=n // 2)],
                                rng.integers(2 * side, 3 * side, size=(n - n // 2, key_dim), dtype=np.int32)])
            cases.append((k, v, np.ascontiguousarray(f)))
        print(f"case: narrow batched build, key_dim {key_dim}, round {rnd}", flush=True)
        assert run_round(ash, maps, oracles, cases, True) == [0] * len(sizes)
        check_maps(maps, oracles)
    assert [m.device_status() for m in maps] == [0] * len(sizes)
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    got = {}
    for narrow in (0, 1):
        blocks, reported = ctypes.c_int64(0), ctypes.c_int64(0)
        L.check(lib.ash_batched_grid(key_dim, narrow, ctypes.byref(blocks), ctypes.byref(reported), sp), "grid")
        assert 0 < blocks.value <= reported.value
        got[narrow] = reported.value
    assert got[1] >= got[0]


@pytest.mark.parametrize("sizes", [[1], [50, 300], [20, 700, 90, 5, 260]])
def test_batched_small_grids(ash, sizes):
    """Launches with fewer blocks than tile queues (a grid of one to a few
    blocks, each block alone on its queue and XCD count), in both builds."""
    rng = np.random.default_rng(70 + len(sizes))
    for shape in ((1, 4), (4, 8)):
        maps = [ash.HashMap(2 * u + 4, 3, [(torch.float32, 8)], probe_group=shape[0], bucket_width=shape[1])
                for u in sizes]
        oracles = [OracleMap(2 * u + 4, 3, [(np.float32, 8)]) for u in sizes]
        print(f"case: small batched grid, sizes {sizes}, shape {shape}", flush=True)
        for rnd in range(2):
            cases = [make_case(rng, max(u // (1 + 2 * rnd), 1)) for u in sizes]
            assert run_round(ash, maps, oracles, cases, True) == [0] * len(sizes)
            check_maps(maps, oracles)
        assert [m.device_status() for m in maps] == [0] * len(sizes)


@pytest.mark.parametrize("grid", ["lane", "stated", "single_op_by_op"])
def test_batched_full_size(ash, grid):
    """The benchmark's 64 maps (distinct counts log-uniform in [1e3, 1e6],
    f32x8 values) in one persistent launch with the shapes the benchmark
    times: the batched tuner's (one lane per key, the narrow build) and the
    stated grid's (W {4, 8, 16, 32} x g {8, 16, 64} x load {0.5, 0.7, 0.85},
    the general build), and the single-map tuner's shapes run op by op (the
    plain path the benchmark compares against).  Every map is fresh, so
    results follow from numpy alone: the insert mask marks first occurrences, their indices are ranks,
    a find returns the rank of its key and the first occurrence's row."""
    import synth
    maps_d = synth.batched()
    maps, ops = [], []
    stated = ([4, 8, 16, 32], [8, 16, 64], [0.5, 0.7, 0.85]) if grid == "stated" else None
    print(f"case: 64 batched maps, {grid} shapes", flush=True)
    for d in maps_d:
        n = len(d["keys"])
        tun, _ = ash.autotune(d["capacity"], n, 0.5, value_specs=[(torch.float32, 8)],
                              batched=grid != "single_op_by_op", grid=stated)
        m = ash.HashMap(d["capacity"], 3, [(torch.float32, 8)], **tun)
        maps.append(m)
        ops.append(dict(map=m, insert_keys=dev(d["keys"]), insert_values=[dev(d["values"])],
                        find_keys=dev(d["find_keys"]), gather=True))
    res = ash.batched(ops, fused=grid != "single_op_by_op")
    torch.cuda.synchronize()
    for d, r, m in zip(maps_d, res, maps):
        keys, vals, fk = d["keys"], d["values"], d["find_keys"]
        packed = np.ascontiguousarray(keys).view(np.dtype((np.void, 12))).ravel()
        _, first, inv = np.unique(packed, return_index=True, return_inverse=True)
        rank = np.empty(len(first), np.int64)
        rank[np.argsort(first)] = np.arange(len(first))  # rank of each distinct key in batch order
        want_mask = np.zeros(len(keys), bool)
        want_mask[first] = True
        assert np.array_equal(host(r["insert_mask"]), want_mask)
        gi = host(r["insert_idx"])
        assert np.array_equal(gi[want_mask], rank[inv[want_mask]].astype(np.int32))
        assert np.all(gi[~want_mask] == -1)
        fpacked = np.ascontiguousarray(fk).view(np.dtype((np.void, 12))).ravel()
        uniq = np.unique(packed)
        pos = np.searchsorted(uniq, fpacked)
        hit = (pos < len(uniq)) & (uniq[np.minimum(pos, len(uniq) - 1)] == fpacked)
        assert np.array_equal(host(r["find_mask"]), hit)
        fi = host(r["find_idx"])
        assert np.array_equal(fi[hit], rank[pos[hit]].astype(np.int32))
        assert np.all(fi[~hit] == -1)
        src = first[pos[hit]]  # the first occurrence's row was stored
        assert np.array_equal(bits(host(r["find_values"][0])[hit]), bits(vals[src]))
        assert m.size() == len(first) and m.device_status() == 0


def test_batched_arrival_failure_runs_op_by_op(ash, monkeypatch):
    """When the blocks of the persistent launch cannot all run at once, they
    leave before touching any map and the call runs the same work op by op,
    with the oracle's results.  The condition is forced from the host:
    ASH_BATCHED_FORCE_ARRIVAL_FAILURE=1 makes the blocks give up without
    counting themselves in, and every kernel still exits normally."""
    from paper_2110_00511_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(48)
    sizes = [20000, 3000, 60000, 9000]
    maps = [ash.HashMap(2 * u, 3, [(torch.float32, 8)], probe_group=1, bucket_width=4) for u in sizes]
    oracles = [OracleMap(2 * u, 3, [(np.float32, 8)]) for u in sizes]
    run_round(ash, maps, oracles, [make_case(rng, u) for u in sizes], True)  # fused, caches the grid
    before = lib.ash_batched_fallbacks()
    monkeypatch.setenv("ASH_BATCHED_FORCE_ARRIVAL_FAILURE", "1")
    print("case: batched launch with a forced arrival failure", flush=True)
    run_round(ash, maps, oracles, [make_case(rng, max(u // 3, 1)) for u in sizes], True)
    assert lib.ash_batched_fallbacks() == before + 1
    monkeypatch.delenv("ASH_BATCHED_FORCE_ARRIVAL_FAILURE")
    check_maps(maps, oracles)
    assert [m.device_status() for m in maps] == [0, 0, 0, 0]
    run_round(ash, maps, oracles, [make_case(rng, max(u // 5, 1)) for u in sizes], True)  # fused again
    assert lib.ash_batched_fallbacks() == before + 1
    check_maps(maps, oracles)
