"""Served map: a request stream through the continuous-batching server must
give every request the results it gets when the requests run one after
another -- checked against the oracle replaying the stream serially, with
requests fused in the mix (all arriving at once, or spread out) and with one
request per device batch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import OracleMap  # noqa: E402
from tests.test_gpu_parity import bits, dev, host  # noqa: E402

FIND, INSERT, ERASE = 0, 1, 2


@pytest.fixture(scope="module")
def ash():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash_mod
    return ash_mod


def make_stream(rng, n_req, side, lo=16, hi=4096, channels=4):
    reqs = []
    kinds = rng.choice(3, size=n_req, p=[0.6, 0.3, 0.1])
    for k in kinds:
        m = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        keys = rng.integers(0, side, size=(m, 3), dtype=np.int32)
        vals = rng.standard_normal((m, channels)).astype(np.float32) if k == INSERT else None
        reqs.append((int(k), keys, vals))
    return reqs


def run_served(ash, capacity, preload, reqs, arrivals, channels=4, tuning=None, **cfg):
    m = ash.HashMap(capacity, 3, [(torch.float32, channels)], **(tuning or {}))
    pk, pv = preload
    m.insert(dev(pk), [dev(pv)])
    torch.cuda.synchronize()
    srv = ash.Server(m, **cfg)
    outs, built, keep = [], [], []
    for kind, keys, vals in reqs:
        n = len(keys)
        o = dict(idx=torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                 mask=torch.full((n,), 7, dtype=torch.uint8, device="cuda"),
                 vals=[torch.zeros((n, channels), dtype=torch.float32, device="cuda")] if kind == FIND else None)
        kd = dev(keys)
        vd = [dev(vals)] if vals is not None else []
        r, k = srv.request(kind, kd, vd, out_idx=o["idx"] if kind != ERASE else None, out_mask=o["mask"],
                           out_values=o["vals"])
        built.append(r)
        keep.append((kd, vd, k, o))
        outs.append(o)
    lat, sts, span = srv.replay(built, arrivals)
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    return m, outs, lat, sts, stats


def check_against_oracle(capacity, preload, reqs, m, outs, channels=4, values=False):
    o = OracleMap(capacity, 3, [(np.float32, channels)])
    pk, pv = preload
    o.insert(pk, [pv])
    written = set(o.active_indices().tolist())
    for (kind, keys, vals), out in zip(reqs, outs):
        if kind == INSERT:
            st, oi, om = o.insert(keys, [vals])
            written.update(oi[om == 1].tolist())
            assert np.array_equal(host(out["mask"]), om)
            assert np.array_equal(host(out["idx"]), oi)
        elif kind == FIND:
            st, oi, om, (ov,) = o.find(keys, gather=True, fill=0)
            assert np.array_equal(host(out["mask"]), om)
            assert np.array_equal(host(out["idx"]), oi)
            assert np.array_equal(bits(host(out["vals"][0])), bits(ov))
        else:
            st, om = o.erase(keys)
            assert np.array_equal(host(out["mask"]), om)
    assert m.size() == o.size
    assert np.array_equal(host(m.heap_buffer()), o.heap())
    act = host(m.active_indices())
    assert np.array_equal(act, o.active_indices())
    assert np.array_equal(host(m.key_buffer())[act], o.key_buffer()[act])
    if values:  # every entry was inserted with its row
        assert np.array_equal(bits(host(m.value_buffer(0))[act]), bits(o.value_buffer(0)[act]))


@pytest.mark.parametrize("mode", ["burst", "spread", "unfused"])
def test_served_results_equal_serial_replay(ash, mode):
    rng = np.random.default_rng(70)
    side, capacity = 40, 60_000
    pre = rng.choice(side ** 3, size=20_000, replace=False)
    pk = np.stack([pre // (side * side), (pre // side) % side, pre % side], axis=1).astype(np.int32)
    pv = rng.standard_normal((len(pk), 4)).astype(np.float32)
    reqs = make_stream(rng, 300, side)
    if mode == "burst":
        arrivals = np.zeros(len(reqs))  # everything waits: maximal fusion
    else:
        arrivals = np.cumsum(rng.exponential(50e-6, size=len(reqs)))
    cfg = dict(fuse=mode != "unfused", max_fused=64, max_batch=1 << 16, in_flight=3)
    m, outs, lat, sts, stats = run_served(ash, capacity, (pk, pv), reqs, arrivals, **cfg)
    assert np.all(sts == 0) and np.all(lat >= 0)
    check_against_oracle(capacity, (pk, pv), reqs, m, outs)
    if mode == "burst":
        assert stats["batches"] < len(reqs)  # requests were fused
    if mode == "unfused":
        assert stats["batches"] == len(reqs)


@pytest.mark.parametrize("case", ["rows_64B", "staged_forced"])
def test_served_staged_batches_equal_serial_replay(ash, case, monkeypatch):
    """Fused batches that go through staging buffers: inserts whose rows
    reach 64 B per key (their rows move in a pass of their own after the
    commit), and every insert and erase batch with ASH_SERVER_STAGED=1.  Both
    must give the serial replay's results, like the batches that run on the
    requests' own buffers."""
    channels = 16 if case == "rows_64B" else 4
    if case == "staged_forced":
        monkeypatch.setenv("ASH_SERVER_STAGED", "1")
    rng = np.random.default_rng(74)
    side, capacity = 40, 60_000
    pre = rng.choice(side ** 3, size=20_000, replace=False)
    pk = np.stack([pre // (side * side), (pre // side) % side, pre % side], axis=1).astype(np.int32)
    pv = rng.standard_normal((len(pk), channels)).astype(np.float32)
    reqs = make_stream(rng, 300, side, channels=channels)
    m, outs, lat, sts, stats = run_served(ash, capacity, (pk, pv), reqs, np.zeros(len(reqs)), channels=channels,
                                          fuse=True, max_fused=64, max_batch=1 << 16, in_flight=3)
    assert np.all(sts == 0) and stats["batches"] < len(reqs)
    check_against_oracle(capacity, (pk, pv), reqs, m, outs, channels=channels, values=True)


def test_served_tight_capacity_matches_serial(ash):
    """Inserts that overflow fail on their own, exactly as in serial order,
    even when the server would fuse them."""
    rng = np.random.default_rng(71)
    side, capacity = 30, 12_000
    pre = rng.choice(side ** 3, size=9_000, replace=False)
    pk = np.stack([pre // (side * side), (pre // side) % side, pre % side], axis=1).astype(np.int32)
    pv = rng.standard_normal((len(pk), 4)).astype(np.float32)
    reqs = make_stream(rng, 200, side, lo=64, hi=3000)
    m, outs, lat, sts, stats = run_served(ash, capacity, (pk, pv), reqs, np.zeros(len(reqs)), fuse=True,
                                          max_fused=32, max_batch=1 << 15, in_flight=2)
    check_against_oracle(capacity, (pk, pv), reqs, m, outs)


def test_fused_finds_mixed_outputs(ash):
    """Finds fused into one batch where some requests gather rows and some do
    not, some skip the index output, and one writes its rows to a view that
    starts 4 bytes into its buffer (the batch then copies in 4-byte units):
    every request still gets exactly the oracle's results and misses' rows
    stay untouched."""
    rng = np.random.default_rng(72)
    side, capacity, ch = 30, 40_000, 8
    pre = rng.choice(side ** 3, size=15_000, replace=False)
    pk = np.stack([pre // (side * side), (pre // side) % side, pre % side], axis=1).astype(np.int32)
    pv = rng.standard_normal((len(pk), ch)).astype(np.float32)
    m = ash.HashMap(capacity, 3, [(torch.float32, ch)])
    m.insert(dev(pk), [dev(pv)])
    o = OracleMap(capacity, 3, [(np.float32, ch)])
    o.insert(pk, [pv])
    torch.cuda.synchronize()
    srv = ash.Server(m, fuse=True, max_fused=64, max_batch=1 << 16, in_flight=2)
    built, outs, keep = [], [], []
    for i in range(40):
        n = int(rng.integers(1, 3000))
        keys = rng.integers(0, side + 5, size=(n, 3), dtype=np.int32)
        gather = i % 3 != 0
        base = torch.full((n * ch + 1,), 7.0, dtype=torch.float32, device="cuda")
        vals = base[1:].view(n, ch) if i == 5 else base[: n * ch].view(n, ch)  # request 5: 4-byte aligned rows
        idx = torch.full((n,), -7, dtype=torch.int32, device="cuda") if i % 4 != 1 else None
        mask = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        kd = dev(keys)
        r, k = srv.request(FIND, kd, [], out_idx=idx, out_mask=mask, out_values=[vals] if gather else None)
        built.append(r)
        keep.append((kd, k, base))
        outs.append((keys, gather, vals, idx, mask))
    lat, sts, span = srv.replay(built, np.zeros(len(built)))
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    assert np.all(sts == 0) and stats["batches"] < len(built)
    for keys, gather, vals, idx, mask in outs:
        st, oi, om, (ov,) = o.find(keys, gather=True, fill=7.0)
        assert np.array_equal(host(mask), om)
        if idx is not None:
            assert np.array_equal(host(idx), oi)
        got = host(vals)
        if gather:
            assert np.array_equal(bits(got), bits(ov))
        else:
            assert np.all(got == 7.0)


@pytest.mark.timeout(900)
def test_served_benchmark_shape(ash):
    """The served benchmark's own configuration: capacity 2^25, 20M keys
    preloaded with f32x8 rows, one lane per key (g = 1, W = 4, max load
    0.5), and the server settings it times (at most 256 requests and 2^22
    positions per fused batch, 4 batches in flight).  The stream, all
    arriving at once: 60 requests from the benchmark's distribution (60%
    find / 30% insert / 10% erase, sizes log-uniform in [256, 2^20], keys
    uniform over the 318^3 universe), then 300 consecutive small finds, 300
    consecutive small inserts and 40 erases (so fused batches carry 256
    requests), then 40 more benchmark requests: about 15M key operations.
    The preload is inserted in sorted key order (the same key set as the
    benchmark's; only the indices it receives differ), which keeps the
    oracle's 20M inserts to under a minute.  Every request's indices, masks
    and gathered rows must equal the oracle replaying the stream one request
    after another, and afterwards the heap, t, the active indices, k^B and
    v^B."""
    import synth
    w = synth.served(n_requests=100)
    order = np.lexsort(w["preload_keys"].T[::-1])
    pk = np.ascontiguousarray(w["preload_keys"][order])
    pv = np.ascontiguousarray(w["preload_values"][order])
    rng = np.random.default_rng(73)
    side, ch = w["side"], w["channels"]
    reqs = []
    for i in range(100):
        if i == 60:  # runs of one kind long enough to fill fused batches
            for kind, count, hi in ((FIND, 300, 4096), (INSERT, 300, 8192), (ERASE, 40, 4096)):
                for _ in range(count):
                    n = int(np.exp(rng.uniform(np.log(256), np.log(hi))))
                    keys = rng.integers(0, side, size=(n, 3), dtype=np.int32)
                    vals = rng.standard_normal((n, ch), dtype=np.float32) if kind == INSERT else None
                    reqs.append((kind, keys, vals))
        keys, vals = synth.request_keys(w, i)
        reqs.append((int(w["kinds"][i]), keys, vals))
    total = sum(len(k) for _, k, _ in reqs)
    print(f"case: served benchmark shape, {len(reqs)} requests, {total} positions, "
          f"preload {len(pk)}", flush=True)
    cfg = dict(fuse=True, max_fused=256, max_batch=1 << 22, in_flight=4)
    tuning = dict(probe_group=1, bucket_width=4, max_load=0.5)
    m, outs, lat, sts, stats = run_served(ash, w["capacity"], (pk, pv), reqs, np.zeros(len(reqs)), channels=ch,
                                          tuning=tuning, **cfg)
    print(f"served: {stats}", flush=True)
    assert np.all(sts == 0) and np.all(lat >= 0)
    assert stats["largest"] == 256  # the long runs filled fused batches
    check_against_oracle(w["capacity"], (pk, pv), reqs, m, outs, channels=ch, values=True)
