"""GPU parity of the neighbor lookups (Listing 3 of Sec. 6.2.4; the 1-cube
and 1-ring lookups of Sec. 6.3) and of set intersection (Sec. 6.4): the HIP
path through the C ABI against the CPU oracle, bit-exact (indices, masks,
selected rows), over probe shapes, neighborhoods, offsets whose sums wrap,
tables with tombstones, every key width, empty and ragged inputs, and the
full-size neighbor search on sampled queries."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import OracleMap  # noqa: E402
from tests.test_gpu_parity import dev, host  # noqa: E402

I32_MIN, I32_MAX = -2 ** 31, 2 ** 31 - 1


@pytest.fixture(scope="module")
def ash():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash_mod
    return ash_mod


def pair(ash, keys, capacity=None, **tuning):
    kd = keys.shape[1]
    cap = capacity or max(2 * len(keys), 16)
    g = ash.HashMap(cap, key_dim=kd, **tuning)
    g.insert(dev(keys))
    o = OracleMap(cap, kd)
    o.insert(keys)
    return g, o


def check_offsets(g, o, queries, offsets):
    gi, gm = g.find_offsets(dev(queries), dev(offsets))
    st, oi, om = o.find_offsets(queries, offsets)
    assert st == 0
    assert gi.shape == (len(queries), len(offsets))
    assert np.array_equal(host(gm).astype(np.uint8), om), "neighbor masks differ"
    assert np.array_equal(host(gi), oi), "neighbor indices differ"
    return om


SHAPES = [(1, 2, 0.5), (1, 4, 0.7), (1, 8, 0.9), (4, 4, 0.5), (16, 8, 0.85), (64, 16, 0.5)]


@pytest.mark.parametrize("g,w,lf", SHAPES)
@pytest.mark.parametrize("kind,radius", [("radius", 1), ("ring", 1), ("cube", 1), ("radius", 2)])
def test_neighborhoods_match_oracle(ash, g, w, lf, kind, radius):
    keys = synth.surface_keys(n=30_000, cell=0.05, seed=21)
    gm, om = pair(ash, keys, probe_group=g, bucket_width=w, max_load=lf)
    rng = np.random.default_rng(22)
    stray = rng.integers(keys.min(), keys.max() + 1, size=(777, 3), dtype=np.int32)
    queries = np.concatenate([keys, stray])  # ragged: not a multiple of any tile
    offsets = host(ash.neighbor_offsets(kind, radius))
    mask = check_offsets(gm, om, queries, offsets)
    assert 0.05 < mask.mean() < 0.95  # a real mix of hits and misses


@pytest.mark.parametrize("kd", [1, 2, 3, 4])
def test_random_offsets_every_key_width(ash, kd):
    rng = np.random.default_rng(30 + kd)
    keys = np.unique(rng.integers(-40, 40, size=(5000, kd), dtype=np.int32), axis=0)
    keys = keys[rng.permutation(len(keys))]
    gm, om = pair(ash, keys)
    queries = rng.integers(-45, 45, size=(3001, kd), dtype=np.int32)
    offsets = rng.integers(-4, 5, size=(13, kd), dtype=np.int32)
    check_offsets(gm, om, queries, offsets)


def test_offset_sums_wrap(ash):
    keys = np.array([[I32_MIN, 0, 5], [I32_MAX, I32_MIN, 0], [0, 0, 0]], np.int32)
    gm, om = pair(ash, keys, capacity=16)
    queries = np.array([[I32_MAX, 0, 5], [I32_MIN, I32_MAX, 0], [1, -1, 0]], np.int32)
    offsets = np.array([[1, 0, 0], [-1, 1, 0], [0, 0, 0], [I32_MAX, 1, 0]], np.int32)
    mask = check_offsets(gm, om, queries, offsets)
    assert mask.sum() == 3


def test_neighbors_after_erase(ash):
    """Tombstones in the probe sequences: erased keys must read as misses and
    keys behind tombstones must still be found."""
    keys = synth.surface_keys(n=40_000, cell=0.04, seed=23)
    gm, om = pair(ash, keys, capacity=len(keys), max_load=0.9, probe_group=1, bucket_width=4)
    gone = keys[::3]
    gm.erase(dev(gone))
    om.erase(gone)
    offsets = host(ash.neighbor_offsets("radius", 1))
    check_offsets(gm, om, keys, offsets)


def test_empty_inputs(ash):
    keys = synth.surface_keys(n=1000, cell=0.05, seed=24)
    gm, om = pair(ash, keys)
    offsets = host(ash.neighbor_offsets("cube", 1))
    check_offsets(gm, om, np.zeros((0, 3), np.int32), offsets)
    check_offsets(gm, om, keys, np.zeros((0, 3), np.int32))
    assert gm.intersect(dev(np.zeros((0, 3), np.int32))).shape == (0, 3)
    empty = ash.HashMap(16, 3)
    idx, mask = empty.find_offsets(dev(keys), dev(offsets))
    assert bool((host(idx) == -1).all()) and not bool(host(mask).any())


@pytest.mark.parametrize("g", [1, 4, 64])
@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 70_001])
def test_intersect_matches_oracle(ash, g, n):
    rng = np.random.default_rng(40 + n)
    a = rng.integers(0, 30, size=(max(n // 2, 1), 3), dtype=np.int32)
    b = rng.integers(0, 40, size=(n, 3), dtype=np.int32)  # duplicates and misses
    gm, om = pair(ash, a, probe_group=g, bucket_width=4)
    got = host(gm.intersect(dev(b)))
    want = om.intersect(b)
    assert np.array_equal(got, want)
    # all hits / no hits
    assert np.array_equal(host(gm.intersect(dev(a))), a)
    assert host(gm.intersect(dev(b + 1000))).shape == (0, 3)


def test_full_size_neighbor_search(ash):
    """The benchmark's shape: the 27-neighborhood of every one of 4.8M surface
    cells.  A seeded sample of queries is checked against the oracle row by
    row; over all queries, the zero offset finds every key at its own index
    and each offset o hits exactly as often as -o (the query set is the key
    set)."""
    keys = synth.surface_keys()
    n = len(keys)
    gm = ash.HashMap(n, 3)
    gm.insert(dev(keys))
    offsets = ash.neighbor_offsets("radius", 1)
    idx, mask = gm.find_offsets(dev(keys), offsets)
    idx, mask = host(idx), host(mask)
    assert idx.shape == (n, 27)
    assert np.array_equal(idx[:, 13], np.arange(n, dtype=np.int32))  # fresh map: p-th key at index p
    hits = mask.sum(axis=0)
    assert np.array_equal(hits, hits[::-1])  # offsets are enumerated symmetrically
    assert np.all(idx[~mask] == -1)
    om = OracleMap(n, 3)
    om.insert(keys)
    sample = np.random.default_rng(25).choice(n, size=20_000, replace=False)
    st, oi, omask = om.find_offsets(keys[sample], host(offsets))
    assert np.array_equal(idx[sample], oi)
    assert np.array_equal(mask[sample].astype(np.uint8), omask)
