"""The separate-chaining backend of the backend ablation (include/ash_slab.h)
against the oracle.  Among equal keys of one batch, whichever position
claims first is inserted (the paper leaves it to the thread schedule), and
indices follow the order in which the heap hands them out to all positions
(three-pass insertion), so the comparison is canonical: the set of inserted
keys, one inserted position per new key, its stored key and row, the size,
the heap's free region, and every find.  Value rows are a function of the
key, so the row stored for a key does not depend on which of its positions
won."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import OracleMap  # noqa: E402
from tests.test_gpu_parity import bits, dev, host  # noqa: E402


@pytest.fixture(scope="module")
def slab():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_00511_amd import ablation
    return ablation


def rows_of(keys, channels):
    """f32 rows determined by the key (an integer mix of its words)."""
    k = keys.astype(np.uint64)
    h = np.full(len(keys), 0x9E3779B97F4A7C15, np.uint64)
    for d in range(keys.shape[1]):
        h = (h ^ k[:, d]) * np.uint64(0xBF58476D1CE4E5B9)
    cols = [((h >> np.uint64(8 * j)) & np.uint64(0xFFFF)).astype(np.float32) for j in range(channels)]
    return np.ascontiguousarray(np.stack(cols, axis=1))


def packed(keys):
    return [tuple(r) for r in keys.tolist()]


def check_insert(keys, g_idx, g_mask, o_mask, kb, vb, vals):
    g_mask = g_mask.astype(bool)
    o_mask = o_mask.astype(bool)
    assert g_mask.sum() == o_mask.sum(), "number of inserted keys differs"
    assert set(packed(keys[g_mask])) == set(packed(keys[o_mask])), "inserted key sets differ"
    assert len(set(packed(keys[g_mask]))) == int(g_mask.sum()), "a key was inserted twice"
    assert np.all(g_idx[~g_mask] == -1)
    ins = g_idx[g_mask]
    assert len(np.unique(ins)) == len(ins), "indices repeat"
    assert np.array_equal(kb[ins], keys[g_mask]), "k^B does not hold the inserted keys"
    if vb is not None:
        assert np.array_equal(bits(vb[ins]), bits(vals[g_mask])), "v^B rows differ"


@pytest.mark.parametrize("key_dim,channels", [(1, 1), (3, 8)])
def test_slab_backend_matches_oracle(slab, key_dim, channels):
    print(f"case: slab backend key_dim={key_dim} channels={channels}", flush=True)
    rng = np.random.default_rng(90 + key_dim)
    cap = 200_000
    side = {1: 100_000, 3: 46}[key_dim]
    m = slab.SlabMap(cap, key_dim, 4 * channels)
    o = OracleMap(cap, key_dim, [(np.float32, channels)])
    live = set()
    for b, n in enumerate((60_000, 50_000, 30_000)):
        keys = rng.integers(-side // 2, side // 2, size=(n, key_dim), dtype=np.int32)
        vals = rows_of(keys, channels)
        st, gi, gm = m.insert(dev(keys), dev(vals))
        assert st == 0
        _, oi, om = o.insert(keys, [vals])
        kb, vb, heap = m.read()
        gi, gm = host(gi), host(gm)
        check_insert(keys, gi, gm, om, kb, vb.view(np.float32) if vb is not None else None, vals)
        live.update(gi[gm == 1].tolist())
        t = m.size()
        assert t == o.size == len(live)
        free = heap[t:]
        assert sorted(free.tolist()) == sorted(set(range(cap)) - live), "heap free region is not the free indices"
        # finds: half present, half absent
        fk = np.concatenate([keys[rng.integers(0, n, size=n // 2)],
                             rng.integers(side, 2 * side, size=(n // 2, key_dim), dtype=np.int32)])
        fi, fm, fv = m.find(dev(fk), gather=True)
        _, ofi, ofm, (ofv,) = o.find(fk, gather=True, fill=0)
        fi, fm = host(fi), host(fm)
        assert np.array_equal(fm, ofm), f"batch {b}: find masks differ"
        hit = fm == 1
        assert np.all(fi[~hit] == -1)
        assert np.array_equal(kb[fi[hit]], fk[hit])
        assert np.array_equal(host(fv).view(np.uint8), bits(ofv)), f"batch {b}: gathered rows differ"


def test_slab_capacity_and_sets(slab):
    from paper_2110_00511_amd import _lib as L
    m = slab.SlabMap(1000, 3, 0)
    keys = np.arange(3 * 900, dtype=np.int32).reshape(900, 3)
    st, gi, gm = m.insert(dev(keys))
    assert st == 0 and m.size() == 900 and bool(host(gm).all())
    st, gi, gm = m.insert(dev(keys[:200]))  # 900 + 200 > 1000: every position takes an index first
    assert st == L.ASH_E_CAPACITY and m.size() == 900
    fi, fm, _ = m.find(dev(keys))
    assert bool(host(fm).all())
    st, gi, gm = m.insert(dev(keys[:100]))  # all present: none inserted, indices returned
    assert st == 0 and not host(gm).any() and m.size() == 900
