"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle: each check compares it with a different
route to the same answer --
  * brute force over every short operation sequence on a tiny key universe,
    against the dictionary model in tests/model.py;
  * closed forms for a fresh map (numpy.unique first occurrences and ranks:
    with h = 0, 1, ..., c-1 the p-th new key gets index p among new keys);
  * invariants of the index heap (Sec. 4.3: the free region h[t:c] is exactly
    the set of indices not in use) and of lookups after erase / rehash;
  * a hand-worked sequence (Sec. 4.3: t rises on allocation, falls on free).
"""
import itertools

import numpy as np
import pytest

from oracle import ORACLE_E_CAPACITY, ORACLE_OK, OracleMap
from tests.model import DictModel


def _tuples(keys):
    return [tuple(int(x) for x in row) for row in np.asarray(keys).reshape(len(keys), -1)]


def _check_heap_invariant(m):
    c, t = m.capacity, m.heap_top
    h = m.heap()
    act = m.active_flags()
    free = np.sort(h[t:c])
    expect = np.flatnonzero(act == 0).astype(np.int32)
    assert t == m.size == int(act.sum())
    assert np.array_equal(free, expect), "free region of the heap is not the complement of the live set"


def test_worked_example_heap_discipline():
    # insert a, b, a, c into a capacity-4 map: the duplicate of a loses.
    m = OracleMap(4, key_dim=1, value_specs=[(np.int32, 1)])
    st, idx, mask = m.insert([[5], [7], [5], [9]], [np.array([[10], [11], [12], [13]])])
    assert st == ORACLE_OK
    assert mask.tolist() == [1, 1, 0, 1] and idx.tolist() == [0, 1, -1, 2]
    assert m.value_buffer(0)[:3, 0].tolist() == [10, 11, 13]
    # erase b twice in one batch: the first frees index 1 (t: 3 -> 2, h[2] = 1)
    st, mask = m.erase([[7], [7]])
    assert mask.tolist() == [1, 0] and m.heap_top == 2 and m.heap()[2] == 1
    # the next new key reuses the freed index from the heap top
    st, idx, mask = m.insert([[8]], [np.array([[14]])])
    assert idx.tolist() == [1] and mask.tolist() == [1]
    st, idx, mask = m.find([[5], [7], [8], [9]])
    assert idx.tolist() == [0, -1, 1, 2] and mask.tolist() == [1, 0, 1, 1]
    _check_heap_invariant(m)


@pytest.mark.parametrize("capacity", [2, 3, 8])
def test_exhaustive_two_op_sequences(capacity):
    """All sequences of two batches (length <= 3 over a 3-key universe) of
    insert / activate / erase, then a find of every key."""
    universe = [(0,), (1,), (2,)]
    batches = [list(b) for L in range(4) for b in itertools.product(universe, repeat=L)]
    ops = ["insert", "activate", "erase"]
    count = 0
    for (op1, b1), (op2, b2) in itertools.product(itertools.product(ops, batches), repeat=2):
        m = OracleMap(capacity, key_dim=1, value_specs=[(np.int32, 1)])
        d = DictModel(capacity)
        for op, b in ((op1, b1), (op2, b2)):
            keys = np.array(b, dtype=np.int32).reshape(-1, 1)
            vals = np.arange(100, 100 + len(b), dtype=np.int32).reshape(-1, 1)
            if op == "erase":
                st, mask = m.erase(keys)
                assert mask.tolist() == d.erase(b)
            else:
                act = op == "activate"
                if act:
                    st, idx, mask = m.activate(keys)
                else:
                    st, idx, mask = m.insert(keys, [vals])
                dst, didx, dmask = d.insert(b, [[int(v) for v in vals[:, 0]]], activate=act)
                assert st == dst and idx.tolist() == didx and mask.tolist() == dmask
        idx, mask = m.find(np.array(universe, dtype=np.int32))[1:]
        didx, dmask = d.find(universe)
        assert idx.tolist() == didx and mask.tolist() == dmask
        assert m.active_indices().tolist() == d.active()
        assert m.heap_top == d.top and m.heap().tolist() == d.heap
        vb = m.value_buffer(0)[:, 0]
        for k, i in d.table.items():
            if d.values.get(i):
                assert vb[i] == d.values[i][0]
        count += 1
    assert count == (len(ops) * len(batches)) ** 2


def test_random_sequences_against_model():
    rng = np.random.default_rng(123)
    for trial in range(300):
        cap = int(rng.integers(1, 12))
        kd = int(rng.integers(1, 5))
        m = OracleMap(cap, key_dim=kd, value_specs=[(np.float32, 2), (np.uint8, 3)])
        d = DictModel(cap)
        for step in range(6):
            n = int(rng.integers(0, 10))
            keys = rng.integers(-2, 2, size=(n, kd), dtype=np.int32)
            tk = _tuples(keys) if n else []
            op = rng.choice(["insert", "insert_grow", "activate", "erase", "find"])
            if op == "erase":
                st, mask = m.erase(keys)
                assert mask.tolist() == d.erase(tk)
            elif op == "find":
                st, idx, mask = m.find(keys)
                didx, dmask = d.find(tk)
                assert idx.tolist() == didx and mask.tolist() == dmask
            else:
                v0 = rng.standard_normal((n, 2)).astype(np.float32)
                v1 = rng.integers(0, 255, size=(n, 3), dtype=np.uint8)
                grow = op == "insert_grow"
                if op == "activate":
                    st, idx, mask = m.activate(keys)
                    dst, didx, dmask = d.insert(tk, activate=True)
                else:
                    st, idx, mask = m.insert(keys, [v0, v1], autogrow=grow)
                    dst, didx, dmask = d.insert(tk, [[tuple(r) for r in v0], [tuple(r) for r in v1]], autogrow=grow)
                assert st == dst and idx.tolist() == didx and mask.tolist() == dmask
                assert m.capacity == d.c
            assert m.heap().tolist() == d.heap and m.heap_top == d.top
            for k, i in d.table.items():
                assert tuple(m.key_buffer()[i]) == k
                vals = d.values.get(i)
                if vals:
                    assert tuple(m.value_buffer(0)[i]) == vals[0]
                    assert tuple(m.value_buffer(1)[i]) == vals[1]
            _check_heap_invariant(m)


def _pack(keys):
    k = keys.astype(np.int64) + (1 << 20)
    return (k[:, 0] << 42) | (k[:, 1] << 21) | k[:, 2]


def test_fresh_insert_matches_unique_first_occurrence():
    rng = np.random.default_rng(7)
    n = 50_000
    keys = rng.integers(-40, 40, size=(n, 3), dtype=np.int32)
    vals = rng.standard_normal((n, 4)).astype(np.float32)
    m = OracleMap(n, 3, [(np.float32, 4)])
    st, idx, mask = m.insert(keys, [vals])
    assert st == ORACLE_OK
    uniq, first = np.unique(_pack(keys), return_index=True)
    want_mask = np.zeros(n, np.uint8)
    want_mask[first] = 1
    assert np.array_equal(mask, want_mask)
    # fresh heap 0..c-1: the winners get consecutive indices in position order
    want_idx = np.full(n, -1, np.int32)
    want_idx[np.sort(first)] = np.arange(len(first), dtype=np.int32)
    assert np.array_equal(idx, want_idx)
    sel = np.flatnonzero(mask)
    assert np.array_equal(m.key_buffer()[idx[sel]], keys[sel])
    assert np.array_equal(m.value_buffer(0)[idx[sel]].view(np.uint32), vals[sel].view(np.uint32))
    # find: membership by binary search over the sorted distinct keys
    q = np.concatenate([keys[rng.integers(0, n, 20_000)], rng.integers(40, 80, size=(20_000, 3), dtype=np.int32)])
    st, fidx, fmask, (out,) = m.find(q, gather=True, fill=-7.0)
    pos = np.searchsorted(uniq, _pack(q))
    hit = (pos < len(uniq)) & (uniq[np.minimum(pos, len(uniq) - 1)] == _pack(q))
    assert np.array_equal(fmask.astype(bool), hit)
    first_of = np.sort(first)
    # the index of a hit is the rank of its key's first occurrence
    rank_of_key = dict(zip(_pack(keys[first_of]).tolist(), range(len(first_of))))
    assert all(fidx[p] == rank_of_key[k] for p, k in zip(np.flatnonzero(hit), _pack(q[hit]).tolist()))
    assert np.all(fidx[~hit] == -1)
    assert np.array_equal(out[hit].view(np.uint32), m.value_buffer(0)[fidx[hit]].view(np.uint32))
    assert np.all(out[~hit] == -7.0)


def test_erase_then_find_invariants():
    rng = np.random.default_rng(11)
    n = 20_000
    keys = rng.integers(0, 30, size=(n, 3), dtype=np.int32)
    vals = rng.standard_normal((n, 1)).astype(np.float32)
    m = OracleMap(2 * n, 3, [(np.float32, 1)])
    m.insert(keys, [vals])
    distinct = len(np.unique(_pack(keys)))
    before_idx = m.find(keys)[1]
    er = keys[rng.choice(n, n // 4, replace=False)]
    st, emask = m.erase(er)
    er_distinct = np.unique(_pack(er), return_index=True)[1]
    want = np.zeros(len(er), np.uint8)
    want[er_distinct] = 1                     # every erased key was present
    assert np.array_equal(emask, want)
    assert m.size == distinct - len(er_distinct)
    st, idx, mask = m.find(keys)
    erased = np.isin(_pack(keys), _pack(er))
    assert np.all(mask[erased] == 0) and np.all(idx[erased] == -1)
    assert np.all(mask[~erased] == 1) and np.array_equal(idx[~erased], before_idx[~erased])
    _check_heap_invariant(m)
    # the re-found keys still return their inserted (first-occurrence) values
    firsts = {}
    for p, k in enumerate(_pack(keys).tolist()):
        firsts.setdefault(k, p)
    live = np.flatnonzero(~erased)
    want_vals = vals[[firsts[k] for k in _pack(keys[live]).tolist()], 0]
    assert np.array_equal(m.value_buffer(0)[idx[live], 0].view(np.uint32), want_vals.view(np.uint32))


def test_capacity_overflow_leaves_map_unchanged_and_autogrow_doubles():
    m = OracleMap(4, 1, [(np.int32, 1)])
    m.insert([[1], [2], [3]], [np.array([[1], [2], [3]])])
    h0, kb0, v0, t0 = m.heap(), m.key_buffer(), m.value_buffer(0), m.heap_top
    st, idx, mask = m.insert([[4], [5], [1]], [np.array([[4], [5], [6]])])
    assert st == ORACLE_E_CAPACITY and idx.tolist() == [-1, -1, -1] and mask.tolist() == [0, 0, 0]
    assert np.array_equal(m.heap(), h0) and np.array_equal(m.key_buffer(), kb0)
    assert np.array_equal(m.value_buffer(0), v0) and m.heap_top == t0
    # with auto-growth the capacity doubles (4 -> 8 is the smallest that fits 5)
    st, idx, mask = m.insert([[4], [5], [6], [1]], [np.array([[4], [5], [6], [7]])], autogrow=True)
    assert st == ORACLE_OK and m.capacity == 8 and mask.tolist() == [1, 1, 1, 0]
    assert idx.tolist() == [3, 4, 5, -1]
    _check_heap_invariant(m)


def test_rehash_keeps_indices_and_values():
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 20, size=(500, 3), dtype=np.int32)
    vals = rng.standard_normal((500, 3)).astype(np.float32)
    m = OracleMap(600, 3, [(np.float32, 3)])
    m.insert(keys, [vals])
    m.erase(keys[:100])
    idx0 = m.find(keys)[1]
    kb0 = m.key_buffer()
    vb0 = m.value_buffer(0)
    h0, t0 = m.heap(), m.heap_top
    assert m.rehash(m.size - 1) != ORACLE_OK and m.rehash(599) != ORACLE_OK
    assert m.rehash(1500) == ORACLE_OK
    assert m.capacity == 1500 and m.heap_top == t0
    assert np.array_equal(m.find(keys)[1], idx0)
    assert np.array_equal(m.key_buffer()[:600], kb0) and np.array_equal(m.value_buffer(0)[:600], vb0)
    assert np.array_equal(m.heap()[:600], h0) and np.array_equal(m.heap()[600:], np.arange(600, 1500))
    _check_heap_invariant(m)


def test_empty_batches():
    m = OracleMap(3, 3, [(np.float32, 1)])
    z = np.zeros((0, 3), np.int32)
    st, idx, mask = m.insert(z, [np.zeros((0, 1), np.float32)])
    assert st == ORACLE_OK and len(idx) == 0
    assert m.erase(z)[0] == ORACLE_OK and m.find(z)[0] == ORACLE_OK
    assert m.size == 0 and m.active_indices().tolist() == []


def test_extreme_int32_keys():
    lo, hi = np.iinfo(np.int32).min, np.iinfo(np.int32).max
    keys = np.array([[lo, lo, lo], [hi, hi, hi], [lo, hi, 0], [-1, -1, -1], [lo, lo, lo]], np.int32)
    m = OracleMap(8, 3)
    st, idx, mask = m.insert(keys)
    assert mask.tolist() == [1, 1, 1, 1, 0] and idx.tolist() == [0, 1, 2, 3, -1]
    assert np.array_equal(m.find(keys)[1], np.array([0, 1, 2, 3, 0], np.int32))
