"""Pins of the oracle's neighbor lookups and set intersection against what
the mathematics fixes, independently of oracle/:

- Listing 3 (Sec. 6.2.4) finds every point's neighbors as finds of the point
  shifted by each offset; on a fresh map the index of the p-th new key is p,
  so expected indices follow from a Python dictionary built over the insert
  batch, with the sums wrapped in numpy's int32 arithmetic;
- on a full grid [0, L)^3 the number of neighbors found has a closed form per
  query: a product (radius and 1-cube lookups, Sec. 6.3) or a sum (1-ring) of
  per-axis counts;
- the intersection of Sec. 6.4 equals a Python set membership filter of the
  second set, order and duplicates kept."""
import itertools

import numpy as np
import pytest

from oracle import OracleMap

I32_MIN, I32_MAX = -2 ** 31, 2 ** 31 - 1


def cube_offsets(r, kd=3):
    return np.array(list(itertools.product(range(-r, r + 1), repeat=kd)), np.int32).reshape(-1, kd)


def fresh_index(keys):
    """key tuple -> buffer index of a fresh map after inserting keys in order."""
    first = {}
    for k in map(tuple, keys.tolist()):
        if k not in first:
            first[k] = len(first)
    return first


@pytest.mark.parametrize("kd", [1, 2, 3, 4])
def test_random_offsets_match_dictionary(kd):
    rng = np.random.default_rng(40 + kd)
    keys = rng.integers(-6, 6, size=(300, kd), dtype=np.int32)
    queries = rng.integers(-8, 8, size=(70, kd), dtype=np.int32)
    offsets = rng.integers(-3, 4, size=(11, kd), dtype=np.int32)
    m = OracleMap(400, kd)
    m.insert(keys)
    index = fresh_index(keys)
    st, idx, mask = m.find_offsets(queries, offsets)
    assert st == 0 and idx.shape == (70, 11) and mask.shape == (70, 11)
    for q in range(len(queries)):
        for o in range(len(offsets)):
            want = index.get(tuple((queries[q] + offsets[o]).tolist()), -1)
            assert idx[q, o] == want
            assert mask[q, o] == (want >= 0)


def test_full_grid_neighbor_counts_closed_form():
    L = 5
    grid = np.array(list(itertools.product(range(L), repeat=3)), np.int32)
    m = OracleMap(len(grid), 3)
    m.insert(grid)
    inner = lambda x: 1 + (x > 0).astype(int) + (x < L - 1).astype(int)  # noqa: E731
    _, idx_r, mask_r = m.find_offsets(grid, cube_offsets(1))
    assert np.array_equal(mask_r.sum(1), np.prod(inner(grid), axis=1))
    # a hit returns the neighbor's own index: lexicographic insertion gives index x*L*L + y*L + z
    off = cube_offsets(1)
    nb = grid[:, None, :] + off[None, :, :]
    lin = (nb[..., 0] * L + nb[..., 1]) * L + nb[..., 2]
    assert np.array_equal(idx_r[mask_r == 1], lin[mask_r == 1])
    assert np.all(idx_r[mask_r == 0] == -1)
    # 1-cube: the 2^3 grid points of the cell whose lowest corner is the query
    cube = np.array(list(itertools.product((0, 1), repeat=3)), np.int32)
    _, _, mask_c = m.find_offsets(grid, cube)
    assert np.array_equal(mask_c.sum(1), np.prod(1 + (grid < L - 1).astype(int), axis=1))
    # 1-ring: the six face neighbors
    ring = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], np.int32)
    _, _, mask_g = m.find_offsets(grid, ring)
    assert np.array_equal(mask_g.sum(1), ((grid > 0).astype(int) + (grid < L - 1).astype(int)).sum(1))
    # the zero offset finds every query itself at its own index
    zero_col = int(np.flatnonzero((off == 0).all(1))[0])
    assert np.array_equal(idx_r[:, zero_col], np.arange(len(grid)))


def test_sums_wrap_modulo_2_32():
    m = OracleMap(8, 3)
    stored = np.array([[I32_MIN, 0, 5], [I32_MAX, I32_MIN, 0]], np.int32)
    m.insert(stored)
    queries = np.array([[I32_MAX, 0, 5], [I32_MIN, I32_MAX, 0]], np.int32)
    offsets = np.array([[1, 0, 0], [-1, 1, 0], [0, 0, 0]], np.int32)
    _, idx, mask = m.find_offsets(queries, offsets)
    # INT32_MAX + 1 wraps to INT32_MIN; INT32_MIN - 1 wraps to INT32_MAX, INT32_MAX + 1 to INT32_MIN
    assert idx.tolist() == [[0, -1, -1], [-1, 1, -1]]
    assert mask.tolist() == [[1, 0, 0], [0, 1, 0]]


def test_erased_keys_are_not_neighbors():
    grid = np.array(list(itertools.product(range(3), repeat=3)), np.int32)
    m = OracleMap(64, 3)
    m.insert(grid)
    gone = grid[::2]
    m.erase(gone)
    kept = {tuple(k) for k in grid[1::2].tolist()}
    _, idx, mask = m.find_offsets(grid, cube_offsets(1))
    for q in range(len(grid)):
        for o, d in enumerate(cube_offsets(1)):
            assert mask[q, o] == (tuple((grid[q] + d).tolist()) in kept)


def test_empty_queries_and_offsets():
    m = OracleMap(4, 3)
    m.insert(np.zeros((1, 3), np.int32))
    st, idx, mask = m.find_offsets(np.zeros((0, 3), np.int32), cube_offsets(1))
    assert st == 0 and idx.shape == (0, 27)
    st, idx, mask = m.find_offsets(np.zeros((4, 3), np.int32), np.zeros((0, 3), np.int32))
    assert st == 0 and idx.shape == (4, 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_intersection_is_an_ordered_membership_filter(seed):
    rng = np.random.default_rng(60 + seed)
    a = rng.integers(0, 7, size=(150, 3), dtype=np.int32)
    b = rng.integers(0, 9, size=(200, 3), dtype=np.int32)  # duplicates and misses
    m = OracleMap(400, 3)
    m.insert(a)
    got = m.intersect(b)
    members = set(map(tuple, a.tolist()))
    want = [row for row in b.tolist() if tuple(row) in members]
    assert got.tolist() == want
    assert len(want) < len(b) and len(want) > 0
    assert m.intersect(np.zeros((0, 3), np.int32)).shape == (0, 3)
    # the set intersection, with numpy's own row operations
    assert np.array_equal(np.unique(got, axis=0),
                          np.array(sorted(members & set(map(tuple, b.tolist()))), np.int32))
