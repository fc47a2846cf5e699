"""Pins of the oracle's voxelization (Sec. 6.1, Listing 1: keys are
floor(xyz / voxel_size) in float32, a hash-set insertion keeps one entry per
voxel).  The independent route is numpy: float32 true division is IEEE
binary32, and numpy.unique(axis=0, return_index, return_inverse,
return_counts) gives the voxels, their first occurrences, the per-point voxel
and the counts; reordering by first occurrence gives the oracle's ids."""
import numpy as np
import pytest

import synth
from oracle import oracle_voxelize


def numpy_voxelize(points, voxel):
    pts = np.asarray(points, dtype=np.float32)
    q = pts / np.float32(voxel)
    f = np.floor(q)
    with np.errstate(invalid="ignore"):
        ok = np.all(np.isfinite(f) & (f >= -2.0 ** 31) & (f < 2.0 ** 31), axis=1)
    keys = f[ok].astype(np.int64).astype(np.int32)
    pv = np.full(len(pts), -1, np.int32)
    if len(keys) == 0:
        return pv, np.zeros((0, 3), np.int32), np.zeros(0, np.int32)
    uniq, first, inv, cnt = np.unique(keys, axis=0, return_index=True, return_inverse=True, return_counts=True)
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    pv[ok] = rank[inv.reshape(-1)]
    return pv, uniq[order].astype(np.int32), cnt[order].astype(np.int32)


def _compare(points, voxel):
    got = oracle_voxelize(points, voxel)
    want = numpy_voxelize(points, voxel)
    for g, w in zip(got, want):
        assert g.shape == w.shape and np.array_equal(g, w)
    return got


@pytest.mark.parametrize("voxel", [0.005, 0.01, 0.05])
def test_surface_points_match_numpy_unique(voxel):
    pts = synth.points(n=200_000, seed=21)
    pv, vk, cnt = _compare(pts, voxel)
    assert cnt.sum() == len(pts) and np.all(pv >= 0)


def test_division_not_reciprocal_at_cell_boundaries():
    # x / s and x * (1/s) differ in binary32 for some x near multiples of s;
    # floor of the true quotient decides the cell.
    s = np.float32(0.1)
    k = np.arange(-3000, 3000, dtype=np.float32)
    x = (k * s).astype(np.float32)
    x = np.concatenate([x, np.nextafter(x, np.float32(np.inf)), np.nextafter(x, np.float32(-np.inf))])
    div = np.floor(x / s)
    mul = np.floor(x * (np.float32(1.0) / s))
    assert np.any(div != mul), "the boundary set must separate division from reciprocal multiply"
    pts = np.stack([x, -x, x * np.float32(0.5)], axis=1)
    pv, vk, cnt = _compare(pts, s)
    assert np.array_equal(vk[pv[: len(x)], 0], div[: len(x)].astype(np.int32))


def test_negative_coordinates_floor_toward_minus_infinity():
    pts = np.array([[-0.001, -0.0, 0.0], [-0.004, 0.001, -0.006], [0.0049, -0.0051, 0.005]], np.float32)
    pv, vk, cnt = _compare(pts, 0.005)
    assert vk[pv[0]].tolist() == [-1, 0, 0]
    assert vk[pv[1]].tolist() == [-1, 0, -2]
    assert vk[pv[2]].tolist() == [0, -2, 1]


def test_rejected_points():
    big = np.float32(3e38)
    pts = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0, 0, -np.inf], [big, 0, 0],
                    [1.0, 1.0, 1.0], [-big, 0, 0], [1.0, 1.0, 1.0]], np.float32)
    pv, vk, cnt = _compare(pts, 0.005)
    assert pv.tolist() == [-1, -1, -1, -1, 0, -1, 0]
    assert vk.tolist() == [[200, 200, 200]] and cnt.tolist() == [2]


def test_int32_range_edges():
    # floor(q) = 2^31 - 128 (largest float below 2^31) is accepted, 2^31 is not;
    # -2^31 is accepted.
    hi = np.float32(2147483520.0)
    pts = np.array([[hi, 0, 0], [np.float32(2.0 ** 31), 0, 0], [np.float32(-2.0 ** 31), 0, 0]], np.float32)
    pv, vk, cnt = _compare(pts, 1.0)
    assert pv.tolist() == [0, -1, 1]
    assert vk.tolist() == [[2147483520, 0, 0], [-2147483648, 0, 0]]


def test_empty_and_single():
    pv, vk, cnt = _compare(np.zeros((0, 3), np.float32), 0.01)
    assert len(pv) == 0 and len(vk) == 0
    pv, vk, cnt = _compare(np.array([[0.5, 0.5, 0.5]], np.float32), 0.01)
    assert pv.tolist() == [0] and cnt.tolist() == [1]


# ---------------------------------------------------------------------------
# Block and in-block voxel coordinates (Sec. 6.2.2).
def test_block_coords_hand_worked():
    """x = -0.1 m, 0.0 m, 0.45 m with 5 cm voxels and 8^3 blocks: voxel
    indices -2, 0, 9 (binary32 quotients -2, 0, 9), blocks -1, 0, 1, local
    coordinates 6, 0, 1."""
    from oracle import oracle_block_coords
    bk, lc, ok = oracle_block_coords(np.array([[-0.1, 0.0, 0.45]], np.float32), 0.05, 8)
    assert ok.tolist() == [1]
    assert bk.tolist() == [[-1, 0, 1]] and lc.tolist() == [[6, 0, 1]]


@pytest.mark.parametrize("voxel,res", [(0.05, 8), (0.004, 16), (0.1, 3)])
def test_block_coords_recompose_voxel_keys(voxel, res):
    """block * res + local is the point's voxelization key; local lies in
    [0, res); away from block boundaries the block equals the paper's
    floor(x / (s * res)) evaluated in float64."""
    from oracle import oracle_block_coords, oracle_voxelize
    rng = np.random.default_rng(7)
    pts = (rng.standard_normal((20_000, 3)) * 3.0).astype(np.float32)
    bk, lc, ok = oracle_block_coords(pts, voxel, res)
    assert ok.all()
    pv, vk, _ = oracle_voxelize(pts, voxel)
    keys = vk[pv]
    assert np.array_equal(bk.astype(np.int64) * res + lc, keys)
    assert lc.min() >= 0 and lc.max() < res
    r = pts.astype(np.float64) / (float(np.float32(voxel)) * res)
    far = np.abs(r - np.round(r)) > 1e-4
    assert far.mean() > 0.99
    assert np.array_equal(bk[far], np.floor(r[far]).astype(np.int64))


def test_block_coords_rejects():
    from oracle import oracle_block_coords
    pts = np.array([[np.nan, 0, 0], [0, np.inf, 0], [3e38, 0, 0], [0.5, 0.5, 0.5]], np.float32)
    bk, lc, ok = oracle_block_coords(pts, 0.01, 8)
    assert ok.tolist() == [0, 0, 0, 1]
    assert not bk[:3].any() and not lc[:3].any()
