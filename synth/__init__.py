"""Seeded synthetic workloads shaped like the ASH paper's experiments.

This module only draws random inputs (numpy PCG64 via default_rng); it holds
none of the hash map's arithmetic and is shared by the tests, the oracle runs
and the benchmark so that every side sees identical bytes.

Workloads (sizes and shapes; the paper's Setups 1-3 of Sec. 5.1 and 6.1 are the
model, extended to 10M keys):
  plain_small   65,536 int32x3 keys uniform in [0,64)^3, value f32 v[p] = p,
                capacity 131,072, a 50%-hit find batch, a 25% erase batch
  plain_large   10M int32x3 keys uniform in a cube of side L chosen for a
                distinct ratio rho in {0.1, 0.5, 0.99}, f32 x C values,
                10M finds at 50% hit, 5M erases
  points        5M float32 xyz points on 20 random spheres/planes in a 10 m
                box with N(0, 1 cm) noise (stand-in for the paper's scans)
  surface_keys  the distinct lattice cells (int32x3) of those points on a
                5 mm grid, in order of first appearance: the key set of a
                neighbor search (Listing 3 of Sec. 6.2.4)
  value_sweep   1M int32x3 keys (distinct ratio ~0.99) and a 50%-hit find
                batch for value rows of 2^j floats (Setup 1's sweep)
  setup1        n int32x3 keys at distinct ratio rho and a 50%-hit find
                batch (Setup 1's capacities 10^3..10^6, rho in {0.1, 0.99})
  setup2        n scalar int32 keys at distinct ratio rho and a 50%-hit find
                batch (Setup 2 of Sec. 5.2)
  batched       64 maps with log-uniform distinct counts in [1e3, 1e6]
  served        request stream over a 318^3 key universe
"""
import math

import numpy as np

# Cube side per distinct ratio for 10M uniform draws: the expected number of
# distinct keys of n draws from L^3 cells is L^3 (1 - exp(-n / L^3)).
PLAIN_LARGE_SIDE = {0.1: 100, 0.5: 184, 0.99: 792}


def plain_small(seed=1):
    """65,536-key insert / find / erase / re-find sequence."""
    rng = np.random.default_rng(seed)
    n = 65536
    keys = rng.integers(0, 64, size=(n, 3), dtype=np.int32)
    values = np.arange(n, dtype=np.float32).reshape(n, 1)
    half = n // 2
    present = keys[rng.choice(n, size=half, replace=False)]
    absent = rng.integers(64, 128, size=(half, 3), dtype=np.int32)
    find_keys = np.concatenate([present, absent])[rng.permutation(n)]
    erase_keys = keys[rng.choice(n, size=n // 4, replace=False)]
    return dict(capacity=131072, keys=keys, values=values,
                find_keys=np.ascontiguousarray(find_keys),
                erase_keys=np.ascontiguousarray(erase_keys))


def plain_large(rho=0.5, channels=8, n=10_000_000, seed=None, with_values=True):
    """10M-key workload at distinct ratio rho with f32 x channels values.

    capacity = 2 * rho * n (twice the nominal distinct count)."""
    if seed is None:
        seed = {0.1: 2, 0.5: 3, 0.99: 4}[rho]
    side = PLAIN_LARGE_SIDE[rho]
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, side, size=(n, 3), dtype=np.int32)
    values = rng.standard_normal((n, channels), dtype=np.float32) if with_values else None
    half = n // 2
    present = keys[rng.integers(0, n, size=half)]
    absent = rng.integers(side, 2 * side, size=(n - half, 3), dtype=np.int32)
    find_keys = np.concatenate([present, absent])[rng.permutation(n)]
    erase_keys = keys[rng.choice(n, size=n // 2, replace=False)]
    return dict(capacity=int(2 * round(rho * n)), side=side, keys=keys, values=values,
                find_keys=np.ascontiguousarray(find_keys),
                erase_keys=np.ascontiguousarray(erase_keys))


def points(n=5_000_000, n_surfaces=20, box=10.0, sigma=0.01, seed=5):
    """Points sampled on random spheres (radius 0.3-2 m) and rectangular
    planes (sides 1-4 m) in a box, counts proportional to area, plus Gaussian
    noise.  Points of one surface are contiguous, in random order."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(n_surfaces):
        if rng.random() < 0.5:
            r = rng.uniform(0.3, 2.0)
            c = rng.uniform(r, box - r, size=3)
            shapes.append(("sphere", c, r, 4.0 * math.pi * r * r))
        else:
            a, b = rng.uniform(1.0, 4.0, size=2)
            c = rng.uniform(2.0, box - 2.0, size=3)
            nrm = rng.standard_normal(3)
            nrm /= np.linalg.norm(nrm)
            u = np.cross(nrm, [1.0, 0.0, 0.0] if abs(nrm[0]) < 0.9 else [0.0, 1.0, 0.0])
            u /= np.linalg.norm(u)
            v = np.cross(nrm, u)
            shapes.append(("plane", c, (a, b, u, v), a * b))
    areas = np.array([s[3] for s in shapes])
    counts = np.floor(n * areas / areas.sum()).astype(np.int64)
    counts[np.argmax(counts)] += n - counts.sum()
    out = []
    for (kind, c, prm, _), m in zip(shapes, counts):
        if kind == "sphere":
            d = rng.standard_normal((m, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            p = c + prm * d
        else:
            a, b, u, v = prm
            s = rng.uniform(-a / 2, a / 2, size=(m, 1))
            t = rng.uniform(-b / 2, b / 2, size=(m, 1))
            p = c + s * u + t * v
        out.append(p + rng.normal(0.0, sigma, size=(m, 3)))
    return np.ascontiguousarray(np.concatenate(out).astype(np.float32))


def surface_keys(n=5_000_000, cell=0.005, seed=5):
    """Distinct lattice cells of the surface points (nearest lattice point of
    a cell-unit grid, in float64), in order of first appearance: integer keys
    with the structure of a scanned surface."""
    pts = points(n=n, seed=seed).astype(np.float64)
    cells = np.rint(pts / cell).astype(np.int32)
    _, first = np.unique(cells, axis=0, return_index=True)
    return np.ascontiguousarray(cells[np.sort(first)])


def value_sweep(n=1_000_000, side=368, seed=8):
    """Keys of the value-size sweep (Setup 1 of Sec. 5.1 at its largest c):
    n int32x3 keys uniform in [0, side)^3 (distinct ratio ~0.99 for the
    defaults) and an n-key find batch, half drawn from the inserted keys and
    half from [side, 2 side)^3.  Value rows are drawn by the caller."""
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, side, size=(n, 3), dtype=np.int32)
    half = n // 2
    present = keys[rng.integers(0, n, size=half)]
    absent = rng.integers(side, 2 * side, size=(n - half, 3), dtype=np.int32)
    find_keys = np.concatenate([present, absent])[rng.permutation(n)]
    return dict(keys=keys, find_keys=np.ascontiguousarray(find_keys))


def cube_for_ratio(n, rho, dims=3):
    """Side L of a cube whose n uniform draws hold about rho * n distinct
    cells: L^d (1 - exp(-n / L^d)) = rho n, solved for x = n / L^d by
    bisection (input generation only)."""
    lo, hi = 1e-9, 1e3
    for _ in range(200):
        x = 0.5 * (lo + hi)
        if (1.0 - math.exp(-x)) / x > rho:
            lo = x
        else:
            hi = x
    return max(2, int(round((n / (0.5 * (lo + hi))) ** (1.0 / dims))))


def setup2(n, rho, seed=11):
    """Setup 2 of Sec. 5.2 at one (c, rho): n int32 scalar keys uniform in
    [0, L) with L sized for distinct ratio rho, and n finds, half drawn from
    the inserted keys and half from [L, 2L)."""
    rng = np.random.default_rng([seed, n, int(round(rho * 100))])
    side = cube_for_ratio(n, rho, dims=1)
    keys = rng.integers(0, side, size=(n, 1), dtype=np.int32)
    half = n // 2
    present = keys[rng.integers(0, n, size=half)]
    absent = rng.integers(side, 2 * side, size=(n - half, 1), dtype=np.int32)
    find_keys = np.concatenate([present, absent])[rng.permutation(n)]
    return dict(keys=keys, find_keys=np.ascontiguousarray(find_keys), side=side)


def setup1(n, rho, seed=10):
    """Setup 1 of Sec. 5.1 at one (c, rho): n int32x3 keys uniform in a cube
    sized for distinct ratio rho (the capacity is n), and n finds, half drawn
    from the inserted keys and half from the cube shifted by its side."""
    rng = np.random.default_rng([seed, n, int(round(rho * 100))])
    side = cube_for_ratio(n, rho)
    keys = rng.integers(0, side, size=(n, 3), dtype=np.int32)
    half = n // 2
    present = keys[rng.integers(0, n, size=half)]
    absent = rng.integers(side, 2 * side, size=(n - half, 3), dtype=np.int32)
    find_keys = np.concatenate([present, absent])[rng.permutation(n)]
    return dict(keys=keys, find_keys=np.ascontiguousarray(find_keys), side=side)


def batched(n_maps=64, channels=8, lo=1e3, hi=1e6, seed=6):
    """Per-map inserts (2 u_m keys, distinct ratio ~0.5) and 50%-hit finds.

    For a target of u distinct keys among 2u uniform draws the cube holds
    x = 2u / y cells with 2 (1 - exp(-y)) = y, i.e. y ~= 1.5936."""
    rng = np.random.default_rng(seed)
    y = 1.5936
    maps = []
    for _ in range(n_maps):
        u = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        side = max(2, int(round((2 * u / y) ** (1.0 / 3.0))))
        keys = rng.integers(0, side, size=(2 * u, 3), dtype=np.int32)
        values = rng.standard_normal((2 * u, channels), dtype=np.float32)
        present = keys[rng.integers(0, 2 * u, size=u)]
        absent = rng.integers(side, 2 * side, size=(u, 3), dtype=np.int32)
        find_keys = np.concatenate([present, absent])[rng.permutation(2 * u)]
        maps.append(dict(capacity=2 * u, keys=keys, values=values,
                         find_keys=np.ascontiguousarray(find_keys)))
    return maps


def served(n_requests=100_000, capacity=1 << 25, side=318, preload=20_000_000,
           channels=8, lo=256, hi=1 << 20, mix=(0.6, 0.3, 0.1), seed=7):
    """Preload keys/values and a request list (kind, keys[, values]) with
    unit-mean exponential inter-arrival gaps (scaled by the caller)."""
    rng = np.random.default_rng(seed)
    cells = rng.choice(side ** 3, size=preload, replace=False)
    pre = np.stack([cells // (side * side), (cells // side) % side, cells % side], axis=1).astype(np.int32)
    pre_values = rng.standard_normal((preload, channels), dtype=np.float32)
    kinds = rng.choice(3, size=n_requests, p=list(mix))  # 0 find, 1 insert, 2 erase
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_requests)).astype(np.int64)
    gaps = rng.exponential(1.0, size=n_requests)
    return dict(capacity=capacity, side=side, preload_keys=pre, preload_values=pre_values,
                kinds=kinds, sizes=sizes, gaps=gaps, channels=channels, seed=seed)


def request_keys(req, i, rng=None):
    """Keys (and values for inserts) of request i, drawn from its own stream."""
    r = np.random.default_rng([req["seed"], i])
    m = int(req["sizes"][i])
    keys = r.integers(0, req["side"], size=(m, 3), dtype=np.int32)
    vals = r.standard_normal((m, req["channels"]), dtype=np.float32) if req["kinds"][i] == 1 else None
    return keys, vals
