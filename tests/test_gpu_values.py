"""Large value rows and the double hash map (Sec. 6.2.3, Listing 2; Setup 1's
value sweep of Sec. 5.1): the row-copy paths against the oracle, bit-exact.

- rows from 4 B to 16 KB (f32 x 2^j), the 8^3 x {1, 3} f32 blocks of
  Listing 2 as two value buffers, and odd row sizes that force narrow copy
  units, through insert (rows copied inside the commit or by the separate row
  pass) and find with gather;
- the local -> global activation of Listing 2 over several frames: a local
  map activates the block coordinates of a frame's points, the first
  occurrences go to the global map (activate, then find), and the local map's
  value row of each block receives its global index."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import OracleMap  # noqa: E402
from tests.test_gpu_parity import Pair, dev, host  # noqa: E402


@pytest.fixture(scope="module")
def ash():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash_mod
    return ash_mod


def row_batch(rng, n, specs):
    keys = rng.integers(0, 24, size=(n, 3), dtype=np.int32)  # about a third of the positions repeat a key
    vals = []
    for dt, e in specs:
        dt = np.dtype(dt)
        raw = rng.integers(0, 256, size=(n, e * dt.itemsize), dtype=np.uint8)
        vals.append(raw.view(dt).reshape(n, e))
    return keys, vals


@pytest.mark.parametrize("specs", [
    [(np.float32, 1 << 4)],                          # 64 B: the separate row pass from its threshold
    [(np.float32, 1 << 9)],                          # 2 KB
    [(np.float32, 1 << 12)],                         # 16 KB
    [(np.float32, 512), (np.float32, 1536)],         # Listing 2's 8^3 x 1 and 8^3 x 3 blocks
    [(np.uint8, 3), (np.float16, 5), (np.float32, 7)],   # 3 B, 10 B, 28 B rows: 1-, 2- and 4-byte units
    [(np.uint8, 67), (np.float16, 33)],              # odd rows over 64 B in total: the row pass with narrow units
    [(np.uint8, 1031), (np.float16, 515)],           # odd rows of 1 KB and more: the unrolled pass, 1- and 2-byte units
], ids=["f32x16", "f32x512", "f32x4096", "blocks8x8x8x1+3", "odd_small", "odd_large", "odd_1k"])
@pytest.mark.parametrize("g", [1, 4])
def test_large_rows_match_oracle(ash, specs, g):
    rng = np.random.default_rng(90 + len(specs))
    pair = Pair(ash, 12_000, 3, specs, probe_group=g, bucket_width=4)
    keys, vals = row_batch(rng, 3001, specs)
    pair.insert(keys, vals)
    pair.check_state()
    keys2, vals2 = row_batch(rng, 2047, specs)  # half present already: their rows must not change
    pair.insert(keys2, vals2)
    find = np.concatenate([keys[:1500], rng.integers(24, 40, size=(1500, 3), dtype=np.int32)])
    pair.find(find)
    pair.erase(keys[::5])
    pair.insert(*row_batch(rng, 999, specs))  # freed indices reused with new rows
    pair.check_state()
    pair.find(find)


def test_double_hash_map_frames(ash):
    """Listing 2 over five frames: the global map (int32x3 block keys -> 8^3 x 1
    and 8^3 x 3 f32 blocks) only ever sees each frame's distinct blocks, and
    the local map links them by index."""
    pts = synth.points(n=200_000, seed=31)
    block = 8 * 0.05  # 8^3 voxels of 5 cm per block
    rng = np.random.default_rng(32)
    gl = Pair(ash, 20_000, 3, [(np.float32, 512), (np.float32, 1536)])
    loc_g = ash.HashMap(100_000, 3, [(torch.int32, 1)])
    for frame in range(5):
        sel = rng.choice(len(pts), size=60_000, replace=False)  # the frame's points
        xyz = np.floor(pts[sel].astype(np.float64) / block).astype(np.int32)
        loc_o = OracleMap(100_000, 3, [(np.int32, 1)])
        loc_g.clear()
        # local map: activate block coordinates; keep the first occurrences
        gi, gm = loc_g.activate(dev(xyz))
        st, oi, om = loc_o.activate(xyz)
        assert np.array_equal(host(gm).astype(np.uint8), om) and np.array_equal(host(gi), oi)
        uniq, i_local = xyz[om == 1], oi[om == 1]
        assert np.array_equal(host(dev(xyz)[gm]), uniq)
        # global map: activate the frame's blocks, then find all of them
        gl.activate(uniq)
        i_global, hit = gl.find(uniq, gather=False)
        assert hit.all()
        # associate local and global maps through indices (Listing 2's last line)
        lv = loc_g.value_buffer(0)
        lv[dev(i_local).long()] = dev(i_global.reshape(-1, 1))
        torch.cuda.synchronize()
        assert np.array_equal(host(lv)[i_local, 0], i_global)
        assert np.array_equal(host(loc_g.key_buffer())[i_local], uniq)
        gl.check_state()
    assert gl.gpu.size() > 0 and gl.gpu.size() == gl.orc.size


def test_value_sweep_full_size_16k_rows(ash):
    """The value sweep's largest shape: 1M keys with 16 KB rows.  A fresh
    map's insert mask marks first occurrences and their indices are ranks;
    every row of v^B and every gathered row of a find must equal the first
    occurrence's input row bit for bit (compared on the device, in chunks),
    and rows of misses stay untouched."""
    d = synth.value_sweep()
    keys, fk = d["keys"], d["find_keys"]
    n = len(keys)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(81)
    vals = torch.randn((n, 4096), dtype=torch.float32, device="cuda", generator=gen)
    m = ash.HashMap(n, 3, [(torch.float32, 4096)])
    gi, gm = m.insert(dev(keys), [vals])
    packed = np.ascontiguousarray(keys).view(np.dtype((np.void, 12))).ravel()
    uniq, first, inv = np.unique(packed, return_index=True, return_inverse=True)
    rank = np.empty(len(first), np.int64)
    rank[np.argsort(first)] = np.arange(len(first))
    want = np.zeros(n, bool)
    want[first] = True
    assert np.array_equal(host(gm), want)
    assert np.array_equal(host(gi)[want], rank[inv[want]].astype(np.int32))
    first_sorted = torch.from_numpy(np.sort(first)).cuda()  # row r of v^B came from position first_sorted[r]
    vb = m.value_buffer(0)
    chunk = 1 << 16
    for r0 in range(0, len(first), chunk):
        r1 = min(r0 + chunk, len(first))
        assert torch.equal(vb[r0:r1].view(torch.int32), vals[first_sorted[r0:r1]].view(torch.int32)), \
            f"v^B rows {r0}..{r1} differ"
    fi, fmask, (fv,) = m.find(dev(fk), gather=True)
    fpacked = np.ascontiguousarray(fk).view(np.dtype((np.void, 12))).ravel()
    pos = np.searchsorted(uniq, fpacked)
    hit = (pos < len(uniq)) & (uniq[np.minimum(pos, len(uniq) - 1)] == fpacked)
    assert np.array_equal(host(fmask), hit)
    hp = torch.from_numpy(np.flatnonzero(hit)).cuda()
    src_pos = torch.from_numpy(first[pos[hit]]).cuda()
    for r0 in range(0, len(hp), chunk):
        r1 = min(r0 + chunk, len(hp))
        assert torch.equal(fv[hp[r0:r1]].view(torch.int32), vals[src_pos[r0:r1]].view(torch.int32)), \
            f"gathered rows {r0}..{r1} of the hits differ"
    mp = torch.from_numpy(np.flatnonzero(~hit)).cuda()
    for r0 in range(0, len(mp), chunk):
        r1 = min(r0 + chunk, len(mp))
        assert not torch.any(fv[mp[r0:r1]].view(torch.int32)), "rows of misses were modified"
    assert m.device_status() == 0


@pytest.mark.parametrize("n_find", [1, 777, 5000])
@pytest.mark.parametrize("specs", [
    [(np.float32, 1024), (np.uint8, 1030)],  # 4 KB and an odd 1030 B row: rows copied by a pass of their own
    [(np.float32, 16)],                      # 64 B rows: copied by the find's own blocks
], ids=["rows_apart", "rows_inside"])
def test_find_rows_without_index_output(ash, n_find, specs):
    """A find that gathers rows while the caller passes no index (or mask)
    output: long rows for a small batch move in a pass of their own after the
    lookup, which reads the indices back from the map's scratch; short rows
    move inside the find.  The gathered rows must equal the oracle's bit for
    bit, and rows of misses stay untouched."""
    import ctypes

    from paper_2110_00511_amd import _lib as L
    rng = np.random.default_rng(95)
    pair = Pair(ash, 6_000, 3, specs)
    keys, vals = row_batch(rng, 4000, specs)
    pair.insert(keys, vals)
    fk = np.concatenate([keys[: n_find // 2], rng.integers(24, 40, size=(n_find - n_find // 2, 3), dtype=np.int32)])
    fk = fk[rng.permutation(n_find)]
    _, oi, om, oout = pair.orc.find(fk, gather=True, fill=0)
    outs = [torch.full((n_find, e), 7, dtype=torch.float32 if dt == np.float32 else torch.uint8, device="cuda")
            for dt, e in specs]
    arr = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
    fkd = dev(fk)
    lib = L.load()
    L.check(lib.ash_find(pair.gpu._m, ctypes.c_void_p(fkd.data_ptr()), n_find, None, None,
                         ctypes.cast(arr, ctypes.c_void_p), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "ash_find")
    hit = om == 1
    for g, o in zip(outs, oout):
        g = host(g)
        assert np.array_equal(g[hit].view(np.uint8), o[hit].view(np.uint8))
        assert np.all(g[~hit] == 7)
