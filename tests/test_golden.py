"""Hand-worked fixtures (tests/golden/*.json, each citing the passage whose
rules it was worked from) run through the oracle here and through the HIP
path in the gpu-marked tests below."""
import json
import os

import numpy as np
import pytest

from oracle import ORACLE_E_CAPACITY, ORACLE_OK, OracleMap, oracle_voxelize

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(HERE, name)) as f:
        return json.load(f)


def heap_steps():
    g = load("heap_worked_example.json")
    return g, [(s, np.array(s["keys"], np.int32).reshape(-1, g["key_dim"])) for s in g["steps"]]


def voxel_points():
    g = load("voxel_worked_example.json")
    pts = np.array([[float(x) for x in row] for row in g["points"]], np.float32)
    return g, pts


def test_heap_worked_example_oracle():
    g, steps = heap_steps()
    m = OracleMap(g["capacity"], g["key_dim"], [(np.int32, 1)])
    for s, keys in steps:
        if s["op"] == "insert":
            st, idx, mask = m.insert(keys, [np.array(s["values"], np.int32).reshape(-1, 1)])
            assert st == (ORACLE_OK if s["status"] == "ok" else ORACLE_E_CAPACITY)
            assert idx.tolist() == s["idx"] and mask.tolist() == s["mask"]
        elif s["op"] == "erase":
            st, mask = m.erase(keys)
            assert mask.tolist() == s["mask"]
        else:
            st, idx, mask, (vals,) = m.find(keys, gather=True, fill=-99)
            assert idx.tolist() == s["idx"] and mask.tolist() == s["mask"]
            assert vals[:, 0].tolist() == [-99 if v is None else v for v in s["values"]]
        if "t" in s:
            assert m.heap_top == s["t"] and m.heap().tolist() == s["heap"]


def test_voxel_worked_example_oracle():
    g, pts = voxel_points()
    pv, vk, cnt = oracle_voxelize(pts, g["voxel"])
    assert pv.tolist() == g["point_voxel"]
    assert vk.tolist() == g["voxel_keys"] and cnt.tolist() == g["voxel_counts"]


@pytest.mark.gpu
def test_heap_worked_example_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash
    g, steps = heap_steps()
    m = ash.HashMap(g["capacity"], g["key_dim"], [(torch.int32, 1)])
    for s, keys in steps:
        k = torch.from_numpy(keys).cuda()
        if s["op"] == "insert":
            idx, mask = m.insert(k, [torch.tensor(s["values"], dtype=torch.int32).reshape(-1, 1).cuda()])
            assert idx.cpu().tolist() == s["idx"] and mask.cpu().int().tolist() == s["mask"]
            assert m.device_status() == (0 if s["status"] == "ok" else 2)
        elif s["op"] == "erase":
            mask = m.erase(k)
            assert mask.cpu().int().tolist() == s["mask"]
        else:
            idx, mask, (vals,) = m.find(k, gather=True)
            assert idx.cpu().tolist() == s["idx"] and mask.cpu().int().tolist() == s["mask"]
            got = vals[:, 0].cpu().tolist()
            assert [v for v, h in zip(got, s["mask"]) if h] == [v for v in s["values"] if v is not None]
        if "t" in s:
            assert m.size() == s["t"] and m.heap_buffer().cpu().tolist() == s["heap"]


@pytest.mark.gpu
def test_voxel_worked_example_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash
    g, pts = voxel_points()
    pv, vk, cnt = ash.voxelize(torch.from_numpy(pts).cuda(), g["voxel"])
    assert pv.cpu().tolist() == g["point_voxel"]
    assert vk.cpu().tolist() == g["voxel_keys"] and cnt.cpu().tolist() == g["voxel_counts"]
