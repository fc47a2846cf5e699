"""Saving and loading a map (Sec. 6.3 keeps a map on disk between stages):
the loaded map holds exactly the saved state -- heap, top, live indices, keys,
value rows -- and goes on handing out the indices the oracle hands out."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from tests.test_gpu_parity import Pair  # noqa: E402


@pytest.fixture(scope="module")
def ash():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00511_amd as ash_mod
    return ash_mod


@pytest.mark.parametrize("kd", [1, 3, 4])
@pytest.mark.parametrize("tuning", [dict(probe_group=4, bucket_width=4), dict(probe_group=1, bucket_width=8)])
def test_save_load_roundtrip_then_continue(ash, tmp_path, kd, tuning):
    rng = np.random.default_rng(50 + kd)
    specs = [(np.float32, 3), (np.uint8, 5)]
    pair = Pair(ash, 30_000, kd, specs)
    batch = lambda n, hi: (rng.integers(-hi, hi, size=(n, kd), dtype=np.int32),  # noqa: E731
                           [rng.standard_normal((n, 3)).astype(np.float32),
                            rng.integers(0, 256, size=(n, 5), dtype=np.uint8)])
    k1, v1 = batch(20_000, 40)
    pair.insert(k1, v1)
    pair.erase(k1[::3])  # freed indices sit on the heap in erase order
    pair.check_state()
    path = tmp_path / "map.ash"
    pair.gpu.save(path)
    pair.gpu = ash.HashMap.load(path, **tuning)
    assert pair.gpu.key_dim == kd and len(pair.gpu.value_specs) == 2
    pair.check_state()
    k2, v2 = batch(9_000, 45)
    pair.insert(k2, v2)  # same indices as the oracle: the heap came back whole
    pair.find(np.concatenate([k1, k2]))
    pair.check_state()


def test_save_load_empty_and_full(ash, tmp_path):
    empty = ash.HashMap(100, 3, [(torch.float32, 2)])
    empty.save(tmp_path / "e.ash")
    e2 = ash.HashMap.load(tmp_path / "e.ash")
    assert e2.size() == 0 and e2.capacity == 100
    zero = ash.HashMap(0, 2)
    zero.save(tmp_path / "z.ash")
    assert ash.HashMap.load(tmp_path / "z.ash").capacity == 0
    pair = Pair(ash, 1000, 3, [(np.int32, 1)])
    keys = np.arange(3000, dtype=np.int32).reshape(1000, 3)
    pair.insert(keys, [np.arange(1000, dtype=np.int32).reshape(-1, 1)])
    pair.gpu.save(tmp_path / "f.ash")
    pair.gpu = ash.HashMap.load(tmp_path / "f.ash")
    pair.check_state()
    pair.find(keys)
