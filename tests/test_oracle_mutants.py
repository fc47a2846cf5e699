"""The pins must catch plausible mistakes in the oracle.

Each case copies ash_oracle.cpp, plants one mistake (a dropped term, a wrong
index or sign, an off-by-one, reciprocal-multiply for division, trunc for
floor ...), compiles it on the CPU and runs the pin suites against it in a
child pytest process; the child must fail."""
import os
import subprocess
import sys

import pytest

from oracle import build_oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ash_oracle.cpp")

MUTANTS = {
    "heap_top_step": ("    m->t += 1;\n", "    m->t += 2;\n"),
    "ignore_heap": ("int32_t i = m->h[m->t];", "int32_t i = (int32_t)m->t;"),
    "erase_keeps_active": ("    m->active[i] = 0;\n    if (out_mask) out_mask[p] = 1;",
                           "    if (out_mask) out_mask[p] = 1;"),
    "erase_push_wrong_slot": ("    m->t -= 1;\n    m->h[m->t] = i;", "    m->h[m->t - 1 > 0 ? m->t - 2 : 0] = i;\n    m->t -= 1;"),
    "capacity_off_by_one": ("if (fresh > m->c - m->t) {", "if (fresh >= m->c - m->t && fresh > 0) {"),
    "no_batch_dedup_in_count": ("if (m->M.count(k) || seen.count(k)) continue;", "if (m->M.count(k)) continue;"),
    "value_from_index_not_position": ("(const uint8_t*)values[j] + p * m->row_bytes[j];",
                                      "(const uint8_t*)values[j] + (int64_t)i * m->row_bytes[j];"),
    "gather_by_position": ("memcpy(dst, &m->vB[j][(int64_t)i * m->row_bytes[j]]",
                           "memcpy(dst, &m->vB[j][(int64_t)p * m->row_bytes[j]]"),
    "key_drops_last_word": ("for (int d = 0; d < key_dim; ++d) k[d] = keys[p * key_dim + d];",
                            "for (int d = 0; d + 1 < key_dim; ++d) k[d] = keys[p * key_dim + d];"),
    "rehash_heap_reversed": ("for (int64_t i = old_c; i < new_capacity; ++i) m->h[i] = (int32_t)i;",
                             "for (int64_t i = old_c; i < new_capacity; ++i) m->h[i] = (int32_t)(new_capacity - 1 - (i - old_c));"),
    "autogrow_plus_one": ("while (grown - m->t < fresh) grown *= 2;", "while (grown - m->t < fresh) grown += 1;"),
    "voxel_reciprocal": ("float q = x / voxel;", "float q = x * (1.0f / voxel);"),
    "voxel_trunc": ("float f = std::floor(q);", "float f = std::trunc(q);"),
    "voxel_range_edge": ("f >= 2147483648.0f", "f > 2147483648.0f"),
    "voxel_count_reset": ("    counts[id] += 1;\n", "    counts[id] = 1;\n"),
    "voxel_rank_off_by_one": ("      id = (int32_t)n_voxels++;",
                              "      id = (int32_t)(n_voxels <= 1 ? 0 : n_voxels - 1);\n      n_voxels++;"),
    "neighbor_offset_subtracted": ("k[d] = (int32_t)(a + b);", "k[d] = (int32_t)(a - b);"),
    "neighbor_offset_major": ("int64_t out = q * n_offsets + o;", "int64_t out = o * n + q;"),
    "neighbor_drops_last_word": ("      for (int d = 0; d < m->key_dim; ++d) {\n        uint32_t a",
                                 "      for (int d = 0; d + 1 < m->key_dim; ++d) {\n        uint32_t a"),
    "block_truncates": ("        if (v[d] % res != 0 && v[d] < 0) b -= 1;  // floor, not truncation\n", "\n"),
    "block_local_remainder": ("        l = v[d] - b * res;", "        l = v[d] % res;"),
    "intersect_keeps_misses": ("if (m->M.find(k) == m->M.end()) continue;", "if (m->M.find(k) != m->M.end()) continue;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} is not unique"
    mpath = tmp_path / "ash_oracle_mutant.cpp"
    mpath.write_text(src.replace(old, new))
    # the mutant must include the original header
    lib = str(tmp_path / "liboracle_mutant.so")
    build_oracle(src=str(mpath), out=lib, extra_flags=("-I" + os.path.join(ROOT, "oracle"), "-w"))
    env = dict(os.environ, ASH_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_voxelize.py"),
                        os.path.join(ROOT, "tests", "test_oracle_neighbors.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
