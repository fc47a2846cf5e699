// ash_oracle.cpp -- sequential CPU oracle for the ASH hash map (test
// infrastructure only; see ash_oracle.h).
//
// The state follows the paper's index-first formulation (Sec. 4.2-4.3):
//   M      : ordered map key -> buffer index (std::map; the hash function of
//            the paper is irrelevant to what is computed, so none is used)
//   kB, vB : key buffer and value buffers of capacity c
//   h, t   : index heap and its top; h starts as 0, 1, ..., c-1 and t = 0
//   active : per-index flag, 1 while the index holds a live key
//
// Readings taken where the paper is silent:
//   * inserting a key that is present changes nothing (lazy insertion,
//     Sec. 4.3.1) -- the stored value is not overwritten, mask 0, idx -1;
//   * in-batch duplicates: the lowest batch position wins (positions are
//     processed in order, so the first occurrence is the one inserted);
//   * idx of a miss / loser is the fixed sentinel -1 (the paper leaves it
//     undefined);
//   * erase of a key that is present frees its index: t -= 1, h[t] = i, in
//     batch order; a later duplicate in the same batch is then a miss;
//   * a batch whose new keys exceed the free indices c - t fails as a whole and
//     leaves the map unchanged, unless auto-growth is asked for, in which case
//     c is doubled until it fits (the x2 rule of Sec. 4.5);
//   * rehash grows c to c' >= c and keeps every live index (h' = h[0..c)
//     followed by c..c'-1); c' = c only rebuilds the table;
//   * voxelize divides in binary32 and floors toward -infinity (Listing 1 of
//     Sec. 6.1 computes floor(xyz / voxel_size) in float32);
//   * a neighbor key is the query plus the offset word by word, wrapping
//     modulo 2^32 (any int32 is a legal key, so no sum is rejected), and the
//     results are laid out query-major, n rows of n_offsets (Listing 3
//     reshapes its results to one row per point);
//   * intersection keeps the queries' order and their duplicates: it is the
//     masked selection of the second set by the find mask (Sec. 6.4).
#include "ash_oracle.h"

#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

namespace {

typedef std::array<int32_t, 4> Key;  // unused trailing words are zero

// Voxel index of one coordinate (Listing 1 of Sec. 6.1): floor(x / voxel)
// with the binary32 quotient; false for a non-finite quotient or a floor
// outside int32.
bool voxel_index(float x, float voxel, int64_t* v) {
  float q = x / voxel;  // binary32 division
  float f = std::floor(q);
  if (!std::isfinite(f) || f < -2147483648.0f || f >= 2147483648.0f)
    return false;
  *v = (int64_t)f;
  return true;
}

Key read_key(const int32_t* keys, int64_t p, int key_dim) {
  Key k = {0, 0, 0, 0};
  for (int d = 0; d < key_dim; ++d) k[d] = keys[p * key_dim + d];
  return k;
}

}  // namespace

struct oracle_map {
  int64_t c;
  int key_dim;
  std::vector<int64_t> row_bytes;
  std::map<Key, int32_t> M;
  std::vector<int32_t> kB;
  std::vector<std::vector<uint8_t>> vB;
  std::vector<int32_t> h;
  int64_t t;
  std::vector<uint8_t> active;
};

extern "C" {

int oracle_create(int64_t capacity, int32_t key_dim, int32_t n_values,
                  const int64_t* row_bytes, oracle_map** out) {
  if (!out || capacity < 0 || key_dim < 1 || key_dim > 4 || n_values < 0)
    return ORACLE_E_INVALID;
  if (n_values > 0 && !row_bytes) return ORACLE_E_INVALID;
  for (int j = 0; j < n_values; ++j)
    if (row_bytes[j] <= 0) return ORACLE_E_INVALID;
  oracle_map* m = new oracle_map;
  m->c = capacity;
  m->key_dim = key_dim;
  m->row_bytes.assign(row_bytes, row_bytes + n_values);
  m->kB.assign(capacity * key_dim, 0);
  m->vB.resize(n_values);
  for (int j = 0; j < n_values; ++j) m->vB[j].assign(capacity * row_bytes[j], 0);
  m->h.resize(capacity);
  for (int64_t i = 0; i < capacity; ++i) m->h[i] = (int32_t)i;
  m->t = 0;
  m->active.assign(capacity, 0);
  *out = m;
  return ORACLE_OK;
}

void oracle_destroy(oracle_map* m) { delete m; }

int oracle_rehash(oracle_map* m, int64_t new_capacity) {
  // Growth only: live indices may sit anywhere below c, so keeping them
  // rules out a smaller capacity.
  if (new_capacity < m->c) return ORACLE_E_INVALID;
  // Keys, values and flags keep their indices; indices c..c'-1 are appended
  // to the heap below the old contents.
  m->kB.resize(new_capacity * m->key_dim, 0);
  for (size_t j = 0; j < m->vB.size(); ++j)
    m->vB[j].resize(new_capacity * m->row_bytes[j], 0);
  m->active.resize(new_capacity, 0);
  int64_t old_c = m->c;
  m->h.resize(new_capacity);
  for (int64_t i = old_c; i < new_capacity; ++i) m->h[i] = (int32_t)i;
  m->c = new_capacity;
  return ORACLE_OK;
}

static int64_t count_new_keys(const oracle_map* m, const int32_t* keys,
                              int64_t n) {
  std::map<Key, int> seen;
  int64_t fresh = 0;
  for (int64_t p = 0; p < n; ++p) {
    Key k = read_key(keys, p, m->key_dim);
    if (m->M.count(k) || seen.count(k)) continue;
    seen[k] = 1;
    ++fresh;
  }
  return fresh;
}

static int insert_impl(oracle_map* m, const int32_t* keys, int64_t n,
                       const void* const* values, bool write_values,
                       int32_t* out_idx, uint8_t* out_mask, int autogrow) {
  if (n < 0 || (n > 0 && !keys)) return ORACLE_E_INVALID;
  int64_t fresh = count_new_keys(m, keys, n);
  if (fresh > m->c - m->t) {
    if (!autogrow) {
      for (int64_t p = 0; p < n; ++p) {
        if (out_idx) out_idx[p] = -1;
        if (out_mask) out_mask[p] = 0;
      }
      return ORACLE_E_CAPACITY;
    }
    int64_t grown = m->c > 0 ? m->c : 1;
    while (grown - m->t < fresh) grown *= 2;
    oracle_rehash(m, grown);
  }
  for (int64_t p = 0; p < n; ++p) {
    Key k = read_key(keys, p, m->key_dim);
    if (m->M.count(k)) {
      if (out_idx) out_idx[p] = -1;
      if (out_mask) out_mask[p] = 0;
      continue;
    }
    int32_t i = m->h[m->t];
    m->t += 1;
    m->M[k] = i;
    m->active[i] = 1;
    for (int d = 0; d < m->key_dim; ++d) m->kB[(int64_t)i * m->key_dim + d] = k[d];
    if (write_values) {
      for (size_t j = 0; j < m->vB.size(); ++j) {
        const uint8_t* src = (const uint8_t*)values[j] + p * m->row_bytes[j];
        memcpy(&m->vB[j][(int64_t)i * m->row_bytes[j]], src, m->row_bytes[j]);
      }
    }
    if (out_idx) out_idx[p] = i;
    if (out_mask) out_mask[p] = 1;
  }
  return ORACLE_OK;
}

int oracle_insert(oracle_map* m, const int32_t* keys, int64_t n,
                  const void* const* values, int32_t* out_idx,
                  uint8_t* out_mask, int autogrow) {
  if (!m->vB.empty() && n > 0 && !values) return ORACLE_E_INVALID;
  return insert_impl(m, keys, n, values, true, out_idx, out_mask, autogrow);
}

int oracle_activate(oracle_map* m, const int32_t* keys, int64_t n,
                    int32_t* out_idx, uint8_t* out_mask, int autogrow) {
  return insert_impl(m, keys, n, nullptr, false, out_idx, out_mask, autogrow);
}

int oracle_find(oracle_map* m, const int32_t* keys, int64_t n,
                int32_t* out_idx, uint8_t* out_mask, void* const* out_values) {
  if (n < 0 || (n > 0 && !keys)) return ORACLE_E_INVALID;
  for (int64_t p = 0; p < n; ++p) {
    Key k = read_key(keys, p, m->key_dim);
    std::map<Key, int32_t>::const_iterator it = m->M.find(k);
    if (it == m->M.end()) {
      if (out_idx) out_idx[p] = -1;
      if (out_mask) out_mask[p] = 0;
      continue;
    }
    int32_t i = it->second;
    if (out_idx) out_idx[p] = i;
    if (out_mask) out_mask[p] = 1;
    if (out_values) {
      for (size_t j = 0; j < m->vB.size(); ++j) {
        uint8_t* dst = (uint8_t*)out_values[j] + p * m->row_bytes[j];
        memcpy(dst, &m->vB[j][(int64_t)i * m->row_bytes[j]], m->row_bytes[j]);
      }
    }
  }
  return ORACLE_OK;
}

int oracle_erase(oracle_map* m, const int32_t* keys, int64_t n,
                 uint8_t* out_mask) {
  if (n < 0 || (n > 0 && !keys)) return ORACLE_E_INVALID;
  for (int64_t p = 0; p < n; ++p) {
    Key k = read_key(keys, p, m->key_dim);
    std::map<Key, int32_t>::iterator it = m->M.find(k);
    if (it == m->M.end()) {
      if (out_mask) out_mask[p] = 0;
      continue;
    }
    int32_t i = it->second;
    m->M.erase(it);
    m->t -= 1;
    m->h[m->t] = i;
    m->active[i] = 0;
    if (out_mask) out_mask[p] = 1;
  }
  return ORACLE_OK;
}

int64_t oracle_active_indices(const oracle_map* m, int32_t* out_idx) {
  int64_t count = 0;
  for (int64_t i = 0; i < m->c; ++i)
    if (m->active[i]) out_idx[count++] = (int32_t)i;
  return count;
}

int64_t oracle_size(const oracle_map* m) { return (int64_t)m->M.size(); }
int64_t oracle_capacity(const oracle_map* m) { return m->c; }
const int32_t* oracle_key_buffer(const oracle_map* m) { return m->kB.data(); }
const void* oracle_value_buffer(const oracle_map* m, int32_t j) {
  return m->vB[j].data();
}
const int32_t* oracle_heap(const oracle_map* m) { return m->h.data(); }
int64_t oracle_heap_top(const oracle_map* m) { return m->t; }
const uint8_t* oracle_active_flags(const oracle_map* m) {
  return m->active.data();
}

int oracle_find_offsets(oracle_map* m, const int32_t* keys, int64_t n,
                        const int32_t* offsets, int64_t n_offsets,
                        int32_t* out_idx, uint8_t* out_mask) {
  if (n < 0 || n_offsets < 0 || (n > 0 && !keys) ||
      (n_offsets > 0 && !offsets))
    return ORACLE_E_INVALID;
  for (int64_t q = 0; q < n; ++q) {
    for (int64_t o = 0; o < n_offsets; ++o) {
      Key k = {0, 0, 0, 0};
      for (int d = 0; d < m->key_dim; ++d) {
        uint32_t a = (uint32_t)keys[q * m->key_dim + d];
        uint32_t b = (uint32_t)offsets[o * m->key_dim + d];
        k[d] = (int32_t)(a + b);  // unsigned sum wraps modulo 2^32
      }
      int64_t out = q * n_offsets + o;
      std::map<Key, int32_t>::const_iterator it = m->M.find(k);
      bool hit = it != m->M.end();
      if (out_idx) out_idx[out] = hit ? it->second : -1;
      if (out_mask) out_mask[out] = hit ? 1 : 0;
    }
  }
  return ORACLE_OK;
}

int64_t oracle_intersect(oracle_map* m, const int32_t* keys, int64_t n,
                         int32_t* out_keys) {
  if (n < 0 || (n > 0 && !keys)) return -1;
  int64_t count = 0;
  for (int64_t p = 0; p < n; ++p) {
    Key k = read_key(keys, p, m->key_dim);
    if (m->M.find(k) == m->M.end()) continue;
    if (out_keys)
      for (int d = 0; d < m->key_dim; ++d)
        out_keys[count * m->key_dim + d] = k[d];
    ++count;
  }
  return count;
}

int64_t oracle_voxelize(const float* points, int64_t n, float voxel,
                        int32_t* point_voxel, int32_t* voxel_keys,
                        int32_t* counts) {
  std::map<std::array<int32_t, 3>, int32_t> ids;
  int64_t n_voxels = 0;
  for (int64_t p = 0; p < n; ++p) {
    std::array<int32_t, 3> k;
    bool ok = true;
    for (int d = 0; d < 3 && ok; ++d) {
      int64_t v = 0;
      ok = voxel_index(points[p * 3 + d], voxel, &v);
      k[d] = (int32_t)v;
    }
    if (!ok) {
      point_voxel[p] = -1;
      continue;
    }
    std::map<std::array<int32_t, 3>, int32_t>::iterator it = ids.find(k);
    int32_t id;
    if (it == ids.end()) {
      id = (int32_t)n_voxels++;
      ids[k] = id;
      for (int d = 0; d < 3; ++d) voxel_keys[(int64_t)id * 3 + d] = k[d];
      counts[id] = 0;
    } else {
      id = it->second;
    }
    counts[id] += 1;
    point_voxel[p] = id;
  }
  return n_voxels;
}

void oracle_block_coords(const float* points, int64_t n, float voxel,
                         int32_t res, int32_t* block_keys,
                         int32_t* local_coords, uint8_t* valid) {
  for (int64_t p = 0; p < n; ++p) {
    int64_t v[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < 3 && ok; ++d) ok = voxel_index(points[p * 3 + d], voxel, &v[d]);
    valid[p] = ok ? 1 : 0;
    for (int d = 0; d < 3; ++d) {
      int64_t b = 0, l = 0;
      if (ok) {
        b = v[d] / res;
        if (v[d] % res != 0 && v[d] < 0) b -= 1;  // floor, not truncation
        l = v[d] - b * res;
      }
      block_keys[p * 3 + d] = (int32_t)b;
      local_coords[p * 3 + d] = (int32_t)l;
    }
  }
}

}  // extern "C"
