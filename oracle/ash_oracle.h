/*
 * ash_oracle.h -- plain, sequential CPU oracle for the ASH spatial hash map.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this library: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header or constant with the
 * HIP implementation under paper_2110_00511_amd/.
 *
 * What it computes (ASH, Dong et al., arXiv 2110.00511):
 *   - key buffer k^B and value buffers {v^B_j} of capacity c, addressed by
 *     buffer indices handed out by an index heap h with top t
 *     (Sec. 4.2, index-first query; Sec. 4.3, index heap; Sec. 4.7, multi-value)
 *   - insert = lazy insertion: a key already present changes nothing, a new key
 *     takes i = h[t], t += 1, and its key/value rows are written (Sec. 4.3.1)
 *   - activate = insert without writing values (Sec. 5.1)
 *   - find returns (index, mask) with mask 0 on a miss (Sec. 4.2, masked query)
 *   - erase frees the index back to the heap: t -= 1, h[t] = i (Sec. 4.3)
 *   - rehash grows the buffers (x2 policy for auto-growth, Sec. 4.5)
 *   - voxelize: keys floor(p / voxel) inserted into a hash set (Sec. 6.1)
 *   - neighbor lookups: finds of every query key shifted by every offset of
 *     a neighborhood (Listing 3, Sec. 6.2.4; Sec. 6.3); set intersection as a find mask
 *     selecting the queries (Sec. 6.4)
 *
 * Batches are processed strictly in position order, which is the
 * "lowest batch position wins" rule for in-batch duplicates.  Readings of the
 * paper where it is silent are listed at the top of ash_oracle.cpp.
 *
 * Parity pins: the functions here are checked against brute force on tiny
 * inputs, numpy.unique closed forms and invariants (tests/test_oracle_*.py).
 * Buffer-index values after erasure are fixed by the heap discipline above;
 * the contents of activated-but-never-written value rows are parity unpinned
 * (the paper leaves them to the user).
 */
#ifndef ASH_ORACLE_H
#define ASH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_E_INVALID = 1,
  ORACLE_E_CAPACITY = 2,
};

typedef struct oracle_map oracle_map;

/* key_dim in [1,4]; n_values >= 0; row_bytes[j] > 0 is the byte size of one
 * row of value buffer j.  Value buffers start zero-filled. */
int oracle_create(int64_t capacity, int32_t key_dim, int32_t n_values,
                  const int64_t* row_bytes, oracle_map** out);
void oracle_destroy(oracle_map* m);

/* keys: n * key_dim int32, row-major.  values: n_values pointers, each to n
 * rows of row_bytes[j].  out_idx / out_mask may be NULL.  With autogrow = 0 a
 * batch that needs more free indices than c - t leaves the map unchanged,
 * writes idx -1 / mask 0 everywhere and returns ORACLE_E_CAPACITY; with
 * autogrow = 1 the capacity is first doubled until the batch fits. */
int oracle_insert(oracle_map* m, const int32_t* keys, int64_t n,
                  const void* const* values, int32_t* out_idx,
                  uint8_t* out_mask, int autogrow);
int oracle_activate(oracle_map* m, const int32_t* keys, int64_t n,
                    int32_t* out_idx, uint8_t* out_mask, int autogrow);
/* out_values may be NULL; rows of misses are left untouched. */
int oracle_find(oracle_map* m, const int32_t* keys, int64_t n,
                int32_t* out_idx, uint8_t* out_mask, void* const* out_values);
int oracle_erase(oracle_map* m, const int32_t* keys, int64_t n,
                 uint8_t* out_mask);
/* Writes the live buffer indices in ascending order; returns their count. */
int64_t oracle_active_indices(const oracle_map* m, int32_t* out_idx);
/* new_capacity >= capacity; indices of live entries are kept. */
int oracle_rehash(oracle_map* m, int64_t new_capacity);

int64_t oracle_size(const oracle_map* m);
int64_t oracle_capacity(const oracle_map* m);
/* Read-only views of the internal state (valid until the next call that can
 * grow the map). */
const int32_t* oracle_key_buffer(const oracle_map* m);
const void* oracle_value_buffer(const oracle_map* m, int32_t j);
const int32_t* oracle_heap(const oracle_map* m);
int64_t oracle_heap_top(const oracle_map* m);
const uint8_t* oracle_active_flags(const oracle_map* m);

/* Neighbor lookup (the radius search of Listing 3, Sec. 6.2.4, and the 1-cube
 * and 1-ring lookups of Sec. 6.3): for every query q and offset o, the find of
 * the key keys[q] + offsets[o] (per word, int32 addition wrapping modulo
 * 2^32) goes to out_idx[q * n_offsets + o] / out_mask[...], query-major.
 * offsets: n_offsets * key_dim int32, row-major.  Outputs may be NULL. */
int oracle_find_offsets(oracle_map* m, const int32_t* keys, int64_t n,
                        const int32_t* offsets, int64_t n_offsets,
                        int32_t* out_idx, uint8_t* out_mask);
/* Set intersection (Sec. 6.4): the query keys that the map holds, in batch
 * order, duplicates kept (a masked selection of the queries by the find
 * mask).  out_keys may be NULL; returns the number of selected rows. */
int64_t oracle_intersect(oracle_map* m, const int32_t* keys, int64_t n,
                         int32_t* out_keys);

/* Voxelization (Sec. 6.1).  points: n * 3 float32.  For every point p and
 * axis d, q = p[d] / voxel in IEEE binary32 (round to nearest even), key =
 * floor(q); a point with a non-finite q or a floor outside int32 is rejected
 * (point_voxel = -1).  Voxel ids are ranks of first occurrence among accepted
 * points.  Writes voxel_keys[id*3+d], counts[id], point_voxel[p]; returns the
 * number of voxels. */
int64_t oracle_voxelize(const float* points, int64_t n, float voxel,
                        int32_t* point_voxel, int32_t* voxel_keys,
                        int32_t* counts);

/* Block and in-block voxel coordinates of points (the coupled lookup of
 * Sec. 6.2.2: a voxel block of res^3 voxels of size `voxel`).  For each
 * axis the voxel index v = floor(p[d] / voxel) is formed exactly as in
 * oracle_voxelize; then block = floor(v / res) (rounding toward -infinity)
 * and local = v - block * res, in [0, res).  Over the reals these equal the
 * paper's floor(x / (s res)) and floor((x - block s res) / s).  A point
 * voxelize rejects gets valid 0 and zero coordinates. */
void oracle_block_coords(const float* points, int64_t n, float voxel,
                         int32_t res, int32_t* block_keys,
                         int32_t* local_coords, uint8_t* valid);

#ifdef __cplusplus
}
#endif

#endif /* ASH_ORACLE_H */
