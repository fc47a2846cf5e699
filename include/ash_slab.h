/*
 * ash_slab.h -- C ABI of the separate-chaining backend kept for the backend
 * ablation (ASH, arXiv 2110.00511, Sec. 4.4 and Sec. 5.3).  It is a
 * benchmark and test subject only: nothing in include/ash.h dispatches to
 * it, and the product map (open addressing) is independent of it.
 *
 * The backend follows the paper's generalisation of a slab hash set with
 * the index heap (Sec. 4.4.1): each bucket is a linked list of slabs of 32
 * words (one 128-byte line: 31 entries and the next-slab link) read by 32
 * lanes at once, and an entry is a buffer index i whose key lives in k^B[i];
 * a probe compares the query with k^B[i] of every occupied entry it meets.
 * Insertion takes the paper's three passes (Sec. 4.4.2):
 *   1. every position p takes the index h[t + p] and writes its key to
 *      k^B (all candidates, so no reader sees a partly written key);
 *   2. positions insert their indices into their buckets' lists, comparing
 *      against the read-only k^B; an entry is claimed with a compare-and-swap
 *      on an empty word, so among equal keys of one batch whichever position
 *      claims first is inserted (the paper leaves the choice to the thread
 *      schedule, and so does this backend);
 *   3. the positions that were inserted keep their indices (h[t..t+w) in
 *      batch order, t += w) and receive their value rows; the other indices
 *      go back to the free part of the heap.
 * Buckets: ceil(2 c / 31) base slabs, so the lists sit about half full when
 * the map holds c keys (the paper uses twice as many buckets as capacity,
 * read here as a load of about 0.5 over the slab entries), plus a pool of
 * overflow slabs.
 *
 * Conventions (as in ash.h): keys, values and outputs are device pointers
 * owned by the caller; key rows of key_dim int32 words; one value buffer of
 * value_bytes per row (0: a hash set); out_idx / out_mask nullable; calls
 * are ordered on `stream`.
 */
#ifndef ASH_SLAB_H
#define ASH_SLAB_H

#include <stdint.h>

#include "ash.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ash_slab* ash_slab_t;

/* capacity in [1, 2^30]; key_dim in [1, 4]; value_bytes in [0, 2^24].
 * Buffers come from hipMalloc.  Synchronizes. */
ash_status_t ash_slab_create(int64_t capacity, int32_t key_dim, int64_t value_bytes, void* stream,
                             ash_slab_t* out);
ash_status_t ash_slab_destroy(ash_slab_t map);
/* Empties the map (fresh heap, empty lists, empty slab pool). */
ash_status_t ash_slab_clear(ash_slab_t map, void* stream);

/* Three-pass insertion (above).  The batch takes n indices before any key is
 * known to be new, so t + n must not exceed c: ASH_E_CAPACITY otherwise,
 * with nothing launched.  A list that needs more overflow slabs than the
 * pool holds fails the insert with ASH_E_CAPACITY (reported by this call,
 * which synchronizes to learn the new size). */
ash_status_t ash_slab_insert(ash_slab_t map, const int32_t* keys, int64_t n, const void* values,
                             int32_t* out_idx, uint8_t* out_mask, void* stream);

/* Query (Sec. 4.3.2 / 4.4.1): out_idx[p] = i with k^B[i] = key, mask 1, and
 * (out_values non-null) row i of v^B; misses give -1 / 0 and untouched
 * rows. */
ash_status_t ash_slab_find(ash_slab_t map, const int32_t* keys, int64_t n, int32_t* out_idx,
                           uint8_t* out_mask, void* out_values, void* stream);

/* Live keys t (synchronizes) and borrowed device pointers to k^B, v^B (NULL
 * for a hash set) and the heap h. */
ash_status_t ash_slab_size(ash_slab_t map, int64_t* out, void* stream);
ash_status_t ash_slab_buffers(ash_slab_t map, int32_t** key_buffer, void** value_buffer,
                              int32_t** heap);

#ifdef __cplusplus
}
#endif

#endif /* ASH_SLAB_H */
