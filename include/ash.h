/*
 * ash.h -- C ABI of the MI355X (gfx950) spatial hash map.
 *
 * The operations follow ASH (Dong, Lao, Kaess, Koltun, "ASH: A Modern Framework
 * for Parallel Spatial Hashing in 3D Perception", arXiv 2110.00511):
 *   - keys live in a key buffer k^B and values in value buffers {v^B_j} of
 *     capacity c; every call returns buffer indices and masks instead of
 *     pointers to pairs, so callers chain tensor ops by advanced indexing
 *     (Sec. 3 and Sec. 4.2, masked index-first query);
 *   - buffer indices come from an index heap h whose top t rises on
 *     allocation and falls on free (Sec. 4.3);
 *   - insert is lazy: a key that is already present changes nothing, values
 *     are copied only for the keys that are actually inserted (Sec. 4.3.1);
 *   - activate inserts keys only, leaving their value rows to the caller
 *     (Sec. 5.1);
 *   - multi-value maps and hash sets (n_values = 0) (Sec. 4.7);
 *   - rehash grows the buffers, x2 for auto-growth (Sec. 4.5);
 *   - voxelize turns points into floor(p / voxel) keys and keeps one entry per
 *     voxel with a hash-set insertion (Sec. 6.1, Listing 1);
 *   - neighbor lookups are finds of keys shifted by a neighborhood's offsets
 *     (Listing 3, Sec. 6.2.4; Sec. 6.3), and set intersection keeps the
 *     queries a map holds (Sec. 6.4).
 *
 * Conventions shared by every entry point:
 *   - Pointers to keys, values, points and per-position outputs are DEVICE
 *     pointers owned by the caller.  Arrays of value-buffer pointers
 *     (values / out_values) are HOST arrays of n_values device pointers.
 *     out_idx / out_mask may be NULL to skip that output.
 *   - keys: n rows of key_dim int32 words, row-major; any int32 value is a
 *     legal key word.  Each value buffer j holds rows of
 *     value_elems[j] * sizeof(value_dtypes[j]) bytes, copied as raw bytes.
 *   - Per-position results: out_idx[p] is the buffer index (int32) or -1,
 *     out_mask[p] is 1 or 0 (uint8).
 *   - In-batch duplicates are resolved deterministically: the lowest batch
 *     position wins.  Indices are handed out in batch order from the heap
 *     top, so results are independent of thread timing.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t, NULL =
 *     the null stream) unless marked "synchronizes".  A map must not be used
 *     from two streams at once.
 *   - Host-detected errors (NULL pointers, bad sizes, n >= 2^31 - 3, allocator
 *     failure) return immediately; nothing is launched and outputs are
 *     untouched.
 *   - A batch whose new keys exceed the free indices c - t is detected on the
 *     device: nothing is inserted (size, heap, index-addressed buffers and
 *     every stored key are as before; slots the batch had claimed become
 *     tombstones, which later inserts reuse), outputs are idx -1 /
 *     mask 0, and ash_device_status() reports ASH_E_CAPACITY.  With
 *     ASH_F_AUTOGROW the map instead grows to the smallest c * 2^k that fits
 *     (this path synchronizes).
 *   - The map owns k^B, v^B, h, the slot table and its bookkeeping, all
 *     obtained from the allocator given at creation (hipMalloc if NULL).
 */
#ifndef ASH_H
#define ASH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ash_map* ash_map_t;

typedef enum {
  ASH_OK = 0,
  ASH_E_INVALID = 1,     /* bad argument */
  ASH_E_CAPACITY = 2,    /* not enough free buffer indices / table slots */
  ASH_E_NOMEM = 3,       /* allocator returned NULL */
  ASH_E_DEVICE = 4,      /* a HIP runtime call failed */
  ASH_E_UNSUPPORTED = 5  /* size or tuning outside what the kernels handle */
} ash_status_t;

/* Value element types; values are moved as raw bytes, the type only sets the
 * element size. */
typedef enum {
  ASH_U8 = 0, ASH_I32 = 1, ASH_F32 = 2, ASH_I64 = 3, ASH_F64 = 4, ASH_F16 = 5, ASH_BF16 = 6
} ash_dtype_t;

/* Device-memory provider.  alloc returns a 256-byte aligned device pointer
 * of at least `bytes` bytes usable on `stream` (NULL on failure; a block that
 * is not 256-byte aligned is freed again and the call fails with
 * ASH_E_NOMEM); free releases it after the work already queued on
 * `stream`. */
typedef struct {
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
  void* ctx;
} ash_allocator_t;

#define ASH_F_AUTOGROW 1u
/* Claims first drop duplicates within each block of 256 positions in LDS, so
 * only one copy of a key per block probes the table.  Results are the same;
 * it pays off when equal keys sit close together in a batch. */
#define ASH_F_LDS_DEDUP 2u

/* Table tuning.  bucket_width W (1..64, power of two) aligns a key's home slot;
 * probe_group g is the number of wavefront lanes that probe one key together:
 * g in {4, 8, 16, 32, 64} lanes each read one slot of a g-slot window, g = 1
 * gives every lane its own key and a window of one bucket (W in {2, 4, 8}).
 * max_load in [0.1, 0.9] sets slots = ceil(capacity / max_load) rounded up to
 * a multiple of W and g.  NULL tuning means W = 4, g = 4, max_load = 0.5,
 * flags = 0. */
typedef struct {
  int32_t bucket_width;
  int32_t probe_group;
  float max_load;
  uint32_t flags;
} ash_tuning_t;

/* Occupancy snapshot (synchronizes). */
typedef struct {
  int64_t size;        /* live keys = heap top t */
  int64_t capacity;    /* c */
  int64_t slots;       /* table slots */
  int64_t used_slots;  /* live + tombstones */
  int64_t tombstones;
} ash_stats_t;

/* Creates an empty map (Sec. 4.3: h = 0..c-1, t = 0).  capacity in
 * [0, 2^31 - 3]; key_dim in [1, 4]; n_values in [0, 8]; value_elems[j] > 0.
 * Besides the device buffers from the allocator, the map holds 64 bytes of
 * pinned host memory (hipHostMalloc) that its kernels write the counters
 * to.  Synchronizes `stream` once the buffers are initialised. */
ash_status_t ash_create(int64_t capacity, int32_t key_dim, int32_t n_values,
                        const ash_dtype_t* value_dtypes, const int64_t* value_elems,
                        const ash_allocator_t* allocator, const ash_tuning_t* tuning,
                        void* stream, ash_map_t* out);
/* Returns the device buffers to the allocator (after the work queued on the
 * null stream) and frees the pinned counter memory once the whole device is
 * idle (this waits for the device). */
ash_status_t ash_destroy(ash_map_t map);

/* Lazy insertion (Sec. 4.3.1): for each new key (first occurrence in batch
 * order) i = h[t], t += 1, k^B[i] = key, v^B_j[i] = values[j][p]; out_idx[p] =
 * i and out_mask[p] = 1.  Keys already present and later duplicates: -1 / 0,
 * nothing stored.  values: host array of n_values device pointers, each to n
 * rows. */
ash_status_t ash_insert(ash_map_t map, const int32_t* keys, int64_t n,
                        const void* const* values, int32_t* out_idx,
                        uint8_t* out_mask, void* stream);

/* Activation (Sec. 5.1): insert without touching value rows. */
ash_status_t ash_activate(ash_map_t map, const int32_t* keys, int64_t n,
                          int32_t* out_idx, uint8_t* out_mask, void* stream);

/* Masked query (Sec. 4.2): out_idx[p] = i with k^B[i] = key and mask 1, or -1
 * / 0 on a miss.  out_values (nullable host array of n_values device pointers
 * to n rows each) receives v^B_j[i] for hits; rows of misses are untouched. */
ash_status_t ash_find(ash_map_t map, const int32_t* keys, int64_t n,
                      int32_t* out_idx, uint8_t* out_mask,
                      void* const* out_values, void* stream);

/* Erase (Sec. 4.3: t falls on free): each present key (first occurrence in
 * batch order) is removed and its index pushed back, t -= 1, h[t] = i, in batch
 * order; out_mask[p] = 1 for those positions, 0 otherwise. */
ash_status_t ash_erase(ash_map_t map, const int32_t* keys, int64_t n,
                       uint8_t* out_mask, void* stream);

/* Neighbor lookups (Listing 3 of Sec. 6.2.4 finds every point's neighbors as
 * finds of the point shifted by each offset; Sec. 6.3 uses 1-cube and 1-ring
 * neighborhoods the same way).  keys: n * key_dim int32 (device);
 * offsets: n_offsets * key_dim int32 (device), row-major.  For query q and
 * offset o, the key keys[q] + offsets[o] (word by word, int32 addition
 * wrapping modulo 2^32) is looked up as by ash_find, and out_idx[q * n_offsets
 * + o] / out_mask[q * n_offsets + o] receive its index and mask (query-major
 * n x n_offsets; either output may be NULL).  n * n_offsets must stay below
 * 2^31 - 3, else ASH_E_INVALID.  Asynchronous. */
ash_status_t ash_find_offsets(ash_map_t map, const int32_t* keys, int64_t n,
                              const int32_t* offsets, int32_t n_offsets,
                              int32_t* out_idx, uint8_t* out_mask,
                              void* stream);

/* Block and in-block voxel coordinates (Sec. 6.2.2: a voxel is found by a
 * lookup of its block, a res^3 grid of voxels, plus direct indexing inside
 * it).  points: n x 3 float32 (device).  Per axis the voxel index v =
 * floor(p / voxel_size) is formed exactly as in ash_voxelize; then
 * out_block_keys = floor(v / block_res) (toward -infinity) and out_local =
 * v - block * block_res, in [0, block_res) -- over the reals the paper's
 * floor(x / (s l)) and floor((x - x_block s l) / s).  Points voxelize would
 * reject get out_valid 0 and zero coordinates.  Outputs: n x 3 int32,
 * n x 3 int32 and n uint8 (device).  voxel_size > 0 and finite, block_res
 * >= 1, n < 2^31 - 3, else ASH_E_INVALID.  Asynchronous. */
ash_status_t ash_block_coords(const float* points, int64_t n, float voxel_size,
                              int32_t block_res, int32_t* out_block_keys,
                              int32_t* out_local, uint8_t* out_valid,
                              void* stream);

/* Standard neighborhoods for ash_find_offsets, written to host memory as rows
 * of key_dim int32, enumerated with the first word slowest:
 *   ASH_NB_RADIUS: every offset with all words in [-radius, radius],
 *                  (2 radius + 1)^key_dim rows, the zero offset included
 *                  (radius 1 in 3-D: the 27 entries of Listing 3);
 *   ASH_NB_CUBE:   every offset with all words in [0, radius]
 *                  (radius 1: the 2^key_dim corners of the 1-cube, Sec. 6.3);
 *   ASH_NB_RING:   every nonzero offset whose word magnitudes sum to at most
 *                  radius (radius 1: the 2 key_dim face neighbors of the
 *                  1-ring, Sec. 6.3).
 * radius in [1, 64]; at most 2^16 rows from at most 2^24 candidates, else
 * ASH_E_INVALID.  out_offsets NULL: only *out_count is written; otherwise it
 * must hold *out_count rows (ask for the count first).  Host only. */
#define ASH_NB_RADIUS 0
#define ASH_NB_CUBE 1
#define ASH_NB_RING 2
ash_status_t ash_neighbor_offsets(int32_t kind, int32_t radius,
                                  int32_t key_dim, int32_t* out_offsets,
                                  int64_t* out_count);

/* Set intersection (Sec. 6.4: build a set from the first keys, query the
 * second and keep the hits): out_keys (device, room for n rows) receives the
 * rows of keys the map holds, in batch order with duplicates kept, and
 * *out_count (host) their number.  Synchronizes. */
ash_status_t ash_intersect(ash_map_t map, const int32_t* keys, int64_t n,
                           int32_t* out_keys, int64_t* out_count,
                           void* stream);

/* Saving and loading (the paper stores a map on disk between processing
 * stages, Sec. 6.3).  ash_save writes the map's logical state to a file and
 * synchronizes; ash_load creates a new map (allocator and tuning as for
 * ash_create) holding exactly that state: the same capacity, heap h and top
 * t, live indices, keys and value rows, so it hands out the indices the saved
 * map would have.  Value rows of free indices are not kept (they read as
 * zero).  The file is little-endian:
 *   char magic[8] = "ASHMAP", 0, 1;
 *   int32 key_dim, n_values; int64 capacity c, size t;
 *   n_values x { int32 dtype, int32 0, int64 elems };
 *   int32 heap[c]; int32 live[t] (ascending); int32 keys[t][key_dim];
 *   for each value buffer j: rows[t][row_bytes_j] (in the order of live).
 * ash_load checks the whole file before any device work (magic, sizes,
 * ascending live indices below c, a free region h[t..c) that holds every
 * other index exactly once, heap entries below t in range, distinct keys, no
 * trailing bytes) and returns ASH_E_INVALID for a
 * file that fails, or that cannot be opened, read or written.  Both
 * synchronize `stream`. */
ash_status_t ash_save(ash_map_t map, const char* path, void* stream);
ash_status_t ash_load(const char* path, const ash_allocator_t* allocator,
                      const ash_tuning_t* tuning, void* stream,
                      ash_map_t* out);

/* Key width, number of value buffers and, when the arrays are given (n_values
 * entries each), the value dtypes and elements per row given at creation.
 * Host only. */
ash_status_t ash_describe(ash_map_t map, int32_t* out_key_dim,
                          int32_t* out_n_values, ash_dtype_t* out_dtypes,
                          int64_t* out_elems);

/* Live buffer indices in ascending order (the active set gathered for
 * rehashing, Sec. 4.5).  out_idx is a device array of at least `size`
 * entries; *out_count (host) receives the count.  Synchronizes. */
ash_status_t ash_active_indices(ash_map_t map, int32_t* out_idx,
                                int64_t* out_count, void* stream);

/* Rehash (Sec. 4.5) to new_capacity >= c: buffers grow, live indices and
 * their rows are kept, h' = h[0..c) followed by c..c'-1, and the slot table is
 * rebuilt without tombstones.  new_capacity == c only cleans the table;
 * new_capacity < c is ASH_E_INVALID (live indices may lie anywhere below c).
 * Buffer pointers obtained earlier become invalid.  Synchronizes. */
ash_status_t ash_rehash(ash_map_t map, int64_t new_capacity, void* stream);

/* Empties the map (state of a fresh ash_create) without reallocating. */
ash_status_t ash_clear(ash_map_t map, void* stream);

/* Live key count t (synchronizes) and capacity c (host-side, no sync). */
ash_status_t ash_size(ash_map_t map, int64_t* out, void* stream);
ash_status_t ash_capacity(ash_map_t map, int64_t* out);
ash_status_t ash_stats(ash_map_t map, ash_stats_t* out, void* stream);

/* Borrowed device pointers to k^B ([c][key_dim] int32), v^B_j ([c][row]) and
 * the index heap h ([c] int32), valid until rehash / auto-growth / destroy
 * (Sec. 4.2: the buffers are exposed for direct access and in-place use). */
ash_status_t ash_key_buffer(ash_map_t map, int32_t** out);
ash_status_t ash_value_buffer(ash_map_t map, int32_t j, void** out);
ash_status_t ash_heap_buffer(ash_map_t map, int32_t** out);

/* Returns and clears the sticky device-side error (ASH_E_CAPACITY after an
 * overflowing batch).  Synchronizes. */
ash_status_t ash_device_status(ash_map_t map, void* stream);

/* Voxelization (Sec. 6.1, Listing 1).  points: n * 3 float32 (device).  For
 * each point and axis, q = p / voxel in IEEE binary32 (correctly rounded
 * division) and key = floor(q); a point whose q is not finite or whose floor
 * lies outside int32 is rejected (out_point_voxel = -1).  Voxel ids are the
 * ranks of first occurrence among accepted points.  Outputs (device):
 * out_point_voxel[n], out_voxel_keys[n][3] and out_voxel_counts[n], of which
 * the first *out_n_voxels rows are written.  *out_n_voxels is a host int64.
 * voxel > 0 and finite.  Workspace comes from `allocator` (hipMalloc if NULL).
 * ASH_E_DEVICE if a HIP call failed or a ranking wait hit its bound (a
 * broken invariant, not expected; the outputs are then not valid).
 * Synchronizes. */
ash_status_t ash_voxelize(const float* points, int64_t n, float voxel,
                          int32_t* out_point_voxel, int32_t* out_voxel_keys,
                          int32_t* out_voxel_counts, int64_t* out_n_voxels,
                          const ash_allocator_t* allocator, void* stream);

/* ash_voxelize without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight per-frame loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks and outputs as
 * ash_voxelize, bit for bit; the workspace is a fixed device array inside the
 * library (38 MiB per GPU, held from library load until the process ends),
 * so n is limited to 1,048,576 points: a larger n returns ASH_E_UNSUPPORTED
 * with nothing launched.  Every call on one GPU shares that array, and each
 * call rewrites what it needs (table, counters, flags) before use: calls
 * that overlap on one GPU (different streams or host threads) race and must
 * be serialized by the caller.  Calls no hipMalloc, hipFree or allocator.
 * Synchronizes. */
ash_status_t ash_voxelize_noalloc(const float* points, int64_t n, float voxel,
                                  int32_t* out_point_voxel, int32_t* out_voxel_keys,
                                  int32_t* out_voxel_counts, int64_t* out_n_voxels,
                                  void* stream);

/* Blocks of the persistent batched launch for maps of this key_dim on the
 * current device: the occupancy the runtime reports (*out_reported, blocks per
 * CU times CUs) and the count the device was seen to run all at once
 * (*out_blocks), which ash_batched uses.  narrow = 1 asks about the kernel
 * build ash_batched launches when every map of the call probes one lane per
 * key (probe_group 1) with bucket_width 2 or 4: it holds fewer registers, so
 * more of its blocks fit; narrow = 0 about the build for every other call.
 * The first call per key_dim, build and device makes an empty launch
 * (touching no map) and synchronizes; later calls return the cached count. */
ash_status_t ash_batched_grid(int32_t key_dim, int32_t narrow, int64_t* out_blocks, int64_t* out_reported,
                              void* stream);

/* Batched maps (many independent maps of uneven sizes at once).  One op is
 * one map's work: an insert batch, then a find batch, with the meaning of
 * ash_insert followed by ash_find on that map (insert_values / find_values
 * are host arrays of n_values device pointers; outputs may be NULL).  With
 * fused = 1 all ops run in one persistent launch whose phases
 * (claims, commits, heap tops, finds) are separated by grid barriers and
 * whose tiles are spread over every resident block, each map keeping its own
 * probe shape; fused = 0 runs the same work op by op through the single-map
 * path.  Maps must be distinct, share key_dim and not use ASH_F_AUTOGROW
 * (ASH_E_UNSUPPORTED otherwise).  Capacity overflow of one map rolls back
 * that map's batch only, as in ash_insert.
 * The fused launch needs all its blocks resident at once.  Its blocks first
 * check in, and if they cannot all run together (other work holds compute
 * units) they leave before touching any map and the call runs the same work
 * op by op, with the same results.  A later phase barrier that gives up
 * (a broken invariant, not expected) returns ASH_E_DEVICE and leaves
 * every map of the call with a sticky device error.  With fused = 1 the
 * call synchronizes `stream` to read the launch's outcome. */
typedef struct {
  ash_map_t map;
  const int32_t* insert_keys;
  int64_t n_insert;
  const void* const* insert_values;
  int32_t* insert_idx;
  uint8_t* insert_mask;
  const int32_t* find_keys;
  int64_t n_find;
  void* const* find_values;
  int32_t* find_idx;
  uint8_t* find_mask;
} ash_batch_op_t;

ash_status_t ash_batched(const ash_batch_op_t* ops, int32_t n_ops, int32_t fused, void* stream);
/* Fused ash_batched calls of this process that failed the arrival check and
 * ran op by op instead (instrumentation).  Setting the environment variable
 * ASH_BATCHED_FORCE_ARRIVAL_FAILURE=1 makes every fused launch fail that
 * check (its blocks leave before touching any map), which tests use to take
 * the fallback on purpose. */
int64_t ash_batched_fallbacks(void);

/* Autotuner for the table shape.  Times insert + find of a synthetic batch on
 * this device -- n_insert keys uniform in a cube sized for the expected ratio
 * of distinct keys, then n_insert finds with half hits -- for every
 * (bucket_width, probe_group, max_load) of the sweep W in {2, 4, 8, 16, 32},
 * g in {1 (W <= 8), 4, 8, 16, 64}, max_load in {0.5, 0.7, 0.85}, and writes
 * the fastest to *out (flags 0) and its time in ms to *out_ms (nullable).
 * Results are cached per (key_dim, value bytes, log2 capacity, log2 n_insert,
 * distinct ratio in tenths).  Synchronizes. */
ash_status_t ash_autotune(int64_t capacity, int32_t key_dim, int32_t n_values,
                          const ash_dtype_t* value_dtypes, const int64_t* value_elems,
                          int64_t n_insert, double distinct_ratio,
                          const ash_allocator_t* allocator, void* stream,
                          ash_tuning_t* out, double* out_ms);

/* The sweep for maps meant for ash_batched: each candidate is timed as the
 * insert and find of one map in the persistent batched launch.  That kernel
 * keeps a fixed number of blocks resident, each taking its tiles one after
 * another, so the sweep keeps the shapes that probe all keys of a tile at
 * once: g = 1 with W in {2, 4}, max_load in {0.5, 0.7, 0.85}.  A launch whose
 * maps all have such shapes runs the kernel build with more blocks resident
 * (ash_batched_grid, narrow = 1).  Cached separately from ash_autotune.
 * Synchronizes. */
ash_status_t ash_autotune_batched(int64_t capacity, int32_t key_dim, int32_t n_values,
                                  const ash_dtype_t* value_dtypes, const int64_t* value_elems,
                                  int64_t n_insert, double distinct_ratio,
                                  const ash_allocator_t* allocator, void* stream,
                                  ash_tuning_t* out, double* out_ms);

/* The tuner over an explicit grid: every valid (bucket_width in widths,
 * probe_group in groups, max_load in loads) is timed as in ash_autotune
 * (fused = 0) or as in ash_autotune_batched (fused = 1); shapes ash_create
 * would refuse are skipped.  Each list holds 1..64 entries; ASH_E_INVALID if
 * no point of the grid is valid.  Cached per workload and grid.
 * Synchronizes. */
ash_status_t ash_autotune_sweep(int64_t capacity, int32_t key_dim, int32_t n_values,
                                const ash_dtype_t* value_dtypes, const int64_t* value_elems,
                                int64_t n_insert, double distinct_ratio,
                                const int32_t* widths, int32_t n_widths,
                                const int32_t* groups, int32_t n_groups,
                                const float* loads, int32_t n_loads, int32_t fused,
                                const ash_allocator_t* allocator, void* stream,
                                ash_tuning_t* out, double* out_ms);

/* Served map (continuous batching).  A server owns one map (the caller must
 * not use the map while it is served) and a worker thread with its own HIP
 * stream.  Requests run in arrival order; requests of one kind that are
 * waiting when the worker is ready are fused into one device batch,
 * concatenated in arrival order, so each request's results equal those of
 * running the requests one after another (lowest batch position = earliest
 * request).  An insert joins a fused batch only while the batch's positions
 * fit the free index-heap slots c - t.  Up to in_flight batches are queued on
 * the device while the next one is formed; a completion thread stamps each
 * request's completion time.  Keys, values and outputs are device buffers
 * owned by the caller; they must hold their data when the request is
 * submitted (the server's stream waits on no other stream) and stay valid
 * until the request completes. */
typedef struct ash_server* ash_server_t;

typedef enum { ASH_REQ_FIND = 0, ASH_REQ_INSERT = 1, ASH_REQ_ERASE = 2 } ash_req_kind_t;

typedef struct {
  int32_t kind;                 /* ash_req_kind_t */
  const int32_t* keys;          /* n rows of key_dim int32 */
  int64_t n;
  const void* const* values;    /* insert: host array of n_values device pointers */
  int32_t* out_idx;             /* insert / find, nullable */
  uint8_t* out_mask;            /* nullable */
  void* const* out_values;      /* find: nullable host array of n_values device pointers */
} ash_request_t;

typedef struct {
  int32_t max_fused;  /* requests per device batch, 1..256 (default 256) */
  int64_t max_batch;  /* positions per fused device batch (default 2^22) */
  int32_t in_flight;  /* device batches queued at once (default 4) */
  int32_t fuse;       /* 0: every request is its own device batch */
} ash_server_config_t;

/* cfg NULL = defaults.  Maps with ASH_F_AUTOGROW are not served
 * (ASH_E_UNSUPPORTED). */
ash_status_t ash_server_create(ash_map_t map, const ash_server_config_t* cfg, ash_server_t* out);
/* Thread safe; *out_ticket identifies the request for ash_server_wait. */
ash_status_t ash_server_submit(ash_server_t server, const ash_request_t* req, int64_t* out_ticket);
/* Blocks until the request completed; returns its status (that of the
 * operation it ran in) and its latency from submission in seconds. */
ash_status_t ash_server_wait(ash_server_t server, int64_t ticket, double* out_latency_s);
/* Submits reqs[i] at arrival_s[i] seconds after the call (a trace replay),
 * then waits for all: latencies from the scheduled arrivals, per-request
 * statuses (nullable outputs) and the time from the call to the last
 * completion. */
ash_status_t ash_server_replay(ash_server_t server, const ash_request_t* reqs, int64_t n,
                               const double* arrival_s, double* out_latency_s, int32_t* out_status,
                               double* out_span_s);
/* Device batches launched, requests they carried and the most requests one
 * batch carried, so far (each output nullable). */
ash_status_t ash_server_stats(ash_server_t server, int64_t* out_batches, int64_t* out_requests,
                              int64_t* out_largest);
/* Runs the remaining requests, then stops the threads and frees the server
 * (not the map). */
ash_status_t ash_server_destroy(ash_server_t server);

/* Per-kernel timing of one map (instrumentation).  While enabled, every
 * kernel the map launches is bracketed by HIP events recorded on the launch
 * stream.  ash_profile_collect synchronizes, writes up to max_entries
 * aggregated records (kernel name, launches, summed milliseconds) and
 * clears the records. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} ash_kernel_time_t;

ash_status_t ash_profile_enable(ash_map_t map, int32_t enable);
ash_status_t ash_profile_collect(ash_map_t map, ash_kernel_time_t* out, int32_t max_entries,
                                 int32_t* n_entries, void* stream);

/* Access-cost microbenchmark (instrumentation; no map is involved).  The
 * map's kernels are bound by random accesses to a large table, so the DRAM
 * cost of one such access is measured on its own: n_access accesses at
 * addresses drawn from a counter-based hash of (seed, access number),
 * uniformly over the table and aligned to the access size.
 *   ASH_ACC_READ / ASH_ACC_STORE: reads / stores of access_bytes in {4, 8,
 *     16, 32, 64, 128, 256}; from 16 bytes on, access_bytes / 16 adjacent
 *     lanes each move one 16-byte unit (a probe group reading a window);
 *   ASH_ACC_CAS64: device-scope 64-bit compare-and-swap, returning
 *     (access_bytes 8);
 *   ASH_ACC_MIN32: device-scope 32-bit atomic minimum, no return
 *     (access_bytes 4);
 *   ASH_ACC_STREAM_READ: one coalesced read of the whole table
 *     (n_access and access_bytes ignored);
 *   ASH_ACC_STREAM_COPY: a coalesced copy of the table's first half onto
 *     its second half (the same).
 * table: device scratch of table_bytes (a multiple of 256, 256-byte
 * aligned); stores, atomics and the copy overwrite it.  *out_ms (nullable)
 * receives the kernel's duration from HIP events on `stream`.  Synchronizes.
 * ASH_E_INVALID for other kinds, sizes or alignments. */
#define ASH_ACC_READ 0
#define ASH_ACC_STORE 1
#define ASH_ACC_CAS64 2
#define ASH_ACC_MIN32 3
#define ASH_ACC_STREAM_READ 4
#define ASH_ACC_STREAM_COPY 5
ash_status_t ash_access_bench(int32_t kind, void* table, int64_t table_bytes, int32_t access_bytes,
                              int64_t n_access, uint64_t seed, double* out_ms, void* stream);

const char* ash_status_string(ash_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* ASH_H */
