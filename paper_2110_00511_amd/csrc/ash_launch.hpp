// ash_launch.hpp -- host-side launchers of the kernels in ash_kernels.hip
// (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ash_device.hpp"

namespace ash {

enum FinalizeMode { kFinalizeInsert = 0, kFinalizeErase = 1, kFinalizeCount = 2, kFinalizeRebuild = 3 };

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
// meta->used / meta->tombs = exact counts of non-EMPTY slots / tombstones.
hipError_t launch_count_slots(int kd, const TableRef& tb, Meta* meta, hipStream_t st);
// Fused served inserts and erases (1 <= nreq <= 256 requests, offsets
// ascending from 0, total = sum of n): gather the requests' keys and (vals
// non-null) values into batch buffers; scatter batch indices (idx nullable)
// and masks to the requests' outputs.  vals is a device array of rows.n
// device pointers.
hipError_t launch_gather_requests(const ReqDesc* d, int nreq, int64_t total, int kd, const RowSet& rows,
                                  int32_t* keys, uint8_t* const* vals, hipStream_t st);
hipError_t launch_scatter_requests(const ReqDesc* d, int nreq, int64_t total, const int32_t* idx, const uint8_t* mask,
                                   hipStream_t st);
// Fused served insert / erase batches reading keys (and value rows) from the
// requests d[0..nreq) (positions in arrival order; the descriptors are in
// args when args.nreq == nreq, else in device memory at d) and
// writing each request's results; n = total positions.  The commit copies
// rows inside (rows under 64 B per key in total).  Otherwise as
// launch_claim / launch_commit / launch_erase_mark / launch_erase_commit.
hipError_t launch_claim_requests(int kd, int g, int w, const TableRef& tb, const ReqArgs& args, const ReqDesc* d,
                                 int nreq, uint32_t n, uint32_t* slot_of, uint8_t* lost, uint32_t* partial, Meta* meta,
                                 hipStream_t st);
hipError_t launch_commit_requests(int kd, const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq,
                                  uint32_t n, const uint32_t* slot_of, uint8_t* lost, int32_t* kB, const int32_t* heap,
                                  uint32_t cap, const ValueSet& vs, Meta* meta, uint64_t* status, int check,
                                  int silent, hipStream_t st);
hipError_t launch_erase_mark_requests(int kd, int g, int w, const TableRef& tb, const ReqArgs& args, const ReqDesc* d,
                                      int nreq, uint32_t n, uint32_t epoch, uint32_t* slot_of, int32_t* found,
                                      uint64_t* owner, uint8_t* lost, hipStream_t st);
hipError_t launch_erase_commit_requests(int kd, const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq,
                                        uint32_t n, const uint32_t* slot_of, const int32_t* found, uint8_t* lost,
                                        int32_t* heap, Meta* meta, uint64_t* status, hipStream_t st);
// A fused served find over n positions of nreq requests (descriptors in args
// or in device memory at d, offsets ascending from 0): keys are read from, and indices,
// masks and (vs.n > 0) the value rows of hits written to, each request's own
// buffers; vs.src are the map's rows, vs.vec must divide every request's
// output address.
hipError_t launch_find_requests(int kd, int g, int w, const TableRef& tb, const ReqArgs& args, const ReqDesc* d,
                                int nreq, uint32_t n, const ValueSet& vs, hipStream_t st);
// dst row r = src row r where mask[r] == 1 (rows of row_bytes, copied in vec-byte units).
hipError_t launch_copy_masked_rows(const uint8_t* mask, const void* src, void* dst, uint64_t rows,
                                   uint32_t row_bytes, uint32_t vec, hipStream_t st);
hipError_t launch_iota(int32_t* h, uint32_t from, uint32_t to, hipStream_t st);
// Table words (a multiple of 4) to EMPTY, h[i] = i for i < c, counters reset:
// one launch.
hipError_t launch_clear_map(uint32_t* table, size_t n_words, int32_t* heap, uint32_t c, Meta* meta, hipStream_t st);
// Voxelization workspace: table words (a multiple of 4) to EMPTY, n_zero words
// from `zero` to 0 (must not overlap meta), counters zero with epoch 1.
hipError_t launch_voxel_init(uint32_t* table, size_t n_table, uint32_t* zero, size_t n_zero, Meta* meta,
                             hipStream_t st);
hipError_t launch_finalize(Meta* m, uint32_t cap, int mode, int silent, int check, const uint64_t* status,
                           uint32_t last_tile, hipStream_t st);
hipError_t launch_sum_partials(const uint32_t* partial, uint32_t count, Meta* meta, hipStream_t st);
// Number of blocks (and per-block counts) of a claim launch over n positions.
uint32_t claim_blocks(int g, uint32_t n);
hipError_t launch_claim(int kd, int g, int w, const TableRef& tb, const int32_t* keys, uint32_t n, uint32_t* slot_of,
                        uint8_t* lost, uint32_t* partial, Meta* meta, hipStream_t st);
// The commit's last tile also finalizes the insert (t, counters, epoch;
// silent = no sticky status on overflow), so no separate finalize follows.
// wlist NULL: value rows are copied inside the commit.  Otherwise n uint32 of
// scratch that receive the winners' positions in rank order, and
// launch_scatter_values must follow to copy the rows.
hipError_t launch_commit(int kd, const TableRef& tb, const int32_t* keys, uint32_t n, const uint32_t* slot_of,
                         uint8_t* lost, int32_t* kB, const int32_t* heap, uint32_t cap, const ValueSet& vs,
                         int32_t* out_idx, uint8_t* out_mask, Meta* meta, uint64_t* status, int check,
                         uint32_t* wlist, int silent, hipStream_t st);
// Value rows of the insert whose commit just finished (n = its batch size).
hipError_t launch_scatter_values(const ValueSet& vs, const uint32_t* wlist, const int32_t* heap, const Meta* meta,
                                 uint32_t n, uint32_t cap, hipStream_t st);
// Value rows of a find's hits in a separate pass: out row p = v^B row idx[p]
// for idx[p] >= 0 (vs as made for a find: src = v^B, dst = outputs).
hipError_t launch_gather_rows(const ValueSet& vs, const int32_t* idx, uint32_t n, uint32_t cap, hipStream_t st);
hipError_t launch_find(int kd, int g, int w, const TableRef& tb, const int32_t* keys, uint32_t n, int32_t* out_idx,
                       uint8_t* out_mask, const ValueSet& vs, hipStream_t st);
// Finds of keys[q] + offsets[o] for q < n / k, o < k (n = queries * k
// positions, < 2^31 - 3); outputs query-major, either may be NULL.
hipError_t launch_find_offsets(int kd, int g, int w, const TableRef& tb, const int32_t* keys, const int32_t* offsets,
                               uint32_t k, uint32_t n, int32_t* out_idx, uint8_t* out_mask, hipStream_t st);
// Rows of keys with mask 1, compacted in order (n >= 1); the count lands in
// meta->result (the last tile finalizes with kFinalizeCount).
hipError_t launch_compact_rows(int kd, const uint8_t* mask, uint32_t n, const int32_t* keys, int32_t* out, Meta* meta,
                               uint64_t* status, hipStream_t st);
hipError_t launch_erase_mark(int kd, int g, int w, const TableRef& tb, const int32_t* keys, uint32_t n,
                             uint32_t epoch, uint32_t* slot_of, int32_t* found, uint64_t* owner, uint8_t* lost,
                             hipStream_t st);
// The last tile also finalizes the erase (t, tombstones, epoch).
hipError_t launch_erase_commit(int kd, const TableRef& tb, uint32_t n, const uint32_t* slot_of, const int32_t* found,
                               uint8_t* lost, int32_t* heap, uint8_t* out_mask, Meta* meta, uint64_t* status,
                               hipStream_t st);
hipError_t launch_active_indices(int kd, const TableRef& tb, uint8_t* flags, uint32_t c, int32_t* out, Meta* meta,
                                 uint64_t* status, hipStream_t st);
hipError_t launch_rebuild(int kd, int g, int w, const TableRef& tb, const uint32_t* old_words, uint32_t old_slots,
                          Meta* meta, hipStream_t st);
hipError_t launch_voxel_claim(int g, int w, const TableRef& tb, const float* pts, float voxel, uint32_t n,
                              uint32_t* slot_of, uint8_t* lost, uint32_t* partial, Meta* meta, hipStream_t st);
// Ranks first points into voxel ids, writes voxel keys, the first points'
// ids and counts of 1, and -1 for rejected points; both kinds get slot_of =
// kNoSlot, so launch_voxel_resolve only handles the remaining points.
hipError_t launch_voxel_commit(const TableRef& tb, const float* pts, float voxel, uint32_t n, uint32_t* slot_of,
                               uint8_t* lost, int32_t* voxel_keys, int32_t* counts, int32_t* point_voxel, Meta* meta,
                               uint64_t* status, hipStream_t st);
// Per point: block keys, in-block voxel coordinates (res >= 1) and a valid flag.
hipError_t launch_block_coords(const float* pts, uint32_t n, float voxel, int32_t res, int32_t* block_keys,
                               int32_t* local, uint8_t* valid, hipStream_t st);
hipError_t launch_voxel_resolve(const TableRef& tb, uint32_t n, const uint32_t* slot_of, int32_t* point_voxel,
                                int32_t* counts, hipStream_t st);

// Inserts then finds of n_items independent maps in one persistent launch.
// items is a device array; tile counts are the flat totals of each phase.
// One persistent launch over the items (grid = min(resident, work) blocks).
// gs (grid_sync_bytes(resident) bytes) must be zero; resident is a block
// count the device runs all at once
// (batched_occupancy gives the upper bound per CU); arrival_spins bounds the
// arrival check (kArrivalSpinLimit); force_fail = 1 makes the check fail (a
// test of the fallback path: no map is touched).  Afterwards gs->count carries
// kArrivalFailed when the blocks were not all resident (no map touched) and
// gs->late is nonzero when a later barrier gave up.  narrow selects the
// build that holds only the one-lane-per-key probes with W <= 4 (every item
// must have g == 1 and W <= 4); it needs fewer registers, so its resident
// block count is its own.
hipError_t launch_batched(int kd, bool narrow, const BatchItem* items, int32_t n_items, uint32_t claim_tiles,
                          uint32_t commit_tiles, uint32_t find_tiles, int32_t any_check, GridSync* gs,
                          uint32_t resident, uint32_t arrival_spins, uint32_t force_fail, hipStream_t st);
hipError_t batched_occupancy(int kd, bool narrow, int* per_cu);

// Synthetic keys of the autotuner (uniform in [0, side)^kd; finds half hits).
hipError_t launch_synth_keys(int32_t* keys, uint32_t n, int kd, uint32_t side, uint64_t seed, int32_t* fkeys,
                             uint32_t nf, hipStream_t st);

}  // namespace ash
