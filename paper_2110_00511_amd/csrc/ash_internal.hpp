// ash_internal.hpp -- host-side state of a map shared by the C-ABI
// implementation files (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ash.h"
#include "ash_device.hpp"

using ash::Meta;
using ash::TableRef;
using ash::ValueSet;

namespace ash_host {

// Value bytes per row from which an insert copies rows in a pass of its own
// after the commit instead of inside it (measured: 4 and 32 B rows copy
// faster inside, 128 B rows 10-15% faster on their own).
constexpr uint32_t kSplitRowBytes = 64;
// Whether a find copies the hits' value rows (row_bytes per key over all
// value buffers) in a pass of its own after the lookup instead of inside
// it.  The find's blocks copy the rows of their own tiles, which overlaps the
// copy with other blocks' probes but leaves most of the chip idle when there
// are few tiles; the separate pass is sized by the bytes to copy.  Measured
// on int32x3 maps with c keys and c finds (half hits), GPU time per find:
//   16 KB rows: 26 against 153 us at c = 10^3, 3.16 against 3.38 ms at 10^6;
//   4 KB rows: 24 against 42 us at 10^3, 77-114 against 80-144 us at 10^5,
//              but 0.90 against 0.85 ms at 10^6;
//   2 KB rows: 23-25 against 25-31 us at 10^3, 28-31 against 27-30 at 10^4;
//   1 KB rows: slower split at every c (23 against 16 us at 10^3).
inline bool find_rows_apart(uint32_t row_bytes, int64_t n) {
  return row_bytes >= 16384 || (row_bytes >= 4096 && n <= (1 << 18)) || (row_bytes >= 2048 && n <= (1 << 12));
}

// Voxelization drops duplicate voxels within each block of points in LDS
// before probing (ASH_F_LDS_DEDUP for its internal set).
constexpr uint32_t kVoxelDedup = 1;

constexpr int64_t kMaxCount = (1ll << 31) - 3;  // positions and indices must fit PENDING(p)
// Standard neighborhoods: at most this many offsets, enumerated from at most
// this many candidates.
constexpr int64_t kMaxNeighborOffsets = 1ll << 16;
constexpr int64_t kMaxNeighborCandidates = 1ll << 24;
constexpr uint64_t kMaxSlots = (1ull << 32) - 128;

#define ASH_HIP(call)                           \
  do {                                          \
    if ((call) != hipSuccess) return ASH_E_DEVICE; \
  } while (0)

#define ASH_TRY(call)                 \
  do {                                \
    ash_status_t st__ = (call);       \
    if (st__ != ASH_OK) return st__;  \
  } while (0)

inline size_t dtype_size(ash_dtype_t t) {
  switch (t) {
    case ASH_U8: return 1;
    case ASH_I32: case ASH_F32: return 4;
    case ASH_I64: case ASH_F64: return 8;
    case ASH_F16: case ASH_BF16: return 2;
    default: return 0;
  }
}

inline bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

struct DevMem {
  ash_allocator_t a{};
  bool custom = false;  // hipMalloc / hipFree unless an allocator was given
  // Kernels load 16-byte slots, CAS 8-byte pairs and fill 16 bytes at a
  // time from the start of each block, so a block that is not 256-byte
  // aligned is handed back and reported as an allocation failure.
  void* get(size_t bytes, hipStream_t st) {
    bytes = std::max<size_t>(bytes, 256);
    if (custom) {
      void* p = a.alloc(a.ctx, bytes, st);
      if (p && ((uintptr_t)p & 255u) != 0) {
        a.free(a.ctx, p, st);
        return nullptr;
      }
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
  }
  void put(void* p, hipStream_t st) {
    if (!p) return;
    if (custom) {
      a.free(a.ctx, p, st);
    } else {
      (void)hipStreamSynchronize(st);
      (void)hipFree(p);
    }
  }
};

// Largest copy unit (16, 8, 4, 2, 1 bytes) dividing the row size and the
// alignment of both base pointers.
inline uint32_t copy_unit(uint32_t row_bytes, const void* a, const void* b) {
  uintptr_t m = (uintptr_t)a | (uintptr_t)b | row_bytes;
  for (uint32_t v = 16; v > 1; v >>= 1)
    if ((m & (v - 1)) == 0) return v;
  return 1;
}

inline uint32_t units_log2(uint32_t row_bytes, uint32_t vec) {
  uint32_t u = row_bytes / vec;
  if (!pow2(u)) return 0xFFu;
  uint32_t l = 0;
  while ((1u << l) < u) ++l;
  return l;
}

// Event records of ash_profile_enable: one (start, stop) pair per launch.
struct ProfRec {
  const char* name;
  hipEvent_t start, stop;
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRec> recs;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

}  // namespace ash_host

struct ash_map {
  ash_host::DevMem mem;
  ash_host::Prof prof;
  int64_t c = 0;
  int key_dim = 3;
  int n_values = 0;
  std::vector<uint32_t> row_bytes;
  std::vector<ash_dtype_t> dtypes;  // as given at creation
  std::vector<int64_t> elems;
  int W = 4, G = 4;
  float max_load = 0.5f;
  uint32_t flags = 0;
  // device state
  uint32_t* table = nullptr;
  uint32_t nslots = 0;
  int32_t* kB = nullptr;
  std::vector<uint8_t*> vB;
  int32_t* heap = nullptr;
  uint64_t* owner = nullptr;  // erase election: (epoch << 32) | ~position
  uint32_t erase_epoch = 0;
  Meta* meta = nullptr;
  // per-call scratch
  uint32_t* slot_of = nullptr;
  int32_t* aux = nullptr;
  uint32_t* partial = nullptr;  // per-block new-key counts of the claim kernel
  uint8_t* lost = nullptr;      // displaced candidates; all zero between calls
  int64_t scratch_n = 0;
  uint64_t* scan_status = nullptr;
  int64_t scan_tiles = 0;
  // host-side upper bounds (exact after any synchronizing call)
  int64_t live_ub = 0;
  int64_t used_ub = 0;
  // An erase ran since the table was last empty or rebuilt, so it may hold
  // tombstones for claims to reuse (skipping them is always correct).
  bool tombs_possible = false;
  // Pinned host memory that every insert and erase finalize copies t, used,
  // tombs and (inserts) the new-key count and batch size to: mirror_h as
  // the host reads it, mirror as the device writes it.  A server reads the
  // counters once a batch is done; inserts read the last new-key fraction.
  Meta* mirror_h = nullptr;
  Meta* mirror = nullptr;
  // The next claim keeps pending keys in their slots (chosen per insert from
  // the last insert's new-key fraction; results are the same either way).
  bool keyed = false;
  // ASH_CLAIM_KEYED=0 / 1 at create fixes the claim variant (-1: chosen per
  // insert from the last insert's new-key fraction); results are the same
  int keyed_override = -1;
  // Buffers of the ash_batched launches that list this map first, kept
  // between calls: on the device the items, the GridSync and the release
  // flags; in pinned host memory a copy of the items (so their upload is a
  // plain DMA) and the launch's GridSync as read back.
  uint8_t* batch_dev = nullptr;
  size_t batch_dev_bytes = 0;
  uint8_t* batch_host = nullptr;
  size_t batch_host_bytes = 0;

  int slot_words() const { return key_dim == 1 ? 2 : (key_dim <= 3 ? 4 : 8); }

  TableRef ref() const {
    TableRef r;
    r.words = table;
    r.nslots = nslots;
    r.bucket_width = (uint32_t)W;
    r.nbuckets = nslots / (uint32_t)W;
    r.window = (uint32_t)(G == 1 ? W : G);
    r.max_windows = nslots / r.window + 1;
    r.dedup = (flags & ASH_F_LDS_DEDUP) ? 1u : 0u;
    r.reuse = tombs_possible ? 1u : 0u;
    r.keyed = keyed ? 1u : 0u;
    r.mirror = mirror;
    return r;
  }
};


namespace ash_host {

// Implemented in ash_api.hip.
ash_status_t read_meta(ash_map* m, Meta* out, hipStream_t st);
ash_status_t ensure_scratch(ash_map* m, int64_t n, hipStream_t st);
// Rebuilds the slot table from the committed slots of m->table (m->nslots of
// them), which it frees; live = number of committed slots.  Synchronizes.
ash_status_t rebuild_table(ash_map* m, int64_t live, hipStream_t st, int64_t room_for = 0);
// Keys of a fused served batch read from its requests' buffers: descriptors
// of nreq requests in arrival order, passed with each launch (args, when
// args->nreq == nreq) or in device memory (d); vs: the insert's value rows
// (dst = v^B; the source rows come from the requests).
struct RequestSource {
  const ash::ReqDesc* d = nullptr;  // device descriptors (when args->nreq == 0)
  const ash::ReqArgs* args = nullptr;  // descriptors passed with each launch
  int nreq = 0;
  ValueSet vs;
};
// Insert of n keys from `keys` (with `values`), or, with rs, from the
// requests rs->d (keys, values and outputs unused; rows must be copied inside
// the commit, and the map may not grow automatically).
ash_status_t insert_impl(ash_map* m, const int32_t* keys, int64_t n, const void* const* values, int32_t* out_idx,
                         uint8_t* out_mask, hipStream_t st, const RequestSource* rs = nullptr);
// Erase of n keys from `keys`, or from the requests rs->d (out_mask unused).
ash_status_t erase_impl(ash_map* m, const int32_t* keys, int64_t n, uint8_t* out_mask, hipStream_t st,
                        const RequestSource* rs = nullptr);

}  // namespace ash_host
