// ash_device.hpp -- device-side building blocks of the gfx950 hash map.
//
// Slot table.  Open addressing over buckets of W slots; a slot of S 32-bit
// words holds the key in place plus a state word:
//     words[0 .. KD-2]  key words k_0 .. k_{KD-2}
//     words[S-2]        "tag word": k_{KD-1} once committed, a 32-bit hash tag
//                        while a claim is pending (for KD = 1 the key itself)
//     words[S-1]        state: EMPTY, TOMBSTONE, PENDING(p) or COMMITTED(i)
// S = 2 (KD = 1), 4 (KD = 2, 3), 8 (KD = 4).  The (tag word, state) pair is
// 8-byte aligned and is claimed with one 64-bit compare-and-swap.
//
// The paper's backends (Sec. 4.3-4.4) are separate chaining; this table is
// bucketed open addressing, read by a group of g lanes of a 64-wide
// wavefront that each load one slot of a g-slot window (the wavefront
// counterpart of the warp-cooperative slab probing the paper builds on).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ash {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kTomb = 0xFFFFFFFEu;
constexpr uint32_t kPending = 0x80000000u;  // PENDING(p) = kPending + p
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint64_t kEmptyPair = ~0ull;
constexpr int kMaxValues = 8;
constexpr int kBlock = 256;        // threads per block of every kernel
constexpr int kScanItems = 4;      // positions per thread in scanning kernels
constexpr int kScanTile = kBlock * kScanItems;

// Sticky status bits kept in Meta::status.
constexpr uint32_t kStatusCapacity = 1u;    // not enough free buffer indices
constexpr uint32_t kStatusTableFull = 2u;   // probe found no empty slot
constexpr uint32_t kStatusScanStall = 4u;   // a look-back wait hit its bound
constexpr uint32_t kStatusGridStall = 8u;   // a persistent launch's blocks did not all run at once
// Polls of a persistent launch's arrival check before its blocks give up
// (about 0.1 s): no table has been touched then.
constexpr uint32_t kArrivalSpinLimit = 1u << 20;
// Polls after which a block that saw the arrival count complete stops waiting
// for its release flag (about 3 s; the flag comes at once unless an invariant
// is broken, and the launch then ends through the phase barriers' bound).
constexpr uint32_t kArrivalWaitLimit = 1u << 26;
// Polls of its later phase barriers (about 1 us apart, so about 8 s).  Once
// every block has arrived, all blocks are resident and every phase ends, so
// these waits only end early for a broken invariant; they must outlast the
// slowest phase of the largest batch, and are bounded so a launch still
// always ends.
constexpr uint32_t kPhaseSpinLimit = 1u << 23;
constexpr uint32_t kLookbackSpinLimit = 1u << 24;

template <int KD>
struct SlotWords {
  static constexpr int value = KD == 1 ? 2 : (KD <= 3 ? 4 : 8);
};

// Device-resident bookkeeping of one map.  Only the finalize kernels write
// t / used / tombs / epoch, so every other kernel may read them with plain
// loads.  No field is a per-wavefront counter: an atomic per wavefront on one
// address serializes (about 11 ns each on MI355X).
struct Meta {
  uint32_t t;       // heap top = number of live keys
  uint32_t claims;  // summed new-key count of the insert in flight (when needed)
  uint32_t used;    // bound on the non-empty slots (live + tombstones); exact after a count
  uint32_t tombs;   // bound on the tombstones; exact after a count
  uint32_t status;  // sticky error bits
  uint32_t epoch;   // tag of the scan status words of the current launch
  uint32_t spare;
  uint32_t result;  // total of the last scanning kernel
  uint32_t fail;    // groups whose probe found no empty slot (claim/rebuild)
  uint32_t last_n;  // mirror only: batch size of the last finalized insert (its result: new keys)
  uint32_t pad[6];
};

// One request of a fused served batch: its positions [off, off + n) of the
// batch, its own key/value inputs and its own outputs (any may be null).
struct ReqDesc {
  int64_t off;
  int64_t n;
  const int32_t* keys;
  const uint8_t* vals[kMaxValues];
  int32_t* out_idx;
  uint8_t* out_mask;
  uint8_t* outv[kMaxValues];
};

// Most requests one fused served batch may carry.
constexpr int kMaxFusedRequestsHost = 256;

// The descriptors of a fused batch of at most kArgRequests requests, passed
// by value with each launch (kernel arguments), so that no upload has to be
// queued before the batch's kernels.  nreq = 0: the kernels read the
// descriptors from device memory instead.
constexpr int kArgRequests = 16;
struct ReqArgs {
  int32_t nreq;
  int32_t pad;
  ReqDesc d[kArgRequests];
};

// Row layout of the value buffers of a map (bytes per row, j < n).
struct RowSet {
  int32_t n;
  uint32_t bytes[kMaxValues];
};

// Barrier words of a persistent launch (zeroed before the launch).  count
// holds the barrier arrivals so far in bits 0-30 and, in bit 31, the flag
// that the arrival check failed (some block gave up before every block had
// arrived; no block then proceeds and no table is touched).  late is set
// when a later phase barrier hit its bound (tables may be half updated;
// every map of the launch then carries kStatusGridStall).
constexpr uint32_t kArrivalFailed = 0x80000000u;
// Barrier words and per-phase tile counters of a persistent launch, each on
// a 128-byte line of its own (the barrier word is polled; each counter takes
// one atomic per tile of its queue).  Zeroed before every launch.
constexpr uint32_t kTileQueues = 8;
constexpr uint32_t kMaxXcc = 16;  // the XCC_ID register holds 4 bits
struct GridSync {
  uint32_t count;   // arrivals at the arrival check
  uint32_t late;    // a phase barrier gave up
  uint32_t n_xcc;   // XCCs the launch's blocks run on
  uint32_t pad0[29];
  uint32_t next[3][kTileQueues][32];  // next[phase][queue][0]: tiles handed out past the queue's first ones
  uint32_t xcc_blocks[kMaxXcc][32];   // [x][0]: blocks on XCC x
  uint32_t xcc_count[kMaxXcc][32];    // [x][0]: phase-barrier arrivals of XCC x's blocks
  uint32_t xcc_done;                  // XCCs whose blocks have all arrived, over all barriers
  uint32_t pad1[31];
};
// After the GridSync, one release flag per block, kFlagWords words apart (a
// 128-byte line each): the block whose arrival completes a barrier writes the
// barrier's number into every flag, and each block polls its own.
constexpr uint32_t kFlagWords = 32;
// Device bytes of the GridSync of a persistent launch of `blocks` blocks,
// with their release flags.
inline size_t grid_sync_bytes(uint32_t blocks) { return sizeof(GridSync) + (size_t)blocks * kFlagWords * 4; }

struct TableRef {
  uint32_t* words;
  uint32_t nslots;
  uint32_t nbuckets;
  uint32_t bucket_width;  // W: a key's home slot is a multiple of W
  uint32_t window;        // slots examined per probe step (G, or W when G == 1)
  uint32_t max_windows;   // probe steps that cover the whole table
  uint32_t dedup;         // 1: claims drop block-local duplicates in LDS first
  uint32_t reuse;         // 1: the table may hold tombstones, which claims may take
  uint32_t keyed;         // 1: claims keep pending keys in their slots (no tombstone reuse then)
  Meta* mirror;           // nullable host-mapped copy of the counters, written by every finalize
};

// ---------------------------------------------------------------------------
// Hashing.  The paper leaves the hash function open.  Words are folded with
// the SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), a
// bijective 64-bit mixer; the home bucket is taken from the high 32 bits by
// multiply-shift range reduction and the pending tag from the low 32 bits.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <int KD>
__device__ __forceinline__ uint64_t key_hash(const int32_t (&k)[KD]) {
  uint64_t h = 0x9e3779b97f4a7c15ull * (uint64_t)KD;
#pragma unroll
  for (int d = 0; d < KD; d += 2) {
    uint64_t w = (uint32_t)k[d];
    if (d + 1 < KD) w |= (uint64_t)(uint32_t)k[d + 1] << 32;
    h = mix64(h ^ w);
  }
  return h;
}

template <int KD>
__device__ __forceinline__ uint32_t pending_tag(const int32_t (&k)[KD], uint64_t h) {
  return KD == 1 ? (uint32_t)k[0] : (uint32_t)h;
}

__device__ __forceinline__ uint32_t home_slot(const TableRef& tb, uint64_t h) {
  uint32_t b = (uint32_t)(((h >> 32) * (uint64_t)tb.nbuckets) >> 32);
  return b * tb.bucket_width;
}

// ---------------------------------------------------------------------------
// Slot access.
template <int S>
struct Slot {
  uint32_t w[S];
};

template <int S>
__device__ __forceinline__ Slot<S> load_slot(const uint32_t* p) {
  Slot<S> s;
  if constexpr (S == 2) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    s.w[0] = v.x; s.w[1] = v.y;
  } else {
#pragma unroll
    for (int q = 0; q < S / 4; ++q) {
      uint4 v = reinterpret_cast<const uint4*>(p)[q];
      s.w[4 * q] = v.x; s.w[4 * q + 1] = v.y; s.w[4 * q + 2] = v.z; s.w[4 * q + 3] = v.w;
    }
  }
  return s;
}

template <int S>
__device__ __forceinline__ void store_slot(uint32_t* p, const Slot<S>& s) {
  if constexpr (S == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(s.w[0], s.w[1]);
  } else {
#pragma unroll
    for (int q = 0; q < S / 4; ++q)
      reinterpret_cast<uint4*>(p)[q] = make_uint4(s.w[4 * q], s.w[4 * q + 1], s.w[4 * q + 2], s.w[4 * q + 3]);
  }
}

// A committed slot holds key k iff its key words and tag word equal k.
template <int KD, int S>
__device__ __forceinline__ bool slot_holds(const Slot<S>& s, const int32_t (&k)[KD]) {
  bool eq = s.w[S - 2] == (uint32_t)k[KD - 1];
#pragma unroll
  for (int d = 0; d < KD - 1; ++d) eq = eq && s.w[d] == (uint32_t)k[d];
  return eq;
}

template <int KD, int S>
__device__ __forceinline__ Slot<S> committed_slot(const int32_t (&k)[KD], uint32_t idx) {
  Slot<S> s;
#pragma unroll
  for (int q = 0; q < S; ++q) s.w[q] = kEmpty;
#pragma unroll
  for (int d = 0; d < KD - 1; ++d) s.w[d] = (uint32_t)k[d];
  s.w[S - 2] = (uint32_t)k[KD - 1];
  s.w[S - 1] = idx;
  return s;
}

__device__ __forceinline__ uint64_t cas_pair(uint32_t* pair, uint64_t expected, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(reinterpret_cast<uint64_t*>(pair), &expected, desired,
                                       __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // value found in memory (== the original expected on success)
}

__device__ __forceinline__ uint32_t atomic_min_u32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t atomic_add_u32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Lane groups of a wavefront.
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

template <int G>
__device__ __forceinline__ uint64_t group_ballot(bool pred) {
  uint64_t b = __ballot(pred);
  if constexpr (G == 64) {
    return b;
  } else {
    const uint32_t shift = lane_id() & ~(uint32_t)(G - 1);
    return (b >> shift) & ((1ull << G) - 1ull);
  }
}

template <int G, typename T>
__device__ __forceinline__ T group_bcast(T v, uint32_t sub) {
  const int src = (int)((lane_id() & ~(uint32_t)(G - 1)) + sub);
  return __shfl(v, src, 64);
}

__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)(__ffsll((unsigned long long)m) - 1); }

// ---------------------------------------------------------------------------
// Ordered ranks: block-wide scan plus single-pass decoupled look-back across
// tiles (Merrill and Garland, "Single-pass Parallel Prefix Scan with
// Decoupled Look-back", 2016).  Tile = blockIdx.x: workgroups are dispatched
// in increasing order, so a tile only waits on tiles that already started.
// Status word of a tile:
//   [63:32] epoch of the launch, [31] inclusive flag, [30:0] count.
__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t inclusive, uint32_t v) {
  return ((uint64_t)epoch << 32) | ((uint64_t)inclusive << 31) | (uint64_t)v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Called by all 64 lanes of one wavefront; returns the exclusive prefix of
// `tile` (uniform over the wave).  Lane j examines predecessor top - j, so
// one probe covers 64 tiles: the prefix is complete at the nearest tile that
// published an inclusive value, provided every tile in between published its
// aggregate.  Every tile of a launch publishes exactly once and a tile only
// waits on tiles with a smaller index, dispatched before it; the wait
// is still bounded so that a broken invariant ends in a sticky error instead
// of a hang.
__device__ inline uint32_t tile_lookback(uint64_t* status, uint32_t tile, uint32_t epoch, uint32_t aggregate,
                                         uint32_t* status_bits) {
  const uint32_t lane = lane_id();
  if (tile == 0) {
    if (lane == 0)
      __hip_atomic_store(status, pack_status(epoch, 1, aggregate), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(status + tile, pack_status(epoch, 0, aggregate), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t excl = 0;
  int64_t top = (int64_t)tile - 1;
  uint32_t spins = 0;
  while (true) {
    const int64_t j = top - (int64_t)lane;
    // positions before tile 0 read as an inclusive zero; tile 0 is always inclusive
    const uint64_t s = j >= 0 ? __hip_atomic_load(status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : pack_status(epoch, 1, 0);
    const bool valid = (uint32_t)(s >> 32) == epoch;
    const uint64_t invalid = __ballot(!valid);
    const uint64_t incl = __ballot(valid && (s & 0x80000000ull));
    if (incl) {
      const uint32_t k = first_lane(incl);
      const uint64_t need = k == 63 ? ~0ull : ((1ull << (k + 1)) - 1ull);
      if ((invalid & need) == 0) {
        excl += wave_sum_u32(lane <= k ? ((uint32_t)s & 0x7FFFFFFFu) : 0u);
        break;
      }
    } else if (invalid == 0) {  // 64 aggregates and no inclusive value: keep walking
      excl += wave_sum_u32((uint32_t)s & 0x7FFFFFFFu);
      top -= 64;
      continue;
    }
    if (++spins == kLookbackSpinLimit) {
      if (lane == 0) __hip_atomic_fetch_or(status_bits, kStatusScanStall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (lane == 0)
    __hip_atomic_store(status + tile, pack_status(epoch, 1, excl + aggregate), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Block-level wrapper: wave 0 runs the look-back, the prefix is broadcast
// through LDS.
__device__ __forceinline__ uint32_t block_lookback(uint64_t* status, uint32_t tile, uint32_t epoch,
                                                   uint32_t aggregate, uint32_t* status_bits, uint32_t* s_prefix) {
  if (threadIdx.x < 64) {
    const uint32_t e = tile_lookback(status, tile, epoch, aggregate, status_bits);
    if (threadIdx.x == 0) *s_prefix = e;
  }
  __syncthreads();
  return *s_prefix;
}

// Exclusive block scan of kScanItems 0/1 flags per thread where the item of
// thread t in row r is position base + r * kBlock + t.  Returns the rank of
// each flagged item among the tile's flagged items (in position order) and the
// tile total.  s_scratch needs kBlock / 64 + 1 uint64 words.
__device__ inline void block_rank_rows(const bool (&flag)[kScanItems], uint32_t (&rank)[kScanItems],
                                       uint32_t& total, uint64_t* s_scratch) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x >> 6;
  constexpr int kWaves = kBlock / 64;
  // four 16-bit counters packed in one 64-bit word (each sum <= kBlock)
  uint64_t v = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) v |= (uint64_t)(flag[r] ? 1u : 0u) << (16 * r);
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == 63) s_scratch[wave] = x;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    uint64_t c = s_scratch[w];
    if ((uint32_t)w < wave) before += c;
    all += c;
  }
  const uint64_t excl = before + x - v;
  uint32_t row_base = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    rank[r] = row_base + (uint32_t)((excl >> (16 * r)) & 0xFFFFu);
    row_base += (uint32_t)((all >> (16 * r)) & 0xFFFFu);
  }
  total = row_base;
  __syncthreads();  // s_scratch may be reused by the caller
}

// ---------------------------------------------------------------------------
// Value rows.  Each buffer j moves rows of row_bytes[j] bytes in units of
// vec[j] bytes (16, 8, 4, 2 or 1, chosen on the host from the row size and
// pointer alignment); consecutive lanes move consecutive units of a row, so
// both the source and destination streams are coalesced.
struct ValueSet {
  int32_t n;
  const uint8_t* src[kMaxValues];
  uint8_t* dst[kMaxValues];
  uint32_t row_bytes[kMaxValues];
  uint32_t vec[kMaxValues];
  uint32_t units_log2[kMaxValues];  // log2(row_bytes / vec), or 0xFF if not a power of two
};

template <typename V>
__device__ inline void copy_rows_t(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, uint32_t row_bytes,
                                   uint32_t units_log2, const uint2* pairs, uint32_t count) {
  const uint32_t units = row_bytes / (uint32_t)sizeof(V);
  const uint32_t total = count * units;
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    uint32_t w, c;
    if (units_log2 != 0xFFu) {
      w = e >> units_log2;
      c = e & (units - 1u);
    } else {
      w = e / units;
      c = e - w * units;
    }
    const uint2 pr = pairs[w];  // (source row, destination row)
    const V v = reinterpret_cast<const V*>(src + (size_t)pr.x * row_bytes)[c];
    reinterpret_cast<V*>(dst + (size_t)pr.y * row_bytes)[c] = v;
  }
}

__device__ inline void copy_rows(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) {
  switch (vs.vec[j]) {
    case 16: copy_rows_t<uint4>(vs.src[j], vs.dst[j], vs.row_bytes[j], vs.units_log2[j], pairs, count); break;
    case 8: copy_rows_t<uint2>(vs.src[j], vs.dst[j], vs.row_bytes[j], vs.units_log2[j], pairs, count); break;
    case 4: copy_rows_t<uint32_t>(vs.src[j], vs.dst[j], vs.row_bytes[j], vs.units_log2[j], pairs, count); break;
    case 2: copy_rows_t<uint16_t>(vs.src[j], vs.dst[j], vs.row_bytes[j], vs.units_log2[j], pairs, count); break;
    default: copy_rows_t<uint8_t>(vs.src[j], vs.dst[j], vs.row_bytes[j], vs.units_log2[j], pairs, count); break;
  }
}

// ---------------------------------------------------------------------------
// Batched maps: one descriptor per (map, insert batch, find batch).  The
// persistent kernel walks flat tile lists; claim0 / commit0 / find0 are the
// first flat tile of this item in each phase.
struct BatchItem {
  TableRef tb;
  int32_t g, w;         // probe shape of the map
  uint32_t cap;
  int32_t check;        // new keys must be summed for the capacity check
  Meta* meta;
  uint64_t* status;     // scan status words of the map
  const int32_t* ikeys;
  uint32_t n_insert;
  uint32_t claim0, commit0, find0;
  uint32_t* slot_of;
  uint8_t* lost;
  uint32_t* partial;
  int32_t* kB;
  const int32_t* heap;
  int32_t* iidx;
  uint8_t* imask;
  const int32_t* fkeys;
  uint32_t n_find;
  int32_t* fidx;
  uint8_t* fmask;
  ValueSet vin;         // insert values -> v^B
  ValueSet vout;        // v^B -> find outputs
};

}  // namespace ash
