// ash_kernels.hip -- gfx950 kernels of the spatial hash map and their
// launchers.  Operation semantics follow ASH (arXiv 2110.00511): lazy
// insertion, activation, masked index query, erase with index-heap free,
// active-set gathering, rehash and voxelization (Sec. 4.2-4.7, 5.1, 6.1).
//
// Insertion is split in two kernels so that no thread ever compares against a
// partially written key (the race that forces the paper's three-pass
// insertion in Sec. 4.4.2 cannot arise):
//   claim  -- each position probes the table; a new key CASes the first EMPTY
//             slot of its probe sequence to (tag, PENDING(p)); a position that
//             meets a PENDING slot of the same key (checked against the
//             read-only input batch) lowers it to PENDING(min) with atomicMin,
//             so every new key ends with exactly one slot holding its lowest
//             batch position;
//   commit -- the position owning its PENDING slot is the winner; winners are
//             ranked in batch order (block scan + decoupled look-back) and take
//             i = h[t + rank]; the key, values and COMMITTED(i) are written.
// A finalize kernel then moves t.  Erase elects the lowest position per
// buffer index with an epoch-tagged atomicMax on owner[i] and pushes winners'
// indices back in batch order.
//
// Traffic model behind the layout (measured on MI355X with rocprofv3): a
// random read fills a 128-byte L2 line, a device-scope atomic is performed at
// the memory side (64 bytes for a 64-bit CAS, 32 for a 32-bit op) and a small
// random store costs a 32-byte write.  So the second pass never re-reads the
// table: positions displaced during the claim are marked in a per-position
// `lost` byte array by whoever displaced them, using the value returned by
// the atomic.

#include "ash_device.hpp"
#include "ash_launch.hpp"

#include <algorithm>

namespace ash {

// ---------------------------------------------------------------------------
// Fused served batches: the requests of a batch occupy consecutive position
// ranges in arrival order.  A block stages the ranges' first positions in LDS
// and finds a position's request by binary search (at most
// kMaxFusedRequests requests per batch).
constexpr int kMaxFusedRequests = kMaxFusedRequestsHost;

__device__ __forceinline__ int request_of(const int64_t* s_off, int nreq, int64_t e) {
  int lo = 0, hi = nreq - 1;  // last request whose first position <= e
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_off[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Stages a fused batch's descriptors in LDS when the launch carries them
// (else they stay in device memory, gd) and the requests' first positions;
// returns where the kernel reads the descriptors.
__device__ __forceinline__ const ReqDesc* stage_requests(const ReqArgs& args, const ReqDesc* gd, int nreq,
                                                         ReqDesc* s_desc, int64_t* s_off) {
  const ReqDesc* d = gd;
  if (args.nreq > 0) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < kArgRequests; ++k)
        if (k < args.nreq) s_desc[k] = args.d[k];
    }
    __syncthreads();
    d = s_desc;
  }
  for (int r = threadIdx.x; r < nreq; r += kBlock) s_off[r] = d[r].off;
  __syncthreads();
  return d;
}

// ---------------------------------------------------------------------------
// Key sources: map keys read from the batch, or voxel keys computed from
// points.  load() returns false for a point that is rejected.
template <int KD>
struct BatchKeys {
  const int32_t* __restrict__ keys;
  __device__ __forceinline__ bool load(uint32_t p, int32_t (&k)[KD]) const {
    const int32_t* r = keys + (size_t)p * KD;
#pragma unroll
    for (int d = 0; d < KD; ++d) k[d] = r[d];
    return true;
  }
};

// Listing 1 of Sec. 6.1: floor(xyz / voxel_size) as int32.  The quotient is
// the correctly rounded binary32 division (the build keeps IEEE division and
// denormals); NaN, infinities and floors outside int32 fail the range test.
struct VoxelKeys {
  const float* __restrict__ points;
  float voxel;
  __device__ __forceinline__ bool load(uint32_t p, int32_t (&k)[3]) const {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float q = points[(size_t)p * 3 + d] / voxel;
      const float f = floorf(q);
      const bool in = f >= -2147483648.0f && f < 2147483648.0f;
      ok = ok && in;
      k[d] = in ? (int32_t)f : 0;
    }
    return ok;
  }
};

// Neighbor keys (Listing 3 of Sec. 6.2.4; the 1-cube and 1-ring lookups of
// Sec. 6.3): position p is query p / k shifted by offset p % k, word by word
// with int32 addition wrapping modulo 2^32.  Positions of one query are
// adjacent, so its key is read once per wavefront from one cache line.
template <int KD>
struct OffsetKeys {
  const int32_t* __restrict__ keys;
  const int32_t* __restrict__ offsets;
  uint32_t k;
  __device__ __forceinline__ bool load(uint32_t p, int32_t (&out)[KD]) const {
    const uint32_t q = p / k;
    const uint32_t o = p - q * k;
#pragma unroll
    for (int d = 0; d < KD; ++d)
      out[d] = (int32_t)((uint32_t)keys[(size_t)q * KD + d] + (uint32_t)offsets[(size_t)o * KD + d]);
    return true;
  }
};

// Keys of a fused served batch, read from the requests' own buffers.
template <int KD>
struct ReqKeys {
  const ReqDesc* __restrict__ d;
  const int64_t* s_off;  // LDS
  int nreq;
  __device__ __forceinline__ bool load(uint32_t p, int32_t (&out)[KD]) const {
    const int r = request_of(s_off, nreq, p);
    const int32_t* k = d[r].keys + (size_t)(p - s_off[r]) * KD;
#pragma unroll
    for (int w = 0; w < KD; ++w) out[w] = k[w];
    return true;
  }
};

template <int KD>
__device__ __forceinline__ bool keys_equal(const int32_t (&a)[KD], const int32_t (&b)[KD]) {
  bool eq = true;
#pragma unroll
  for (int d = 0; d < KD; ++d) eq = eq && a[d] == b[d];
  return eq;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-shared scratch of the tile functions.  Every kernel declares one and
// passes it down, so a persistent kernel that dispatches several probe shapes
// holds a single copy.
// Block-local duplicate removal of a claim: the block's keys, an LDS hash
// table of 2 * kBlock entries (owner thread, lowest thread with that key) and
// each thread's representative and claim result.
struct DedupLds {
  int32_t keys[kBlock][4];
  uint32_t own[2 * kBlock];
  uint32_t low[2 * kBlock];
  uint32_t rep[kBlock];
  uint32_t out[kBlock];
};

struct TileLds {
  union {
    uint2 pairs[kScanTile];  // (source row, destination row) of value copies
    DedupLds dd;
  };
  uint64_t scan[kBlock / 64 + 1];  // block_rank_rows
  uint32_t count[16];              // per-wavefront partial sums (up to 1024 threads)
  uint32_t prefix;                 // look-back result
  uint32_t hits;                   // gathered rows of a find tile
};

// ---------------------------------------------------------------------------
// Fill / init kernels.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t n4 = n / 4;
  uint4* p4 = reinterpret_cast<uint4*>(p);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) p4[i] = make_uint4(v, v, v, v);
  for (size_t i = n4 * 4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t* __restrict__ h, uint32_t from, uint32_t to) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = from + blockIdx.x * blockDim.x + threadIdx.x; i < to; i += stride) h[i] = (int32_t)i;
}

__device__ __forceinline__ void reset_meta(Meta* m) {
  m->t = 0; m->claims = 0; m->used = 0; m->tombs = 0; m->status = 0; m->result = 0; m->fail = 0;
  m->epoch = m->epoch + 1u == 0u ? 1u : m->epoch + 1u;
}

// A voxelization workspace made ready in one launch: the table's words
// EMPTY (n_table a multiple of 4), n_zero words from `zero` cleared (the lost
// bytes and scan status words), and the counters zero with epoch 1.
__global__ __launch_bounds__(kBlock) void k_voxel_init(uint32_t* __restrict__ table, size_t n_table,
                                                       uint32_t* __restrict__ zero, size_t n_zero, Meta* meta) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4* t4 = reinterpret_cast<uint4*>(table);
  for (size_t i = i0; i < n_table / 4; i += stride) t4[i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
  for (size_t i = i0; i < n_zero; i += stride) zero[i] = 0u;
  if (i0 == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(meta);
    for (size_t k = 0; k < sizeof(Meta) / 4; ++k) w[k] = 0u;
    meta->epoch = 1u;
  }
}

// A map emptied in one launch: every table word EMPTY (n_words, a multiple
// of 4), the heap back to h[i] = i for i < c, and the counters reset.
__global__ __launch_bounds__(kBlock) void k_clear_map(uint32_t* __restrict__ table, size_t n_words,
                                                      int32_t* __restrict__ heap, uint32_t c, Meta* meta) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4* t4 = reinterpret_cast<uint4*>(table);
  for (size_t i = i0; i < n_words / 4; i += stride) t4[i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
  for (size_t i = i0; i < c; i += stride) heap[i] = (int32_t)i;
  if (i0 == 0) reset_meta(meta);
}

// Positions per block of the probing kernels: 256 (G lanes per position, so a
// group takes G positions in turn).
template <int G>
__host__ __device__ constexpr uint32_t rounds_for_dev() { return 256u / (kBlock / G); }

// ---------------------------------------------------------------------------
// Probe windows.  One probe step examines `kSize` consecutive slots starting
// at `base`: either G lanes of a wavefront hold one slot each (G > 1, group
// decisions by ballot and lane broadcast), or one lane holds a whole bucket
// of WL slots (G == 1, decisions by local bit masks).  Member L of a window
// is slot base + L.  Results of mask() and of the uniform accessors are the
// same on every lane of a group.
template <int KD, int G, int WL>
struct Window {
  static constexpr int S = SlotWords<KD>::value;
  static constexpr int kPer = G == 1 ? WL : 1;
  static constexpr int kSize = G == 1 ? WL : G;
  Slot<S> v[kPer];
  uint32_t at[kPer];

  __device__ __forceinline__ void load(const TableRef& tb, uint32_t base, uint32_t sub) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      uint32_t s = base + (G == 1 ? (uint32_t)j : sub);
      if (s >= tb.nslots) s -= tb.nslots;
      at[j] = s;
      v[j] = load_slot<S>(tb.words + (size_t)s * S);
    }
  }

  template <typename F>
  __device__ __forceinline__ uint64_t mask(F&& pred) const {
    if constexpr (G == 1) {
      uint64_t m = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const Slot<S> sl = v[j];
        m |= pred(sl) ? (1ull << j) : 0ull;
      }
      return m;
    } else {
      const Slot<S> sl = v[0];
      return group_ballot<G>(pred(sl));
    }
  }

  // The same, with each member's slot number passed to the predicate.
  template <typename F>
  __device__ __forceinline__ uint64_t mask_at(F&& pred) const {
    if constexpr (G == 1) {
      uint64_t m = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j) m |= pred(v[j], at[j]) ? (1ull << j) : 0ull;
      return m;
    } else {
      return group_ballot<G>(pred(v[0], at[0]));
    }
  }

  // (member selection in lane mode is an OR of masked words, which keeps the
  // window in registers; a select chain would be folded into an indexed
  // load from a stack copy)
  __device__ __forceinline__ uint32_t word(uint32_t L, int w) const {
    if constexpr (G == 1) {
      uint32_t r = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j) r |= v[j].w[w] & (0u - (uint32_t)(L == (uint32_t)j));
      return r;
    } else {
      return group_bcast<G>(v[0].w[w], L);
    }
  }

  __device__ __forceinline__ uint32_t slot(uint32_t L) const {
    if constexpr (G == 1) {
      uint32_t r = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j) r |= at[j] & (0u - (uint32_t)(L == (uint32_t)j));
      return r;
    } else {
      return group_bcast<G>(at[0], L);
    }
  }

  // Replaces member L's tag word and state (on the lane that holds it).
  __device__ __forceinline__ void set_pair(uint32_t L, uint32_t sub, uint32_t tagw, uint32_t st) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t member = G == 1 ? (uint32_t)j : sub;
      const uint32_t m = 0u - (uint32_t)(member == L);  // blend, not an indexed store
      v[j].w[S - 2] = (v[j].w[S - 2] & ~m) | (tagw & m);
      v[j].w[S - 1] = (v[j].w[S - 1] & ~m) | (st & m);
    }
  }
};

// Broadcast of a 64-bit value from the group leader (sub-lane 0).
template <int G>
__device__ __forceinline__ uint64_t leader_bcast64(uint64_t x) {
  if constexpr (G == 1) {
    return x;
  } else {
    const uint32_t lo = group_bcast<G>((uint32_t)x, 0u);
    const uint32_t hi = group_bcast<G>((uint32_t)(x >> 32), 0u);
    return ((uint64_t)hi << 32) | lo;
  }
}

// ---------------------------------------------------------------------------
// Claim (insert / activate / voxelize pass 1).  A group of G lanes (or one
// lane when G == 1) owns one position at a time.  Every position ends as
//   - a loser: the key was committed by an earlier call, or a lower position
//     of the same key already holds the pending slot;
//   - a candidate: it CASed the slot, or lowered PENDING(q) to PENDING(p) with
//     an atomicMin that returned q > p -- in which case it sets lost[q], since
//     q can no longer win.
// After the kernel, the winner of each claimed slot is its unique candidate
// with lost == 0.  Map claims write slot_of[p] = slot for candidates and
// kNoSlot for losers; voxel claims (kVoxel) keep the slot for every accepted
// point and mark candidates with kCandidate (the table has < 2^31 slots).
constexpr uint32_t kCandidate = 0x80000000u;

// Block-local duplicate removal (one thread per position of the block's 256
// positions): every valid key enters an LDS hash table, where the first
// thread to reach an entry owns it and every thread with that key lowers the
// entry's minimum.  dd.rep[t] is then the lowest thread holding t's key, or
// kNoSlot when position t has no valid key; dd.keys holds the keys.  Only
// representatives probe the table: a later copy of a key in the same block
// cannot be the batch's first occurrence.
template <int KD, typename Src>
__device__ __forceinline__ void block_dedup(const Src& src, uint32_t n, uint32_t tile_base, DedupLds& dd) {
  constexpr uint32_t kEntries = 2 * kBlock;
  const uint32_t t = threadIdx.x;
  const uint32_t p = tile_base + t;
  int32_t k[KD];
  bool valid = false;
  if (p < n) valid = src.load(p, k);
#pragma unroll
  for (int d = 0; d < KD; ++d) dd.keys[t][d] = valid ? k[d] : 0;
  dd.own[t] = kNoSlot;
  dd.own[t + kBlock] = kNoSlot;
  dd.low[t] = kNoSlot;
  dd.low[t + kBlock] = kNoSlot;
  __syncthreads();
  uint32_t j = 0;
  if (valid) {
    j = (uint32_t)(key_hash<KD>(k) >> 20) & (kEntries - 1);
    while (true) {  // at most kBlock owners in kEntries entries: ends at a free or matching entry
      const uint32_t o = atomicCAS(&dd.own[j], kNoSlot, t);
      if (o == kNoSlot) break;
      bool eq = true;
#pragma unroll
      for (int d = 0; d < KD; ++d) eq = eq && dd.keys[o][d] == k[d];
      if (eq) break;
      j = (j + 1) & (kEntries - 1);
    }
    atomicMin(&dd.low[j], t);
  }
  __syncthreads();
  dd.rep[t] = valid ? dd.low[j] : kNoSlot;
  __syncthreads();
}

// Claims on a table without reusable tombstones keep a pending slot's key
// in the slot once someone has read it: the pending tag word is the key's
// last word, and a position that compares against a pending slot whose other
// key words still read 0xFFFFFFFF (a slot claimed from EMPTY keeps those
// until written; EMPTY slots are never written otherwise) reads the pending
// position's key from the batch and writes its other words into the slot
// with one write-through store.  Later positions of that key then compare
// against the slot alone.  Every such store writes the slot's own key (all
// positions pending on a slot share it), so concurrent stores agree.  Keys
// seen only once cost nothing extra.  With key_dim 4 the three words would
// need two stores, so that case keeps a hash tag.
template <int KD, int S>
__device__ __forceinline__ void publish_key_words(uint32_t* slot, const int32_t (&k)[KD]) {
  if constexpr (KD == 2) {
    __hip_atomic_store(slot, (uint32_t)k[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if constexpr (KD == 3) {
    const uint64_t w = (uint64_t)(uint32_t)k[0] | ((uint64_t)(uint32_t)k[1] << 32);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(slot), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int KD, int G, int WL, typename Src, bool kVoxel, bool kReuse = false, bool kKeep = false>
__device__ __forceinline__ void claim_tile(const TableRef& tb, const Src& src, uint32_t n, uint32_t tile,
                                           uint32_t rounds, uint32_t* __restrict__ slot_of,
                                           uint8_t* __restrict__ lost, uint32_t* __restrict__ partial, Meta* meta,
                                           TileLds& lds) {
  using Win = Window<KD, G, WL>;
  constexpr int S = Win::S;
  constexpr uint32_t kGroups = kBlock / G;
  constexpr bool kKeyed = kKeep && !kReuse && (KD == 2 || KD == 3);  // pending keys kept in their slots
  const uint32_t sub = G == 1 ? 0u : (threadIdx.x & (G - 1));
  const uint32_t grp = threadIdx.x / G;
  const uint32_t tile_base = tile * kGroups * rounds;  // 256 positions per tile
  const bool dedup = tb.dedup != 0;
  if (dedup) block_dedup<KD>(src, n, tile_base, lds.dd);
  uint32_t claimed = 0;
  uint32_t unresolved = 0;
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint32_t p = tile_base + r * kGroups + grp;
    if (p >= n) break;
    int32_t k[KD];
    bool valid, copy = false;
    if (dedup) {  // keys staged in LDS; block-local copies skip the probe
      const uint32_t rp = lds.dd.rep[p - tile_base];
      valid = rp != kNoSlot;
      copy = valid && rp != p - tile_base;
#pragma unroll
      for (int d = 0; d < KD; ++d) k[d] = lds.dd.keys[p - tile_base][d];
    } else {
      valid = src.load(p, k);
    }
    uint32_t out = kNoSlot;
    if (valid && !copy) {
      const uint64_t h = key_hash<KD>(k);
      const uint32_t tag = kKeyed ? (uint32_t)k[KD - 1] : pending_tag<KD>(k, h);
      const uint64_t desired = ((uint64_t)(kPending + p) << 32) | tag;
      uint32_t base = home_slot(tb, h);
      bool resolved = false;
      // The first reusable slot of the sequence: a tombstone seen before the
      // first EMPTY slot (which confirms the key is absent), with the window
      // it was seen in, for a rescan when its CAS fails.
      uint32_t r_slot = kNoSlot, r_base = 0, r_w = 0;
      uint64_t r_pair = 0;
      for (uint32_t w = 0; w < tb.max_windows && !resolved; ++w) {
        Win win;
        win.load(tb, base, sub);
        bool rescan = false;
        while (true) {
          // key committed by an earlier call: not new
          const uint64_t mc = win.mask([&](const Slot<S> sl) {
            return sl.w[S - 1] < kPending && slot_holds<KD, S>(sl, k);
          });
          if (mc) {
            if (kVoxel) out = win.slot(first_lane(mc));
            resolved = true;
            break;
          }
          // same key pending in this batch (compared against the read-only batch)
          const uint64_t mp = win.mask_at([&](const Slot<S> sl, uint32_t slot_no) {
            const uint32_t st = sl.w[S - 1];
            if (!(st >= kPending && st < kTomb && sl.w[S - 2] == tag && st - kPending < n)) return false;
            if constexpr (KD == 1) {
              return true;  // the tag word of a 1-word key is the key
            } else {
              if constexpr (kKeyed) {  // the tag word is the last key word
                bool unset = true, eq = true;
#pragma unroll
                for (int d = 0; d < KD - 1; ++d) {
                  unset = unset && sl.w[d] == kEmpty;
                  eq = eq && sl.w[d] == (uint32_t)k[d];
                }
                if (!unset) return eq;
              }
              int32_t kq[KD];
              src.load(st - kPending, kq);
              if constexpr (kKeyed) publish_key_words<KD, S>(tb.words + (size_t)slot_no * S, kq);
              return keys_equal<KD>(kq, k);
            }
          });
          if (mp) {
            const uint32_t L = first_lane(mp);
            const uint32_t q = win.word(L, S - 1) - kPending;
            const uint32_t s = win.slot(L);
            uint32_t cand = 0;
            if (p < q && sub == 0) {
              const uint32_t old = __hip_atomic_fetch_min(tb.words + (size_t)s * S + S - 1, kPending + p,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (old > kPending + p) {  // p now holds the slot; the previous holder lost
                const uint32_t prev = old - kPending;
                if (prev < n) lost[prev] = 1;
                cand = 1;
              }
            }
            cand = G == 1 ? cand : group_bcast<G>(cand, 0u);
            if (kVoxel) out = s | (cand ? kCandidate : 0u);
            else out = cand ? s : kNoSlot;
            resolved = true;
            break;
          }
          const uint64_t me = win.mask([&](const Slot<S> sl) { return sl.w[S - 1] == kEmpty; });
          if (kReuse && r_slot == kNoSlot) {
            const uint64_t mt = win.mask([&](const Slot<S> sl) { return sl.w[S - 1] == kTomb; });
            if (mt && (!me || first_lane(mt) < first_lane(me))) {
              const uint32_t L = first_lane(mt);
              r_slot = win.slot(L);
              r_pair = ((uint64_t)win.word(L, S - 1) << 32) | win.word(L, S - 2);
              r_base = base;
              r_w = w;
            }
          }
          if (!me) break;  // no empty slot in this window: next window
          // The key is absent: claim the first reusable slot, a tombstone
          // seen on the way or else this EMPTY slot.  Every claimer of a key
          // targets the first slot it sees reusable, and slots only stop
          // being reusable during a claim, so claimers of one key meet there.
          const bool tomb = kReuse && r_slot != kNoSlot;
          const uint32_t L = first_lane(me);
          const uint32_t s = tomb ? r_slot : win.slot(L);
          const uint64_t expect = tomb ? r_pair : kEmptyPair;
          uint64_t found = 0;
          if (sub == 0) found = cas_pair(tb.words + (size_t)s * S + S - 2, expect, desired);
          found = leader_bcast64<G>(found);
          if (found == expect) {
            // A map claim keeping pending keys publishes its key words right
            // away, so later positions of the key compare against the slot
            // instead of reading the batch (a reader that comes first still
            // sees them unset and reads the batch).
            if constexpr (kKeyed && !kVoxel)
              if (sub == 0) publish_key_words<KD, S>(tb.words + (size_t)s * S, k);
            out = kVoxel ? (s | kCandidate) : s;
            claimed += sub == 0 ? 1u : 0u;
            resolved = true;
            break;
          }
          if (tomb) {
            if ((uint32_t)(found >> 32) == kTomb) {  // still a tombstone (an older tag word was seen)
              r_pair = found;
              continue;
            }
            // the tombstone was taken: look again from its window
            r_slot = kNoSlot;
            base = r_base;
            w = r_w - 1u;  // the loop's increment brings it back to r_w
            rescan = true;
            break;
          }
          // someone filled the EMPTY slot first: look at what is there now
          win.set_pair(L, sub, (uint32_t)found, (uint32_t)(found >> 32));
        }
        if (rescan) continue;
        base += tb.window;
        if (base >= tb.nslots) base -= tb.nslots;
      }
      if (!resolved) unresolved = 1;
    }
    if (sub == 0) {
      if (kVoxel && dedup) lds.dd.out[p - tile_base] = out;
      if (!(kVoxel && copy)) slot_of[p] = out;
    }
  }
  if (kVoxel && dedup) {  // a voxel's later points in the block resolve through their representative's slot
    __syncthreads();
    const uint32_t t = threadIdx.x;
    const uint32_t rp = lds.dd.rep[t];
    if (tile_base + t < n && rp != kNoSlot && rp != t) {
      const uint32_t o = lds.dd.out[rp];
      slot_of[tile_base + t] = o == kNoSlot ? kNoSlot : (o & ~kCandidate);
    }
  }
  // Per-block count of new keys (a single shared counter would serialize
  // one atomic per wavefront); k_sum_partials adds them up when needed.
  const uint32_t wc = wave_sum(claimed);
  const uint32_t wu = wave_sum(unresolved);
  if (lane_id() == 0) {
    lds.count[threadIdx.x >> 6] = wc;
    if (wu) atomic_add_u32(&meta->fail, 1u);  // only when the table is full
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) c += lds.count[w];
    partial[tile] = c;
  }
  __syncthreads();  // the scratch is reused by the next tile of a persistent block
}

template <int KD, int G, int WL, typename Src, bool kVoxel, bool kReuse, bool kKeep>
__global__ __launch_bounds__(kBlock) void k_claim(TableRef tb, Src src, uint32_t n, uint32_t rounds,
                                                  uint32_t* __restrict__ slot_of, uint8_t* __restrict__ lost,
                                                  uint32_t* __restrict__ partial, Meta* meta) {
  __shared__ TileLds lds;
  claim_tile<KD, G, WL, Src, kVoxel, kReuse, kKeep>(tb, src, n, blockIdx.x, rounds, slot_of, lost, partial, meta,
                                                     lds);
}

// meta->claims = sum of the claim kernel's per-block counts (one block).
template <int kThreads>
__device__ __forceinline__ void sum_partials_block(const uint32_t* __restrict__ partial, uint32_t count, Meta* meta,
                                                   TileLds& lds) {
  uint32_t* s_sum = lds.count;
  uint32_t v = 0;
  for (uint32_t i = threadIdx.x; i < count; i += kThreads) v += partial[i];
  v = wave_sum(v);
  if (lane_id() == 0) s_sum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kThreads / 64; ++w) t += s_sum[w];
    meta->claims = t;
  }
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_sum_partials(const uint32_t* __restrict__ partial, uint32_t count,
                                                        Meta* meta) {
  __shared__ TileLds lds;
  sum_partials_block<1024>(partial, count, meta, lds);
}

// Moves the heap top and resets per-launch counters.  Runs after the
// scanning kernel, so every block of that kernel has read t / epoch.  The
// number of keys an insert added is the scan total of its commit (0 when the
// batch was rolled back).
// total: the scan total of the launch being finalized (winners of an insert
// or erase, the count of a compaction); n: the insert's batch size.
// used and tombs are upper bounds (an insert may reuse tombstones, a rolled
// back insert leaves tombstones); k_count_slots makes them exact.
__device__ __forceinline__ void finalize_total(Meta* m, uint32_t cap, int mode, int silent, int check,
                                               uint32_t total, uint32_t n = 0) {
  if (mode == kFinalizeInsert) {
    const bool overflow = m->fail != 0 || (check && m->claims > cap - m->t);
    if (!overflow) {
      m->t += total;
      m->used += total;
      m->result = total;
    } else {
      m->result = 0;
      m->used += n;  // claimed slots were rolled back to tombstones
      m->tombs += n;
      if (!silent)
        __hip_atomic_fetch_or(&m->status, m->fail ? kStatusTableFull : kStatusCapacity, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    }
    m->claims = 0;
    m->fail = 0;
  } else if (mode == kFinalizeErase) {
    m->t -= total;
    m->tombs += total;
    m->result = total;
  } else if (mode == kFinalizeCount) {
    m->result = total;
  } else if (mode == kFinalizeRebuild) {
    m->result = m->fail ? 1u : 0u;  // this rebuild's own outcome (status is sticky across calls)
    if (m->fail) __hip_atomic_fetch_or(&m->status, kStatusTableFull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    m->fail = 0;
  }
  m->epoch = m->epoch + 1u == 0u ? 1u : m->epoch + 1u;
}

// Copies the counters a host reader tracks to the table's mirror, if any
// (vector stores to host-mapped memory, visible once the kernel is done):
// t and the slot counts, and after an insert of n positions its new-key
// count, which the host uses to choose the next insert's claim variant.
__device__ __forceinline__ void publish_counts(const TableRef& tb, const Meta* m, uint32_t insert_n = 0) {
  if (!tb.mirror) return;
  tb.mirror->t = m->t;
  tb.mirror->used = m->used;
  tb.mirror->tombs = m->tombs;
  if (insert_n) {
    tb.mirror->result = m->result;
    tb.mirror->last_n = insert_n;
  }
  __threadfence_system();
}

__device__ __forceinline__ void finalize_map(Meta* m, uint32_t cap, int mode, int silent, int check,
                                             const uint64_t* status, uint32_t last_tile, uint32_t n = 0) {
  const uint32_t total = mode == kFinalizeRebuild ? 0u : (uint32_t)status[last_tile] & 0x7FFFFFFFu;
  finalize_total(m, cap, mode, silent, check, total, n);
}

// Where a find's, commit's or erase's results go: batch-indexed outputs
// (DirectOut), or the requests of a fused served batch (ReqOut).  put()
// writes a position's index (kNoSlot for a miss or a loser) and mask; rows()
// copies the value rows of a find tile's hits, given as (buffer index,
// position) pairs.
struct DirectOut {
  int32_t* __restrict__ idx;
  uint8_t* __restrict__ mask;
  __device__ __forceinline__ void put(uint32_t p, uint32_t i) const {
    const bool hit = i != kNoSlot;
    if (idx) idx[p] = hit ? (int32_t)i : -1;
    if (mask) mask[p] = hit ? 1 : 0;
  }
  __device__ __forceinline__ void rows(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) const {
    copy_rows(vs, j, pairs, count);
  }
};

struct ReqOut {
  const ReqDesc* __restrict__ d;
  const int64_t* s_off;  // LDS
  int nreq;
  __device__ __forceinline__ void put(uint32_t p, uint32_t i) const {
    const int r = request_of(s_off, nreq, p);
    const size_t q = p - s_off[r];
    const bool hit = i != kNoSlot;
    if (d[r].out_idx) d[r].out_idx[q] = hit ? (int32_t)i : -1;
    if (d[r].out_mask) d[r].out_mask[q] = hit ? 1 : 0;
  }
  template <typename V>
  __device__ __forceinline__ void rows_t(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) const {
    const uint32_t row = vs.row_bytes[j];
    const uint32_t units = row / (uint32_t)sizeof(V);
    for (uint32_t e = threadIdx.x; e < count * units; e += blockDim.x) {
      const uint32_t w = e / units;
      const uint32_t c = e - w * units;
      const uint2 pr = pairs[w];  // (buffer index, position)
      const int r = request_of(s_off, nreq, pr.y);
      uint8_t* dst = d[r].outv[j];
      if (!dst) continue;
      const V v = reinterpret_cast<const V*>(vs.src[j] + (size_t)pr.x * row)[c];
      reinterpret_cast<V*>(dst + (size_t)(pr.y - s_off[r]) * row)[c] = v;
    }
  }
  __device__ __forceinline__ void rows(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) const {
    switch (vs.vec[j]) {
      case 16: rows_t<uint4>(vs, j, pairs, count); break;
      case 8: rows_t<uint2>(vs, j, pairs, count); break;
      case 4: rows_t<uint32_t>(vs, j, pairs, count); break;
      case 2: rows_t<uint16_t>(vs, j, pairs, count); break;
      default: rows_t<uint8_t>(vs, j, pairs, count); break;
    }
  }
};


// Where a commit's value rows come from: the batch's rows (DirectRowsIn, row p
// of vs.src), or the requests of a fused served batch (ReqRowsIn: row p is
// row p - off[r] of its request's values).  copy() moves the rows of a tile's
// winners, given as (position, buffer index) pairs, to v^B.
struct DirectRowsIn {
  __device__ __forceinline__ void copy(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) const {
    copy_rows(vs, j, pairs, count);
  }
};

struct ReqRowsIn {
  const ReqDesc* __restrict__ d;
  const int64_t* s_off;  // LDS
  int nreq;
  template <typename V>
  __device__ __forceinline__ void copy_t(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) const {
    const uint32_t row = vs.row_bytes[j];
    const uint32_t units = row / (uint32_t)sizeof(V);
    for (uint32_t e = threadIdx.x; e < count * units; e += blockDim.x) {
      const uint32_t w = e / units;
      const uint32_t c = e - w * units;
      const uint2 pr = pairs[w];  // (position, buffer index)
      const int r = request_of(s_off, nreq, pr.x);
      const V v = reinterpret_cast<const V*>(d[r].vals[j] + (size_t)(pr.x - s_off[r]) * row)[c];
      reinterpret_cast<V*>(vs.dst[j] + (size_t)pr.y * row)[c] = v;
    }
  }
  __device__ __forceinline__ void copy(const ValueSet& vs, int j, const uint2* pairs, uint32_t count) const {
    switch (vs.vec[j]) {
      case 16: copy_t<uint4>(vs, j, pairs, count); break;
      case 8: copy_t<uint2>(vs, j, pairs, count); break;
      case 4: copy_t<uint32_t>(vs, j, pairs, count); break;
      case 2: copy_t<uint16_t>(vs, j, pairs, count); break;
      default: copy_t<uint8_t>(vs, j, pairs, count); break;
    }
  }
};

// ---------------------------------------------------------------------------
// Commit (insert / activate pass 2).  Winners are the candidates not marked
// lost; they are ranked in batch order and take i = h[t + rank].  The lost
// bytes read here are cleared again, so the array is all zero between calls.
// Value rows are copied by the block right after the ranking (kInline), or
// left to k_scatter_values: then each winner writes its position at its
// global rank, wlist[prefix + rank] = p, and the rows move after the
// finalize in a separate pass over the winners only.  The block copy is a
// dependent chain per tile, which costs little for short rows; the separate
// pass keeps many more loads in flight and wins for long rows.
template <int KD, bool kInline, typename Src, typename Out, typename Rows>
__device__ __forceinline__ void commit_tile_src(const TableRef& tb, const Src& src, const Out& out, const Rows& rows,
                                                uint32_t n, uint32_t tile, const uint32_t* __restrict__ slot_of,
                                                uint8_t* __restrict__ lost, int32_t* __restrict__ kB,
                                                const int32_t* __restrict__ heap, uint32_t cap, const ValueSet& vs,
                                                Meta* meta, uint64_t* __restrict__ status, int check,
                                                uint32_t* __restrict__ wlist, int fin, TileLds& lds) {
  constexpr int S = SlotWords<KD>::value;
  uint2* s_pairs = lds.pairs;
  const uint32_t t0 = meta->t;
  // With check == 0 the host has proved t + new keys <= c (its bound on t
  // plus n); otherwise meta->claims holds the summed count of new keys.
  const bool overflow = meta->fail != 0 || (check && meta->claims > cap - t0);
  const uint32_t base = tile * kScanTile;
  bool win[kScanItems];
  uint32_t slot[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    slot[r] = kNoSlot;
    win[r] = false;
    if (p < n) {
      slot[r] = slot_of[p];
      const uint8_t l = lost[p];
      if (l) lost[p] = 0;
      win[r] = slot[r] != kNoSlot && l == 0;
    }
  }
  if (overflow) {
    // Roll the claims back to tombstones: a claimed slot may have been a
    // tombstone that other keys' probe sequences run through, and a
    // tombstone is correct in either case (the occupied-slot count stays an
    // upper bound).
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      if (win[r]) *reinterpret_cast<uint2*>(tb.words + (size_t)slot[r] * S + S - 2) = make_uint2(kEmpty, kTomb);
      win[r] = false;  // every position reports a miss; tiles still publish
    }
  }
  uint32_t rank[kScanItems];
  uint32_t total;
  block_rank_rows(win, rank, total, lds.scan);
  const uint32_t prefix = block_lookback(status, tile, meta->epoch, total, &meta->status, &lds.prefix);
  // fin >= 0: the last tile finalizes the insert (fin = silent flag).  Its
  // look-back saw every other tile publish, and each tile publishes only
  // after reading t, the epoch and the claim counters, so none reads them
  // after this point; the next kernel sees the update at the launch boundary.
  if (fin >= 0 && threadIdx.x == 0 && tile == (n - 1) / kScanTile) {
    finalize_total(meta, cap, kFinalizeInsert, fin, check, prefix + total, n);
    publish_counts(tb, meta, n);
  }
  bool bad = false;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    if (p >= n) continue;
    if (win[r] && t0 + prefix + rank[r] >= cap) bad = true;  // cannot happen: winners == claims
    if (win[r] && t0 + prefix + rank[r] < cap) {
      const uint32_t i = (uint32_t)heap[t0 + prefix + rank[r]];
      int32_t k[KD];
      src.load(p, k);
#pragma unroll
      for (int d = 0; d < KD; ++d) kB[(size_t)i * KD + d] = k[d];
      store_slot<S>(tb.words + (size_t)slot[r] * S, committed_slot<KD, S>(k, i));
      if constexpr (kInline) s_pairs[rank[r]] = make_uint2(p, i);
      else if (wlist) wlist[prefix + rank[r]] = p;
      out.put(p, i);
    } else {
      out.put(p, kNoSlot);
    }
  }
  if constexpr (kInline) {
    if (vs.n > 0 && !__syncthreads_or(bad)) {
      for (int j = 0; j < vs.n; ++j) rows.copy(vs, j, s_pairs, total);
    }
  }
  __syncthreads();  // LDS is reused by the next tile of a persistent block
}

template <int KD, bool kInline>
__device__ __forceinline__ void commit_tile(const TableRef& tb, const int32_t* __restrict__ keys, uint32_t n,
                                            uint32_t tile, const uint32_t* __restrict__ slot_of,
                                            uint8_t* __restrict__ lost, int32_t* __restrict__ kB,
                                            const int32_t* __restrict__ heap, uint32_t cap, const ValueSet& vs,
                                            int32_t* __restrict__ out_idx, uint8_t* __restrict__ out_mask,
                                            Meta* meta, uint64_t* __restrict__ status, int check,
                                            uint32_t* __restrict__ wlist, int fin, TileLds& lds) {
  commit_tile_src<KD, kInline>(tb, BatchKeys<KD>{keys}, DirectOut{out_idx, out_mask}, DirectRowsIn{}, n, tile,
                               slot_of, lost, kB, heap, cap, vs, meta, status, check, wlist, fin, lds);
}

// Value rows of an insert's winners, after its finalize: the finalize left
// the number of winners in meta->result and moved t past their indices, so
// winner w (in batch order) went to i = h[t - total + w] from position
// wlist[w].  dst row i = src row p, in units of V; threads past the winners
// only read the two counters.  Each thread takes U units a grid stride
// apart and issues all their loads before any store, so U (wlist, heap, row)
// chains are in flight per thread; that pays for rows of 1 KB and more
// (16 KB rows: 7.25 -> 6.55 ms for 1M rows) and costs up to 40% below.
constexpr uint32_t kUnrollRowBytes = 1024;

template <typename V, int U>
__global__ __launch_bounds__(kBlock) void k_scatter_values(const uint32_t* __restrict__ wlist,
                                                           const int32_t* __restrict__ heap, const Meta* meta,
                                                           const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                           uint32_t row_bytes, uint32_t units_log2, uint32_t n,
                                                           uint32_t cap) {
  const uint32_t total = meta->result;
  const uint32_t base = meta->t - total;
  const uint32_t units = row_bytes / (uint32_t)sizeof(V);
  const uint64_t items = (uint64_t)total * units;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t e0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e0 < items; e0 += stride * U) {
    V v[U];
    V* to[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      to[k] = nullptr;
      const uint64_t e = e0 + (uint64_t)k * stride;
      if (e >= items) continue;
      uint32_t w, c;
      if (units_log2 != 0xFFu) {
        w = (uint32_t)(e >> units_log2);
        c = (uint32_t)e & (units - 1u);
      } else {
        w = (uint32_t)(e / units);
        c = (uint32_t)(e - (uint64_t)w * units);
      }
      const uint32_t p = wlist[w];
      const uint32_t i = (uint32_t)heap[base + w];
      if (p >= n || i >= cap) continue;  // cannot happen: every winner listed itself
      v[k] = reinterpret_cast<const V*>(src + (size_t)p * row_bytes)[c];
      to[k] = reinterpret_cast<V*>(dst + (size_t)i * row_bytes) + c;
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (to[k]) *to[k] = v[k];
  }
}

// Value rows of a find's hits, after the find: dst row p = src row idx[p]
// for every p whose idx is a buffer index; rows of misses (idx -1) stay
// untouched.  A pass over n * units items sized by the row bytes keeps the
// whole chip copying even when n is small and rows are long, which a copy
// by the find's own blocks (one block per tile of positions) does not.
// Each thread takes U units a grid stride apart and loads them all before
// storing any.
template <typename V, int U>
__global__ __launch_bounds__(kBlock) void k_gather_rows(const int32_t* __restrict__ idx,
                                                        const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                        uint32_t row_bytes, uint32_t units_log2, uint32_t n,
                                                        uint32_t cap) {
  const uint32_t units = row_bytes / (uint32_t)sizeof(V);
  const uint64_t items = (uint64_t)n * units;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t e0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e0 < items; e0 += stride * U) {
    V v[U];
    V* to[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      to[k] = nullptr;
      const uint64_t e = e0 + (uint64_t)k * stride;
      if (e >= items) continue;
      uint32_t p, c;
      if (units_log2 != 0xFFu) {
        p = (uint32_t)(e >> units_log2);
        c = (uint32_t)e & (units - 1u);
      } else {
        p = (uint32_t)(e / units);
        c = (uint32_t)(e - (uint64_t)p * units);
      }
      const int32_t i = idx[p];
      if (i < 0 || (uint32_t)i >= cap) continue;  // a miss
      v[k] = reinterpret_cast<const V*>(src + (size_t)(uint32_t)i * row_bytes)[c];
      to[k] = reinterpret_cast<V*>(dst + (size_t)p * row_bytes) + c;
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (to[k]) *to[k] = v[k];
  }
}

template <int KD, bool kInline>
__global__ __launch_bounds__(kBlock) void k_commit(TableRef tb, const int32_t* __restrict__ keys, uint32_t n,
                                                   const uint32_t* __restrict__ slot_of, uint8_t* __restrict__ lost,
                                                   int32_t* __restrict__ kB, const int32_t* __restrict__ heap,
                                                   uint32_t cap, ValueSet vs, int32_t* __restrict__ out_idx,
                                                   uint8_t* __restrict__ out_mask, Meta* meta,
                                                   uint64_t* __restrict__ status, int check,
                                                   uint32_t* __restrict__ wlist, int silent) {
  __shared__ TileLds lds;
  commit_tile<KD, kInline>(tb, keys, n, blockIdx.x, slot_of, lost, kB, heap, cap, vs, out_idx, out_mask, meta,
                           status, check, wlist, silent, lds);
}

__global__ void k_finalize(Meta* m, uint32_t cap, int mode, int silent, int check, const uint64_t* status,
                           uint32_t last_tile) {
  finalize_map(m, cap, mode, silent, check, status, last_tile);
}

// ---------------------------------------------------------------------------
// Find (masked query, Sec. 4.2) with optional value gather.  Probing stops at
// the first window that holds an EMPTY slot: a key is always claimed at the
// first EMPTY slot of its sequence and slots never return to EMPTY outside a
// rebuild.
template <int KD, int G, int WL, typename Src, typename Out = DirectOut>
__device__ __forceinline__ void find_tile(const TableRef& tb, const Src& src, uint32_t n,
                                          uint32_t tile, uint32_t rounds, const Out& out, const ValueSet& vs,
                                          TileLds& lds) {
  using Win = Window<KD, G, WL>;
  constexpr int S = Win::S;
  constexpr uint32_t kGroups = kBlock / G;
  uint2* s_pairs = lds.pairs;
  uint32_t& s_hits = lds.hits;
  const uint32_t sub = G == 1 ? 0u : (threadIdx.x & (G - 1));
  const uint32_t grp = threadIdx.x / G;
  const uint32_t tile_base = tile * kGroups * rounds;
  if (vs.n > 0) {
    if (threadIdx.x == 0) s_hits = 0;
    __syncthreads();
  }
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint32_t p = tile_base + r * kGroups + grp;
    if (p >= n) break;
    int32_t k[KD];
    src.load(p, k);
    const uint64_t h = key_hash<KD>(k);
    uint32_t base = home_slot(tb, h);
    uint32_t idx = kNoSlot;
    for (uint32_t w = 0; w < tb.max_windows; ++w) {
      Win win;
      win.load(tb, base, sub);
      const uint64_t mh = win.mask([&](const Slot<S> sl) {
        return sl.w[S - 1] < kPending && slot_holds<KD, S>(sl, k);
      });
      if (mh) {
        idx = win.word(first_lane(mh), S - 1);
        break;
      }
      if (win.mask([&](const Slot<S> sl) { return sl.w[S - 1] == kEmpty; })) break;
      base += tb.window;
      if (base >= tb.nslots) base -= tb.nslots;
    }
    if (sub == 0) {
      out.put(p, idx);
      if (idx != kNoSlot && vs.n > 0) s_pairs[atomicAdd(&s_hits, 1u)] = make_uint2(idx, p);
    }
  }
  if (vs.n > 0) {
    __syncthreads();
    const uint32_t hits = s_hits;
    for (int j = 0; j < vs.n; ++j) out.rows(vs, j, s_pairs, hits);
    __syncthreads();  // LDS is reused by the next tile of a persistent block
  }
}

template <int KD, int G, int WL>
__global__ __launch_bounds__(kBlock) void k_find(TableRef tb, const int32_t* __restrict__ keys, uint32_t n,
                                                 uint32_t rounds, int32_t* __restrict__ out_idx,
                                                 uint8_t* __restrict__ out_mask, ValueSet vs) {
  __shared__ TileLds lds;
  find_tile<KD, G, WL>(tb, BatchKeys<KD>{keys}, n, blockIdx.x, rounds, DirectOut{out_idx, out_mask}, vs, lds);
}

// A fused served find: keys come from the requests' buffers and every
// result goes straight to its request (vs: the map's rows as sources; rows
// are copied for requests that asked for them).
template <int KD, int G, int WL>
__global__ __launch_bounds__(kBlock) void k_find_requests(TableRef tb, ReqArgs args, const ReqDesc* __restrict__ gd, int nreq,
                                                          uint32_t n, uint32_t rounds, ValueSet vs) {
  __shared__ TileLds lds;
  __shared__ int64_t s_off[kMaxFusedRequests];
  __shared__ ReqDesc s_desc[kArgRequests];
  const ReqDesc* d = stage_requests(args, gd, nreq, s_desc, s_off);
  find_tile<KD, G, WL>(tb, ReqKeys<KD>{d, s_off, nreq}, n, blockIdx.x, rounds, ReqOut{d, s_off, nreq}, vs, lds);
}

// Neighbor lookups: a find over n * k shifted keys, results query-major.
template <int KD, int G, int WL>
__global__ __launch_bounds__(kBlock) void k_find_offsets(TableRef tb, OffsetKeys<KD> src, uint32_t n,
                                                         uint32_t rounds, int32_t* __restrict__ out_idx,
                                                         uint8_t* __restrict__ out_mask) {
  __shared__ TileLds lds;
  ValueSet none;
  none.n = 0;
  find_tile<KD, G, WL>(tb, src, n, blockIdx.x, rounds, DirectOut{out_idx, out_mask}, none, lds);
}

// ---------------------------------------------------------------------------
// Erase pass 1: locate each key and elect the lowest position per buffer
// index.  owner[i] holds (epoch << 32) | ~p of the call that wrote it, and
// positions race with a 64-bit atomicMax: entries of earlier calls (smaller
// epoch) lose to any position of this call, and within the call the largest
// ~p is the lowest p -- so owner never needs clearing.  The returned value
// tells each position whether it displaced an earlier holder (lost[holder]
// = 1) or lost itself.
template <int KD, int G, int WL, typename Src>
__device__ __forceinline__ void erase_mark_tile(const TableRef& tb, const Src& src, uint32_t n, uint32_t tile,
                                                uint32_t rounds, uint32_t epoch, uint32_t* __restrict__ slot_of,
                                                int32_t* __restrict__ found_idx, uint64_t* __restrict__ owner,
                                                uint8_t* __restrict__ lost) {
  using Win = Window<KD, G, WL>;
  constexpr int S = Win::S;
  constexpr uint32_t kGroups = kBlock / G;
  const uint32_t sub = G == 1 ? 0u : (threadIdx.x & (G - 1));
  const uint32_t grp = threadIdx.x / G;
  const uint32_t tile_base = tile * kGroups * rounds;
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint32_t p = tile_base + r * kGroups + grp;
    if (p >= n) break;
    int32_t k[KD];
    src.load(p, k);
    const uint64_t h = key_hash<KD>(k);
    uint32_t base = home_slot(tb, h);
    uint32_t idx = kNoSlot, where = kNoSlot;
    for (uint32_t w = 0; w < tb.max_windows; ++w) {
      Win win;
      win.load(tb, base, sub);
      const uint64_t mh = win.mask([&](const Slot<S> sl) {
        return sl.w[S - 1] < kPending && slot_holds<KD, S>(sl, k);
      });
      if (mh) {
        const uint32_t L = first_lane(mh);
        idx = win.word(L, S - 1);
        where = win.slot(L);
        break;
      }
      if (win.mask([&](const Slot<S> sl) { return sl.w[S - 1] == kEmpty; })) break;
      base += tb.window;
      if (base >= tb.nslots) base -= tb.nslots;
    }
    if (sub == 0) {
      bool cand = false;
      if (idx != kNoSlot) {
        const uint64_t mine = ((uint64_t)epoch << 32) | (uint64_t)(~p);
        const uint64_t old = __hip_atomic_fetch_max(owner + idx, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(old >> 32) != epoch) {
          cand = true;  // first position of this call for the index
        } else {
          const uint32_t prev = ~(uint32_t)old;
          cand = prev > p;
          if (cand && prev < n) lost[prev] = 1;
        }
      }
      slot_of[p] = cand ? where : kNoSlot;
      found_idx[p] = cand ? (int32_t)idx : -1;
    }
  }
}

template <int KD, int G, int WL>
__global__ __launch_bounds__(kBlock) void k_erase_mark(TableRef tb, const int32_t* __restrict__ keys, uint32_t n,
                                                       uint32_t rounds, uint32_t epoch,
                                                       uint32_t* __restrict__ slot_of,
                                                       int32_t* __restrict__ found_idx, uint64_t* __restrict__ owner,
                                                       uint8_t* __restrict__ lost) {
  erase_mark_tile<KD, G, WL>(tb, BatchKeys<KD>{keys}, n, blockIdx.x, rounds, epoch, slot_of, found_idx, owner, lost);
}

// Erase pass 2: winners (candidates not marked lost) tombstone their slot and
// push their index back on the heap in batch order: the r-th winner writes
// h[t - 1 - r].  Out receives each position's mask (put with kNoSlot: 0).
template <int KD, typename Out>
__device__ __forceinline__ void erase_commit_tile(const TableRef& tb, uint32_t n, uint32_t tile,
                                                  const uint32_t* __restrict__ slot_of,
                                                  const int32_t* __restrict__ found_idx, uint8_t* __restrict__ lost,
                                                  int32_t* __restrict__ heap, const Out& out, Meta* meta,
                                                  uint64_t* __restrict__ status, uint32_t* s_prefix,
                                                  uint64_t* s_scan) {
  constexpr int S = SlotWords<KD>::value;
  const uint32_t t0 = meta->t;
  const uint32_t base = tile * kScanTile;
  bool win[kScanItems];
  int32_t idx[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    idx[r] = -1;
    win[r] = false;
    if (p < n) {
      idx[r] = found_idx[p];
      const uint8_t l = lost[p];
      if (l) lost[p] = 0;
      win[r] = idx[r] >= 0 && l == 0;
    }
  }
  uint32_t rank[kScanItems];
  uint32_t total;
  block_rank_rows(win, rank, total, s_scan);
  block_lookback(status, tile, meta->epoch, total, &meta->status, s_prefix);
  const uint32_t prefix = *s_prefix;
  // the last tile finalizes the erase (every tile read t and the epoch before
  // publishing, see commit_tile)
  if (threadIdx.x == 0 && tile == (n - 1) / kScanTile) {
    finalize_total(meta, 0u, kFinalizeErase, 0, 0, prefix + total);
    publish_counts(tb, meta);
  }
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    if (p >= n) continue;
    if (win[r] && prefix + rank[r] < t0) {  // winners are distinct live indices: always true
      heap[t0 - 1u - (prefix + rank[r])] = idx[r];
      tb.words[(size_t)slot_of[p] * S + S - 1] = kTomb;
    }
    out.put(p, win[r] ? 0u : kNoSlot);
  }
}

template <int KD>
__global__ __launch_bounds__(kBlock) void k_erase_commit(TableRef tb, uint32_t n, const uint32_t* __restrict__ slot_of,
                                                         const int32_t* __restrict__ found_idx,
                                                         uint8_t* __restrict__ lost, int32_t* __restrict__ heap,
                                                         uint8_t* __restrict__ out_mask, Meta* meta,
                                                         uint64_t* __restrict__ status) {
  __shared__ uint32_t s_prefix;
  __shared__ uint64_t s_scan[kBlock / 64 + 1];
  erase_commit_tile<KD>(tb, n, blockIdx.x, slot_of, found_idx, lost, heap, DirectOut{nullptr, out_mask}, meta, status,
                        &s_prefix, s_scan);
}

// ---------------------------------------------------------------------------
// Fused served batches of inserts or erases read the keys (and value rows)
// from the requests' own buffers and write each request's results there: the
// same passes as above over a key source and an output that map a batch
// position to its request (the offsets staged in LDS), with no staging copy
// in or out.  Value rows are copied inside the commit (rows under 64 B per
// key in total; longer rows take the staged path).

template <int KD, int G, int WL, bool kReuse, bool kKeep>
__global__ __launch_bounds__(kBlock) void k_claim_requests(TableRef tb, ReqArgs args, const ReqDesc* __restrict__ gd, int nreq,
                                                           uint32_t n, uint32_t rounds, uint32_t* __restrict__ slot_of,
                                                           uint8_t* __restrict__ lost, uint32_t* __restrict__ partial,
                                                           Meta* meta) {
  __shared__ TileLds lds;
  __shared__ int64_t s_off[kMaxFusedRequests];
  __shared__ ReqDesc s_desc[kArgRequests];
  const ReqDesc* d = stage_requests(args, gd, nreq, s_desc, s_off);
  claim_tile<KD, G, WL, ReqKeys<KD>, false, kReuse, kKeep>(tb, ReqKeys<KD>{d, s_off, nreq}, n, blockIdx.x, rounds,
                                                            slot_of, lost, partial, meta, lds);
}

template <int KD>
__global__ __launch_bounds__(kBlock) void k_commit_requests(TableRef tb, ReqArgs args, const ReqDesc* __restrict__ gd, int nreq,
                                                            uint32_t n, const uint32_t* __restrict__ slot_of,
                                                            uint8_t* __restrict__ lost, int32_t* __restrict__ kB,
                                                            const int32_t* __restrict__ heap, uint32_t cap,
                                                            ValueSet vs, Meta* meta, uint64_t* __restrict__ status,
                                                            int check, int silent) {
  __shared__ TileLds lds;
  __shared__ int64_t s_off[kMaxFusedRequests];
  __shared__ ReqDesc s_desc[kArgRequests];
  const ReqDesc* d = stage_requests(args, gd, nreq, s_desc, s_off);
  commit_tile_src<KD, true>(tb, ReqKeys<KD>{d, s_off, nreq}, ReqOut{d, s_off, nreq}, ReqRowsIn{d, s_off, nreq}, n,
                            blockIdx.x, slot_of, lost, kB, heap, cap, vs, meta, status, check, nullptr, silent, lds);
}

template <int KD, int G, int WL>
__global__ __launch_bounds__(kBlock) void k_erase_mark_requests(TableRef tb, ReqArgs args, const ReqDesc* __restrict__ gd, int nreq,
                                                                uint32_t n, uint32_t rounds, uint32_t epoch,
                                                                uint32_t* __restrict__ slot_of,
                                                                int32_t* __restrict__ found_idx,
                                                                uint64_t* __restrict__ owner,
                                                                uint8_t* __restrict__ lost) {
  __shared__ int64_t s_off[kMaxFusedRequests];
  __shared__ ReqDesc s_desc[kArgRequests];
  const ReqDesc* d = stage_requests(args, gd, nreq, s_desc, s_off);
  erase_mark_tile<KD, G, WL>(tb, ReqKeys<KD>{d, s_off, nreq}, n, blockIdx.x, rounds, epoch, slot_of, found_idx, owner,
                             lost);
}

template <int KD>
__global__ __launch_bounds__(kBlock) void k_erase_commit_requests(TableRef tb, ReqArgs args, const ReqDesc* __restrict__ gd, int nreq,
                                                                  uint32_t n, const uint32_t* __restrict__ slot_of,
                                                                  const int32_t* __restrict__ found_idx,
                                                                  uint8_t* __restrict__ lost,
                                                                  int32_t* __restrict__ heap, Meta* meta,
                                                                  uint64_t* __restrict__ status) {
  __shared__ uint32_t s_prefix;
  __shared__ uint64_t s_scan[kBlock / 64 + 1];
  __shared__ int64_t s_off[kMaxFusedRequests];
  __shared__ ReqDesc s_desc[kArgRequests];
  const ReqDesc* d = stage_requests(args, gd, nreq, s_desc, s_off);
  erase_commit_tile<KD>(tb, n, blockIdx.x, slot_of, found_idx, lost, heap, ReqOut{d, s_off, nreq}, meta, status,
                        &s_prefix, s_scan);
}

// ---------------------------------------------------------------------------
// Exact occupancy: meta->used += non-EMPTY slots and meta->tombs += tombstones
// (both zeroed before the launch), one atomic pair per block.
template <int S>
__global__ __launch_bounds__(kBlock) void k_count_slots(TableRef tb, Meta* meta) {
  __shared__ uint32_t s_used[kBlock / 64], s_tomb[kBlock / 64];
  uint32_t used = 0, tomb = 0;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < tb.nslots; s += gridDim.x * kBlock) {
    const uint32_t st = tb.words[(size_t)s * S + S - 1];
    used += st != kEmpty ? 1u : 0u;
    tomb += st == kTomb ? 1u : 0u;
  }
  used = wave_sum(used);
  tomb = wave_sum(tomb);
  if (lane_id() == 0) {
    s_used[threadIdx.x >> 6] = used;
    s_tomb[threadIdx.x >> 6] = tomb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t u = 0, t = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      u += s_used[w];
      t += s_tomb[w];
    }
    atomic_add_u32(&meta->used, u);
    atomic_add_u32(&meta->tombs, t);
  }
}

hipError_t launch_count_slots(int kd, const TableRef& tb, Meta* meta, hipStream_t st) {
  hipError_t e = launch_fill_u32(&meta->used, 0u, 2, st);  // used and tombs are adjacent
  if (e != hipSuccess) return e;
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((tb.nslots + kBlock - 1) / kBlock, 1024));
  switch (kd) {
    case 1: hipLaunchKernelGGL(k_count_slots<2>, dim3(grid), dim3(kBlock), 0, st, tb, meta); break;
    case 2:
    case 3: hipLaunchKernelGGL(k_count_slots<4>, dim3(grid), dim3(kBlock), 0, st, tb, meta); break;
    case 4: hipLaunchKernelGGL(k_count_slots<8>, dim3(grid), dim3(kBlock), 0, st, tb, meta); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Active indices (ascending): flags[i] = 1 for every committed slot, then a
// compaction of the flags.
template <int S>
__global__ __launch_bounds__(kBlock) void k_mark_live(TableRef tb, uint8_t* __restrict__ flags, uint32_t c) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < tb.nslots; s += stride) {
    const uint32_t st = tb.words[(size_t)s * S + S - 1];
    if (st < kPending && st < c) flags[st] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_compact_flags(const uint8_t* __restrict__ flags, uint32_t c,
                                                          int32_t* __restrict__ out, Meta* meta,
                                                          uint64_t* __restrict__ status) {
  __shared__ uint32_t s_prefix;
  __shared__ uint64_t s_scan[kBlock / 64 + 1];
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kScanTile;
  bool on[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r * kBlock + threadIdx.x;
    on[r] = i < c && flags[i] != 0;
  }
  uint32_t rank[kScanItems];
  uint32_t total;
  block_rank_rows(on, rank, total, s_scan);
  block_lookback(status, tile, meta->epoch, total, &meta->status, &s_prefix);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r)
    if (on[r]) out[s_prefix + rank[r]] = (int32_t)(base + r * kBlock + threadIdx.x);
}

// Set intersection (Sec. 6.4): the rows of the queries whose find mask is 1,
// compacted in batch order.  The last tile's look-back sees every tile's
// count, so it also finalizes (meta->result = number of rows).
template <int KD>
__global__ __launch_bounds__(kBlock) void k_compact_rows(const uint8_t* __restrict__ mask, uint32_t n,
                                                         const int32_t* __restrict__ keys,
                                                         int32_t* __restrict__ out, Meta* meta,
                                                         uint64_t* __restrict__ status) {
  __shared__ uint32_t s_prefix;
  __shared__ uint64_t s_scan[kBlock / 64 + 1];
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kScanTile;
  bool on[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t i = base + r * kBlock + threadIdx.x;
    on[r] = i < n && mask[i] != 0;
  }
  uint32_t rank[kScanItems];
  uint32_t total;
  block_rank_rows(on, rank, total, s_scan);
  const uint32_t prefix = block_lookback(status, tile, meta->epoch, total, &meta->status, &s_prefix);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    if (!on[r]) continue;
    const size_t i = base + r * kBlock + threadIdx.x;
    const size_t o = prefix + rank[r];
#pragma unroll
    for (int d = 0; d < KD; ++d) out[o * KD + d] = keys[i * KD + d];
  }
  if (threadIdx.x == 0 && tile == (n - 1) / kScanTile) finalize_total(meta, 0u, kFinalizeCount, 0, 0, prefix + total);
}

// ---------------------------------------------------------------------------
// Rebuild (rehash, Sec. 4.5): every committed slot of the old table is
// inserted into a fresh table as (key, COMMITTED(i)); tombstones are dropped.
// Keys are distinct, so a position only looks for EMPTY slots: the leader
// CASes (k_{KD-1}, i) into the first one and then writes the other key words.
template <int KD, int G, int WL>
__global__ __launch_bounds__(kBlock) void k_rebuild(TableRef tb, const uint32_t* __restrict__ old_words,
                                                    uint32_t old_slots, uint32_t rounds, Meta* meta) {
  using Win = Window<KD, G, WL>;
  constexpr int S = Win::S;
  constexpr uint32_t kGroups = kBlock / G;
  const uint32_t sub = G == 1 ? 0u : (threadIdx.x & (G - 1));
  const uint32_t grp = threadIdx.x / G;
  const uint32_t tile_base = blockIdx.x * kGroups * rounds;
  uint32_t unresolved = 0;
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint32_t os = tile_base + r * kGroups + grp;
    if (os >= old_slots) break;
    const Slot<S> old = load_slot<S>(old_words + (size_t)os * S);
    const uint32_t i = old.w[S - 1];
    if (i >= kPending) continue;  // empty or tombstone
    int32_t k[KD];
#pragma unroll
    for (int d = 0; d < KD - 1; ++d) k[d] = (int32_t)old.w[d];
    k[KD - 1] = (int32_t)old.w[S - 2];
    const uint64_t h = key_hash<KD>(k);
    const uint64_t desired = ((uint64_t)i << 32) | (uint32_t)k[KD - 1];
    uint32_t base = home_slot(tb, h);
    bool done = false;
    for (uint32_t w = 0; w < tb.max_windows && !done; ++w) {
      Win win;
      win.load(tb, base, sub);
      while (true) {
        const uint64_t me = win.mask([&](const Slot<S> sl) { return sl.w[S - 1] == kEmpty; });
        if (!me) break;
        const uint32_t L = first_lane(me);
        const uint32_t s = win.slot(L);
        uint64_t found = 0;
        if (sub == 0) {
          uint32_t* sp = tb.words + (size_t)s * S;
          found = cas_pair(sp + S - 2, kEmptyPair, desired);
          if (found == kEmptyPair) {
#pragma unroll
            for (int d = 0; d < KD - 1; ++d) sp[d] = (uint32_t)k[d];
          }
        }
        found = leader_bcast64<G>(found);
        if (found == kEmptyPair) {
          done = true;
          break;
        }
        win.set_pair(L, sub, (uint32_t)found, (uint32_t)(found >> 32));
      }
      base += tb.window;
      if (base >= tb.nslots) base -= tb.nslots;
    }
    if (!done) unresolved = 1;
  }
  if (wave_sum(unresolved) && lane_id() == 0) atomic_add_u32(&meta->fail, 1u);
}

// ---------------------------------------------------------------------------
// Voxelization pass 2: the first occurrence of each voxel (its winner) gets
// the id rank-of-first-occurrence; its slot becomes COMMITTED(id).
__global__ __launch_bounds__(kBlock) void k_voxel_commit(TableRef tb, VoxelKeys src, uint32_t n,
                                                         uint32_t* __restrict__ slot_of,
                                                         uint8_t* __restrict__ lost,
                                                         int32_t* __restrict__ voxel_keys,
                                                         int32_t* __restrict__ counts,
                                                         int32_t* __restrict__ point_voxel, Meta* meta,
                                                         uint64_t* __restrict__ status) {
  constexpr int S = SlotWords<3>::value;
  __shared__ uint32_t s_prefix;
  __shared__ uint64_t s_scan[kBlock / 64 + 1];
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kScanTile;
  bool win[kScanItems];
  uint32_t slot[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    slot[r] = kNoSlot;
    win[r] = false;
    if (p < n) {
      const uint32_t so = slot_of[p];
      const uint8_t l = lost[p];
      if (l) lost[p] = 0;
      win[r] = so != kNoSlot && (so & kCandidate) && l == 0;
      slot[r] = so & ~kCandidate;
      if (so == kNoSlot) point_voxel[p] = -1;  // rejected point
    }
  }
  uint32_t rank[kScanItems];
  uint32_t total;
  block_rank_rows(win, rank, total, s_scan);
  block_lookback(status, tile, meta->epoch, total, &meta->status, &s_prefix);
  // the last tile's look-back saw every tile: it records the voxel count
  if (threadIdx.x == 0 && tile == gridDim.x - 1) meta->claims = s_prefix + total;
  // Where most points of a tile open a voxel (a fine voxelization), the
  // tile does not write voxel ids into slots (one random store per voxel);
  // the few later points find such an id through the voxel's first point
  // instead (the slot still holds PENDING(first point); see
  // k_voxel_resolve, which handles either state per slot).
  const uint32_t tile_points = n - base < kScanTile ? n - base : kScanTile;
  const bool publish = 2u * total <= tile_points;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    if (!win[r]) continue;
    const uint32_t p = base + r * kBlock + threadIdx.x;
    const uint32_t id = s_prefix + rank[r];
    int32_t k[3];
    src.load(p, k);
    voxel_keys[(size_t)id * 3 + 0] = k[0];
    voxel_keys[(size_t)id * 3 + 1] = k[1];
    voxel_keys[(size_t)id * 3 + 2] = k[2];
    // a voxel's first point is resolved here: it counts itself, and the
    // resolve pass skips it
    counts[id] = 1;
    point_voxel[p] = (int32_t)id;
    slot_of[p] = kNoSlot;
    if (publish) tb.words[(size_t)slot[r] * S + S - 1] = id;
  }
}

// Block and in-block voxel coordinates (the coupled lookup of Sec. 6.2.2):
// per axis the voxel index v = floor(p / voxel), formed as in voxelization,
// then block = floor(v / res) and local = v - block * res in [0, res).
// Equal over the reals to the paper's floor(x / (s res)) and
// floor((x - block s res) / s), and exact in integers.  Rejected points get
// valid 0 and zero coordinates.  One thread per point; an HBM-bound stream.
__global__ __launch_bounds__(kBlock) void k_block_coords(const float* __restrict__ pts, uint32_t n, float voxel,
                                                         int32_t res, int32_t* __restrict__ block_keys,
                                                         int32_t* __restrict__ local, uint8_t* __restrict__ valid) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int32_t v[3];
  const bool ok = VoxelKeys{pts, voxel}.load(p, v);
  valid[p] = ok ? 1 : 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int64_t b = 0, l = 0;  // 64-bit: b * res may leave int32 near its ends
    if (ok) {
      b = v[d] / res;
      if (v[d] % res != 0 && v[d] < 0) b -= 1;
      l = v[d] - b * res;
    }
    block_keys[(size_t)p * 3 + d] = (int32_t)b;
    local[(size_t)p * 3 + d] = (int32_t)l;
  }
}

// Voxelization pass 3: voxel ids and counts of the points the commit left:
// every accepted point that is not its voxel's first (the commit resolved
// first points and rejected ones, and set their slot_of to kNoSlot).  The
// slot holds the voxel's id, or, when the commit did not write ids into
// slots, PENDING(first point), whose id the commit wrote to point_voxel.
__global__ __launch_bounds__(kBlock) void k_voxel_resolve(TableRef tb, uint32_t n, const uint32_t* __restrict__ slot_of,
                                                          int32_t* __restrict__ point_voxel,
                                                          int32_t* __restrict__ counts) {
  constexpr int S = SlotWords<3>::value;
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t so = slot_of[p];
  if (so == kNoSlot) return;
  uint32_t id = tb.words[(size_t)(so & ~kCandidate) * S + S - 1];
  if (id >= kPending && id < kTomb) {
    const uint32_t first = id - kPending;
    id = first < n ? (uint32_t)point_voxel[first] : kNoSlot;  // the first point's id (always < n)
  }
  if (id >= n) {  // cannot happen once every claimed slot is committed
    point_voxel[p] = -1;
    return;
  }
  point_voxel[p] = (int32_t)id;
  atomic_add_u32(reinterpret_cast<uint32_t*>(counts) + id, 1u);
}

// ---------------------------------------------------------------------------
// Batched maps in one persistent cooperative launch.  Phases, separated by
// grid barriers: claims of every item -> (per-map new-key sums, only when a
// capacity check is needed) -> commits (each map's last tile finalizes the
// map) -> finds.  Each phase walks a flat list of tiles handed out in
// increasing order to the resident blocks (for_each_tile); all blocks are
// co-resident, so the per-map look-back of the commit phase (which only
// waits on lower tiles of the same map) always completes.  Each item keeps
// its own probe shape.
// The item that holds tile t of a phase: the last item whose first tile is
// <= t.  A block visits its tiles in increasing order, so it moves its
// current item forward instead of searching (usually one check per tile).
template <uint32_t BatchItem::*kFirst>
__device__ __forceinline__ int advance_item(const BatchItem* __restrict__ items, int n_items, int cur, uint32_t t) {
  while (cur + 1 < n_items && items[cur + 1].*kFirst <= t) ++cur;
  return cur;
}

// kNarrow: a build for launches whose items all probe one lane per key with
// W <= 4 (what the batched tuner picks); leaving the wider windows out of
// the kernel lowers its register count, so more blocks stay resident.
template <int KD, bool kNarrow>
__device__ __forceinline__ void batched_claim(const BatchItem& it, uint32_t tile, TileLds& lds) {
  const BatchKeys<KD> src{it.ikeys};
  if constexpr (kNarrow) {
    if (it.w == 2) claim_tile<KD, 1, 2, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<1>(), it.slot_of, it.lost, it.partial, it.meta, lds);
    else claim_tile<KD, 1, 4, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<1>(), it.slot_of, it.lost, it.partial, it.meta, lds);
    return;
  }
  switch (it.g == 1 ? it.w : 100 + it.g) {
    case 2: claim_tile<KD, 1, 2, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<1>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 4: claim_tile<KD, 1, 4, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<1>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 8: claim_tile<KD, 1, 8, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<1>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 104: claim_tile<KD, 4, 1, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<4>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 108: claim_tile<KD, 8, 1, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<8>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 116: claim_tile<KD, 16, 1, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<16>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 132: claim_tile<KD, 32, 1, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<32>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    case 164: claim_tile<KD, 64, 1, BatchKeys<KD>, false>(it.tb, src, it.n_insert, tile, rounds_for_dev<64>(), it.slot_of, it.lost, it.partial, it.meta, lds); break;
    default: break;
  }
}

template <int KD, bool kNarrow>
__device__ __forceinline__ void batched_find(const BatchItem& it, uint32_t tile, TileLds& lds) {
  if constexpr (kNarrow) {
    if (it.w == 2) find_tile<KD, 1, 2>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<1>(), DirectOut{it.fidx, it.fmask}, it.vout, lds);
    else find_tile<KD, 1, 4>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<1>(), DirectOut{it.fidx, it.fmask}, it.vout, lds);
    return;
  }
  switch (it.g == 1 ? it.w : 100 + it.g) {
    case 2: find_tile<KD, 1, 2>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<1>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 4: find_tile<KD, 1, 4>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<1>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 8: find_tile<KD, 1, 8>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<1>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 104: find_tile<KD, 4, 1>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<4>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 108: find_tile<KD, 8, 1>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<8>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 116: find_tile<KD, 16, 1>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<16>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 132: find_tile<KD, 32, 1>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<32>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    case 164: find_tile<KD, 64, 1>(it.tb, BatchKeys<KD>{it.fkeys}, it.n_find, tile, rounds_for_dev<64>(), DirectOut{it.fidx, it.fmask}, it.vout, lds); break;
    default: break;
  }
}

// Grid barriers of the persistent launch: an arrival check, then the phase
// barriers (grid_barrier).
//
// The arrival check comes before any table is touched, and it either lets
// every block through or none.  Each block counts itself in on gs->count;
// the block whose arrival brings the count to gridDim.x writes every block's
// release flag, and a block passes when it sees its flag.  A block that has
// waited arrival_spins polls gives up by setting kArrivalFailed with a
// compare-and-swap that only succeeds while some block has not arrived.  So
// once the count is complete no give-up can succeed, and once a give-up has
// succeeded the count never reads gridDim.x, no flag is written and no block
// passes (blocks that start later see kArrivalFailed in the value their
// arrival returns; waiting blocks reread the count).  If the blocks cannot
// all be resident at once, the resident ones give up and leave, the rest
// then start, see the flag and leave, and the launch ends with no map
// changed.  With force_fail (a test of that path) no block counts itself in,
// so the first block to give up always succeeds.
//
// Later barriers wait on blocks that are all resident (each passed the
// arrival check and stays until it exits), so they only end early after a
// broken invariant: the bound then sets gs->late and marks every map.
// The XCC (accelerator complex die, with its own L2) the calling wave runs on.
__device__ __forceinline__ uint32_t xcc_id() {
  return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kMaxXcc - 1u);  // XCC_ID[3:0]
}

// Barrier state of a block of the persistent launch (thread 0's copy is the
// one used).
struct BarrierState {
  uint32_t passed = 0;      // phase barriers passed
  uint32_t xcc = 0;         // this block's XCC
  uint32_t xcc_blocks = 0;  // blocks of the launch on that XCC
  uint32_t n_xcc = 0;       // XCCs the launch runs on
};

__device__ __forceinline__ uint32_t* release_flag(GridSync* gs, uint32_t b) {
  return reinterpret_cast<uint32_t*>(gs + 1) + (size_t)b * kFlagWords;
}

__device__ __forceinline__ bool arrival_check(GridSync* gs, uint32_t arrival_spins, uint32_t force_fail,
                                              BarrierState& bs, uint32_t* s_sh) {
  __syncthreads();
  uint32_t c = 0;
  if (threadIdx.x == 0) {
    // Relaxed atomics: no block has written anything yet, and what the
    // blocks read next was written before the launch (a release per block
    // would write back its XCC's L2 once per block).  A block first counts
    // itself on its XCC (and the XCC, when it is the first there), waits for
    // those atomics to be done, and only then counts itself in, so a block
    // that sees every arrival also sees every XCC count.
    bs.xcc = xcc_id();
    if (!force_fail) {
      if (__hip_atomic_fetch_add(&gs->xcc_blocks[bs.xcc][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
        __hip_atomic_fetch_add(&gs->n_xcc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
    }
    c = force_fail ? __hip_atomic_load(&gs->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    s_sh[1] = (!force_fail && c == gridDim.x) ? 1u : 0u;  // this arrival completed the count
  }
  __syncthreads();
  if (s_sh[1] != 0u)  // every block has arrived: let them all through (flag value 1)
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += kBlock)
      __hip_atomic_store(release_flag(gs, b), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) {
    if (force_fail) arrival_spins = 0;
    const uint32_t* flag = release_flag(gs, blockIdx.x);
    bool ok = false;
    uint32_t spins = 0;
    while (true) {
      if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = true;
        break;
      }
      if ((c & kArrivalFailed) != 0u || spins == kArrivalWaitLimit) break;  // (the limit: a broken invariant)
      if (c < gridDim.x && spins >= arrival_spins) {
        uint32_t expected = c;  // give up only while some block has not arrived
        if (__hip_atomic_compare_exchange_strong(&gs->count, &expected, c | kArrivalFailed, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          break;
        c = expected;  // the count moved: look again
        continue;
      }
      ++spins;
      __builtin_amdgcn_s_sleep(2);
      if ((spins & 7u) == 0u) c = __hip_atomic_load(&gs->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (ok) {
      bs.xcc_blocks = __hip_atomic_load(&gs->xcc_blocks[bs.xcc][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bs.n_xcc = __hip_atomic_load(&gs->n_xcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_sh[0] = ok ? 1u : 0u;
  }
  __syncthreads();
  return s_sh[0] != 0u;
}

// A phase barrier, in two levels.  Every wave first waits until its stores
// of the phase are in its XCC's L2; each block then counts itself on its XCC
// (a relaxed atomic).  The block that completes its XCC's count writes that
// L2 back once (a release fence at agent scope), for every block of the XCC,
// and counts the XCC done; the block that completes the count of XCCs
// acquires and writes the barrier's number into every block's release flag.
// Each block waits on its own flag, then acquires.  So a barrier costs one
// L2 write-back per XCC instead of one per block (each write-back stalls the
// XCC's L2 under the blocks still at work), and the polls are spread over
// one line per block instead of queueing on one word at the memory side.
__device__ __forceinline__ bool grid_barrier(GridSync* gs, BarrierState& bs, const BatchItem* __restrict__ items,
                                             int32_t n_items, uint32_t* s_sh) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the L2
  __syncthreads();
  const uint32_t gen = ++bs.passed;
  if (threadIdx.x == 0) {
    const bool ok = __hip_atomic_load(&gs->late, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    uint32_t last = 0;
    if (ok) {
      const uint32_t c = __hip_atomic_fetch_add(&gs->xcc_count[bs.xcc][0], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) + 1u;
      if (c == gen * bs.xcc_blocks) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the whole XCC's writes of the phase
        const uint32_t d = __hip_atomic_fetch_add(&gs->xcc_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (d == gen * bs.n_xcc) {
          last = 1u;
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
    }
    s_sh[0] = ok ? 1u : 0u;
    s_sh[1] = last;
  }
  __syncthreads();
  if (s_sh[1] != 0u) {  // every block has arrived: release them all
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += kBlock)
      __hip_atomic_store(release_flag(gs, b), gen + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) {
    bool ok = s_sh[0] != 0u;
    if (ok) {
      const uint32_t* flag = release_flag(gs, blockIdx.x);
      uint32_t spins = 0;
      while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen + 1u) {
        ++spins;
        if (spins == kPhaseSpinLimit ||
            ((spins & 63u) == 0u && __hip_atomic_load(&gs->late, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(32);  // about 1 us
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (!ok && __hip_atomic_exchange(&gs->late, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      for (int32_t m = 0; m < n_items; ++m)  // the first block to give up marks every map
        __hip_atomic_fetch_or(&items[m].meta->status, kStatusGridStall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_sh[0] = ok ? 1u : 0u;
  }
  __syncthreads();
  return s_sh[0] != 0u;
}

// Tiles of one phase, handed out at run time.  The tiles are dealt over K =
// min(kTileQueues, gridDim.x) queues (tile t is in queue t mod K), and
// block b serves queue b mod K: its first tile is b itself, and each later
// one comes from the queue's counter, fetched while the block works on its
// current tile.  Blocks that run faster take more tiles (on a CU the older
// waves win issue priority, so a static share leaves the later-placed
// blocks last), and a phase ends with its work instead of with the slowest
// block's share.  A single counter for all tiles would take one atomic per
// tile on one address, which serializes at the memory side; K counters on
// lines of their own split that.  Within a queue tiles go out in increasing
// order, so the commit's look-back (which waits only on lower tiles of its
// map) still always completes: take the lowest tile that has been handed out
// and is unfinished; its block works on it (a block's fetched next tile is
// above its current one), and a lower tile not yet handed out would sit in a
// queue whose blocks all work on still lower tiles, so every lower tile is
// done.
template <typename F>
__device__ __forceinline__ void for_each_tile(uint32_t (*next)[32], uint32_t n_tiles, uint32_t* s_next, F&& body) {
  const uint32_t K = gridDim.x < kTileQueues ? gridDim.x : kTileQueues;
  const uint32_t q = blockIdx.x % K;
  const uint32_t first = (gridDim.x - q + K - 1) / K;  // blocks of queue q, which take its first tiles
  uint32_t* ctr = &next[q][0];
  uint32_t t = blockIdx.x;
  while (t < n_tiles) {
    uint32_t nxt = 0;
    if (threadIdx.x == 0) nxt = q + K * (first + atomic_add_u32(ctr, 1u));
    body(t);
    __syncthreads();  // every thread has read *s_next for this tile
    if (threadIdx.x == 0) *s_next = nxt;
    __syncthreads();
    t = *s_next;
  }
}

template <int KD, bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_batched(const BatchItem* __restrict__ items, int32_t n_items,
                                                    uint32_t claim_tiles, uint32_t commit_tiles, uint32_t find_tiles,
                                                    int32_t any_check, GridSync* gs, uint32_t arrival_spins,
                                                    uint32_t force_fail) {
  __shared__ TileLds lds;
  __shared__ uint32_t s_next, s_sh[2];
  BarrierState bs;
  if (!arrival_check(gs, arrival_spins, force_fail, bs, s_sh)) return;  // all blocks resident, or none works
  int cur = 0;
  for_each_tile(gs->next[0], claim_tiles, &s_next, [&](uint32_t t) {
    cur = advance_item<&BatchItem::claim0>(items, n_items, cur, t);
    const BatchItem& it = items[cur];
    batched_claim<KD, kNarrow>(it, t - it.claim0, lds);
  });
  if (!grid_barrier(gs, bs, items, n_items, s_sh)) return;
  if (any_check) {
    for (int m = blockIdx.x; m < n_items; m += gridDim.x) {
      const BatchItem& it = items[m];
      if (it.check && it.n_insert) sum_partials_block<kBlock>(it.partial, (it.n_insert + 255u) / 256u, it.meta, lds);
    }
    if (!grid_barrier(gs, bs, items, n_items, s_sh)) return;
  }
  cur = 0;
  for_each_tile(gs->next[1], commit_tiles, &s_next, [&](uint32_t t) {
    cur = advance_item<&BatchItem::commit0>(items, n_items, cur, t);
    const BatchItem& it = items[cur];
    // each map's last commit tile finalizes that map (as in k_commit)
    commit_tile<KD, true>(it.tb, it.ikeys, it.n_insert, t - it.commit0, it.slot_of, it.lost, it.kB, it.heap, it.cap,
                          it.vin, it.iidx, it.imask, it.meta, it.status, it.check, nullptr, 0, lds);
  });
  if (!grid_barrier(gs, bs, items, n_items, s_sh)) return;
  cur = 0;
  for_each_tile(gs->next[2], find_tiles, &s_next, [&](uint32_t t) {
    cur = advance_item<&BatchItem::find0>(items, n_items, cur, t);
    const BatchItem& it = items[cur];
    batched_find<KD, kNarrow>(it, t - it.find0, lds);
  });
}

// ---------------------------------------------------------------------------
// Synthetic workload of the autotuner: key words uniform in [0, side) from a
// counter-based hash of (seed, word index); find keys alternate between a
// key of the insert batch (recomputed, not read back) and a key from
// [side, 2 side), which is never inserted.
__device__ __forceinline__ int32_t synth_word(uint64_t seed, uint64_t i, uint32_t side) {
  return (int32_t)(((mix64(seed ^ (i * 0x9e3779b97f4a7c15ull)) >> 32) * (uint64_t)side) >> 32);
}

__global__ __launch_bounds__(kBlock) void k_synth_keys(int32_t* __restrict__ keys, uint32_t n, int kd,
                                                       uint32_t side, uint64_t seed, int32_t* __restrict__ fkeys,
                                                       uint32_t nf) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    for (int d = 0; d < kd; ++d) keys[(size_t)p * kd + d] = synth_word(seed, (uint64_t)p * kd + d, side);
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nf; q += stride) {
    if (q & 1u) {
      for (int d = 0; d < kd; ++d)
        fkeys[(size_t)q * kd + d] = (int32_t)side + synth_word(seed + 1, (uint64_t)q * kd + d, side);
    } else {
      const uint32_t src = (uint32_t)(((mix64(seed + 2 + q) >> 32) * (uint64_t)n) >> 32);
      for (int d = 0; d < kd; ++d) fkeys[(size_t)q * kd + d] = synth_word(seed, (uint64_t)src * kd + d, side);
    }
  }
}

hipError_t launch_synth_keys(int32_t* keys, uint32_t n, int kd, uint32_t side, uint64_t seed, int32_t* fkeys,
                             uint32_t nf, hipStream_t st) {
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((std::max(n, nf) + kBlock - 1) / kBlock, 8192));
  hipLaunchKernelGGL(k_synth_keys, dim3(grid), dim3(kBlock), 0, st, keys, n, kd, side, seed, fkeys, nf);
  return hipGetLastError();
}

// Copies the rows whose mask byte is 1 (a served find's hits from the fused
// batch back to the request's own buffer; rows of misses stay untouched).
template <typename U>
__global__ __launch_bounds__(kBlock) void k_copy_masked_rows(const uint8_t* __restrict__ mask,
                                                             const U* __restrict__ src, U* __restrict__ dst,
                                                             uint64_t rows, uint32_t units) {
  const uint64_t total = rows * units;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (uint64_t)gridDim.x * kBlock) {
    const uint64_t r = e / units;
    if (mask[r]) dst[e] = src[e];
  }
}

hipError_t launch_copy_masked_rows(const uint8_t* mask, const void* src, void* dst, uint64_t rows,
                                   uint32_t row_bytes, uint32_t vec, hipStream_t st) {
  if (rows == 0 || row_bytes == 0) return hipSuccess;
  const uint32_t units = row_bytes / vec;
  const uint32_t grid = std::max<uint32_t>(1, (uint32_t)std::min<uint64_t>((rows * units + kBlock - 1) / kBlock, 8192));
  switch (vec) {
    case 16:
      hipLaunchKernelGGL(k_copy_masked_rows<uint4>, dim3(grid), dim3(kBlock), 0, st, mask, (const uint4*)src,
                         (uint4*)dst, rows, units);
      break;
    case 8:
      hipLaunchKernelGGL(k_copy_masked_rows<uint2>, dim3(grid), dim3(kBlock), 0, st, mask, (const uint2*)src,
                         (uint2*)dst, rows, units);
      break;
    case 4:
      hipLaunchKernelGGL(k_copy_masked_rows<uint32_t>, dim3(grid), dim3(kBlock), 0, st, mask, (const uint32_t*)src,
                         (uint32_t*)dst, rows, units);
      break;
    case 2:
      hipLaunchKernelGGL(k_copy_masked_rows<uint16_t>, dim3(grid), dim3(kBlock), 0, st, mask, (const uint16_t*)src,
                         (uint16_t*)dst, rows, units);
      break;
    default:
      hipLaunchKernelGGL(k_copy_masked_rows<uint8_t>, dim3(grid), dim3(kBlock), 0, st, mask, (const uint8_t*)src,
                         (uint8_t*)dst, rows, row_bytes);
      break;
  }
  return hipGetLastError();
}

// Fused served batches (gather and scatter for inserts and erases; fused
// finds read and write the requests' buffers directly, see k_find_requests).
// Rows move in 4-byte words when the row size allows, else byte by byte.
__device__ __forceinline__ void copy_row(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, uint32_t bytes) {
  if ((bytes & 3u) == 0 && (((uintptr_t)src | (uintptr_t)dst) & 3u) == 0) {
    for (uint32_t w = 0; w < bytes / 4; ++w)
      reinterpret_cast<uint32_t*>(dst)[w] = reinterpret_cast<const uint32_t*>(src)[w];
  } else {
    for (uint32_t b = 0; b < bytes; ++b) dst[b] = src[b];
  }
}

// Concatenates the requests' keys (and insert values) into the batch buffers.
__global__ __launch_bounds__(kBlock) void k_gather_requests(const ReqDesc* __restrict__ d, int nreq, int64_t total,
                                                            int kd, RowSet rows, int32_t* __restrict__ keys,
                                                            uint8_t* const* __restrict__ vals) {
  __shared__ int64_t s_off[kMaxFusedRequests];
  for (int r = threadIdx.x; r < nreq; r += kBlock) s_off[r] = d[r].off;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int r = request_of(s_off, nreq, e);
    const int64_t q = e - s_off[r];
    const int32_t* src = d[r].keys + q * kd;
    for (int w = 0; w < kd; ++w) keys[e * kd + w] = src[w];
    for (int j = 0; j < rows.n; ++j)
      if (vals && d[r].vals[j]) copy_row(d[r].vals[j] + q * rows.bytes[j], vals[j] + e * rows.bytes[j], rows.bytes[j]);
  }
}

// Hands each request of a fused insert or erase its part of the batch
// results: indices and masks.
__global__ __launch_bounds__(kBlock) void k_scatter_requests(const ReqDesc* __restrict__ d, int nreq, int64_t total,
                                                             const int32_t* __restrict__ idx,
                                                             const uint8_t* __restrict__ mask) {
  __shared__ int64_t s_off[kMaxFusedRequests];
  for (int r = threadIdx.x; r < nreq; r += kBlock) s_off[r] = d[r].off;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int r = request_of(s_off, nreq, e);
    const int64_t q = e - s_off[r];
    if (idx && d[r].out_idx) d[r].out_idx[q] = idx[e];
    if (d[r].out_mask) d[r].out_mask[q] = mask[e];
  }
}

hipError_t launch_gather_requests(const ReqDesc* d, int nreq, int64_t total, int kd, const RowSet& rows,
                                  int32_t* keys, uint8_t* const* vals, hipStream_t st) {
  if (nreq < 1 || nreq > kMaxFusedRequests) return hipErrorInvalidValue;
  if (total == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<int64_t>((total + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_gather_requests, dim3(grid), dim3(kBlock), 0, st, d, nreq, total, kd, rows, keys, vals);
  return hipGetLastError();
}

hipError_t launch_scatter_requests(const ReqDesc* d, int nreq, int64_t total, const int32_t* idx, const uint8_t* mask,
                                   hipStream_t st) {
  if (nreq < 1 || nreq > kMaxFusedRequests) return hipErrorInvalidValue;
  if (total == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<int64_t>((total + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_scatter_requests, dim3(grid), dim3(kBlock), 0, st, d, nreq, total, idx, mask);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint32_t grid = (uint32_t)std::min<size_t>((n / 4 + kBlock - 1) / kBlock + 1, 65536);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kBlock), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* h, uint32_t from, uint32_t to, hipStream_t st) {
  if (to <= from) return hipSuccess;
  uint32_t grid = std::min<uint32_t>(cdiv(to - from, kBlock), 65536);
  hipLaunchKernelGGL(k_iota, dim3(grid), dim3(kBlock), 0, st, h, from, to);
  return hipGetLastError();
}

hipError_t launch_voxel_init(uint32_t* table, size_t n_table, uint32_t* zero, size_t n_zero, Meta* meta,
                             hipStream_t st) {
  if (n_table % 4 != 0) return hipErrorInvalidValue;
  const size_t work = std::max<size_t>(n_table / 4, n_zero);
  const uint32_t grid = (uint32_t)std::max<size_t>(1, std::min<size_t>((work + kBlock - 1) / kBlock, 65536));
  hipLaunchKernelGGL(k_voxel_init, dim3(grid), dim3(kBlock), 0, st, table, n_table, zero, n_zero, meta);
  return hipGetLastError();
}

hipError_t launch_clear_map(uint32_t* table, size_t n_words, int32_t* heap, uint32_t c, Meta* meta, hipStream_t st) {
  if (n_words % 4 != 0) return hipErrorInvalidValue;
  const size_t work = std::max<size_t>(n_words / 4, c);
  const uint32_t grid = (uint32_t)std::max<size_t>(1, std::min<size_t>((work + kBlock - 1) / kBlock, 65536));
  hipLaunchKernelGGL(k_clear_map, dim3(grid), dim3(kBlock), 0, st, table, n_words, heap, c, meta);
  return hipGetLastError();
}

hipError_t launch_finalize(Meta* m, uint32_t cap, int mode, int silent, int check, const uint64_t* status,
                           uint32_t last_tile, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1), 0, st, m, cap, mode, silent, check, status, last_tile);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const uint32_t* partial, uint32_t count, Meta* meta, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, partial, count, meta);
  return hipGetLastError();
}

// Positions per block of the probing kernels: 256 (G lanes per position, so
// a group takes G positions in turn).
template <int G>
static inline uint32_t rounds_for() { return 256u / (kBlock / G); }

uint32_t claim_blocks(int g, uint32_t n) { return cdiv(n, 256u); }

template <int KD, int G, int WL>
struct ClaimK {
  static hipError_t run(const TableRef& tb, const int32_t* keys, uint32_t n, uint32_t* slot_of, uint8_t* lost,
                        uint32_t* partial, Meta* meta, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    const dim3 grid(cdiv(n, (kBlock / G) * rounds));
    // tombstones are reused only where an erase may have left some
    if (tb.reuse)
      hipLaunchKernelGGL((k_claim<KD, G, WL, BatchKeys<KD>, false, true, false>), grid, dim3(kBlock), 0, st, tb,
                         BatchKeys<KD>{keys}, n, rounds, slot_of, lost, partial, meta);
    else if (tb.keyed)
      hipLaunchKernelGGL((k_claim<KD, G, WL, BatchKeys<KD>, false, false, true>), grid, dim3(kBlock), 0, st, tb,
                         BatchKeys<KD>{keys}, n, rounds, slot_of, lost, partial, meta);
    else
      hipLaunchKernelGGL((k_claim<KD, G, WL, BatchKeys<KD>, false, false, false>), grid, dim3(kBlock), 0, st, tb,
                         BatchKeys<KD>{keys}, n, rounds, slot_of, lost, partial, meta);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct ClaimRequestsK {
  static hipError_t run(const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq, uint32_t n,
                        uint32_t* slot_of, uint8_t* lost, uint32_t* partial, Meta* meta, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    const dim3 grid(cdiv(n, (kBlock / G) * rounds));
    if (tb.reuse)
      hipLaunchKernelGGL((k_claim_requests<KD, G, WL, true, false>), grid, dim3(kBlock), 0, st, tb, args, d, nreq, n,
                         rounds, slot_of, lost, partial, meta);
    else if (tb.keyed)
      hipLaunchKernelGGL((k_claim_requests<KD, G, WL, false, true>), grid, dim3(kBlock), 0, st, tb, args, d, nreq, n,
                         rounds, slot_of, lost, partial, meta);
    else
      hipLaunchKernelGGL((k_claim_requests<KD, G, WL, false, false>), grid, dim3(kBlock), 0, st, tb, args, d, nreq, n,
                         rounds, slot_of, lost, partial, meta);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct EraseMarkRequestsK {
  static hipError_t run(const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq, uint32_t n,
                        uint32_t epoch, uint32_t* slot_of, int32_t* found, uint64_t* owner, uint8_t* lost,
                        hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_erase_mark_requests<KD, G, WL>), dim3(cdiv(n, (kBlock / G) * rounds)), dim3(kBlock), 0, st,
                       tb, args, d, nreq, n, rounds, epoch, slot_of, found, owner, lost);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct FindK {
  static hipError_t run(const TableRef& tb, const int32_t* keys, uint32_t n, int32_t* out_idx, uint8_t* out_mask,
                        const ValueSet& vs, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_find<KD, G, WL>), dim3(cdiv(n, (kBlock / G) * rounds)), dim3(kBlock), 0, st, tb, keys, n,
                       rounds, out_idx, out_mask, vs);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct FindRequestsK {
  static hipError_t run(const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq, uint32_t n,
                        const ValueSet& vs, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_find_requests<KD, G, WL>), dim3(cdiv(n, (kBlock / G) * rounds)), dim3(kBlock), 0, st, tb,
                       args, d, nreq, n, rounds, vs);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct FindOffsetsK {
  static hipError_t run(const TableRef& tb, const int32_t* keys, const int32_t* offsets, uint32_t k, uint32_t n,
                        int32_t* out_idx, uint8_t* out_mask, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_find_offsets<KD, G, WL>), dim3(cdiv(n, (kBlock / G) * rounds)), dim3(kBlock), 0, st, tb,
                       OffsetKeys<KD>{keys, offsets, k}, n, rounds, out_idx, out_mask);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct EraseMarkK {
  static hipError_t run(const TableRef& tb, const int32_t* keys, uint32_t n, uint32_t epoch, uint32_t* slot_of,
                        int32_t* found, uint64_t* owner, uint8_t* lost, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_erase_mark<KD, G, WL>), dim3(cdiv(n, (kBlock / G) * rounds)), dim3(kBlock), 0, st, tb,
                       keys, n, rounds, epoch, slot_of, found, owner, lost);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct RebuildK {
  static hipError_t run(const TableRef& tb, const uint32_t* old_words, uint32_t old_slots, Meta* meta,
                        hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_rebuild<KD, G, WL>), dim3(cdiv(old_slots, (kBlock / G) * rounds)), dim3(kBlock), 0, st,
                       tb, old_words, old_slots, rounds, meta);
    return hipGetLastError();
  }
};

template <int KD, int G, int WL>
struct VoxelClaimK {
  static hipError_t run(const TableRef& tb, const float* pts, float voxel, uint32_t n, uint32_t* slot_of,
                        uint8_t* lost, uint32_t* partial, Meta* meta, hipStream_t st) {
    const uint32_t rounds = rounds_for<G>();
    hipLaunchKernelGGL((k_claim<3, G, WL, VoxelKeys, true, false, true>), dim3(cdiv(n, (kBlock / G) * rounds)), dim3(kBlock), 0,
                       st, tb, VoxelKeys{pts, voxel}, n, rounds, slot_of, lost, partial, meta);
    return hipGetLastError();
  }
};

// Dispatch on the probe shape: G lanes per key (WL = 1), or one lane per key
// reading a bucket of WL slots (G = 1).
template <int KD, template <int, int, int> class F, typename... A>
static hipError_t with_probe(int g, int w, A&&... a) {
  if (g == 1) {
    switch (w) {
      case 2: return F<KD, 1, 2>::run(a...);
      case 4: return F<KD, 1, 4>::run(a...);
      case 8: return F<KD, 1, 8>::run(a...);
      default: return hipErrorInvalidValue;
    }
  }
  switch (g) {
    case 4: return F<KD, 4, 1>::run(a...);
    case 8: return F<KD, 8, 1>::run(a...);
    case 16: return F<KD, 16, 1>::run(a...);
    case 32: return F<KD, 32, 1>::run(a...);
    case 64: return F<KD, 64, 1>::run(a...);
    default: return hipErrorInvalidValue;
  }
}

template <template <int, int, int> class F, typename... A>
static hipError_t with_kd_probe(int kd, int g, int w, A&&... a) {
  switch (kd) {
    case 1: return with_probe<1, F>(g, w, a...);
    case 2: return with_probe<2, F>(g, w, a...);
    case 3: return with_probe<3, F>(g, w, a...);
    case 4: return with_probe<4, F>(g, w, a...);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_claim(int kd, int g, int w, const TableRef& tb, const int32_t* keys, uint32_t n, uint32_t* slot_of,
                        uint8_t* lost, uint32_t* partial, Meta* meta, hipStream_t st) {
  return with_kd_probe<ClaimK>(kd, g, w, tb, keys, n, slot_of, lost, partial, meta, st);
}

template <int KD>
static hipError_t commit_k(const TableRef& tb, const int32_t* keys, uint32_t n, const uint32_t* slot_of,
                           uint8_t* lost, int32_t* kB, const int32_t* heap, uint32_t cap, const ValueSet& vs,
                           int32_t* out_idx, uint8_t* out_mask, Meta* meta, uint64_t* status, int check,
                           uint32_t* wlist, int silent, hipStream_t st) {
  if (wlist)
    hipLaunchKernelGGL((k_commit<KD, false>), dim3(cdiv(n, kScanTile)), dim3(kBlock), 0, st, tb, keys, n, slot_of,
                       lost, kB, heap, cap, vs, out_idx, out_mask, meta, status, check, wlist, silent);
  else
    hipLaunchKernelGGL((k_commit<KD, true>), dim3(cdiv(n, kScanTile)), dim3(kBlock), 0, st, tb, keys, n, slot_of,
                       lost, kB, heap, cap, vs, out_idx, out_mask, meta, status, check, wlist, silent);
  return hipGetLastError();
}

template <typename V, int U>
static void scatter_values_k(const ValueSet& vs, int j, const uint32_t* wlist, const int32_t* heap, const Meta* meta,
                             uint32_t n, uint32_t cap, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL((k_scatter_values<V, U>), dim3(grid), dim3(kBlock), 0, st, wlist, heap, meta, vs.src[j],
                     vs.dst[j], vs.row_bytes[j], vs.units_log2[j], n, cap);
}

template <typename V>
static void scatter_values_v(const ValueSet& vs, int j, const uint32_t* wlist, const int32_t* heap, const Meta* meta,
                             uint32_t n, uint32_t cap, uint32_t grid, hipStream_t st) {
  if (vs.row_bytes[j] >= kUnrollRowBytes)
    scatter_values_k<V, 4>(vs, j, wlist, heap, meta, n, cap, grid, st);
  else
    scatter_values_k<V, 1>(vs, j, wlist, heap, meta, n, cap, grid, st);
}

hipError_t launch_scatter_values(const ValueSet& vs, const uint32_t* wlist, const int32_t* heap, const Meta* meta,
                                 uint32_t n, uint32_t cap, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int j = 0; j < vs.n && e == hipSuccess; ++j) {
    const uint64_t units = vs.row_bytes[j] / vs.vec[j];
    // sized for every position winning; the kernel reads the actual count
    const uint32_t grid =
        (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(((uint64_t)n * units + kBlock - 1) / kBlock, 16384));
    switch (vs.vec[j]) {
      case 16: scatter_values_v<uint4>(vs, j, wlist, heap, meta, n, cap, grid, st); break;
      case 8: scatter_values_v<uint2>(vs, j, wlist, heap, meta, n, cap, grid, st); break;
      case 4: scatter_values_v<uint32_t>(vs, j, wlist, heap, meta, n, cap, grid, st); break;
      case 2: scatter_values_v<uint16_t>(vs, j, wlist, heap, meta, n, cap, grid, st); break;
      default: scatter_values_v<uint8_t>(vs, j, wlist, heap, meta, n, cap, grid, st); break;
    }
    e = hipGetLastError();
  }
  return e;
}

template <typename V>
static void gather_rows_v(const ValueSet& vs, int j, const int32_t* idx, uint32_t n, uint32_t cap, uint32_t grid,
                          hipStream_t st) {
  if (vs.row_bytes[j] >= kUnrollRowBytes)
    hipLaunchKernelGGL((k_gather_rows<V, 4>), dim3(grid), dim3(kBlock), 0, st, idx, vs.src[j], vs.dst[j],
                       vs.row_bytes[j], vs.units_log2[j], n, cap);
  else
    hipLaunchKernelGGL((k_gather_rows<V, 1>), dim3(grid), dim3(kBlock), 0, st, idx, vs.src[j], vs.dst[j],
                       vs.row_bytes[j], vs.units_log2[j], n, cap);
}

hipError_t launch_gather_rows(const ValueSet& vs, const int32_t* idx, uint32_t n, uint32_t cap, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int j = 0; j < vs.n && e == hipSuccess; ++j) {
    const uint64_t units = vs.row_bytes[j] / vs.vec[j];
    const uint32_t grid =
        (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(((uint64_t)n * units + kBlock - 1) / kBlock, 16384));
    switch (vs.vec[j]) {
      case 16: gather_rows_v<uint4>(vs, j, idx, n, cap, grid, st); break;
      case 8: gather_rows_v<uint2>(vs, j, idx, n, cap, grid, st); break;
      case 4: gather_rows_v<uint32_t>(vs, j, idx, n, cap, grid, st); break;
      case 2: gather_rows_v<uint16_t>(vs, j, idx, n, cap, grid, st); break;
      default: gather_rows_v<uint8_t>(vs, j, idx, n, cap, grid, st); break;
    }
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_commit(int kd, const TableRef& tb, const int32_t* keys, uint32_t n, const uint32_t* slot_of,
                         uint8_t* lost, int32_t* kB, const int32_t* heap, uint32_t cap, const ValueSet& vs,
                         int32_t* out_idx, uint8_t* out_mask, Meta* meta, uint64_t* status, int check,
                         uint32_t* wlist, int silent, hipStream_t st) {
  switch (kd) {
    case 1: return commit_k<1>(tb, keys, n, slot_of, lost, kB, heap, cap, vs, out_idx, out_mask, meta, status, check, wlist, silent, st);
    case 2: return commit_k<2>(tb, keys, n, slot_of, lost, kB, heap, cap, vs, out_idx, out_mask, meta, status, check, wlist, silent, st);
    case 3: return commit_k<3>(tb, keys, n, slot_of, lost, kB, heap, cap, vs, out_idx, out_mask, meta, status, check, wlist, silent, st);
    case 4: return commit_k<4>(tb, keys, n, slot_of, lost, kB, heap, cap, vs, out_idx, out_mask, meta, status, check, wlist, silent, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_find(int kd, int g, int w, const TableRef& tb, const int32_t* keys, uint32_t n, int32_t* out_idx,
                       uint8_t* out_mask, const ValueSet& vs, hipStream_t st) {
  return with_kd_probe<FindK>(kd, g, w, tb, keys, n, out_idx, out_mask, vs, st);
}

// The batch's descriptors: nreq of them, either all in the launch arguments
// or all in device memory.
static bool args_fit(const ReqArgs& args, int nreq) {
  return nreq >= 1 && nreq <= kMaxFusedRequests && args.nreq >= 0 && args.nreq <= kArgRequests &&
         (args.nreq == 0 || args.nreq == nreq);
}

hipError_t launch_find_requests(int kd, int g, int w, const TableRef& tb, const ReqArgs& args, const ReqDesc* d,
                                int nreq, uint32_t n, const ValueSet& vs, hipStream_t st) {
  if (!args_fit(args, nreq)) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  return with_kd_probe<FindRequestsK>(kd, g, w, tb, args, d, nreq, n, vs, st);
}

hipError_t launch_find_offsets(int kd, int g, int w, const TableRef& tb, const int32_t* keys, const int32_t* offsets,
                               uint32_t k, uint32_t n, int32_t* out_idx, uint8_t* out_mask, hipStream_t st) {
  return with_kd_probe<FindOffsetsK>(kd, g, w, tb, keys, offsets, k, n, out_idx, out_mask, st);
}

hipError_t launch_compact_rows(int kd, const uint8_t* mask, uint32_t n, const int32_t* keys, int32_t* out, Meta* meta,
                               uint64_t* status, hipStream_t st) {
  const dim3 grid(cdiv(n, kScanTile));
  switch (kd) {
    case 1: hipLaunchKernelGGL(k_compact_rows<1>, grid, dim3(kBlock), 0, st, mask, n, keys, out, meta, status); break;
    case 2: hipLaunchKernelGGL(k_compact_rows<2>, grid, dim3(kBlock), 0, st, mask, n, keys, out, meta, status); break;
    case 3: hipLaunchKernelGGL(k_compact_rows<3>, grid, dim3(kBlock), 0, st, mask, n, keys, out, meta, status); break;
    case 4: hipLaunchKernelGGL(k_compact_rows<4>, grid, dim3(kBlock), 0, st, mask, n, keys, out, meta, status); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_erase_mark(int kd, int g, int w, const TableRef& tb, const int32_t* keys, uint32_t n,
                             uint32_t epoch, uint32_t* slot_of, int32_t* found, uint64_t* owner, uint8_t* lost,
                             hipStream_t st) {
  return with_kd_probe<EraseMarkK>(kd, g, w, tb, keys, n, epoch, slot_of, found, owner, lost, st);
}

template <int KD>
static hipError_t erase_commit_k(const TableRef& tb, uint32_t n, const uint32_t* slot_of, const int32_t* found,
                                 uint8_t* lost, int32_t* heap, uint8_t* out_mask, Meta* meta, uint64_t* status,
                                 hipStream_t st) {
  hipLaunchKernelGGL((k_erase_commit<KD>), dim3(cdiv(n, kScanTile)), dim3(kBlock), 0, st, tb, n, slot_of, found,
                     lost, heap, out_mask, meta, status);
  return hipGetLastError();
}

hipError_t launch_erase_commit(int kd, const TableRef& tb, uint32_t n, const uint32_t* slot_of, const int32_t* found,
                               uint8_t* lost, int32_t* heap, uint8_t* out_mask, Meta* meta, uint64_t* status,
                               hipStream_t st) {
  switch (kd) {
    case 1: return erase_commit_k<1>(tb, n, slot_of, found, lost, heap, out_mask, meta, status, st);
    case 2: return erase_commit_k<2>(tb, n, slot_of, found, lost, heap, out_mask, meta, status, st);
    case 3: return erase_commit_k<3>(tb, n, slot_of, found, lost, heap, out_mask, meta, status, st);
    case 4: return erase_commit_k<4>(tb, n, slot_of, found, lost, heap, out_mask, meta, status, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_claim_requests(int kd, int g, int w, const TableRef& tb, const ReqArgs& args, const ReqDesc* d,
                                 int nreq, uint32_t n, uint32_t* slot_of, uint8_t* lost, uint32_t* partial, Meta* meta,
                                 hipStream_t st) {
  if (!args_fit(args, nreq) || tb.dedup) return hipErrorInvalidValue;
  return with_kd_probe<ClaimRequestsK>(kd, g, w, tb, args, d, nreq, n, slot_of, lost, partial, meta, st);
}

template <int KD>
static hipError_t commit_requests_k(const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq, uint32_t n,
                                    const uint32_t* slot_of, uint8_t* lost, int32_t* kB, const int32_t* heap,
                                    uint32_t cap, const ValueSet& vs, Meta* meta, uint64_t* status, int check,
                                    int silent, hipStream_t st) {
  hipLaunchKernelGGL((k_commit_requests<KD>), dim3(cdiv(n, kScanTile)), dim3(kBlock), 0, st, tb, args, d, nreq, n,
                     slot_of, lost, kB, heap, cap, vs, meta, status, check, silent);
  return hipGetLastError();
}

hipError_t launch_commit_requests(int kd, const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq,
                                  uint32_t n, const uint32_t* slot_of, uint8_t* lost, int32_t* kB, const int32_t* heap,
                                  uint32_t cap, const ValueSet& vs, Meta* meta, uint64_t* status, int check,
                                  int silent, hipStream_t st) {
  if (!args_fit(args, nreq)) return hipErrorInvalidValue;
  switch (kd) {
    case 1: return commit_requests_k<1>(tb, args, d, nreq, n, slot_of, lost, kB, heap, cap, vs, meta, status, check, silent, st);
    case 2: return commit_requests_k<2>(tb, args, d, nreq, n, slot_of, lost, kB, heap, cap, vs, meta, status, check, silent, st);
    case 3: return commit_requests_k<3>(tb, args, d, nreq, n, slot_of, lost, kB, heap, cap, vs, meta, status, check, silent, st);
    case 4: return commit_requests_k<4>(tb, args, d, nreq, n, slot_of, lost, kB, heap, cap, vs, meta, status, check, silent, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_erase_mark_requests(int kd, int g, int w, const TableRef& tb, const ReqArgs& args, const ReqDesc* d,
                                      int nreq, uint32_t n, uint32_t epoch, uint32_t* slot_of, int32_t* found,
                                      uint64_t* owner, uint8_t* lost, hipStream_t st) {
  if (!args_fit(args, nreq)) return hipErrorInvalidValue;
  return with_kd_probe<EraseMarkRequestsK>(kd, g, w, tb, args, d, nreq, n, epoch, slot_of, found, owner, lost, st);
}

template <int KD>
static hipError_t erase_commit_requests_k(const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq,
                                          uint32_t n, const uint32_t* slot_of, const int32_t* found, uint8_t* lost,
                                          int32_t* heap, Meta* meta, uint64_t* status, hipStream_t st) {
  hipLaunchKernelGGL((k_erase_commit_requests<KD>), dim3(cdiv(n, kScanTile)), dim3(kBlock), 0, st, tb, args, d, nreq,
                     n, slot_of, found, lost, heap, meta, status);
  return hipGetLastError();
}

hipError_t launch_erase_commit_requests(int kd, const TableRef& tb, const ReqArgs& args, const ReqDesc* d, int nreq,
                                        uint32_t n, const uint32_t* slot_of, const int32_t* found, uint8_t* lost,
                                        int32_t* heap, Meta* meta, uint64_t* status, hipStream_t st) {
  if (!args_fit(args, nreq)) return hipErrorInvalidValue;
  switch (kd) {
    case 1: return erase_commit_requests_k<1>(tb, args, d, nreq, n, slot_of, found, lost, heap, meta, status, st);
    case 2: return erase_commit_requests_k<2>(tb, args, d, nreq, n, slot_of, found, lost, heap, meta, status, st);
    case 3: return erase_commit_requests_k<3>(tb, args, d, nreq, n, slot_of, found, lost, heap, meta, status, st);
    case 4: return erase_commit_requests_k<4>(tb, args, d, nreq, n, slot_of, found, lost, heap, meta, status, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_active_indices(int kd, const TableRef& tb, uint8_t* flags, uint32_t c, int32_t* out, Meta* meta,
                                 uint64_t* status, hipStream_t st) {
  const uint32_t grid = std::min<uint32_t>(cdiv(tb.nslots, kBlock), 8192);
  switch (kd) {
    case 1: hipLaunchKernelGGL(k_mark_live<2>, dim3(grid), dim3(kBlock), 0, st, tb, flags, c); break;
    case 2:
    case 3: hipLaunchKernelGGL(k_mark_live<4>, dim3(grid), dim3(kBlock), 0, st, tb, flags, c); break;
    case 4: hipLaunchKernelGGL(k_mark_live<8>, dim3(grid), dim3(kBlock), 0, st, tb, flags, c); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact_flags, dim3(cdiv(c, kScanTile)), dim3(kBlock), 0, st, flags, c, out, meta, status);
  return hipGetLastError();
}

hipError_t launch_rebuild(int kd, int g, int w, const TableRef& tb, const uint32_t* old_words, uint32_t old_slots,
                          Meta* meta, hipStream_t st) {
  return with_kd_probe<RebuildK>(kd, g, w, tb, old_words, old_slots, meta, st);
}

hipError_t launch_voxel_claim(int g, int w, const TableRef& tb, const float* pts, float voxel, uint32_t n,
                              uint32_t* slot_of, uint8_t* lost, uint32_t* partial, Meta* meta, hipStream_t st) {
  return with_probe<3, VoxelClaimK>(g, w, tb, pts, voxel, n, slot_of, lost, partial, meta, st);
}

hipError_t launch_voxel_commit(const TableRef& tb, const float* pts, float voxel, uint32_t n, uint32_t* slot_of,
                               uint8_t* lost, int32_t* voxel_keys, int32_t* counts, int32_t* point_voxel, Meta* meta,
                               uint64_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_voxel_commit, dim3(cdiv(n, kScanTile)), dim3(kBlock), 0, st, tb, VoxelKeys{pts, voxel}, n,
                     slot_of, lost, voxel_keys, counts, point_voxel, meta, status);
  return hipGetLastError();
}

hipError_t launch_block_coords(const float* pts, uint32_t n, float voxel, int32_t res, int32_t* block_keys,
                               int32_t* local, uint8_t* valid, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_coords, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, pts, n, voxel, res, block_keys,
                     local, valid);
  return hipGetLastError();
}

hipError_t launch_voxel_resolve(const TableRef& tb, uint32_t n, const uint32_t* slot_of, int32_t* point_voxel,
                                int32_t* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_voxel_resolve, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, tb, n, slot_of, point_voxel,
                     counts);
  return hipGetLastError();
}

template <int KD, bool kNarrow>
static hipError_t batched_k(const BatchItem* items, int32_t n_items, uint32_t claim_tiles, uint32_t commit_tiles,
                            uint32_t find_tiles, int32_t any_check, GridSync* gs, uint32_t resident,
                            uint32_t arrival_spins, uint32_t force_fail, hipStream_t st) {
  // n_items == 0 launches all `resident` blocks with no work: a residency probe
  const uint32_t work = std::max(std::max(claim_tiles, commit_tiles), std::max(find_tiles, (uint32_t)n_items));
  const uint32_t grid = n_items == 0 ? resident : std::max<uint32_t>(1, std::min<uint32_t>(resident, work));
  hipLaunchKernelGGL((k_batched<KD, kNarrow>), dim3(grid), dim3(kBlock), 0, st, items, n_items, claim_tiles,
                     commit_tiles, find_tiles, any_check, gs, arrival_spins, force_fail);
  return hipGetLastError();
}

template <bool kNarrow>
static hipError_t batched_occupancy_k(int kd, int* per_cu) {
  switch (kd) {
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batched<1, kNarrow>, kBlock, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batched<2, kNarrow>, kBlock, 0);
    case 3: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batched<3, kNarrow>, kBlock, 0);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batched<4, kNarrow>, kBlock, 0);
    default: return hipErrorInvalidValue;
  }
}

hipError_t batched_occupancy(int kd, bool narrow, int* per_cu) {
  return narrow ? batched_occupancy_k<true>(kd, per_cu) : batched_occupancy_k<false>(kd, per_cu);
}

template <bool kNarrow>
static hipError_t launch_batched_k(int kd, const BatchItem* items, int32_t n_items, uint32_t claim_tiles,
                                   uint32_t commit_tiles, uint32_t find_tiles, int32_t any_check, GridSync* gs,
                                   uint32_t resident, uint32_t arrival_spins, uint32_t force_fail, hipStream_t st) {
  switch (kd) {
    case 1: return batched_k<1, kNarrow>(items, n_items, claim_tiles, commit_tiles, find_tiles, any_check, gs,
                                         resident, arrival_spins, force_fail, st);
    case 2: return batched_k<2, kNarrow>(items, n_items, claim_tiles, commit_tiles, find_tiles, any_check, gs,
                                         resident, arrival_spins, force_fail, st);
    case 3: return batched_k<3, kNarrow>(items, n_items, claim_tiles, commit_tiles, find_tiles, any_check, gs,
                                         resident, arrival_spins, force_fail, st);
    case 4: return batched_k<4, kNarrow>(items, n_items, claim_tiles, commit_tiles, find_tiles, any_check, gs,
                                         resident, arrival_spins, force_fail, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batched(int kd, bool narrow, const BatchItem* items, int32_t n_items, uint32_t claim_tiles,
                          uint32_t commit_tiles, uint32_t find_tiles, int32_t any_check, GridSync* gs,
                          uint32_t resident, uint32_t arrival_spins, uint32_t force_fail, hipStream_t st) {
  return narrow ? launch_batched_k<true>(kd, items, n_items, claim_tiles, commit_tiles, find_tiles, any_check, gs,
                                         resident, arrival_spins, force_fail, st)
                : launch_batched_k<false>(kd, items, n_items, claim_tiles, commit_tiles, find_tiles, any_check, gs,
                                          resident, arrival_spins, force_fail, st);
}

}  // namespace ash
