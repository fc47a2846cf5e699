// ash_slab.hip -- the separate-chaining ("slab") backend of the backend
// ablation (Sec. 4.4 and Sec. 5.3 of ASH, arXiv 2110.00511); declared in
// include/ash_slab.h.  Benchmark and test subject only: no entry point of
// include/ash.h reaches these kernels.
//
// A bucket is a linked list of slabs.  A slab is one 128-byte line of 32
// words: words 0..30 hold buffer indices (or kSlabEmpty), word 31 the next
// slab of the list (kNoNext at the end).  32 lanes of a 64-wide wavefront
// read one slab together, so one probe step is one coalesced line; keys are
// not in the slab but in k^B, read once per occupied entry a probe meets
// (the index is the delegate key of the integer-only hash set, Sec. 4.4.1).
// Slab ids below nbuckets are the buckets' first slabs, the rest the
// overflow pool, taken with an atomic counter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "ash.h"
#include "ash_device.hpp"
#include "ash_internal.hpp"
#include "ash_launch.hpp"
#include "ash_slab.h"

namespace ash {
namespace {

constexpr uint32_t kSlabWords = 32;
constexpr uint32_t kSlabEntries = 31;
constexpr uint32_t kSlabEmpty = 0xFFFFFFFFu;
constexpr uint32_t kNoNext = 0xFFFFFFFFu;
constexpr int kSlabRounds = 4;  // positions per 32-lane group and block

struct SlabMeta {
  uint32_t t;         // heap top
  uint32_t pool_top;  // overflow slabs taken
  uint32_t fail;      // a list needed more slabs than the pool holds
  uint32_t result;    // keys the last insert added
  uint32_t status;    // look-back stall bits
  uint32_t pad[11];
};

struct SlabRef {
  uint32_t* slabs;
  uint32_t nbuckets;
  uint32_t pool;  // overflow slabs
  uint32_t max_steps;  // slabs a list can have: 1 + pool
};

template <int KD>
__device__ __forceinline__ uint32_t slab_bucket(const SlabRef& sr, const int32_t (&k)[KD]) {
  const uint64_t h = key_hash<KD>(k);
  return (uint32_t)(((h >> 32) * (uint64_t)sr.nbuckets) >> 32);
}

template <int KD>
__device__ __forceinline__ bool key_at(const int32_t* __restrict__ kB, uint32_t i, const int32_t (&k)[KD]) {
  bool eq = true;
#pragma unroll
  for (int d = 0; d < KD; ++d) eq = eq && kB[(size_t)i * KD + d] == k[d];
  return eq;
}

// Pass 1: every position takes the index h[t + p] and writes its key there.
template <int KD>
__global__ __launch_bounds__(kBlock) void k_slab_take(const SlabMeta* meta, const int32_t* __restrict__ heap,
                                                      const int32_t* __restrict__ keys, uint32_t n,
                                                      int32_t* __restrict__ kB, uint32_t* __restrict__ idx_of) {
  const uint32_t t0 = meta->t;
  for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
    const uint32_t i = (uint32_t)heap[t0 + p];
    idx_of[p] = i;
#pragma unroll
    for (int d = 0; d < KD; ++d) kB[(size_t)i * KD + d] = keys[(size_t)p * KD + d];
  }
}

// Pass 2: each position inserts its index into its bucket's list unless an
// entry with an equal key is there (k^B is read-only now).  An entry is
// claimed by a compare-and-swap of the first empty word the group sees;
// words only ever go from empty to an index, so two equal keys can never
// both be inserted: the later one sees the earlier one's entry before any
// empty word it could take.
template <int KD>
__global__ __launch_bounds__(kBlock) void k_slab_insert(SlabRef sr, SlabMeta* meta, const int32_t* __restrict__ keys,
                                                        uint32_t n, const int32_t* __restrict__ kB,
                                                        const uint32_t* __restrict__ idx_of,
                                                        uint8_t* __restrict__ won) {
  constexpr uint32_t kGroups = kBlock / kSlabWords;
  const uint32_t lane = threadIdx.x & (kSlabWords - 1);
  const uint32_t grp = threadIdx.x / kSlabWords;
  const uint32_t base = blockIdx.x * kGroups * kSlabRounds;
  for (int r = 0; r < kSlabRounds; ++r) {
    const uint32_t p = base + r * kGroups + grp;
    if (p >= n) break;
    int32_t k[KD];
#pragma unroll
    for (int d = 0; d < KD; ++d) k[d] = keys[(size_t)p * KD + d];
    const uint32_t mine = idx_of[p];
    uint32_t slab = slab_bucket<KD>(sr, k);
    uint8_t result = 0;
    for (uint32_t step = 0; step <= sr.max_steps; ++step) {
      uint32_t* words = sr.slabs + (size_t)slab * kSlabWords;
      const uint32_t w = __hip_atomic_load(words + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool entry = lane < kSlabEntries && w != kSlabEmpty;
      if (group_ballot<kSlabWords>(entry && key_at<KD>(kB, w, k))) break;  // present: not inserted
      const uint64_t empty = group_ballot<kSlabWords>(lane < kSlabEntries && w == kSlabEmpty);
      if (empty) {
        const uint32_t L = first_lane(empty);
        uint32_t old = 0;
        if (lane == L) {
          uint32_t expected = kSlabEmpty;
          __hip_atomic_compare_exchange_strong(words + L, &expected, mine, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
          old = expected;
        }
        old = group_bcast<kSlabWords>(old, L);
        if (old == kSlabEmpty) {
          result = 1;
          break;
        }
        --step;  // the word was taken: look at this slab again
        continue;
      }
      uint32_t next = group_bcast<kSlabWords>(w, kSlabWords - 1);
      if (next == kNoNext) {  // the list is full: link a slab from the pool
        uint32_t got = 0;
        if (lane == 0) {
          const uint32_t s = __hip_atomic_fetch_add(&meta->pool_top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (s >= sr.pool) {
            __hip_atomic_fetch_or(&meta->fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            got = kNoNext;
          } else {
            uint32_t expected = kNoNext;
            __hip_atomic_compare_exchange_strong(words + kSlabWords - 1, &expected, sr.nbuckets + s,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            got = expected == kNoNext ? sr.nbuckets + s : expected;  // another group linked first: follow its slab
          }
        }
        next = group_bcast<kSlabWords>(got, 0u);
        if (next == kNoNext) break;  // pool exhausted (the insert reports a capacity error)
      }
      slab = next;
    }
    if (lane == 0) won[p] = result;
  }
}

// Pass 3: inserted positions keep their indices, in batch order, as
// h[t .. t + w); the others return theirs to h[t + w .. t + n) (last first).
// Block scan plus decoupled look-back over 1024-position tiles; the last
// tile moves t.
__global__ __launch_bounds__(kBlock) void k_slab_commit(SlabMeta* meta, uint32_t n, const uint8_t* __restrict__ won,
                                                        const uint32_t* __restrict__ idx_of,
                                                        int32_t* __restrict__ heap, int32_t* __restrict__ out_idx,
                                                        uint8_t* __restrict__ out_mask, uint32_t* __restrict__ wlist,
                                                        uint64_t* __restrict__ status, uint32_t epoch) {
  __shared__ uint32_t s_prefix, s_t0;
  __shared__ uint64_t s_scan[kBlock / 64 + 1];
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kScanTile;
  // t is read before this tile publishes its count, so the last tile, whose
  // look-back waits for every count, moves it only after all tiles read it
  if (threadIdx.x == 0) s_t0 = __hip_atomic_load(&meta->t, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t t0 = s_t0;
  bool win[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    win[r] = p < n && won[p] != 0;
  }
  uint32_t rank[kScanItems];
  uint32_t total;
  block_rank_rows(win, rank, total, s_scan);
  const uint32_t prefix = block_lookback(status, tile, epoch, total, &meta->status, &s_prefix);
  if (threadIdx.x == 0 && tile == (n - 1) / kScanTile) {
    meta->t = t0 + prefix + total;
    meta->result = prefix + total;
  }
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint32_t p = base + r * kBlock + threadIdx.x;
    if (p >= n) continue;
    const uint32_t i = idx_of[p];
    const uint32_t before = prefix + rank[r];  // inserted positions before p
    if (win[r]) {
      heap[t0 + before] = (int32_t)i;
      if (wlist) wlist[before] = p;
    } else {
      heap[t0 + n - 1 - (p - before)] = (int32_t)i;
    }
    if (out_idx) out_idx[p] = win[r] ? (int32_t)i : -1;
    if (out_mask) out_mask[p] = win[r] ? 1 : 0;
  }
}

// Value rows of the inserted positions: v^B[i] = values[p] for winner w =
// (p = wlist[w], i = h[t - result + w]), in 4-byte units (rows of 4 bytes
// and more that are 4-byte multiples) or bytes.
template <typename U>
__global__ __launch_bounds__(kBlock) void k_slab_values(const SlabMeta* meta, const uint32_t* __restrict__ wlist,
                                                        const int32_t* __restrict__ heap, const uint8_t* __restrict__ src,
                                                        uint8_t* __restrict__ dst, uint32_t row_bytes) {
  const uint32_t total = meta->result;
  const uint32_t t0 = meta->t - total;
  const uint32_t units = row_bytes / (uint32_t)sizeof(U);
  const uint64_t items = (uint64_t)total * units;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < items; e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t w = (uint32_t)(e / units);
    const uint32_t c = (uint32_t)(e - (uint64_t)w * units);
    const uint32_t p = wlist[w];
    const uint32_t i = (uint32_t)heap[t0 + w];
    reinterpret_cast<U*>(dst + (size_t)i * row_bytes)[c] = reinterpret_cast<const U*>(src + (size_t)p * row_bytes)[c];
  }
}

// Query: walk the list comparing against k^B of every occupied entry.
template <int KD>
__global__ __launch_bounds__(kBlock) void k_slab_find(SlabRef sr, const int32_t* __restrict__ keys, uint32_t n,
                                                      const int32_t* __restrict__ kB, int32_t* __restrict__ out_idx,
                                                      uint8_t* __restrict__ out_mask) {
  constexpr uint32_t kGroups = kBlock / kSlabWords;
  const uint32_t lane = threadIdx.x & (kSlabWords - 1);
  const uint32_t grp = threadIdx.x / kSlabWords;
  const uint32_t base = blockIdx.x * kGroups * kSlabRounds;
  for (int r = 0; r < kSlabRounds; ++r) {
    const uint32_t p = base + r * kGroups + grp;
    if (p >= n) break;
    int32_t k[KD];
#pragma unroll
    for (int d = 0; d < KD; ++d) k[d] = keys[(size_t)p * KD + d];
    uint32_t slab = slab_bucket<KD>(sr, k);
    uint32_t found = kSlabEmpty;
    for (uint32_t step = 0; step <= sr.max_steps; ++step) {
      const uint32_t w = sr.slabs[(size_t)slab * kSlabWords + lane];
      const bool entry = lane < kSlabEntries && w != kSlabEmpty;
      const uint64_t m = group_ballot<kSlabWords>(entry && key_at<KD>(kB, w, k));
      if (m) {
        found = group_bcast<kSlabWords>(w, first_lane(m));
        break;
      }
      slab = group_bcast<kSlabWords>(w, kSlabWords - 1);
      if (slab == kNoNext) break;
    }
    if (lane == 0) {
      if (out_idx) out_idx[p] = found == kSlabEmpty ? -1 : (int32_t)found;
      if (out_mask) out_mask[p] = found == kSlabEmpty ? 0 : 1;
    }
  }
}

// Rows of the hits: out[p] = v^B[idx[p]] where idx[p] >= 0.
template <typename U>
__global__ __launch_bounds__(kBlock) void k_slab_gather(const int32_t* __restrict__ idx, uint32_t n,
                                                        const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                        uint32_t row_bytes) {
  const uint32_t units = row_bytes / (uint32_t)sizeof(U);
  const uint64_t items = (uint64_t)n * units;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < items; e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t p = (uint32_t)(e / units);
    const uint32_t c = (uint32_t)(e - (uint64_t)p * units);
    const int32_t i = idx[p];
    if (i >= 0)
      reinterpret_cast<U*>(dst + (size_t)p * row_bytes)[c] =
          reinterpret_cast<const U*>(src + (size_t)i * row_bytes)[c];
  }
}

__global__ void k_slab_reset(SlabMeta* m) {
  m->t = 0;
  m->pool_top = 0;
  m->fail = 0;
  m->result = 0;
  m->status = 0;
}

inline uint32_t cdiv32(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace
}  // namespace ash

using namespace ash_host;

struct ash_slab {
  int64_t c = 0;
  int32_t key_dim = 0;
  int64_t value_bytes = 0;
  ash::SlabRef sr{};
  int32_t* kB = nullptr;
  uint8_t* vB = nullptr;
  int32_t* heap = nullptr;
  ash::SlabMeta* meta = nullptr;
  uint32_t* idx_of = nullptr;
  uint8_t* won = nullptr;
  uint32_t* wlist = nullptr;
  int32_t* fidx = nullptr;  // find indices when the caller skips them but gathers rows
  uint64_t* status = nullptr;
  int64_t scratch_n = 0;
  int64_t t_ub = 0;
  uint32_t epoch = 0;
};

namespace {

void slab_free(ash_slab* m) {
  for (void* p : {(void*)m->sr.slabs, (void*)m->kB, (void*)m->vB, (void*)m->heap, (void*)m->meta, (void*)m->idx_of,
                  (void*)m->won, (void*)m->wlist, (void*)m->fidx, (void*)m->status})
    if (p) (void)hipFree(p);
}

ash_status_t slab_scratch(ash_slab* m, int64_t n) {
  if (n <= m->scratch_n) return ASH_OK;
  for (void* p : {(void*)m->idx_of, (void*)m->won, (void*)m->wlist, (void*)m->fidx, (void*)m->status})
    if (p) (void)hipFree(p);
  m->idx_of = nullptr;
  m->won = nullptr;
  m->wlist = nullptr;
  m->fidx = nullptr;
  m->status = nullptr;
  m->scratch_n = 0;
  const int64_t tiles = (n + ash::kScanTile - 1) / ash::kScanTile + 1;
  if (hipMalloc(&m->idx_of, (size_t)n * 4) != hipSuccess || hipMalloc(&m->won, (size_t)n) != hipSuccess ||
      hipMalloc(&m->wlist, (size_t)n * 4) != hipSuccess || hipMalloc(&m->fidx, (size_t)n * 4) != hipSuccess ||
      hipMalloc(&m->status, (size_t)tiles * 8) != hipSuccess)
    return ASH_E_NOMEM;
  ASH_HIP(hipMemset(m->status, 0, (size_t)tiles * 8));  // epoch 0: older than every launch
  m->epoch = 0;
  m->scratch_n = n;
  return ASH_OK;
}

ash_status_t slab_reset(ash_slab* m, hipStream_t st) {
  const size_t words = (size_t)(m->sr.nbuckets + m->sr.pool) * ash::kSlabWords;
  ASH_HIP(ash::launch_fill_u32(m->sr.slabs, ash::kSlabEmpty, words, st));
  ASH_HIP(ash::launch_iota(m->heap, 0, (uint32_t)m->c, st));
  hipLaunchKernelGGL(ash::k_slab_reset, dim3(1), dim3(1), 0, st, m->meta);
  ASH_HIP(hipGetLastError());
  m->t_ub = 0;
  return ASH_OK;
}

template <template <int> class K, typename... A>
hipError_t by_kd(int kd, dim3 grid, hipStream_t st, A... a) {
  switch (kd) {
    case 1: hipLaunchKernelGGL(K<1>::f, grid, dim3(ash::kBlock), 0, st, a...); break;
    case 2: hipLaunchKernelGGL(K<2>::f, grid, dim3(ash::kBlock), 0, st, a...); break;
    case 3: hipLaunchKernelGGL(K<3>::f, grid, dim3(ash::kBlock), 0, st, a...); break;
    case 4: hipLaunchKernelGGL(K<4>::f, grid, dim3(ash::kBlock), 0, st, a...); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KD>
struct TakeK {
  static constexpr auto f = ash::k_slab_take<KD>;
};
template <int KD>
struct InsertK {
  static constexpr auto f = ash::k_slab_insert<KD>;
};
template <int KD>
struct FindK {
  static constexpr auto f = ash::k_slab_find<KD>;
};

}  // namespace

extern "C" {

ash_status_t ash_slab_create(int64_t capacity, int32_t key_dim, int64_t value_bytes, void* stream, ash_slab_t* out) {
  if (!out || capacity < 1 || capacity > (1ll << 30) || key_dim < 1 || key_dim > 4) return ASH_E_INVALID;
  if (value_bytes < 0 || value_bytes > (1ll << 24)) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  ash_slab* m = new ash_slab;
  m->c = capacity;
  m->key_dim = key_dim;
  m->value_bytes = value_bytes;
  const uint64_t nb = (2 * (uint64_t)capacity + ash::kSlabEntries - 1) / ash::kSlabEntries;
  m->sr.nbuckets = (uint32_t)std::max<uint64_t>(nb, 1);
  m->sr.pool = m->sr.nbuckets / 8 + 64;
  m->sr.max_steps = m->sr.pool + 1;
  const size_t slab_bytes = (size_t)(m->sr.nbuckets + m->sr.pool) * ash::kSlabWords * 4;
  bool ok = hipMalloc(&m->sr.slabs, slab_bytes) == hipSuccess &&
            hipMalloc(&m->kB, (size_t)capacity * key_dim * 4) == hipSuccess &&
            hipMalloc(&m->heap, (size_t)capacity * 4) == hipSuccess &&
            hipMalloc(&m->meta, sizeof(ash::SlabMeta)) == hipSuccess &&
            (value_bytes == 0 || hipMalloc(&m->vB, (size_t)capacity * value_bytes) == hipSuccess);
  ok = ok && slab_scratch(m, 1024) == ASH_OK && slab_reset(m, st) == ASH_OK && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    slab_free(m);
    delete m;
    return ASH_E_NOMEM;
  }
  *out = m;
  return ASH_OK;
}

ash_status_t ash_slab_destroy(ash_slab_t m) {
  if (!m) return ASH_E_INVALID;
  (void)hipDeviceSynchronize();
  slab_free(m);
  delete m;
  return ASH_OK;
}

ash_status_t ash_slab_clear(ash_slab_t m, void* stream) {
  if (!m) return ASH_E_INVALID;
  return slab_reset(m, (hipStream_t)stream);
}

ash_status_t ash_slab_insert(ash_slab_t m, const int32_t* keys, int64_t n, const void* values, int32_t* out_idx,
                             uint8_t* out_mask, void* stream) {
  if (!m || n < 0 || (n > 0 && !keys) || (n > 0 && m->value_bytes > 0 && !values)) return ASH_E_INVALID;
  if (n == 0) return ASH_OK;
  hipStream_t st = (hipStream_t)stream;
  if (m->t_ub + n > m->c) {
    int64_t t = 0;
    ASH_TRY(ash_slab_size(m, &t, stream));
    if (t + n > m->c) return ASH_E_CAPACITY;  // every position takes an index first
  }
  ASH_TRY(slab_scratch(m, n));
  const uint32_t un = (uint32_t)n;
  m->epoch = m->epoch + 1 == 0 ? 1 : m->epoch + 1;
  ASH_HIP(by_kd<TakeK>(m->key_dim, dim3(std::min<uint32_t>(ash::cdiv32(un, ash::kBlock), 65536)), st,
                       (const ash::SlabMeta*)m->meta, (const int32_t*)m->heap, keys, un, m->kB, m->idx_of));
  const uint32_t per_block = (ash::kBlock / ash::kSlabWords) * ash::kSlabRounds;
  ASH_HIP(by_kd<InsertK>(m->key_dim, dim3(ash::cdiv32(un, per_block)), st, m->sr, m->meta, keys, un,
                         (const int32_t*)m->kB, (const uint32_t*)m->idx_of, m->won));
  hipLaunchKernelGGL(ash::k_slab_commit, dim3(ash::cdiv32(un, ash::kScanTile)), dim3(ash::kBlock), 0, st, m->meta, un,
                     (const uint8_t*)m->won, (const uint32_t*)m->idx_of, m->heap, out_idx, out_mask,
                     m->value_bytes > 0 ? m->wlist : nullptr, m->status, m->epoch);
  ASH_HIP(hipGetLastError());
  if (m->value_bytes > 0) {
    const uint32_t grid = std::min<uint32_t>(ash::cdiv32((uint64_t)n * (m->value_bytes / 4 + 1), ash::kBlock), 65536);
    if (m->value_bytes % 4 == 0 && ((uintptr_t)values & 3u) == 0)
      hipLaunchKernelGGL(ash::k_slab_values<uint32_t>, dim3(grid), dim3(ash::kBlock), 0, st,
                         (const ash::SlabMeta*)m->meta, (const uint32_t*)m->wlist, (const int32_t*)m->heap,
                         (const uint8_t*)values, m->vB, (uint32_t)m->value_bytes);
    else
      hipLaunchKernelGGL(ash::k_slab_values<uint8_t>, dim3(grid), dim3(ash::kBlock), 0, st,
                         (const ash::SlabMeta*)m->meta, (const uint32_t*)m->wlist, (const int32_t*)m->heap,
                         (const uint8_t*)values, m->vB, (uint32_t)m->value_bytes);
    ASH_HIP(hipGetLastError());
  }
  ash::SlabMeta h;
  ASH_HIP(hipMemcpyAsync(&h, m->meta, sizeof(h), hipMemcpyDeviceToHost, st));
  ASH_HIP(hipStreamSynchronize(st));
  m->t_ub = h.t;
  if (h.status) return ASH_E_DEVICE;
  return h.fail ? ASH_E_CAPACITY : ASH_OK;
}

ash_status_t ash_slab_find(ash_slab_t m, const int32_t* keys, int64_t n, int32_t* out_idx, uint8_t* out_mask,
                           void* out_values, void* stream) {
  if (!m || n < 0 || (n > 0 && !keys)) return ASH_E_INVALID;
  if (n == 0) return ASH_OK;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t un = (uint32_t)n;
  int32_t* idx = out_idx;
  if (!idx && out_values && m->value_bytes > 0) {
    ASH_TRY(slab_scratch(m, n));
    idx = m->fidx;
  }
  const uint32_t per_block = (ash::kBlock / ash::kSlabWords) * ash::kSlabRounds;
  ASH_HIP(by_kd<FindK>(m->key_dim, dim3(ash::cdiv32(un, per_block)), st, m->sr, keys, un, (const int32_t*)m->kB, idx,
                       out_mask));
  if (out_values && m->value_bytes > 0) {
    const uint32_t grid = std::min<uint32_t>(ash::cdiv32((uint64_t)n * (m->value_bytes / 4 + 1), ash::kBlock), 65536);
    if (m->value_bytes % 4 == 0 && ((uintptr_t)out_values & 3u) == 0)
      hipLaunchKernelGGL(ash::k_slab_gather<uint32_t>, dim3(grid), dim3(ash::kBlock), 0, st, (const int32_t*)idx, un,
                         (const uint8_t*)m->vB, (uint8_t*)out_values, (uint32_t)m->value_bytes);
    else
      hipLaunchKernelGGL(ash::k_slab_gather<uint8_t>, dim3(grid), dim3(ash::kBlock), 0, st, (const int32_t*)idx, un,
                         (const uint8_t*)m->vB, (uint8_t*)out_values, (uint32_t)m->value_bytes);
    ASH_HIP(hipGetLastError());
  }
  return ASH_OK;
}

ash_status_t ash_slab_size(ash_slab_t m, int64_t* out, void* stream) {
  if (!m || !out) return ASH_E_INVALID;
  ash::SlabMeta h;
  ASH_HIP(hipMemcpyAsync(&h, m->meta, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream));
  ASH_HIP(hipStreamSynchronize((hipStream_t)stream));
  m->t_ub = h.t;
  *out = h.t;
  return ASH_OK;
}

ash_status_t ash_slab_buffers(ash_slab_t m, int32_t** key_buffer, void** value_buffer, int32_t** heap) {
  if (!m) return ASH_E_INVALID;
  if (key_buffer) *key_buffer = m->kB;
  if (value_buffer) *value_buffer = m->vB;
  if (heap) *heap = m->heap;
  return ASH_OK;
}

}  // extern "C"
