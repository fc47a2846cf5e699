// ash_membench.hip -- access-cost microbenchmark (instrumentation).
//
// The hash map's kernels are bound by random accesses to a large table: one
// window read per probe step, one claim CAS per new key, one slot store per
// committed key.  What such an access costs in DRAM traffic and time is a
// property of the memory system, not of the method, so it is measured here
// with kernels that do nothing else: n accesses at addresses drawn from a
// counter-based hash (the SplitMix64 output function of i) over a table of
// the caller's size, each access aligned to its own size.  Reads and stores
// of A >= 16 bytes are made by A / 16 consecutive lanes of a wavefront,
// one 16-byte unit each (as a g-lane probe group reads a window); smaller
// ones by one lane.  A streaming read and a streaming copy of the table give
// the reference that byte counters are calibrated against.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ash.h"
#include "ash_device.hpp"
#include "ash_internal.hpp"

namespace ash {
namespace {

constexpr int kUnroll = 8;  // independent accesses in flight per lane

__device__ __forceinline__ uint64_t unit_of(uint64_t seed, uint64_t a, uint64_t units) {
  return __umul64hi(mix64(seed ^ (a * 0x9e3779b97f4a7c15ull)), units);
}

__device__ __forceinline__ uint32_t fold(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t fold(uint2 v) { return v.x ^ v.y; }
__device__ __forceinline__ uint32_t fold(uint4 v) { return v.x ^ v.y ^ v.z ^ v.w; }

template <typename V>
__device__ __forceinline__ V splat(uint32_t x);
template <>
__device__ __forceinline__ uint32_t splat<uint32_t>(uint32_t x) { return x; }
template <>
__device__ __forceinline__ uint2 splat<uint2>(uint32_t x) { return make_uint2(x, ~x); }
template <>
__device__ __forceinline__ uint4 splat<uint4>(uint32_t x) { return make_uint4(x, ~x, x + 1u, x - 1u); }

// Random reads (kStore = false) or stores of A bytes: lanes of a group of L
// move unit sub of access a at table + unit_of(a) * A + sub * sizeof(V).
template <typename V, int L, bool kStore>
__global__ __launch_bounds__(kBlock) void k_acc_random(uint8_t* __restrict__ table, uint64_t units,
                                                       uint64_t n, uint64_t seed) {
  constexpr uint32_t A = sizeof(V) * L;
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t groups = (uint64_t)gridDim.x * kBlock / L;
  const uint64_t grp = tid / L;
  const uint32_t sub = (uint32_t)(tid % L);
  uint32_t acc = 0;
  for (uint64_t a0 = grp; a0 < n; a0 += groups * kUnroll) {
    V v[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const uint64_t a = a0 + (uint64_t)j * groups;
      if (a >= n) continue;
      V* p = reinterpret_cast<V*>(table + unit_of(seed, a, units) * A) + sub;
      if constexpr (kStore) *p = splat<V>((uint32_t)a);
      else v[j] = *p;
    }
    if constexpr (!kStore) {
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (a0 + (uint64_t)j * groups < n) acc ^= fold(v[j]);
    }
  }
  if (!kStore && acc == 0x9e3779b9u && tid == 0) *reinterpret_cast<uint32_t*>(table) = acc;  // keeps the loads
}

// Device-scope 64-bit compare-and-swap (returning) at random 8-byte words.
__global__ __launch_bounds__(kBlock) void k_acc_cas64(uint8_t* __restrict__ table, uint64_t units, uint64_t n,
                                                      uint64_t seed) {
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint64_t acc = 0;
  for (uint64_t a = tid; a < n; a += stride) {
    uint64_t* p = reinterpret_cast<uint64_t*>(table) + unit_of(seed, a, units);
    uint64_t expected = a;
    __hip_atomic_compare_exchange_strong(p, &expected, a ^ seed, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    acc ^= expected;
  }
  if (acc == 0x9e3779b97f4a7c15ull) *reinterpret_cast<uint64_t*>(table) = acc;
}

// Device-scope 32-bit atomic minimum (no return) at random 4-byte words.
__global__ __launch_bounds__(kBlock) void k_acc_min32(uint8_t* __restrict__ table, uint64_t units, uint64_t n,
                                                      uint64_t seed) {
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t a = tid; a < n; a += stride) {
    uint32_t* p = reinterpret_cast<uint32_t*>(table) + unit_of(seed, a, units);
    __hip_atomic_fetch_min(p, (uint32_t)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Streaming read of the whole table (16 bytes per lane and step).
__global__ __launch_bounds__(kBlock) void k_acc_stream_read(uint8_t* __restrict__ table, uint64_t n16) {
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint4* p = reinterpret_cast<const uint4*>(table);
  uint32_t acc = 0;
  for (uint64_t i = tid; i < n16; i += stride) acc ^= fold(p[i]);
  if (acc == 0x9e3779b9u && tid == 0) *reinterpret_cast<uint32_t*>(table) = acc;
}

// Streaming copy of the table's first half onto its second half.
__global__ __launch_bounds__(kBlock) void k_acc_stream_copy(uint8_t* __restrict__ table, uint64_t half16) {
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint4* src = reinterpret_cast<const uint4*>(table);
  uint4* dst = reinterpret_cast<uint4*>(table) + half16;
  for (uint64_t i = tid; i < half16; i += stride) dst[i] = src[i];
}

template <typename V, int L, bool kStore>
void launch_random(uint8_t* table, uint64_t units, uint64_t n, uint64_t seed, hipStream_t st) {
  const uint64_t threads = std::max<uint64_t>(1, (n * L + kUnroll - 1) / kUnroll);
  const uint32_t grid = (uint32_t)std::min<uint64_t>((threads + kBlock - 1) / kBlock, 16384);
  hipLaunchKernelGGL((k_acc_random<V, L, kStore>), dim3(grid), dim3(kBlock), 0, st, table, units, n, seed);
}

template <bool kStore>
bool launch_sized(int access_bytes, uint8_t* table, uint64_t units, uint64_t n, uint64_t seed, hipStream_t st) {
  switch (access_bytes) {
    case 4: launch_random<uint32_t, 1, kStore>(table, units, n, seed, st); return true;
    case 8: launch_random<uint2, 1, kStore>(table, units, n, seed, st); return true;
    case 16: launch_random<uint4, 1, kStore>(table, units, n, seed, st); return true;
    case 32: launch_random<uint4, 2, kStore>(table, units, n, seed, st); return true;
    case 64: launch_random<uint4, 4, kStore>(table, units, n, seed, st); return true;
    case 128: launch_random<uint4, 8, kStore>(table, units, n, seed, st); return true;
    case 256: launch_random<uint4, 16, kStore>(table, units, n, seed, st); return true;
    default: return false;
  }
}

}  // namespace
}  // namespace ash

using namespace ash_host;

extern "C" ash_status_t ash_access_bench(int32_t kind, void* table, int64_t table_bytes, int32_t access_bytes,
                                         int64_t n_access, uint64_t seed, double* out_ms, void* stream) {
  if (!table || ((uintptr_t)table & 255u) != 0 || table_bytes < 256 || (table_bytes & 255) != 0)
    return ASH_E_INVALID;
  if (n_access < 0 || n_access > (1ll << 40)) return ASH_E_INVALID;
  const bool sized = kind == ASH_ACC_READ || kind == ASH_ACC_STORE;
  if (sized && !(access_bytes == 4 || access_bytes == 8 || access_bytes == 16 || access_bytes == 32 ||
                 access_bytes == 64 || access_bytes == 128 || access_bytes == 256))
    return ASH_E_INVALID;
  if (kind == ASH_ACC_CAS64 && access_bytes != 8) return ASH_E_INVALID;
  if (kind == ASH_ACC_MIN32 && access_bytes != 4) return ASH_E_INVALID;
  if (kind < ASH_ACC_READ || kind > ASH_ACC_STREAM_COPY) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  uint8_t* t = (uint8_t*)table;
  const uint64_t tb = (uint64_t)table_bytes;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return ASH_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ASH_E_DEVICE;
  }
  const uint64_t n = (uint64_t)n_access;
  const uint32_t stream_grid = 8192;
  bool ok = hipEventRecord(e0, st) == hipSuccess;
  if (ok) {
    switch (kind) {
      case ASH_ACC_READ: ok = ash::launch_sized<false>(access_bytes, t, tb / access_bytes, n, seed, st); break;
      case ASH_ACC_STORE: ok = ash::launch_sized<true>(access_bytes, t, tb / access_bytes, n, seed, st); break;
      case ASH_ACC_CAS64:
        hipLaunchKernelGGL(ash::k_acc_cas64, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256 + 1, 16384)),
                           dim3(ash::kBlock), 0, st, t, tb / 8, n, seed);
        break;
      case ASH_ACC_MIN32:
        hipLaunchKernelGGL(ash::k_acc_min32, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256 + 1, 16384)),
                           dim3(ash::kBlock), 0, st, t, tb / 4, n, seed);
        break;
      case ASH_ACC_STREAM_READ:
        hipLaunchKernelGGL(ash::k_acc_stream_read, dim3(stream_grid), dim3(ash::kBlock), 0, st, t, tb / 16);
        break;
      default:
        hipLaunchKernelGGL(ash::k_acc_stream_copy, dim3(stream_grid), dim3(ash::kBlock), 0, st, t, tb / 32);
        break;
    }
    ok = ok && hipGetLastError() == hipSuccess;
  }
  ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  float ms = 0.0f;
  ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return ASH_E_DEVICE;
  if (out_ms) *out_ms = ms;
  return ASH_OK;
}
