// ash_io.hip -- saving a map to a file and loading it back (the paper keeps a
// map on disk between processing stages, Sec. 6.3), and describing a map.
//
// A file holds the map's whole logical state: capacity, the index heap h with
// its top t, the live buffer indices with their keys and value rows.  Loading
// restores exactly that state, so the loaded map hands out the same indices
// as the saved one would have; the slot table is rebuilt from the live
// (key, index) pairs by the same kernel that rehashing uses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ash.h"
#include "ash_device.hpp"
#include "ash_internal.hpp"
#include "ash_launch.hpp"

using namespace ash_host;

namespace {

constexpr char kMagic[8] = {'A', 'S', 'H', 'M', 'A', 'P', 0, 1};

struct Header {
  int32_t key_dim;
  int32_t n_values;
  int64_t capacity;
  int64_t size;
};

struct File {
  std::FILE* f = nullptr;
  explicit File(std::FILE* p) : f(p) {}
  ~File() {
    if (f) std::fclose(f);
  }
  bool write(const void* p, size_t bytes) { return bytes == 0 || std::fwrite(p, 1, bytes, f) == bytes; }
  bool read(void* p, size_t bytes) { return bytes == 0 || std::fread(p, 1, bytes, f) == bytes; }
};

bool valid_dtype(int32_t t) { return t >= ASH_U8 && t <= ASH_BF16; }

}  // namespace

extern "C" {

ash_status_t ash_describe(ash_map_t m, int32_t* out_key_dim, int32_t* out_n_values, ash_dtype_t* out_dtypes,
                          int64_t* out_elems) {
  if (!m || !out_key_dim || !out_n_values) return ASH_E_INVALID;
  *out_key_dim = m->key_dim;
  *out_n_values = m->n_values;
  for (int j = 0; j < m->n_values; ++j) {
    if (out_dtypes) out_dtypes[j] = m->dtypes[j];
    if (out_elems) out_elems[j] = m->elems[j];
  }
  return ASH_OK;
}

ash_status_t ash_save(ash_map_t m, const char* path, void* stream) {
  if (!m || !path) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  Meta h;
  ASH_TRY(read_meta(m, &h, st));
  const int64_t c = m->c;
  const int64_t t = h.t;
  std::vector<int32_t> live(std::max<int64_t>(t, 1));
  if (c > 0) {
    int32_t* d_live = (int32_t*)m->mem.get((size_t)c * 4, st);
    if (!d_live) return ASH_E_NOMEM;
    int64_t count = 0;
    ash_status_t rc = ash_active_indices(m, d_live, &count, stream);
    if (rc == ASH_OK && count != t) rc = ASH_E_DEVICE;  // live slots and heap top disagree
    if (rc == ASH_OK && t > 0 &&
        hipMemcpyAsync(live.data(), d_live, (size_t)t * 4, hipMemcpyDeviceToHost, st) != hipSuccess)
      rc = ASH_E_DEVICE;
    m->mem.put(d_live, st);
    ASH_TRY(rc);
  }
  // The heap, k^B and every v^B go to the host whole; live rows are picked there.
  std::vector<int32_t> heap(c), kB((size_t)c * m->key_dim);
  std::vector<std::vector<uint8_t>> vB(m->n_values);
  if (c > 0) {
    ASH_HIP(hipMemcpyAsync(heap.data(), m->heap, (size_t)c * 4, hipMemcpyDeviceToHost, st));
    ASH_HIP(hipMemcpyAsync(kB.data(), m->kB, (size_t)c * m->key_dim * 4, hipMemcpyDeviceToHost, st));
    for (int j = 0; j < m->n_values; ++j) {
      vB[j].resize((size_t)c * m->row_bytes[j]);
      ASH_HIP(hipMemcpyAsync(vB[j].data(), m->vB[j], vB[j].size(), hipMemcpyDeviceToHost, st));
    }
  }
  ASH_HIP(hipStreamSynchronize(st));

  File f(std::fopen(path, "wb"));
  if (!f.f) return ASH_E_INVALID;
  const Header hd{m->key_dim, m->n_values, c, t};
  bool ok = f.write(kMagic, sizeof(kMagic)) && f.write(&hd, sizeof(hd));
  for (int j = 0; j < m->n_values && ok; ++j) {
    const int32_t dt[2] = {(int32_t)m->dtypes[j], 0};
    ok = f.write(dt, sizeof(dt)) && f.write(&m->elems[j], 8);
  }
  ok = ok && f.write(heap.data(), (size_t)c * 4) && f.write(live.data(), (size_t)t * 4);
  for (int64_t r = 0; r < t && ok; ++r) ok = f.write(&kB[(size_t)live[r] * m->key_dim], (size_t)m->key_dim * 4);
  for (int j = 0; j < m->n_values && ok; ++j)
    for (int64_t r = 0; r < t && ok; ++r)
      ok = f.write(&vB[j][(size_t)live[r] * m->row_bytes[j]], m->row_bytes[j]);
  ok = ok && std::fflush(f.f) == 0;
  return ok ? ASH_OK : ASH_E_INVALID;
}

ash_status_t ash_load(const char* path, const ash_allocator_t* allocator, const ash_tuning_t* tuning, void* stream,
                      ash_map_t* out) {
  if (!path || !out) return ASH_E_INVALID;
  File f(std::fopen(path, "rb"));
  if (!f.f) return ASH_E_INVALID;
  // --- everything is read and checked before any device work
  char magic[8];
  Header hd;
  if (!f.read(magic, 8) || std::memcmp(magic, kMagic, 8) != 0 || !f.read(&hd, sizeof(hd))) return ASH_E_INVALID;
  if (hd.key_dim < 1 || hd.key_dim > 4 || hd.n_values < 0 || hd.n_values > ash::kMaxValues) return ASH_E_INVALID;
  if (hd.capacity < 0 || hd.capacity > kMaxCount || hd.size < 0 || hd.size > hd.capacity) return ASH_E_INVALID;
  const int kd = hd.key_dim;
  const int64_t c = hd.capacity, t = hd.size;
  std::vector<ash_dtype_t> dtypes(hd.n_values);
  std::vector<int64_t> elems(hd.n_values);
  std::vector<uint64_t> rb(hd.n_values);
  for (int j = 0; j < hd.n_values; ++j) {
    int32_t dt[2];
    if (!f.read(dt, sizeof(dt)) || !f.read(&elems[j], 8) || !valid_dtype(dt[0])) return ASH_E_INVALID;
    dtypes[j] = (ash_dtype_t)dt[0];
    if (elems[j] <= 0 || elems[j] > (1 << 24)) return ASH_E_INVALID;
    rb[j] = dtype_size(dtypes[j]) * (uint64_t)elems[j];
    if (rb[j] > (1u << 24)) return ASH_E_INVALID;
  }
  std::vector<int32_t> heap(c), live(t), keys((size_t)t * kd);
  if (!f.read(heap.data(), (size_t)c * 4) || !f.read(live.data(), (size_t)t * 4) ||
      !f.read(keys.data(), keys.size() * 4))
    return ASH_E_INVALID;
  std::vector<std::vector<uint8_t>> rows(hd.n_values);
  for (int j = 0; j < hd.n_values; ++j) {
    rows[j].resize((size_t)t * rb[j]);
    if (!f.read(rows[j].data(), rows[j].size())) return ASH_E_INVALID;
  }
  char extra;
  if (std::fread(&extra, 1, 1, f.f) != 0) return ASH_E_INVALID;  // trailing bytes
  // live indices ascend (hence are distinct) below c; the heap's free region
  // h[t..c) holds every other index once (Sec. 4.3: allocation takes h[t],
  // a free writes h[t - 1], so entries below t are stale and only in range)
  std::vector<uint8_t> seen(c, 0);
  for (int64_t r = 0; r < t; ++r) {
    if (live[r] < 0 || live[r] >= c) return ASH_E_INVALID;
    if (r > 0 && live[r] <= live[r - 1]) return ASH_E_INVALID;
    seen[live[r]] = 1;
  }
  for (int64_t r = 0; r < c; ++r) {
    const int32_t i = heap[r];
    if (i < 0 || i >= c) return ASH_E_INVALID;
    if (r >= t) {
      if (seen[i]) return ASH_E_INVALID;  // live, or twice in the free region
      seen[i] = 2;
    }
  }
  {  // keys are distinct
    std::vector<std::array<int32_t, 4>> sorted(t);
    for (int64_t r = 0; r < t; ++r) {
      sorted[r] = {0, 0, 0, 0};
      for (int d = 0; d < kd; ++d) sorted[r][d] = keys[(size_t)r * kd + d];
    }
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return ASH_E_INVALID;
  }

  // --- a fresh map, then its state
  ash_map_t m = nullptr;
  ASH_TRY(ash_create(c, kd, hd.n_values, dtypes.data(), elems.data(), allocator, tuning, stream, &m));
  hipStream_t st = (hipStream_t)stream;
  ash_status_t rc = ASH_OK;
  uint32_t* pairs = nullptr;
  std::vector<int32_t> kB((size_t)c * kd, 0);
  std::vector<std::vector<uint8_t>> vB(hd.n_values);
  for (int64_t r = 0; r < t; ++r)
    std::memcpy(&kB[(size_t)live[r] * kd], &keys[(size_t)r * kd], (size_t)kd * 4);
  for (int j = 0; j < hd.n_values; ++j) {
    vB[j].assign((size_t)c * rb[j], 0);
    for (int64_t r = 0; r < t; ++r) std::memcpy(&vB[j][(size_t)live[r] * rb[j]], &rows[j][(size_t)r * rb[j]], rb[j]);
  }
  // (key, index) pairs laid out as committed slots, for the table rebuild
  const int S = m->slot_words();
  std::vector<uint32_t> slots((size_t)t * S, 0);
  for (int64_t r = 0; r < t; ++r) {
    uint32_t* w = &slots[(size_t)r * S];
    for (int d = 0; d < kd - 1; ++d) w[d] = (uint32_t)keys[(size_t)r * kd + d];
    w[S - 2] = (uint32_t)keys[(size_t)r * kd + kd - 1];
    w[S - 1] = (uint32_t)live[r];
  }
  if (c > 0) {
    if (hipMemcpyAsync(m->heap, heap.data(), (size_t)c * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(m->kB, kB.data(), kB.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = ASH_E_DEVICE;
    for (int j = 0; j < hd.n_values && rc == ASH_OK; ++j)
      if (hipMemcpyAsync(m->vB[j], vB[j].data(), vB[j].size(), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = ASH_E_DEVICE;
  }
  if (rc == ASH_OK && t > 0) {
    pairs = (uint32_t*)m->mem.get(slots.size() * 4, st);
    if (!pairs) rc = ASH_E_NOMEM;
    if (rc == ASH_OK && hipMemcpyAsync(pairs, slots.data(), slots.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = ASH_E_DEVICE;
  }
  Meta h;
  if (rc == ASH_OK) rc = read_meta(m, &h, st);  // also waits for the uploads above (host vectors stay valid)
  if (rc == ASH_OK) {
    h.t = (uint32_t)t;
    if (hipMemcpyAsync(m->meta, &h, sizeof(Meta), hipMemcpyHostToDevice, st) != hipSuccess) rc = ASH_E_DEVICE;
  }
  if (rc == ASH_OK && t > 0) {
    // the pairs stand in for an old table of t slots; the rebuild frees them
    m->mem.put(m->table, st);
    m->table = pairs;
    m->nslots = (uint32_t)t;
    pairs = nullptr;
    rc = rebuild_table(m, t, st);
  }
  if (rc == ASH_OK && hipStreamSynchronize(st) != hipSuccess) rc = ASH_E_DEVICE;
  if (pairs) m->mem.put(pairs, st);
  if (rc != ASH_OK) {
    ash_destroy(m);
    return rc;
  }
  m->live_ub = t;
  m->used_ub = t;
  *out = m;
  return ASH_OK;
}

}  // extern "C"
