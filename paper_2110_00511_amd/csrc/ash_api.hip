// ash_api.hip -- host side of the C ABI declared in include/ash.h: argument
// checks, buffer ownership, capacity policy and launch sequencing.  Every
// step of every operation runs in the kernels of ash_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ash.h"
#include "ash_device.hpp"
#include "ash_internal.hpp"
#include "ash_launch.hpp"

using namespace ash_host;

namespace ash_host {

// Slots for a capacity: ceil(c / max_load) rounded up to the larger of W and
// G (both powers of two), at least 64.
ash_status_t slots_for(int64_t c, float max_load, int W, int G, uint32_t* out) {
  const uint64_t unit = (uint64_t)std::max(W, G);
  double want = std::ceil((double)c / (double)max_load);
  uint64_t s = std::max<uint64_t>((uint64_t)want, 64);
  s = (s + unit - 1) / unit * unit;
  if (s > kMaxSlots) return ASH_E_UNSUPPORTED;
  *out = (uint32_t)s;
  return ASH_OK;
}

// Runs one launch, bracketed by events when profiling is on.
template <typename F>
hipError_t timed(ash_map* m, const char* name, hipStream_t st, F&& launch) {
  if (!m->prof.on) return launch();
  hipEvent_t a = m->prof.next(), b = m->prof.next();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  m->prof.recs.push_back({name, a, b});
  return e;
}

ash_status_t read_meta(ash_map* m, Meta* out, hipStream_t st) {
  ASH_HIP(hipMemcpyAsync(out, m->meta, sizeof(Meta), hipMemcpyDeviceToHost, st));
  ASH_HIP(hipStreamSynchronize(st));
  m->live_ub = out->t;
  m->used_ub = out->used;
  return ASH_OK;
}

ash_status_t ensure_scratch(ash_map* m, int64_t n, hipStream_t st) {
  if (n > m->scratch_n) {
    m->mem.put(m->slot_of, st);
    m->mem.put(m->aux, st);
    m->mem.put(m->partial, st);
    m->mem.put(m->lost, st);
    const size_t lost_bytes = ((size_t)n + 3) / 4 * 4;
    m->slot_of = (uint32_t*)m->mem.get((size_t)n * 4, st);
    m->aux = (int32_t*)m->mem.get((size_t)n * 4, st);
    m->partial = (uint32_t*)m->mem.get(((size_t)n / 256 + 2) * 4, st);
    m->lost = (uint8_t*)m->mem.get(lost_bytes, st);
    if (!m->slot_of || !m->aux || !m->partial || !m->lost) {
      m->scratch_n = 0;
      return ASH_E_NOMEM;
    }
    ASH_HIP(ash::launch_fill_u32((uint32_t*)m->lost, 0u, lost_bytes / 4, st));
    m->scratch_n = n;
  }
  const int64_t tiles = (std::max(n, m->c) + ash::kScanTile - 1) / ash::kScanTile + 1;
  if (tiles > m->scan_tiles) {
    m->mem.put(m->scan_status, st);
    m->scan_status = (uint64_t*)m->mem.get((size_t)tiles * 8, st);
    if (!m->scan_status) {
      m->scan_tiles = 0;
      return ASH_E_NOMEM;
    }
    ASH_HIP(ash::launch_fill_u32((uint32_t*)m->scan_status, 0u, (size_t)tiles * 2, st));
    m->scan_tiles = tiles;
  }
  return ASH_OK;
}

void free_buffers(ash_map* m, hipStream_t st) {
  m->mem.put(m->table, st);
  m->mem.put(m->kB, st);
  for (uint8_t* p : m->vB) m->mem.put(p, st);
  m->mem.put(m->heap, st);
  m->mem.put(m->owner, st);
  m->table = nullptr;
  m->kB = nullptr;
  m->vB.assign(m->vB.size(), nullptr);
  m->heap = nullptr;
  m->owner = nullptr;
}

// Rebuilds the slot table of `m` (new slot array, tombstones dropped) from the
// committed slots of the old table, sized for max(c, room_for) keys.
ash_status_t rebuild_table(ash_map* m, int64_t live, hipStream_t st, int64_t room_for) {
  uint32_t nslots;
  ASH_TRY(slots_for(std::max(m->c, room_for), m->max_load, m->W, m->G, &nslots));
  uint32_t* fresh = (uint32_t*)m->mem.get((size_t)nslots * m->slot_words() * 4, st);
  if (!fresh) return ASH_E_NOMEM;
  ASH_HIP(ash::launch_fill_u32(fresh, ash::kEmpty, (size_t)nslots * m->slot_words(), st));
  uint32_t* old = m->table;
  const uint32_t old_slots = m->nslots;
  m->table = fresh;
  m->nslots = nslots;
  ASH_HIP(timed(m, "rebuild", st, [&] {
    return ash::launch_rebuild(m->key_dim, m->G, m->W, m->ref(), old, old_slots, m->meta, st);
  }));
  m->mem.put(old, st);
  ASH_HIP(timed(m, "finalize", st, [&] { return ash::launch_finalize(m->meta, (uint32_t)m->c, ash::kFinalizeRebuild, 0, 0, m->scan_status, 0, st); }));
  // live keys now occupy exactly `live` slots and there are no tombstones
  Meta h;
  ASH_TRY(read_meta(m, &h, st));
  h.used = (uint32_t)live;
  h.tombs = 0;
  ASH_HIP(hipMemcpyAsync(m->meta, &h, sizeof(Meta), hipMemcpyHostToDevice, st));
  ASH_HIP(hipStreamSynchronize(st));
  m->used_ub = live;
  m->tombs_possible = false;
  return h.result ? ASH_E_CAPACITY : ASH_OK;  // this rebuild found no slot for some key
}

ash_status_t grow(ash_map* m, int64_t new_c, hipStream_t st) {
  Meta h;
  ASH_TRY(read_meta(m, &h, st));
  const int64_t live = h.t;
  if (new_c < m->c) return ASH_E_INVALID;
  if (new_c > kMaxCount) return ASH_E_UNSUPPORTED;
  if (new_c != m->c) {
    uint32_t probe_slots;
    ASH_TRY(slots_for(new_c, m->max_load, m->W, m->G, &probe_slots));
    const int64_t keep = m->c;
    int32_t* kB = (int32_t*)m->mem.get((size_t)new_c * m->key_dim * 4, st);
    int32_t* heap = (int32_t*)m->mem.get((size_t)new_c * 4, st);
    uint64_t* owner = (uint64_t*)m->mem.get((size_t)new_c * 8, st);
    std::vector<uint8_t*> vB(m->n_values, nullptr);
    bool ok = kB && heap && owner;
    for (int j = 0; j < m->n_values && ok; ++j) {
      vB[j] = (uint8_t*)m->mem.get((size_t)new_c * m->row_bytes[j], st);
      ok = vB[j] != nullptr;
    }
    if (!ok) {
      m->mem.put(kB, st);
      m->mem.put(heap, st);
      m->mem.put(owner, st);
      for (uint8_t* p : vB) m->mem.put(p, st);
      return ASH_E_NOMEM;
    }
    // Live indices are < c and keep their rows; the heap keeps its contents
    // and receives c .. new_c-1 above them (h' = h ++ [c, c')).
    if (keep > 0) {
      ASH_HIP(hipMemcpyAsync(kB, m->kB, (size_t)keep * m->key_dim * 4, hipMemcpyDeviceToDevice, st));
      ASH_HIP(hipMemcpyAsync(heap, m->heap, (size_t)keep * 4, hipMemcpyDeviceToDevice, st));
      for (int j = 0; j < m->n_values; ++j)
        ASH_HIP(hipMemcpyAsync(vB[j], m->vB[j], (size_t)keep * m->row_bytes[j], hipMemcpyDeviceToDevice, st));
    }
    if (new_c > keep) ASH_HIP(ash::launch_iota(heap, (uint32_t)keep, (uint32_t)new_c, st));
    // a zero owner entry carries epoch 0, older than every erase call
    ASH_HIP(ash::launch_fill_u32((uint32_t*)owner, 0u, (size_t)new_c * 2, st));
    m->erase_epoch = 0;
    m->mem.put(m->kB, st);
    m->mem.put(m->heap, st);
    m->mem.put(m->owner, st);
    for (uint8_t* p : m->vB) m->mem.put(p, st);
    m->kB = kB;
    m->heap = heap;
    m->owner = owner;
    m->vB = vB;
    m->c = new_c;
    ASH_TRY(ensure_scratch(m, 0, st));
  }
  return rebuild_table(m, live, st);
}

// Keeps probe sequences short under erase churn: when the slots that may be
// in use after this insert could pass a quarter of the way from the live
// limit c to a full table (5/8 of the slots at max_load 0.5), count them
// exactly and, if needed, rebuild without tombstones.  Linear probing forms
// long clusters as occupancy rises: at 3/4 of the slots the longest probe of
// a few hundred random misses is about twice as long as at 5/8.
ash_status_t maybe_clean(ash_map* m, int64_t n, hipStream_t st) {
  const int64_t limit = m->c + ((int64_t)m->nslots - m->c) / 4;
  if (m->used_ub + std::min(n, m->c) <= limit) return ASH_OK;
  Meta h;
  ASH_TRY(read_meta(m, &h, st));
  if ((int64_t)h.used + std::min<int64_t>(n, m->c - h.t) <= limit) return ASH_OK;
  // the device's count is a bound too (inserts reuse tombstones): count exactly
  ASH_HIP(ash::launch_count_slots(m->key_dim, m->ref(), m->meta, st));
  ASH_TRY(read_meta(m, &h, st));
  if ((int64_t)h.used + std::min<int64_t>(n, m->c - h.t) <= limit) return ASH_OK;
  return rebuild_table(m, h.t, st);
}

ash_status_t check_keys(ash_map* m, const int32_t* keys, int64_t n) {
  if (!m) return ASH_E_INVALID;
  if (n < 0 || n > kMaxCount) return ASH_E_INVALID;
  if (n > 0 && !keys) return ASH_E_INVALID;
  return ASH_OK;
}

ValueSet make_values(const ash_map* m, const void* const* src, void* const* dst, bool to_buffer) {
  ValueSet vs;
  std::memset(&vs, 0, sizeof(vs));
  vs.n = m->n_values;
  for (int j = 0; j < m->n_values; ++j) {
    const uint8_t* s = to_buffer ? (const uint8_t*)src[j] : m->vB[j];
    uint8_t* d = to_buffer ? m->vB[j] : (uint8_t*)dst[j];
    vs.src[j] = s;
    vs.dst[j] = d;
    vs.row_bytes[j] = m->row_bytes[j];
    vs.vec[j] = copy_unit(m->row_bytes[j], s, d);
    vs.units_log2[j] = units_log2(m->row_bytes[j], vs.vec[j]);
  }
  return vs;
}

ash_status_t insert_impl(ash_map* m, const int32_t* keys, int64_t n, const void* const* values, int32_t* out_idx,
                         uint8_t* out_mask, hipStream_t st, const RequestSource* rs) {
  if (rs) {
    if (!m || n < 0 || n > kMaxCount || !rs->args || rs->nreq < 1 || (rs->args->nreq == 0 && !rs->d) ||
        (m->flags & ASH_F_AUTOGROW) || (m->flags & ASH_F_LDS_DEDUP))
      return ASH_E_INVALID;
  } else {
    ASH_TRY(check_keys(m, keys, n));
  }
  if (n == 0) return ASH_OK;
  if (values) {
    for (int j = 0; j < m->n_values; ++j)
      if (!values[j]) return ASH_E_INVALID;
  }
  ValueSet vs;
  std::memset(&vs, 0, sizeof(vs));
  if (rs) vs = rs->vs;
  else if (values && m->n_values > 0) vs = make_values(m, values, nullptr, true);
  ASH_TRY(ensure_scratch(m, n, st));
  ASH_TRY(maybe_clean(m, n, st));
  // Keeping pending keys in their slots pays when most positions repeat a
  // key (the later copies compare against the slot instead of reading the
  // batch) and costs a store per repeated key otherwise: measured on 10M
  // keys, the claim takes 280 against 379 us with 90% repeats, 497 against
  // 466 us with 50%.  The last finalized insert's new-key fraction (possibly
  // an earlier call's) decides; results do not depend on the choice.
  {
    const volatile Meta* mr = m->mirror_h;
    const uint64_t last_n = mr->last_n, last_new = mr->result;
    m->keyed = last_n > 0 && last_new * 10 <= last_n * 4;
    if (m->keyed_override >= 0) m->keyed = m->keyed_override != 0;
  }
  const uint32_t un = (uint32_t)n;
  const uint32_t blocks = ash::claim_blocks(m->G, un);
  auto claim = [&]() -> ash_status_t {
    // the profile names the claim variant that ran (results are the same)
    const char* label = m->tombs_possible ? "claim_reuse" : (m->keyed ? "claim_keyed" : "claim");
    ASH_HIP(timed(m, label, st, [&] {
      if (rs)
        return ash::launch_claim_requests(m->key_dim, m->G, m->W, m->ref(), *rs->args, rs->d, rs->nreq, un,
                                          m->slot_of, m->lost, m->partial, m->meta, st);
      return ash::launch_claim(m->key_dim, m->G, m->W, m->ref(), keys, un, m->slot_of, m->lost, m->partial, m->meta,
                               st);
    }));
    return ASH_OK;
  };
  auto sum = [&]() -> ash_status_t {
    ASH_HIP(timed(m, "sum_partials", st, [&] { return ash::launch_sum_partials(m->partial, blocks, m->meta, st); }));
    return ASH_OK;
  };
  auto commit = [&](int check, int silent, int32_t* oi, uint8_t* om) -> ash_status_t {
    // Rows of 64 bytes or more move in a separate pass over the winners, whose
    // positions go to aux (erase's scratch, idle during an insert); shorter
    // rows are copied inside the commit.
    uint32_t row_total = 0;
    for (int j = 0; j < vs.n; ++j) row_total += vs.row_bytes[j];
    if (rs) {
      if (row_total >= kSplitRowBytes) return ASH_E_INVALID;  // request rows are copied inside the commit only
      ASH_HIP(timed(m, "commit", st, [&] {
        return ash::launch_commit_requests(m->key_dim, m->ref(), *rs->args, rs->d, rs->nreq, un, m->slot_of, m->lost,
                                           m->kB, m->heap, (uint32_t)m->c, vs, m->meta, m->scan_status, check, silent,
                                           st);
      }));
      return ASH_OK;
    }
    uint32_t* wlist = row_total >= kSplitRowBytes ? reinterpret_cast<uint32_t*>(m->aux) : nullptr;
    ASH_HIP(timed(m, "commit", st, [&] {  // its last tile also finalizes the insert
      return ash::launch_commit(m->key_dim, m->ref(), keys, un, m->slot_of, m->lost, m->kB, m->heap,
                                (uint32_t)m->c, vs, oi, om, m->meta, m->scan_status, check, wlist, silent, st);
    }));
    if (wlist)
      ASH_HIP(timed(m, "values", st, [&] {
        return ash::launch_scatter_values(vs, wlist, m->heap, m->meta, un, (uint32_t)m->c, st);
      }));
    return ASH_OK;
  };
  // The capacity check needs the batch's count of new keys; when the host's
  // bound on t plus n fits in c it cannot fail and the count is skipped.
  int check = m->live_ub + n > m->c ? 1 : 0;
  if (check && (m->flags & ASH_F_AUTOGROW)) {
    Meta h;
    ASH_TRY(read_meta(m, &h, st));
    check = (int64_t)h.t + n > m->c ? 1 : 0;
    if (check) {
      // The counting claim must not run out of slots: give the table room for
      // every position of the batch first.
      if ((int64_t)h.used + n > (int64_t)m->c + ((int64_t)m->nslots - m->c) / 2)
        ASH_TRY(rebuild_table(m, h.t, st, (int64_t)h.t + n));
      ASH_TRY(claim());
      ASH_TRY(sum());
      ASH_TRY(read_meta(m, &h, st));
      if (!h.fail && (int64_t)h.t + h.claims > m->c) {
        // Roll the claims back silently, grow x2 until the batch fits, redo.
        const int64_t need = (int64_t)h.t + h.claims;
        ASH_TRY(commit(1, 1, nullptr, nullptr));
        int64_t new_c = std::max<int64_t>(m->c, 1);
        while (new_c < need) new_c *= 2;
        if (new_c > kMaxCount) return ASH_E_CAPACITY;
        ASH_TRY(grow(m, new_c, st));
        if (values && m->n_values > 0) vs = make_values(m, values, nullptr, true);
        ASH_TRY(ensure_scratch(m, n, st));
        ASH_TRY(claim());
        check = 0;
      }
      ASH_TRY(commit(check, 0, out_idx, out_mask));
      m->live_ub = std::min(m->c, m->live_ub + n);
      m->used_ub += std::min(n, m->c);
      return ASH_OK;
    }
  }
  ASH_TRY(claim());
  if (check) ASH_TRY(sum());
  ASH_TRY(commit(check, 0, out_idx, out_mask));
  m->live_ub = std::min(m->c, m->live_ub + n);
  m->used_ub += std::min(n, m->c);
  return ASH_OK;
}

ash_status_t reset_state(ash_map* m, hipStream_t st) {
  ASH_HIP(ash::launch_clear_map(m->table, (size_t)m->nslots * m->slot_words(), m->heap, (uint32_t)m->c, m->meta,
                                st));
  m->live_ub = 0;
  m->used_ub = 0;
  m->tombs_possible = false;
  return ASH_OK;
}

ash_status_t erase_impl(ash_map* m, const int32_t* keys, int64_t n, uint8_t* out_mask, hipStream_t st,
                        const RequestSource* rs) {
  if (rs) {
    if (!m || n < 0 || n > kMaxCount || !rs->args || rs->nreq < 1 || (rs->args->nreq == 0 && !rs->d))
      return ASH_E_INVALID;
  } else {
    ASH_TRY(check_keys(m, keys, n));
  }
  if (n == 0) return ASH_OK;
  ASH_TRY(ensure_scratch(m, n, st));
  const uint32_t un = (uint32_t)n;
  if (++m->erase_epoch == 0) {  // epochs wrapped: start the owner entries afresh
    ASH_HIP(ash::launch_fill_u32((uint32_t*)m->owner, 0u, (size_t)m->c * 2, st));
    m->erase_epoch = 1;
  }
  const uint32_t epoch = m->erase_epoch;
  ASH_HIP(timed(m, "erase_mark", st, [&] {
    if (rs)
      return ash::launch_erase_mark_requests(m->key_dim, m->G, m->W, m->ref(), *rs->args, rs->d, rs->nreq, un, epoch,
                                             m->slot_of, m->aux, m->owner, m->lost, st);
    return ash::launch_erase_mark(m->key_dim, m->G, m->W, m->ref(), keys, un, epoch, m->slot_of, m->aux, m->owner,
                                  m->lost, st);
  }));
  m->tombs_possible = true;
  ASH_HIP(timed(m, "erase_commit", st, [&] {  // its last tile also finalizes the erase
    if (rs)
      return ash::launch_erase_commit_requests(m->key_dim, m->ref(), *rs->args, rs->d, rs->nreq, un, m->slot_of,
                                               m->aux, m->lost, m->heap, m->meta, m->scan_status, st);
    return ash::launch_erase_commit(m->key_dim, m->ref(), un, m->slot_of, m->aux, m->lost, m->heap, out_mask, m->meta,
                                    m->scan_status, st);
  }));
  return ASH_OK;
}

}  // namespace ash_host

extern "C" {

ash_status_t ash_create(int64_t capacity, int32_t key_dim, int32_t n_values, const ash_dtype_t* value_dtypes,
                        const int64_t* value_elems, const ash_allocator_t* allocator, const ash_tuning_t* tuning,
                        void* stream, ash_map_t* out) {
  if (!out || capacity < 0 || capacity > kMaxCount || key_dim < 1 || key_dim > 4) return ASH_E_INVALID;
  if (n_values < 0 || n_values > ash::kMaxValues) return ASH_E_INVALID;
  if (n_values > 0 && (!value_dtypes || !value_elems)) return ASH_E_INVALID;
  if (allocator && (!allocator->alloc || !allocator->free)) return ASH_E_INVALID;
  std::vector<uint32_t> rb(n_values);
  for (int j = 0; j < n_values; ++j) {
    const size_t es = dtype_size(value_dtypes[j]);
    if (es == 0 || value_elems[j] <= 0) return ASH_E_INVALID;
    const uint64_t bytes = es * (uint64_t)value_elems[j];
    if (bytes > (1u << 24)) return ASH_E_UNSUPPORTED;
    rb[j] = (uint32_t)bytes;
  }
  int W = 4, G = 4;
  float lf = 0.5f;
  uint32_t flags = 0;
  if (tuning) {
    W = tuning->bucket_width;
    G = tuning->probe_group;
    lf = tuning->max_load;
    flags = tuning->flags;
  }
  if (!pow2(W) || W > 64) return ASH_E_INVALID;
  if (G != 1 && G != 4 && G != 8 && G != 16 && G != 32 && G != 64) return ASH_E_INVALID;
  if (G == 1 && W != 2 && W != 4 && W != 8) return ASH_E_INVALID;  // one lane reads a bucket
  if (!(lf >= 0.1f && lf <= 0.9f)) return ASH_E_INVALID;
  if (flags & ~(ASH_F_AUTOGROW | ASH_F_LDS_DEDUP)) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;

  ash_map* m = new ash_map;
  m->mem.custom = allocator != nullptr;
  if (allocator) m->mem.a = *allocator;
  m->c = capacity;
  m->key_dim = key_dim;
  m->n_values = n_values;
  m->row_bytes = rb;
  m->dtypes.assign(value_dtypes, value_dtypes + n_values);
  m->elems.assign(value_elems, value_elems + n_values);
  m->W = W;
  m->G = G;
  m->max_load = lf;
  m->flags = flags;
  m->vB.assign(n_values, nullptr);
  {
    const char* v = std::getenv("ASH_CLAIM_KEYED");
    if (v && (v[0] == '0' || v[0] == '1') && v[1] == '\0') m->keyed_override = v[0] - '0';
  }
  ash_status_t s = slots_for(capacity, lf, W, G, &m->nslots);
  if (s != ASH_OK) {
    delete m;
    return s;
  }
  m->table = (uint32_t*)m->mem.get((size_t)m->nslots * m->slot_words() * 4, st);
  m->kB = (int32_t*)m->mem.get((size_t)capacity * key_dim * 4, st);
  m->heap = (int32_t*)m->mem.get((size_t)capacity * 4, st);
  m->owner = (uint64_t*)m->mem.get((size_t)capacity * 8, st);
  m->meta = (Meta*)m->mem.get(sizeof(Meta), st);
  bool ok = m->table && m->kB && m->heap && m->owner && m->meta;
  for (int j = 0; j < n_values && ok; ++j) {
    m->vB[j] = (uint8_t*)m->mem.get((size_t)capacity * rb[j], st);
    ok = m->vB[j] != nullptr;
  }
  if (ok) ok = ensure_scratch(m, 0, st) == ASH_OK;
  if (ok) {
    ok = hipHostMalloc((void**)&m->mirror_h, sizeof(Meta), hipHostMallocDefault) == hipSuccess;
    if (!ok) m->mirror_h = nullptr;
    if (ok) {
      std::memset(m->mirror_h, 0, sizeof(Meta));
      ok = hipHostGetDevicePointer((void**)&m->mirror, m->mirror_h, 0) == hipSuccess;
    }
  }
  if (!ok) {
    ash_destroy(m);
    return ASH_E_NOMEM;
  }
  if (ash::launch_fill_u32((uint32_t*)m->meta, 0u, sizeof(Meta) / 4, st) != hipSuccess ||
      ash::launch_fill_u32((uint32_t*)m->owner, 0u, (size_t)capacity * 2, st) != hipSuccess ||
      reset_state(m, st) != ASH_OK || hipStreamSynchronize(st) != hipSuccess) {
    ash_destroy(m);
    return ASH_E_DEVICE;
  }
  *out = m;
  return ASH_OK;
}

ash_status_t ash_destroy(ash_map_t m) {
  if (!m) return ASH_E_INVALID;
  hipStream_t st = nullptr;
  free_buffers(m, st);
  m->mem.put(m->meta, st);
  m->mem.put(m->slot_of, st);
  m->mem.put(m->aux, st);
  m->mem.put(m->partial, st);
  m->mem.put(m->lost, st);
  m->mem.put(m->scan_status, st);
  m->mem.put(m->batch_dev, st);
  for (hipEvent_t e : m->prof.pool) (void)hipEventDestroy(e);
  if (m->mirror_h || m->batch_host) {
    (void)hipDeviceSynchronize();  // no finalize may still write the mirror
    if (m->mirror_h) (void)hipHostFree(m->mirror_h);
    if (m->batch_host) (void)hipHostFree(m->batch_host);
  }
  delete m;
  return ASH_OK;
}

ash_status_t ash_profile_enable(ash_map_t m, int32_t enable) {
  if (!m) return ASH_E_INVALID;
  m->prof.on = enable != 0;
  return ASH_OK;
}

ash_status_t ash_profile_collect(ash_map_t m, ash_kernel_time_t* out, int32_t max_entries, int32_t* n_entries,
                                 void* stream) {
  if (!m || !n_entries || max_entries < 0 || (max_entries > 0 && !out)) return ASH_E_INVALID;
  ASH_HIP(hipStreamSynchronize((hipStream_t)stream));
  std::vector<ash_kernel_time_t> agg;
  for (const ProfRec& r : m->prof.recs) {
    float ms = 0.0f;
    ASH_HIP(hipEventSynchronize(r.stop));
    ASH_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    size_t k = 0;
    while (k < agg.size() && std::strcmp(agg[k].name, r.name) != 0) ++k;
    if (k == agg.size()) {
      ash_kernel_time_t t;
      std::memset(&t, 0, sizeof(t));
      std::strncpy(t.name, r.name, sizeof(t.name) - 1);
      agg.push_back(t);
    }
    agg[k].launches += 1;
    agg[k].total_ms += ms;
  }
  m->prof.recs.clear();
  m->prof.used = 0;
  const int32_t n = (int32_t)std::min<size_t>(agg.size(), (size_t)max_entries);
  for (int32_t k = 0; k < n; ++k) out[k] = agg[k];
  *n_entries = n;
  return ASH_OK;
}

ash_status_t ash_insert(ash_map_t m, const int32_t* keys, int64_t n, const void* const* values, int32_t* out_idx,
                        uint8_t* out_mask, void* stream) {
  if (m && m->n_values > 0 && n > 0 && !values) return ASH_E_INVALID;
  return insert_impl(m, keys, n, m && m->n_values > 0 ? values : nullptr, out_idx, out_mask, (hipStream_t)stream);
}

ash_status_t ash_activate(ash_map_t m, const int32_t* keys, int64_t n, int32_t* out_idx, uint8_t* out_mask,
                          void* stream) {
  return insert_impl(m, keys, n, nullptr, out_idx, out_mask, (hipStream_t)stream);
}

ash_status_t ash_find(ash_map_t m, const int32_t* keys, int64_t n, int32_t* out_idx, uint8_t* out_mask,
                      void* const* out_values, void* stream) {
  ASH_TRY(check_keys(m, keys, n));
  if (n == 0) return ASH_OK;
  hipStream_t st = (hipStream_t)stream;
  ValueSet vs;
  std::memset(&vs, 0, sizeof(vs));
  if (out_values && m->n_values > 0) {
    for (int j = 0; j < m->n_values; ++j)
      if (!out_values[j]) return ASH_E_INVALID;
    vs = make_values(m, nullptr, out_values, false);
  }
  uint32_t row_total = 0;
  for (int j = 0; j < vs.n; ++j) row_total += vs.row_bytes[j];
  if (vs.n > 0 && find_rows_apart(row_total, n)) {
    // Long rows move in a pass of their own, sized by the bytes to copy (the
    // find's blocks alone leave most of the chip idle when n is small).
    int32_t* idx = out_idx;
    if (!idx) {
      ASH_TRY(ensure_scratch(m, n, st));
      idx = m->aux;
    }
    ValueSet none;
    std::memset(&none, 0, sizeof(none));
    ASH_HIP(timed(m, "find", st, [&] {
      return ash::launch_find(m->key_dim, m->G, m->W, m->ref(), keys, (uint32_t)n, idx, out_mask, none, st);
    }));
    ASH_HIP(timed(m, "gather", st, [&] { return ash::launch_gather_rows(vs, idx, (uint32_t)n, (uint32_t)m->c, st); }));
    return ASH_OK;
  }
  ASH_HIP(timed(m, "find", st, [&] { return ash::launch_find(m->key_dim, m->G, m->W, m->ref(), keys, (uint32_t)n, out_idx, out_mask, vs, st); }));
  return ASH_OK;
}

ash_status_t ash_erase(ash_map_t m, const int32_t* keys, int64_t n, uint8_t* out_mask, void* stream) {
  return erase_impl(m, keys, n, out_mask, (hipStream_t)stream);
}

ash_status_t ash_find_offsets(ash_map_t m, const int32_t* keys, int64_t n, const int32_t* offsets, int32_t n_offsets,
                              int32_t* out_idx, uint8_t* out_mask, void* stream) {
  ASH_TRY(check_keys(m, keys, n));
  if (n_offsets < 0 || (n_offsets > 0 && !offsets)) return ASH_E_INVALID;
  if (n_offsets > 0 && n > kMaxCount / n_offsets) return ASH_E_INVALID;
  const int64_t total = n * n_offsets;
  if (total == 0) return ASH_OK;
  hipStream_t st = (hipStream_t)stream;
  ASH_HIP(timed(m, "find_offsets", st, [&] {
    return ash::launch_find_offsets(m->key_dim, m->G, m->W, m->ref(), keys, offsets, (uint32_t)n_offsets,
                                    (uint32_t)total, out_idx, out_mask, st);
  }));
  return ASH_OK;
}

ash_status_t ash_intersect(ash_map_t m, const int32_t* keys, int64_t n, int32_t* out_keys, int64_t* out_count,
                           void* stream) {
  ASH_TRY(check_keys(m, keys, n));
  if (!out_count || (n > 0 && !out_keys)) return ASH_E_INVALID;
  if (n == 0) {
    *out_count = 0;
    return ASH_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  ASH_TRY(ensure_scratch(m, n, st));  // look-back status words for n positions
  uint8_t* mask = (uint8_t*)m->mem.get((size_t)n, st);
  if (!mask) return ASH_E_NOMEM;
  ValueSet none;
  std::memset(&none, 0, sizeof(none));
  ash_status_t rc = ASH_OK;
  if (timed(m, "find", st, [&] {
        return ash::launch_find(m->key_dim, m->G, m->W, m->ref(), keys, (uint32_t)n, nullptr, mask, none, st);
      }) != hipSuccess ||
      timed(m, "compact_rows", st, [&] {  // its last tile writes the count
        return ash::launch_compact_rows(m->key_dim, mask, (uint32_t)n, keys, out_keys, m->meta, m->scan_status, st);
      }) != hipSuccess)
    rc = ASH_E_DEVICE;
  Meta h;
  if (rc == ASH_OK) rc = read_meta(m, &h, st);
  m->mem.put(mask, st);
  if (rc == ASH_OK) *out_count = h.result;
  return rc;
}

ash_status_t ash_block_coords(const float* points, int64_t n, float voxel_size, int32_t block_res,
                              int32_t* out_block_keys, int32_t* out_local, uint8_t* out_valid, void* stream) {
  if (n < 0 || n > kMaxCount || block_res < 1 || !(voxel_size > 0.0f) || !std::isfinite(voxel_size))
    return ASH_E_INVALID;
  if (n > 0 && (!points || !out_block_keys || !out_local || !out_valid)) return ASH_E_INVALID;
  if (n == 0) return ASH_OK;
  ASH_HIP(ash::launch_block_coords(points, (uint32_t)n, voxel_size, block_res, out_block_keys, out_local, out_valid,
                                   (hipStream_t)stream));
  return ASH_OK;
}

ash_status_t ash_neighbor_offsets(int32_t kind, int32_t radius, int32_t key_dim, int32_t* out_offsets,
                                  int64_t* out_count) {
  if (!out_count || key_dim < 1 || key_dim > 4 || radius < 1 || radius > 64) return ASH_E_INVALID;
  if (kind != ASH_NB_RADIUS && kind != ASH_NB_CUBE && kind != ASH_NB_RING) return ASH_E_INVALID;
  // candidates: every word in [lo, radius], enumerated with the first word slowest
  const int64_t lo = kind == ASH_NB_CUBE ? 0 : -radius;
  const int64_t side = radius - lo + 1;
  int64_t cand = 1;
  for (int d = 0; d < key_dim; ++d) cand *= side;  // <= 129^4
  if (cand > kMaxNeighborCandidates) return ASH_E_INVALID;
  int64_t count = 0;
  int32_t w[4];
  for (int64_t c = 0; c < cand; ++c) {
    int64_t r = c, l1 = 0;
    for (int d = key_dim - 1; d >= 0; --d) {
      w[d] = (int32_t)(lo + r % side);
      r /= side;
      l1 += w[d] < 0 ? -w[d] : w[d];
    }
    if (kind == ASH_NB_RING && (l1 == 0 || l1 > radius)) continue;
    if (count >= kMaxNeighborOffsets) return ASH_E_INVALID;
    if (out_offsets)
      for (int d = 0; d < key_dim; ++d) out_offsets[count * key_dim + d] = w[d];
    ++count;
  }
  *out_count = count;
  return ASH_OK;
}

ash_status_t ash_active_indices(ash_map_t m, int32_t* out_idx, int64_t* out_count, void* stream) {
  if (!m || !out_count || (m->c > 0 && !out_idx)) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  if (m->c == 0) {
    *out_count = 0;
    return ASH_OK;
  }
  const size_t flag_bytes = ((size_t)m->c + 3) / 4 * 4;
  uint8_t* flags = (uint8_t*)m->mem.get(flag_bytes, st);
  if (!flags) return ASH_E_NOMEM;
  const uint32_t last_tile = (uint32_t)((m->c + ash::kScanTile - 1) / ash::kScanTile - 1);
  ash_status_t rc = ASH_OK;
  if (ash::launch_fill_u32((uint32_t*)flags, 0u, flag_bytes / 4, st) != hipSuccess ||
      timed(m, "active_indices", st, [&] {
        return ash::launch_active_indices(m->key_dim, m->ref(), flags, (uint32_t)m->c, out_idx, m->meta,
                                          m->scan_status, st);
      }) != hipSuccess ||
      timed(m, "finalize", st, [&] {
        return ash::launch_finalize(m->meta, (uint32_t)m->c, ash::kFinalizeCount, 0, 0, m->scan_status, last_tile, st);
      }) != hipSuccess)
    rc = ASH_E_DEVICE;
  Meta h;
  if (rc == ASH_OK) rc = read_meta(m, &h, st);
  m->mem.put(flags, st);
  if (rc == ASH_OK) *out_count = h.result;
  return rc;
}

ash_status_t ash_rehash(ash_map_t m, int64_t new_capacity, void* stream) {
  if (!m || new_capacity < 0) return ASH_E_INVALID;
  return grow(m, new_capacity, (hipStream_t)stream);
}

ash_status_t ash_clear(ash_map_t m, void* stream) {
  if (!m) return ASH_E_INVALID;
  return reset_state(m, (hipStream_t)stream);
}

ash_status_t ash_size(ash_map_t m, int64_t* out, void* stream) {
  if (!m || !out) return ASH_E_INVALID;
  Meta h;
  ASH_TRY(read_meta(m, &h, (hipStream_t)stream));
  *out = h.t;
  return ASH_OK;
}

ash_status_t ash_capacity(ash_map_t m, int64_t* out) {
  if (!m || !out) return ASH_E_INVALID;
  *out = m->c;
  return ASH_OK;
}

ash_status_t ash_stats(ash_map_t m, ash_stats_t* out, void* stream) {
  if (!m || !out) return ASH_E_INVALID;
  Meta h;
  ASH_HIP(ash::launch_count_slots(m->key_dim, m->ref(), m->meta, (hipStream_t)stream));
  ASH_TRY(read_meta(m, &h, (hipStream_t)stream));
  out->size = h.t;
  out->capacity = m->c;
  out->slots = m->nslots;
  out->used_slots = h.used;
  out->tombstones = h.tombs;
  return ASH_OK;
}

ash_status_t ash_key_buffer(ash_map_t m, int32_t** out) {
  if (!m || !out) return ASH_E_INVALID;
  *out = m->kB;
  return ASH_OK;
}

ash_status_t ash_value_buffer(ash_map_t m, int32_t j, void** out) {
  if (!m || !out || j < 0 || j >= m->n_values) return ASH_E_INVALID;
  *out = m->vB[j];
  return ASH_OK;
}

ash_status_t ash_heap_buffer(ash_map_t m, int32_t** out) {
  if (!m || !out) return ASH_E_INVALID;
  *out = m->heap;
  return ASH_OK;
}

ash_status_t ash_device_status(ash_map_t m, void* stream) {
  if (!m) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  Meta h;
  ASH_TRY(read_meta(m, &h, st));
  if (h.status == 0) return ASH_OK;
  const uint32_t zero = 0;
  ASH_HIP(hipMemcpyAsync(&m->meta->status, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
  ASH_HIP(hipStreamSynchronize(st));
  return (h.status & (ash::kStatusScanStall | ash::kStatusGridStall)) ? ASH_E_DEVICE : ASH_E_CAPACITY;
}

}  // extern "C"

namespace {

// Workspace of one voxelization over n points (one block, 256-byte aligned
// parts): the slot table (16 B slots, max load 0.5, W = g = 4), slot_of,
// per-block claim counts, lost bytes, and the scan status words followed by
// the Meta of the call.
struct VoxelWork {
  uint32_t nslots = 0;
  size_t table = 0, slot_of = 0, partial = 0, lost = 0, status = 0, bytes = 0;
  int64_t tiles = 0;
  size_t lost_bytes = 0;
};

constexpr int kVoxW = 4, kVoxG = 4;  // four lanes per point, 4-slot buckets:
// against one lane per point, equal at 5 mm and 1 cm, 3% faster at 2 cm and
// 8% at 5 cm (5M points)
constexpr float kVoxLoad = 0.5f;

ash_status_t voxel_work(int64_t n, VoxelWork* w) {
  ASH_TRY(slots_for(n, kVoxLoad, kVoxW, kVoxG, &w->nslots));
  if (w->nslots >= 0x7FFFFFFFu) return ASH_E_UNSUPPORTED;  // slot_of keeps a candidate bit
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  w->tiles = (n + ash::kScanTile - 1) / ash::kScanTile;
  w->lost_bytes = ((size_t)n + 3) / 4 * 4;
  const uint32_t blocks = ash::claim_blocks(kVoxG, (uint32_t)n);
  size_t o = 0;
  w->table = o;
  o += up((size_t)w->nslots * 16);
  w->slot_of = o;
  o += up((size_t)n * 4);
  w->partial = o;
  o += up((size_t)blocks * 4);
  w->lost = o;
  o += up(w->lost_bytes);
  w->status = o;
  o += up((size_t)w->tiles * 8 + sizeof(Meta));
  w->bytes = o;
  return ASH_OK;
}

// The kernels of one voxelization on a workspace laid out by voxel_work.
ash_status_t voxelize_run(const float* points, int64_t n, float voxel, int32_t* out_point_voxel,
                          int32_t* out_voxel_keys, int32_t* out_voxel_counts, int64_t* out_n_voxels,
                          const VoxelWork& w, uint8_t* base, hipStream_t st) {
  const uint32_t un = (uint32_t)n;
  uint32_t* table = (uint32_t*)(base + w.table);
  uint32_t* slot_of = (uint32_t*)(base + w.slot_of);
  uint32_t* partial = (uint32_t*)(base + w.partial);
  uint8_t* lost = base + w.lost;
  uint64_t* status = (uint64_t*)(base + w.status);
  Meta* meta = (Meta*)(status + w.tiles);
  TableRef tb;
  tb.words = table;
  tb.nslots = w.nslots;
  tb.bucket_width = kVoxW;
  tb.nbuckets = w.nslots / kVoxW;
  tb.window = kVoxG == 1 ? kVoxW : kVoxG;
  tb.max_windows = w.nslots / tb.window + 1;
  tb.dedup = kVoxelDedup;
  tb.reuse = 0;
  tb.keyed = 1;  // (the voxel claim always keeps pending keys in their slots)
  tb.mirror = nullptr;
  Meta h;
  // every part that must start in a known state is written here by kernels
  // (the workspace may hold an earlier call's contents): an empty table,
  // zero status words and lost bytes, and zero counters with epoch 1
  // (one launch: the lost bytes and the status words are one range, the
  // counters follow it)
  const bool ok = ash::launch_voxel_init(table, (size_t)w.nslots * 4, (uint32_t*)lost,
                                         (w.status - w.lost) / 4 + (size_t)w.tiles * 2, meta, st) == hipSuccess &&
                  ash::launch_voxel_claim(kVoxG, kVoxW, tb, points, voxel, un, slot_of, lost, partial, meta, st) ==
                      hipSuccess &&
                  ash::launch_voxel_commit(tb, points, voxel, un, slot_of, lost, out_voxel_keys, out_voxel_counts,
                                           out_point_voxel, meta, status, st) == hipSuccess &&
                  ash::launch_voxel_resolve(tb, un, slot_of, out_point_voxel, out_voxel_counts, st) == hipSuccess &&
                  hipMemcpyAsync(&h, meta, sizeof(Meta), hipMemcpyDeviceToHost, st) == hipSuccess &&
                  hipStreamSynchronize(st) == hipSuccess;
  if (!ok) return ASH_E_DEVICE;
  if (h.status & ash::kStatusScanStall) return ASH_E_DEVICE;  // a look-back wait hit its bound: ids not valid
  if (h.fail) return ASH_E_CAPACITY;
  *out_n_voxels = h.claims;
  return ASH_OK;
}

ash_status_t voxelize_args(const float* points, int64_t n, float voxel, int32_t* out_point_voxel,
                           int32_t* out_voxel_keys, int32_t* out_voxel_counts, int64_t* out_n_voxels) {
  if (!out_n_voxels || n < 0 || n > kMaxCount) return ASH_E_INVALID;
  if (!(voxel > 0.0f) || !std::isfinite(voxel)) return ASH_E_INVALID;
  if (n > 0 && (!points || !out_point_voxel || !out_voxel_keys || !out_voxel_counts)) return ASH_E_INVALID;
  return ASH_OK;
}

// Workspace of ash_voxelize_noalloc: a file-scope device array of which each
// GPU holds its own copy (at its own address) until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it is
// a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns on each device, taken once per device with that
// device current and kept in g_scratch_at.  Every call on one GPU shares the
// array, so calls that overlap on one GPU race.
constexpr int64_t kNoAllocVoxelPoints = 1 << 20;
constexpr size_t kNoAllocVoxelBytes = 38ull << 20;  // voxel_work(2^20 points) takes 37.1 MiB
__device__ __align__(256) uint8_t scratch[kNoAllocVoxelBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_at[kMaxDevices] = {};

ash_status_t scratch_address(uint8_t** out) {
  int dev = 0;
  ASH_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return ASH_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ASH_E_DEVICE;
    g_scratch_at[dev] = (uint8_t*)p;
  }
  *out = g_scratch_at[dev];
  return ASH_OK;
}

}  // namespace

extern "C" {

ash_status_t ash_voxelize_noalloc(const float* points, int64_t n, float voxel, int32_t* out_point_voxel,
                                  int32_t* out_voxel_keys, int32_t* out_voxel_counts, int64_t* out_n_voxels,
                                  void* stream) {
  ASH_TRY(voxelize_args(points, n, voxel, out_point_voxel, out_voxel_keys, out_voxel_counts, out_n_voxels));
  if (n > kNoAllocVoxelPoints) return ASH_E_UNSUPPORTED;
  if (n == 0) {
    *out_n_voxels = 0;
    return ASH_OK;
  }
  VoxelWork w;
  ASH_TRY(voxel_work(n, &w));
  if (w.bytes > kNoAllocVoxelBytes) return ASH_E_UNSUPPORTED;
  uint8_t* base = nullptr;
  ASH_TRY(scratch_address(&base));
  // voxelize_run writes every part of the workspace that must start in a
  // known state (table, status words, lost bytes, counters) with kernels
  return voxelize_run(points, n, voxel, out_point_voxel, out_voxel_keys, out_voxel_counts, out_n_voxels, w, base,
                      (hipStream_t)stream);
}

ash_status_t ash_voxelize(const float* points, int64_t n, float voxel, int32_t* out_point_voxel,
                          int32_t* out_voxel_keys, int32_t* out_voxel_counts, int64_t* out_n_voxels,
                          const ash_allocator_t* allocator, void* stream) {
  ASH_TRY(voxelize_args(points, n, voxel, out_point_voxel, out_voxel_keys, out_voxel_counts, out_n_voxels));
  if (allocator && (!allocator->alloc || !allocator->free)) return ASH_E_INVALID;
  if (n == 0) {
    *out_n_voxels = 0;
    return ASH_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  VoxelWork w;
  ASH_TRY(voxel_work(n, &w));
  DevMem mem;
  mem.custom = allocator != nullptr;
  if (allocator) mem.a = *allocator;
  uint8_t* base = (uint8_t*)mem.get(w.bytes, st);
  if (!base) return ASH_E_NOMEM;
  const ash_status_t rc = voxelize_run(points, n, voxel, out_point_voxel, out_voxel_keys, out_voxel_counts,
                                       out_n_voxels, w, base, st);
  mem.put(base, st);
  return rc;
}

// Blocks of the persistent batched kernel that the device runs all at once,
// found once per (key_dim, build, device): an empty launch at the occupancy
// the runtime reports, lowered one block per CU at a time until every block
// passes the kernel's arrival check.  A failed try costs the barrier's
// bounded wait and touches no map.
std::mutex g_resident_mu;
std::map<std::tuple<int, bool, int>, uint32_t> g_resident;

static ash_status_t batched_resident(int kd, bool narrow, DevMem& mem, hipStream_t st, uint32_t* out) {
  int dev = 0, cus = 0, per_cu = 0;
  ASH_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lock(g_resident_mu);
    auto it = g_resident.find({kd, narrow, dev});
    if (it != g_resident.end()) {
      *out = it->second;
      return ASH_OK;
    }
  }
  ASH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  ASH_HIP(ash::batched_occupancy(kd, narrow, &per_cu));
  if (cus < 1 || per_cu < 1) return ASH_E_DEVICE;
  const size_t gs_bytes = ash::grid_sync_bytes((uint32_t)(cus * per_cu));
  ash::GridSync* gs = (ash::GridSync*)mem.get(gs_bytes, st);
  if (!gs) return ASH_E_NOMEM;
  uint32_t found = 0;
  ash_status_t rc = ASH_OK;
  for (int b = per_cu; b >= 1 && found == 0 && rc == ASH_OK; --b) {
    ash::GridSync h;
    if (ash::launch_fill_u32((uint32_t*)gs, 0u, gs_bytes / 4, st) != hipSuccess ||
        ash::launch_batched(kd, narrow, nullptr, 0, 0, 0, 0, 0, gs, (uint32_t)(cus * b), ash::kArrivalSpinLimit, 0u,
                            st) !=
            hipSuccess ||
        hipMemcpyAsync(&h, gs, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = ASH_E_DEVICE;
    } else if ((h.count & ash::kArrivalFailed) == 0u && h.late == 0u) {  // every block passed every barrier
      found = (uint32_t)(cus * b);
    }
  }
  mem.put(gs, st);
  if (rc != ASH_OK) return rc;
  if (found == 0) return ASH_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_resident_mu);
  g_resident[{kd, narrow, dev}] = found;
  *out = found;
  return ASH_OK;
}

ash_status_t ash_batched_grid(int32_t key_dim, int32_t narrow, int64_t* out_blocks, int64_t* out_reported,
                              void* stream) {
  if (key_dim < 1 || key_dim > 4 || (narrow != 0 && narrow != 1) || !out_blocks) return ASH_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0, per_cu = 0;
  ASH_HIP(hipGetDevice(&dev));
  ASH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  ASH_HIP(ash::batched_occupancy(key_dim, narrow != 0, &per_cu));
  DevMem mem;
  uint32_t resident = 0;
  ASH_TRY(batched_resident(key_dim, narrow != 0, mem, st, &resident));
  *out_blocks = resident;
  if (out_reported) *out_reported = (int64_t)cus * per_cu;
  return ASH_OK;
}

}  // extern "C"

namespace {

// Launches of the persistent batched kernel that failed their arrival check
// and ran op by op instead.
std::atomic<int64_t> batched_fallbacks{0};

// ASH_BATCHED_FORCE_ARRIVAL_FAILURE=1 makes the arrival check of the
// persistent launch fail (its blocks give up without counting themselves
// in), so a test can take the fallback path while every kernel exits
// normally.
uint32_t force_arrival_failure() {
  const char* v = std::getenv("ASH_BATCHED_FORCE_ARRIVAL_FAILURE");
  return v && v[0] == '1' && v[1] == '\0' ? 1u : 0u;
}

// The single-map path, op by op: each op's insert, then its find.
ash_status_t batched_op_by_op(const ash_batch_op_t* ops, int32_t n_ops, hipStream_t st) {
  for (int32_t i = 0; i < n_ops; ++i) {
    const ash_batch_op_t& op = ops[i];
    ASH_TRY(insert_impl(op.map, op.insert_keys, op.n_insert, op.map->n_values > 0 ? op.insert_values : nullptr,
                        op.insert_idx, op.insert_mask, st));
    ASH_TRY(ash_find(op.map, op.find_keys, op.n_find, op.find_idx, op.find_mask, op.find_values, (void*)st));
  }
  return ASH_OK;
}

}  // namespace

extern "C" {

ash_status_t ash_batched(const ash_batch_op_t* ops, int32_t n_ops, int32_t fused, void* stream) {
  if (n_ops < 0 || (n_ops > 0 && !ops)) return ASH_E_INVALID;
  if (n_ops == 0) return ASH_OK;
  hipStream_t st = (hipStream_t)stream;
  const int kd = ops[0].map ? ops[0].map->key_dim : 0;
  std::vector<ash_map*> seen;
  for (int32_t i = 0; i < n_ops; ++i) {
    const ash_batch_op_t& op = ops[i];
    ash_map* m = op.map;
    if (!m || m->key_dim != kd) return ASH_E_INVALID;
    if (m->flags & ASH_F_AUTOGROW) return ASH_E_UNSUPPORTED;
    if (std::find(seen.begin(), seen.end(), m) != seen.end()) return ASH_E_INVALID;
    seen.push_back(m);
    ASH_TRY(check_keys(m, op.insert_keys, op.n_insert));
    ASH_TRY(check_keys(m, op.find_keys, op.n_find));
    if (m->n_values > 0 && op.n_insert > 0) {
      if (!op.insert_values) return ASH_E_INVALID;
      for (int j = 0; j < m->n_values; ++j)
        if (!op.insert_values[j]) return ASH_E_INVALID;
    }
    if (op.find_values)
      for (int j = 0; j < m->n_values; ++j)
        if (!op.find_values[j]) return ASH_E_INVALID;
  }
  if (!fused) return batched_op_by_op(ops, n_ops, st);
  std::vector<ash::BatchItem> items(n_ops);
  uint32_t claim_tiles = 0, commit_tiles = 0, find_tiles = 0;
  int32_t any_check = 0;
  bool narrow = true;  // every map probes one lane per key with W <= 4
  for (int32_t i = 0; i < n_ops; ++i) {
    const ash_batch_op_t& op = ops[i];
    ash_map* m = op.map;
    narrow = narrow && m->G == 1 && (m->W == 2 || m->W == 4);
    ASH_TRY(ensure_scratch(m, std::max<int64_t>(op.n_insert, 1), st));
    ASH_TRY(maybe_clean(m, op.n_insert, st));
    ash::BatchItem& it = items[i];
    std::memset(&it, 0, sizeof(it));
    it.tb = m->ref();
    it.g = m->G;
    it.w = m->W;
    it.cap = (uint32_t)m->c;
    it.check = m->live_ub + op.n_insert > m->c ? 1 : 0;
    any_check |= it.check;
    it.meta = m->meta;
    it.status = m->scan_status;
    it.ikeys = op.insert_keys;
    it.n_insert = (uint32_t)op.n_insert;
    it.claim0 = claim_tiles;
    it.commit0 = commit_tiles;
    it.find0 = find_tiles;
    claim_tiles += (uint32_t)((op.n_insert + 255) / 256);
    commit_tiles += (uint32_t)((op.n_insert + ash::kScanTile - 1) / ash::kScanTile);
    find_tiles += (uint32_t)((op.n_find + 255) / 256);
    it.slot_of = m->slot_of;
    it.lost = m->lost;
    it.partial = m->partial;
    it.kB = m->kB;
    it.heap = m->heap;
    it.iidx = op.insert_idx;
    it.imask = op.insert_mask;
    it.fkeys = op.find_keys;
    it.n_find = (uint32_t)op.n_find;
    it.fidx = op.find_idx;
    it.fmask = op.find_mask;
    if (m->n_values > 0 && op.n_insert > 0) it.vin = make_values(m, op.insert_values, nullptr, true);
    if (m->n_values > 0 && op.find_values) it.vout = make_values(m, nullptr, op.find_values, false);
  }
  ash_map* m0 = ops[0].map;
  uint32_t resident = 0;
  ASH_TRY(batched_resident(kd, narrow, m0->mem, st, &resident));
  const size_t item_bytes = (sizeof(ash::BatchItem) * (size_t)n_ops + 255) / 256 * 256;
  const size_t gs_bytes = ash::grid_sync_bytes(resident);
  const size_t bytes = item_bytes + gs_bytes;
  if (m0->batch_dev_bytes < bytes) {
    m0->mem.put(m0->batch_dev, st);
    m0->batch_dev_bytes = 0;
    m0->batch_dev = (uint8_t*)m0->mem.get(bytes, st);
    if (!m0->batch_dev) return ASH_E_NOMEM;
    m0->batch_dev_bytes = bytes;
  }
  const size_t host_bytes = item_bytes + sizeof(ash::GridSync);
  if (m0->batch_host_bytes < host_bytes) {  // every call ends synchronized, so no copy still reads the old one
    if (m0->batch_host) (void)hipHostFree(m0->batch_host);
    m0->batch_host = nullptr;
    m0->batch_host_bytes = 0;
    ASH_HIP(hipHostMalloc((void**)&m0->batch_host, host_bytes, hipHostMallocDefault));
    m0->batch_host_bytes = host_bytes;
  }
  uint8_t* dev = m0->batch_dev;
  ash::BatchItem* dev_items = (ash::BatchItem*)dev;
  ash::GridSync* gs = (ash::GridSync*)(dev + item_bytes);
  std::memcpy(m0->batch_host, items.data(), sizeof(ash::BatchItem) * (size_t)n_ops);
  ash::GridSync& h = *(ash::GridSync*)(m0->batch_host + item_bytes);
  ash_status_t rc = ASH_OK;
  const uint32_t force_fail = force_arrival_failure();
  if (hipMemcpyAsync(dev_items, m0->batch_host, sizeof(ash::BatchItem) * (size_t)n_ops, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      ash::launch_fill_u32((uint32_t*)gs, 0u, gs_bytes / 4, st) != hipSuccess ||
      timed(m0, "batched", st, [&] {
        return ash::launch_batched(kd, narrow, dev_items, n_ops, claim_tiles, commit_tiles, find_tiles, any_check,
                                   gs, resident, ash::kArrivalSpinLimit, force_fail, st);
      }) != hipSuccess ||
      hipMemcpyAsync(&h, gs, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    rc = ASH_E_DEVICE;
  if (rc != ASH_OK) return rc;
  if (h.count & ash::kArrivalFailed) {
    // The blocks could not all run at once (other work holds CUs): the launch
    // left before touching any map, so the same work runs op by op.
    batched_fallbacks.fetch_add(1);
    return batched_op_by_op(ops, n_ops, st);
  }
  if (h.late) return ASH_E_DEVICE;  // every map of the launch carries kStatusGridStall
  for (int32_t i = 0; i < n_ops; ++i) {
    ash_map* m = ops[i].map;
    m->live_ub = std::min(m->c, m->live_ub + ops[i].n_insert);
    m->used_ub += std::min(ops[i].n_insert, m->c);
  }
  return ASH_OK;
}

int64_t ash_batched_fallbacks(void) { return batched_fallbacks.load(); }

namespace {

// (key_dim, value bytes, log2 capacity, log2 batch, distinct ratio in
// tenths, fused, the swept grid)
typedef std::tuple<int, int64_t, int, int, int, int, std::vector<int32_t>> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<ash_tuning_t, double>> g_tune_cache;

int log2_floor(int64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    ++l;
  }
  return l;
}

// Cube side whose n uniform draws give about `ratio * n` distinct keys:
// L^d (1 - exp(-n / L^d)) = ratio * n, solved for x = n / L^d by bisection.
uint32_t cube_side(int64_t n, int kd, double ratio) {
  ratio = std::min(std::max(ratio, 1e-3), 0.999);
  double lo = 1e-6, hi = 1e3;
  for (int it = 0; it < 200; ++it) {
    const double x = 0.5 * (lo + hi);
    if ((1.0 - std::exp(-x)) / x > ratio) lo = x;
    else hi = x;
  }
  const double cells = (double)n / (0.5 * (lo + hi));
  return (uint32_t)std::max(2.0, std::ceil(std::pow(cells, 1.0 / kd)));
}

// The shapes ash_create accepts, for a sweep.
bool valid_shape(int32_t w, int32_t g, float lf) {
  if (!pow2(w) || w > 64) return false;
  if (g != 1 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64) return false;
  if (g == 1 && w != 2 && w != 4 && w != 8) return false;
  return lf >= 0.1f && lf <= 0.9f;
}

}  // namespace

// Every (bucket_width, probe_group, max_load) of the grid is timed on a
// synthetic batch: clear + insert + find through the single-map path, or as
// one map of the persistent batched launch (fused).
static ash_status_t autotune_impl(int64_t capacity, int32_t key_dim, int32_t n_values,
                                  const ash_dtype_t* value_dtypes, const int64_t* value_elems, int64_t n_insert,
                                  double distinct_ratio, const std::vector<int32_t>& widths,
                                  const std::vector<int32_t>& groups, const std::vector<float>& loads, bool fused,
                                  const ash_allocator_t* allocator, void* stream, ash_tuning_t* out, double* out_ms) {
  if (!out || capacity <= 0 || capacity > kMaxCount || key_dim < 1 || key_dim > 4) return ASH_E_INVALID;
  if (n_insert <= 0 || n_insert > kMaxCount || !(distinct_ratio > 0.0) || distinct_ratio > 1.0) return ASH_E_INVALID;
  if (n_values < 0 || n_values > ash::kMaxValues || (n_values > 0 && (!value_dtypes || !value_elems)))
    return ASH_E_INVALID;
  if (widths.empty() || groups.empty() || loads.empty()) return ASH_E_INVALID;
  bool any = false;
  for (int32_t g : groups)
    for (int32_t w : widths)
      for (float lf : loads) any = any || valid_shape(w, g, lf);
  if (!any) return ASH_E_INVALID;
  int64_t row = 0;
  for (int j = 0; j < n_values; ++j) row += (int64_t)dtype_size(value_dtypes[j]) * value_elems[j];
  std::vector<int32_t> grid;  // the grid is part of the cache key
  for (int32_t w : widths) grid.push_back(w);
  grid.push_back(-1);
  for (int32_t g : groups) grid.push_back(g);
  grid.push_back(-1);
  for (float lf : loads) grid.push_back((int32_t)std::lround(lf * 1000.0f));
  const TuneKey key(key_dim, row, log2_floor(capacity), log2_floor(n_insert), (int)std::lround(distinct_ratio * 10),
                    fused ? 1 : 0, grid);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *out = it->second.first;
      if (out_ms) *out_ms = it->second.second;
      return ASH_OK;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  DevMem mem;
  mem.custom = allocator != nullptr;
  if (allocator) mem.a = *allocator;
  const uint32_t n = (uint32_t)n_insert;
  int32_t* keys = (int32_t*)mem.get((size_t)n * key_dim * 4, st);
  int32_t* fkeys = (int32_t*)mem.get((size_t)n * key_dim * 4, st);
  std::vector<void*> vals(n_values, nullptr);
  bool ok = keys && fkeys;
  for (int j = 0; j < n_values && ok; ++j) {
    vals[j] = mem.get((size_t)n * dtype_size(value_dtypes[j]) * value_elems[j], st);
    ok = vals[j] != nullptr;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  ok = ok && ash::launch_synth_keys(keys, n, key_dim, cube_side(n_insert, key_dim, distinct_ratio), 0x5eedull, fkeys,
                                   n, st) == hipSuccess;
  ash_tuning_t best;
  std::memset(&best, 0, sizeof(best));
  double best_ms = 1e30;
  for (int32_t g : groups) {
    for (int32_t w : widths) {
      for (float lf : loads) {
        if (!ok) break;
        if (!valid_shape(w, g, lf)) continue;
        ash_tuning_t t = {w, g, lf, 0u};
        ash_map* m = nullptr;
        if (ash_create(capacity, key_dim, n_values, value_dtypes, value_elems, allocator, &t, stream, &m) != ASH_OK)
          continue;  // e.g. not enough memory for this load factor
        double ms = 1e30;
        for (int rep = 0; rep < 4 && ok; ++rep) {
          ash_batch_op_t op = {m, keys, n_insert, n_values ? vals.data() : nullptr, nullptr, nullptr,
                               fkeys, n_insert, nullptr, nullptr, nullptr};
          ok = ash_clear(m, stream) == ASH_OK && hipEventRecord(e0, st) == hipSuccess &&
               (fused ? ash_batched(&op, 1, 1, stream) == ASH_OK
                      : insert_impl(m, keys, n_insert, n_values ? vals.data() : nullptr, nullptr, nullptr, st) ==
                                ASH_OK &&
                            ash_find(m, fkeys, n_insert, nullptr, nullptr, nullptr, stream) == ASH_OK) &&
               hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
          float f = 0.0f;
          if (ok && rep > 0 && hipEventElapsedTime(&f, e0, e1) == hipSuccess) ms = std::min(ms, (double)f);
        }
        ash_destroy(m);
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  mem.put(keys, st);
  mem.put(fkeys, st);
  for (void* v : vals) mem.put(v, st);
  if (!ok) return ASH_E_DEVICE;
  if (best_ms >= 1e30) return ASH_E_NOMEM;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = {best, best_ms};
  }
  *out = best;
  if (out_ms) *out_ms = best_ms;
  return ASH_OK;
}

ash_status_t ash_autotune(int64_t capacity, int32_t key_dim, int32_t n_values, const ash_dtype_t* value_dtypes,
                          const int64_t* value_elems, int64_t n_insert, double distinct_ratio,
                          const ash_allocator_t* allocator, void* stream, ash_tuning_t* out, double* out_ms) {
  return autotune_impl(capacity, key_dim, n_values, value_dtypes, value_elems, n_insert, distinct_ratio,
                       {2, 4, 8, 16, 32}, {1, 4, 8, 16, 64}, {0.5f, 0.7f, 0.85f}, false, allocator, stream, out,
                       out_ms);
}

// In the persistent batched launch every resident block takes its tiles one
// after another, so a tile's latency is not hidden by other blocks: a lane
// per key probes all 256 keys of a tile at once, while g >= 4 runs g rounds
// in sequence.  The batched sweep therefore keeps g = 1, and W <= 4: a launch
// whose maps all have those shapes runs the narrow build of the kernel (more
// blocks resident), and one map with W = 8 would move the whole launch to
// the general build, which a one-map timing does not see.
ash_status_t ash_autotune_batched(int64_t capacity, int32_t key_dim, int32_t n_values,
                                  const ash_dtype_t* value_dtypes, const int64_t* value_elems, int64_t n_insert,
                                  double distinct_ratio, const ash_allocator_t* allocator, void* stream,
                                  ash_tuning_t* out, double* out_ms) {
  return autotune_impl(capacity, key_dim, n_values, value_dtypes, value_elems, n_insert, distinct_ratio, {2, 4}, {1},
                       {0.5f, 0.7f, 0.85f}, true, allocator, stream, out, out_ms);
}

ash_status_t ash_autotune_sweep(int64_t capacity, int32_t key_dim, int32_t n_values, const ash_dtype_t* value_dtypes,
                                const int64_t* value_elems, int64_t n_insert, double distinct_ratio,
                                const int32_t* widths, int32_t n_widths, const int32_t* groups, int32_t n_groups,
                                const float* loads, int32_t n_loads, int32_t fused,
                                const ash_allocator_t* allocator, void* stream, ash_tuning_t* out, double* out_ms) {
  if (n_widths < 1 || n_groups < 1 || n_loads < 1 || !widths || !groups || !loads) return ASH_E_INVALID;
  if (n_widths > 64 || n_groups > 64 || n_loads > 64) return ASH_E_INVALID;
  return autotune_impl(capacity, key_dim, n_values, value_dtypes, value_elems, n_insert, distinct_ratio,
                       std::vector<int32_t>(widths, widths + n_widths), std::vector<int32_t>(groups, groups + n_groups),
                       std::vector<float>(loads, loads + n_loads), fused != 0, allocator, stream, out, out_ms);
}

const char* ash_status_string(ash_status_t s) {
  switch (s) {
    case ASH_OK: return "ok";
    case ASH_E_INVALID: return "invalid argument";
    case ASH_E_CAPACITY: return "capacity exceeded";
    case ASH_E_NOMEM: return "allocation failed";
    case ASH_E_DEVICE: return "HIP runtime error";
    case ASH_E_UNSUPPORTED: return "unsupported size or tuning";
    default: return "unknown status";
  }
}

}  // extern "C"
