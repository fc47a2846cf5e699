// ash_serve.hip -- served map: continuous batching of insert / find / erase
// requests on one device-resident map (host runtime around the C ABI).
//
// A worker thread owns the map and a HIP stream.  Requests are admitted in
// arrival order; consecutive requests of the same kind that are waiting when
// the worker is ready are fused into one device batch, concatenated in
// arrival order, so that the lowest-batch-position rule of insert and erase
// makes an earlier request win exactly as it would when the requests run one
// after another.  Finds never fuse with inserts or erases, and batches run in
// order on one stream, so every request sees the map that serial execution
// would show it.  An insert joins a fused batch only while the positions of
// the batch fit the free heap slots c - t: a fused insert can therefore never
// overflow where the separate requests would not.  A completion thread waits
// on each batch's event and stamps the completion time of its requests.  Up
// to `in_flight` batches are queued on the device while the worker forms the
// next one, so arrivals overlap with device work.
//
// The host never waits for the device to learn t: the last tile of every
// insert or erase commit writes the map's counters to a host-mapped mirror
// (no copy is queued), the completion thread reads the mirror when such a
// batch retires, and the bound the worker uses is those counters plus what
// the batches still in flight may add (their insert positions).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ash.h"
#include "ash_internal.hpp"
#include "ash_launch.hpp"

using namespace ash_host;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  ash_request_t r;
  std::vector<const void*> values;
  std::vector<void*> out_values;
  double arrival = 0.0;  // seconds since the server started
  double done = -1.0;
  ash_status_t status = ASH_OK;
  bool finished = false;
};

// Staging of one fused batch in flight.
struct Stage {
  int64_t cap = 0;
  int32_t* keys = nullptr;
  std::vector<uint8_t*> vals;
  int32_t* idx = nullptr;
  uint8_t* mask = nullptr;
  ash::ReqDesc* hdesc = nullptr;  // pinned host descriptors of the batch's requests
  ash::ReqDesc* ddesc = nullptr;  // their device copy
  uint8_t** dvals = nullptr;      // device array of the staging value row pointers
};

struct Batch {
  std::vector<Req*> reqs;
  hipEvent_t done = nullptr;
  int stage = -1;
  int64_t add_live = 0;  // upper bound on what the batch adds to t
  int64_t add_used = 0;  // ... and to the occupied slots
  bool snap = false;     // an insert or erase: its finalize updated the counter mirror
};

}  // namespace

struct ash_server {
  ash_map* map = nullptr;
  ash_server_config_t cfg;
  hipStream_t stream = nullptr;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_queue, cv_flight, cv_done;
  std::deque<Req*> queue;                  // submitted, not launched yet
  std::deque<Batch> flight;                // launched, not completed yet
  std::vector<std::unique_ptr<Req>> reqs;  // every request by ticket
  std::vector<Stage> stages;
  std::vector<int> free_stages;
  std::vector<hipEvent_t> free_events;
  int64_t conf_t = 0, conf_used = 0;    // read from the mirror when a batch retires
  int64_t add_live = 0, add_used = 0;  // summed over the batches in flight
  bool stop = false;
  bool worker_done = false;
  bool staged = false;  // fused inserts and erases through staging buffers (ASH_SERVER_STAGED=1)
  int device = 0;
  int64_t batches = 0, fused_requests = 0, largest = 0;
  std::thread worker, completer;
};

namespace {

double now_s(const ash_server* s) { return std::chrono::duration<double>(Clock::now() - s->t0).count(); }

ash_status_t stage_alloc(ash_server* s, Stage& g) {
  ash_map* m = s->map;
  const int64_t n = s->cfg.max_batch;
  g.cap = n;
  if (hipMalloc(&g.keys, (size_t)n * m->key_dim * 4) != hipSuccess) return ASH_E_NOMEM;
  if (hipMalloc(&g.idx, (size_t)n * 4) != hipSuccess) return ASH_E_NOMEM;
  if (hipMalloc(&g.mask, (size_t)n) != hipSuccess) return ASH_E_NOMEM;
  g.vals.assign(m->n_values, nullptr);
  for (int j = 0; j < m->n_values; ++j)
    if (hipMalloc(&g.vals[j], (size_t)n * m->row_bytes[j]) != hipSuccess) return ASH_E_NOMEM;
  const size_t dbytes = sizeof(ash::ReqDesc) * ash::kMaxFusedRequestsHost;
  if (hipHostMalloc((void**)&g.hdesc, dbytes, hipHostMallocDefault) != hipSuccess) {
    g.hdesc = nullptr;
    return ASH_E_NOMEM;
  }
  if (hipMalloc(&g.ddesc, dbytes) != hipSuccess) return ASH_E_NOMEM;
  const size_t pbytes = sizeof(uint8_t*) * std::max(m->n_values, 1);
  if (hipMalloc(&g.dvals, pbytes) != hipSuccess) return ASH_E_NOMEM;
  if (m->n_values > 0 &&
      hipMemcpy(g.dvals, g.vals.data(), sizeof(uint8_t*) * m->n_values, hipMemcpyHostToDevice) != hipSuccess)
    return ASH_E_DEVICE;
  return ASH_OK;
}

void stage_free(Stage& g) {
  (void)hipFree(g.keys);
  (void)hipFree(g.idx);
  (void)hipFree(g.mask);
  for (uint8_t* p : g.vals) (void)hipFree(p);
  if (g.hdesc) (void)hipHostFree(g.hdesc);
  (void)hipFree(g.ddesc);
  (void)hipFree(g.dvals);
}

// Runs one request directly on its own buffers.
ash_status_t run_one(ash_server* s, Req* q) {
  ash_map* m = s->map;
  const ash_request_t& r = q->r;
  switch (r.kind) {
    case ASH_REQ_INSERT:
      return insert_impl(m, r.keys, r.n, m->n_values > 0 ? q->values.data() : nullptr, r.out_idx, r.out_mask,
                         s->stream);
    case ASH_REQ_FIND:
      return ash_find(m, r.keys, r.n, r.out_idx, r.out_mask, q->out_values.empty() ? nullptr : q->out_values.data(),
                      s->stream);
    case ASH_REQ_ERASE:
      return ash_erase(m, r.keys, r.n, r.out_mask, s->stream);
    default:
      return ASH_E_INVALID;
  }
}

// Runs requests of one kind as one device batch.  A find is one kernel that
// reads the keys from, and writes the results to, the requests' own buffers;
// inserts and erases run their two passes over the requests' buffers the
// same way (insert rows under 64 B per key in total).  The kernels of such a
// batch carry the descriptors of up to kArgRequests requests in their
// arguments; larger batches upload them once.  Otherwise, or with
// ASH_SERVER_STAGED=1 at create, inserts and erases go through staging
// buffers: a descriptor upload, a gather kernel in, the operation, a scatter
// kernel out.
ash_status_t run_fused(ash_server* s, const std::vector<Req*>& run, Stage& g) {
  ash_map* m = s->map;
  hipStream_t st = s->stream;
  const int kind = run[0]->r.kind;
  const int nreq = (int)run.size();
  bool gather = false;
  int64_t off = 0;
  for (int k = 0; k < nreq; ++k) {  // descriptors in arrival order
    const Req* q = run[k];
    ash::ReqDesc& d = g.hdesc[k];
    std::memset(&d, 0, sizeof(d));
    d.off = off;
    d.n = q->r.n;
    d.keys = q->r.keys;
    if (kind == ASH_REQ_INSERT)
      for (int j = 0; j < m->n_values; ++j) d.vals[j] = (const uint8_t*)q->values[j];
    d.out_idx = kind != ASH_REQ_ERASE ? q->r.out_idx : nullptr;
    d.out_mask = q->r.out_mask;
    if (kind == ASH_REQ_FIND && !q->out_values.empty()) {
      gather = true;
      for (int j = 0; j < m->n_values; ++j) d.outv[j] = (uint8_t*)q->out_values[j];
    }
    off += q->r.n;
  }
  ash::RowSet rows;
  std::memset(&rows, 0, sizeof(rows));
  rows.n = m->n_values;
  for (int j = 0; j < m->n_values; ++j) rows.bytes[j] = m->row_bytes[j];
  uint32_t row_total = 0;
  for (int j = 0; j < m->n_values; ++j) row_total += m->row_bytes[j];
  const bool direct = kind == ASH_REQ_FIND || (!s->staged && !(m->flags & ASH_F_LDS_DEDUP) &&
                                               (kind == ASH_REQ_ERASE || row_total < kSplitRowBytes));
  // A direct batch of few requests passes its descriptors with each launch;
  // otherwise they are uploaded once.
  ash::ReqArgs args;
  args.nreq = 0;
  args.pad = 0;
  if (direct && nreq <= ash::kArgRequests) {
    args.nreq = nreq;
    std::memcpy(args.d, g.hdesc, sizeof(ash::ReqDesc) * nreq);
  } else {
    ASH_HIP(hipMemcpyAsync(g.ddesc, g.hdesc, sizeof(ash::ReqDesc) * nreq, hipMemcpyHostToDevice, st));
  }
  if (kind == ASH_REQ_FIND) {
    // one kernel: keys read from the requests, results written to them
    ValueSet vs;
    std::memset(&vs, 0, sizeof(vs));
    if (gather && m->n_values > 0) {
      vs.n = m->n_values;
      for (int j = 0; j < m->n_values; ++j) {
        vs.src[j] = m->vB[j];
        vs.row_bytes[j] = m->row_bytes[j];
        uint32_t vec = 16;
        for (int k = 0; k < nreq; ++k)
          if (g.hdesc[k].outv[j]) vec = std::min(vec, copy_unit(m->row_bytes[j], m->vB[j], g.hdesc[k].outv[j]));
        vs.vec[j] = vec;
        vs.units_log2[j] = units_log2(m->row_bytes[j], vec);
      }
    }
    ASH_HIP(ash::launch_find_requests(m->key_dim, m->G, m->W, m->ref(), args, g.ddesc, nreq, (uint32_t)off, vs, st));
    return ASH_OK;
  }
  if (direct) {
    RequestSource rs;
    rs.d = g.ddesc;
    rs.args = &args;
    rs.nreq = nreq;
    std::memset(&rs.vs, 0, sizeof(rs.vs));
    if (kind == ASH_REQ_INSERT && m->n_values > 0) {
      rs.vs.n = m->n_values;
      for (int j = 0; j < m->n_values; ++j) {
        rs.vs.dst[j] = m->vB[j];
        rs.vs.row_bytes[j] = m->row_bytes[j];
        uint32_t vec = 16;
        for (int k = 0; k < nreq; ++k) vec = std::min(vec, copy_unit(m->row_bytes[j], g.hdesc[k].vals[j], m->vB[j]));
        rs.vs.vec[j] = vec;
        rs.vs.units_log2[j] = units_log2(m->row_bytes[j], vec);
      }
    }
    if (kind == ASH_REQ_INSERT) return insert_impl(m, nullptr, off, nullptr, nullptr, nullptr, st, &rs);
    return erase_impl(m, nullptr, off, nullptr, st, &rs);
  }
  ASH_HIP(ash::launch_gather_requests(g.ddesc, nreq, off, m->key_dim, rows, g.keys,
                                      kind == ASH_REQ_INSERT && m->n_values > 0 ? g.dvals : nullptr, st));
  std::vector<const void*> vin(g.vals.begin(), g.vals.end());
  switch (kind) {
    case ASH_REQ_INSERT:
      ASH_TRY(insert_impl(m, g.keys, off, m->n_values > 0 ? vin.data() : nullptr, g.idx, g.mask, st));
      break;
    case ASH_REQ_ERASE:
      ASH_TRY(ash_erase(m, g.keys, off, g.mask, st));
      break;
    default:
      return ASH_E_INVALID;
  }
  ASH_HIP(ash::launch_scatter_requests(g.ddesc, nreq, off, kind == ASH_REQ_INSERT ? g.idx : nullptr, g.mask, st));
  return ASH_OK;
}

// Bounds on t and on the occupied slots once every launched batch has run.
int64_t live_bound(const ash_server* s) { return std::min(s->map->c, s->conf_t + s->add_live); }
int64_t used_bound(const ash_server* s) { return s->conf_used + s->add_used; }

// Free heap slots the next insert batch may assume.
int64_t insert_room(const ash_server* s) { return s->map->c - live_bound(s); }

// Takes the longest run at the queue head that may share a device batch
// (called with the queue lock held; only the worker pops the queue).
std::vector<Req*> take_run(ash_server* s) {
  std::vector<Req*> run;
  Req* head = s->queue.front();
  s->queue.pop_front();
  run.push_back(head);
  if (!s->cfg.fuse || head->r.n > s->cfg.max_batch) return run;
  const int kind = head->r.kind;
  int64_t total = head->r.n;
  int64_t room = INT64_MAX;
  if (kind == ASH_REQ_INSERT) {
    room = insert_room(s);
    if (total > room) return run;  // runs alone: it fails or succeeds exactly as on its own
  }
  while (!s->queue.empty() && (int)run.size() < s->cfg.max_fused) {
    Req* q = s->queue.front();
    if (q->r.kind != kind || total + q->r.n > s->cfg.max_batch || total + q->r.n > room) break;
    total += q->r.n;
    run.push_back(q);
    s->queue.pop_front();
  }
  return run;
}

void worker_loop(ash_server* s) {
  (void)hipSetDevice(s->device);
  while (true) {
    std::vector<Req*> run;
    int stage = -1;
    hipEvent_t ev = nullptr;
    ash_map* m = s->map;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_queue.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) return;  // stop requested and nothing left
      // a free stage and event: wait for the completion thread to retire a batch
      s->cv_done.wait(lk, [&] { return !s->free_stages.empty() && !s->free_events.empty(); });
      run = take_run(s);
      stage = s->free_stages.back();
      s->free_stages.pop_back();
      ev = s->free_events.back();
      s->free_events.pop_back();
      // the map's own checks (capacity count, tombstone cleaning) start from
      // the server's bounds instead of the ones it accumulated alone
      m->live_ub = live_bound(s);
      m->used_ub = used_bound(s);
    }
    const int kind = run[0]->r.kind;
    int64_t total = 0;
    for (Req* q : run) total += q->r.n;
    ash_status_t rc = run.size() == 1 ? run_one(s, run[0]) : run_fused(s, run, s->stages[stage]);
    // counters after the batch (a find changes neither t nor the occupied slots)
    const bool snap = kind != ASH_REQ_FIND;
    if (hipEventRecord(ev, s->stream) != hipSuccess && rc == ASH_OK) rc = ASH_E_DEVICE;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (Req* q : run) q->status = rc;
      Batch b;
      b.reqs = run;
      b.done = ev;
      b.stage = stage;
      b.snap = snap;
      if (kind == ASH_REQ_INSERT) {
        b.add_live = total;
        b.add_used = std::min(total, m->c);
      }
      s->add_live += b.add_live;
      s->add_used += b.add_used;
      s->flight.push_back(b);
      s->batches += 1;
      s->fused_requests += (int64_t)run.size();
      s->largest = std::max<int64_t>(s->largest, (int64_t)run.size());
    }
    s->cv_flight.notify_one();
  }
}

void completer_loop(ash_server* s) {
  (void)hipSetDevice(s->device);
  while (true) {
    Batch b;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_flight.wait(lk, [&] { return !s->flight.empty() || s->worker_done; });
      if (s->flight.empty()) return;
      b = s->flight.front();
    }
    const hipError_t e = hipEventSynchronize(b.done);
    const double t = now_s(s);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->flight.pop_front();
      s->add_live -= b.add_live;
      s->add_used -= b.add_used;
      if (e == hipSuccess && b.snap) {
        // The mirror holds this batch's counters or those of a later batch
        // (still in flight, so its additions are also in add_live): either
        // way conf + add stays an upper bound.
        const volatile Meta* mr = s->map->mirror_h;
        s->conf_t = mr->t;
        s->conf_used = mr->used;
      }
      for (Req* q : b.reqs) {
        if (e != hipSuccess && q->status == ASH_OK) q->status = ASH_E_DEVICE;
        q->done = t;
        q->finished = true;
      }
      s->free_stages.push_back(b.stage);
      s->free_events.push_back(b.done);
    }
    s->cv_done.notify_all();
  }
}

// Device resources of a server: stream, staging, events, the map's scratch
// sized for a full batch, and the exact starting counters (also written to
// the map's counter mirror, which the completion thread reads).
ash_status_t setup(ash_server* s) {
  const ash_server_config_t& c = s->cfg;
  if (hipGetDevice(&s->device) != hipSuccess) return ASH_E_DEVICE;
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return ASH_E_DEVICE;
  s->stages.resize(c.in_flight);
  for (int i = 0; i < c.in_flight; ++i) {
    if (c.fuse) ASH_TRY(stage_alloc(s, s->stages[i]));
    s->free_stages.push_back(i);
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return ASH_E_DEVICE;
    s->free_events.push_back(e);
  }
  Meta h;
  ASH_TRY(ensure_scratch(s->map, c.fuse ? c.max_batch : 1, s->stream));
  ASH_TRY(read_meta(s->map, &h, s->stream));
  s->map->mirror_h->t = h.t;  // nothing is in flight: the counters are exact
  s->map->mirror_h->used = h.used;
  s->map->mirror_h->tombs = h.tombs;
  s->conf_t = h.t;
  s->conf_used = h.used;
  return ASH_OK;
}

// Frees what setup() made (the threads are not running or have been joined).
void release(ash_server* s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (Stage& g : s->stages) stage_free(g);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);

  if (s->stream) (void)hipStreamDestroy(s->stream);
}

}  // namespace

extern "C" {

ash_status_t ash_server_create(ash_map_t map, const ash_server_config_t* cfg, ash_server_t* out) {
  if (!map || !out) return ASH_E_INVALID;
  if (map->flags & ASH_F_AUTOGROW) return ASH_E_UNSUPPORTED;  // admission needs a fixed capacity
  ash_server_config_t c = {256, 1 << 22, 4, 1};
  if (cfg) c = *cfg;
  if (c.max_fused < 1 || c.max_fused > ash::kMaxFusedRequestsHost || c.max_batch < 1 || c.max_batch > (1ll << 30) ||
      c.in_flight < 1 || c.in_flight > 64)
    return ASH_E_INVALID;
  std::unique_ptr<ash_server> s(new ash_server);
  s->map = map;
  s->cfg = c;
  {
    const char* v = std::getenv("ASH_SERVER_STAGED");
    s->staged = v && v[0] == '1' && v[1] == '\0';
  }
  ash_status_t rc = setup(s.get());
  if (rc != ASH_OK) {
    release(s.get());
    return rc;
  }
  s->t0 = Clock::now();
  ash_server* raw = s.release();
  raw->worker = std::thread(worker_loop, raw);
  raw->completer = std::thread(completer_loop, raw);
  *out = raw;
  return ASH_OK;
}

ash_status_t ash_server_submit(ash_server_t s, const ash_request_t* req, int64_t* out_ticket) {
  if (!s || !req || !out_ticket) return ASH_E_INVALID;
  ash_map* m = s->map;
  const ash_request_t& r = *req;
  if (r.kind < ASH_REQ_FIND || r.kind > ASH_REQ_ERASE || r.n < 0 || (r.n > 0 && !r.keys)) return ASH_E_INVALID;
  if (r.kind == ASH_REQ_INSERT && m->n_values > 0 && r.n > 0 && !r.values) return ASH_E_INVALID;
  std::unique_ptr<Req> q(new Req);
  q->r = r;
  if (r.kind == ASH_REQ_INSERT && m->n_values > 0 && r.values) q->values.assign(r.values, r.values + m->n_values);
  if (r.kind == ASH_REQ_FIND && r.out_values) q->out_values.assign(r.out_values, r.out_values + m->n_values);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return ASH_E_INVALID;
    q->arrival = now_s(s);
    *out_ticket = (int64_t)s->reqs.size();
    s->queue.push_back(q.get());
    s->reqs.push_back(std::move(q));
  }
  s->cv_queue.notify_one();
  return ASH_OK;
}

ash_status_t ash_server_wait(ash_server_t s, int64_t ticket, double* out_latency_s) {
  if (!s) return ASH_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket < 0 || ticket >= (int64_t)s->reqs.size()) return ASH_E_INVALID;
  Req* q = s->reqs[ticket].get();
  s->cv_done.wait(lk, [&] { return q->finished; });
  if (out_latency_s) *out_latency_s = q->done - q->arrival;
  return q->status;
}

ash_status_t ash_server_replay(ash_server_t s, const ash_request_t* reqs, int64_t n, const double* arrival_s,
                               double* out_latency_s, int32_t* out_status, double* out_span_s) {
  if (!s || n < 0 || (n > 0 && (!reqs || !arrival_s))) return ASH_E_INVALID;
  const double base = now_s(s);
  std::vector<int64_t> tickets(n);
  for (int64_t i = 0; i < n; ++i) {
    const double due = base + arrival_s[i];
    double t = now_s(s);
    while (t < due) {  // submit at the scheduled arrival time
      if (due - t > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(due - t - 100e-6));
      t = now_s(s);
    }
    ASH_TRY(ash_server_submit(s, &reqs[i], &tickets[i]));
    std::lock_guard<std::mutex> lk(s->mu);
    s->reqs[tickets[i]]->arrival = due;  // latency counts from the scheduled arrival
  }
  double last = base;
  for (int64_t i = 0; i < n; ++i) {
    double lat = 0.0;
    const ash_status_t st = ash_server_wait(s, tickets[i], &lat);
    if (out_latency_s) out_latency_s[i] = lat;
    if (out_status) out_status[i] = st;
    std::lock_guard<std::mutex> lk(s->mu);
    last = std::max(last, s->reqs[tickets[i]]->done);
  }
  if (out_span_s) *out_span_s = last - base;
  return ASH_OK;
}

ash_status_t ash_server_stats(ash_server_t s, int64_t* out_batches, int64_t* out_requests, int64_t* out_largest) {
  if (!s) return ASH_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (out_batches) *out_batches = s->batches;
  if (out_requests) *out_requests = s->fused_requests;
  if (out_largest) *out_largest = s->largest;
  return ASH_OK;
}

ash_status_t ash_server_destroy(ash_server_t s) {
  if (!s) return ASH_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_queue.notify_all();
  s->worker.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->worker_done = true;
  }
  s->cv_flight.notify_all();
  s->completer.join();
  release(s);
  delete s;
  return ASH_OK;
}

}  // extern "C"
