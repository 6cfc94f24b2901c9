// Batching and serving runtime over the plan's asynchronous estimate (include/pkm.h).
//
// Batch: many estimates (mocks of uneven mesh size, each with all its (l, m) fields) issued
// as one unit.  Estimates on distinct plans run on the plans' own streams and overlap on
// the device; estimates sharing a plan run in order on its stream.  The whole issue sequence
// can be captured once into a HIP graph (fork/join over the plans' streams) and replayed
// with one launch.
//
// Server: a request loop that admits multipole requests of different sizes and l_max as
// they arrive, by HBM footprint and a cap on concurrent estimates, keeps plans (meshes and
// tables) resident for reuse, overlaps the admitted estimates on separate streams, and
// records per-request latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pkm.h"
#include "internal.hpp"

namespace {

struct PinnedBuf {
  double* p = nullptr;
  size_t n = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { release(); }
  hipError_t resize(size_t count) {
    if (count <= n) return hipSuccess;
    release();
    hipError_t e = hipHostMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) n = count;
    else p = nullptr;
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace

// ===========================================================================================
// Batch
// ===========================================================================================
struct BatchItem {
  pkm_plan* plan = nullptr;
  pkm_catalog data{}, rand{};
  bool has_rand = false;
  uint64_t gen = 0;  // the plan's generation when the item was added
  std::unique_ptr<PinnedBuf> slot;
};

struct pkm_batch {
  int device = 0;
  hipStream_t origin = nullptr;
  std::vector<BatchItem> items;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t fork = nullptr, t0 = nullptr, t1 = nullptr;
  std::vector<hipEvent_t> joins;
  bool ran = false;
  std::string err;
};

namespace {

pkm_status hip_fail(pkm_batch* b, hipError_t e, const char* what) {
  b->err = std::string(what) + " failed: " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? PKM_ENOMEM : PKM_EDEVICE;
}

void drop_graph(pkm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Distinct plan streams of the batch, in first-use order.
std::vector<hipStream_t> batch_streams(const pkm_batch* b) {
  std::vector<hipStream_t> v;
  for (const auto& it : b->items) {
    hipStream_t s = pkm_internal::stream_of(it.plan);
    if (std::find(v.begin(), v.end(), s) == v.end()) v.push_back(s);
  }
  return v;
}

// Fork from origin, every item on its plan's stream, join back on origin.
pkm_status issue(pkm_batch* b) {
  const auto streams = batch_streams(b);
  hipError_t e = hipEventRecord(b->fork, b->origin);
  if (e != hipSuccess) return hip_fail(b, e, "fork event");
  for (hipStream_t s : streams)
    if ((e = hipStreamWaitEvent(s, b->fork, 0)) != hipSuccess) return hip_fail(b, e, "stream wait");
  for (size_t i = 0; i < b->items.size(); ++i) {
    BatchItem& it = b->items[i];
    const pkm_status st =
        pkm_internal::enqueue(it.plan, &it.data, it.has_rand ? &it.rand : nullptr, it.slot->p, false);
    if (st != PKM_OK) {
      b->err = "item " + std::to_string(i) + ": " + pkm_internal::error_of(it.plan);
      return st;
    }
  }
  while (b->joins.size() < streams.size()) {
    hipEvent_t ev;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(b, e, "event");
    b->joins.push_back(ev);
  }
  for (size_t k = 0; k < streams.size(); ++k) {
    if ((e = hipEventRecord(b->joins[k], streams[k])) != hipSuccess) return hip_fail(b, e, "join event");
    if ((e = hipStreamWaitEvent(b->origin, b->joins[k], 0)) != hipSuccess) return hip_fail(b, e, "join wait");
  }
  return PKM_OK;
}

}  // namespace

extern "C" {

pkm_status pkm_batch_create(int32_t device_id, pkm_batch** out) {
  if (!out) return PKM_EINVAL;
  pkm_batch* b = new (std::nothrow) pkm_batch();
  if (!b) return PKM_ENOMEM;
  b->device = device_id;
  hipError_t e = hipSetDevice(device_id);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&b->t0);
  if (e == hipSuccess) e = hipEventCreate(&b->t1);
  if (e != hipSuccess) {
    pkm_batch_destroy(b);
    return e == hipErrorOutOfMemory ? PKM_ENOMEM : PKM_EDEVICE;
  }
  *out = b;
  return PKM_OK;
}

pkm_status pkm_batch_add(pkm_batch* b, pkm_plan* plan, const pkm_catalog* data, const pkm_catalog* randoms,
                         int32_t* index_out) {
  if (!b) return PKM_EINVAL;
  if (!plan || !data) { b->err = "need a plan and a data catalog"; return PKM_EINVAL; }
  if (!pkm_internal::prepared(plan)) { b->err = "plan not prepared (pkm_prepare)"; return PKM_EORDER; }
  if (pkm_internal::device_of(plan) != b->device) { b->err = "plan lives on another device"; return PKM_EINVAL; }
  if (pkm_internal::stream_of(plan) == nullptr) {
    b->err = "batched plans need their own stream (not the null stream)";
    return PKM_EINVAL;
  }
  if (!data->on_device || (randoms && !randoms->on_device)) {
    b->err = "batched estimates take device-resident catalogs";
    return PKM_EINVAL;
  }
  if (pkm_check_catalogs(data, randoms) != PKM_OK) {
    b->err = "invalid catalogs (empty, missing arrays or n-bar, or above PKM_MAX_PARTICLES)";
    return PKM_EINVAL;
  }
  BatchItem it;
  it.plan = plan;
  it.gen = pkm_internal::generation(plan);
  it.data = *data;
  if (randoms) { it.rand = *randoms; it.has_rand = true; }
  it.slot.reset(new (std::nothrow) PinnedBuf());
  if (!it.slot) return PKM_ENOMEM;
  (void)hipSetDevice(b->device);
  hipError_t e = it.slot->resize(pkm_internal::slot_doubles(plan));
  if (e != hipSuccess) return hip_fail(b, e, "hipHostMalloc");
  b->items.push_back(std::move(it));
  drop_graph(b);
  b->ran = false;
  if (index_out) *index_out = (int32_t)(b->items.size() - 1);
  return PKM_OK;
}

pkm_status pkm_batch_run(pkm_batch* b, int32_t use_graph, double* ms_out) {
  if (!b) return PKM_EINVAL;
  if (b->items.empty()) { b->err = "empty batch"; return PKM_EINVAL; }
  // an item whose plan was re-prepared or reallocated since it was added would run kernels
  // (recorded or issued) on freed buffers or overrun its result slot: refuse before issuing
  for (size_t i = 0; i < b->items.size(); ++i) {
    const BatchItem& it = b->items[i];
    if (pkm_internal::generation(it.plan) != it.gen || !pkm_internal::prepared(it.plan) ||
        it.slot->n < pkm_internal::slot_doubles(it.plan)) {
      drop_graph(b);
      b->ran = false;
      b->err = "item " + std::to_string(i) + ": its plan changed after pkm_batch_add (add the items again)";
      return PKM_EORDER;
    }
  }
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(b, e, "hipSetDevice");
  b->ran = false;
  if (use_graph && !b->exec) {
    if ((e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(b, e, "begin capture");
    const pkm_status st = issue(b);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->origin, &g);
    if (st != PKM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e2 != hipSuccess) return hip_fail(b, e2, "end capture");
    b->graph = g;
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
      drop_graph(b);
      return hip_fail(b, e, "graph instantiate");
    }
  }
  if ((e = hipEventRecord(b->t0, b->origin)) != hipSuccess) return hip_fail(b, e, "event");
  if (use_graph) {
    if ((e = hipGraphLaunch(b->exec, b->origin)) != hipSuccess) return hip_fail(b, e, "graph launch");
  } else {
    const pkm_status st = issue(b);
    if (st != PKM_OK) return st;
  }
  if ((e = hipEventRecord(b->t1, b->origin)) != hipSuccess) return hip_fail(b, e, "event");
  if ((e = hipStreamSynchronize(b->origin)) != hipSuccess) return hip_fail(b, e, "synchronize");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, b->t0, b->t1);
  if (ms_out) *ms_out = ms;
  b->ran = true;
  return PKM_OK;
}

pkm_status pkm_batch_result(pkm_batch* b, int32_t index, pkm_result* out) {
  if (!b) return PKM_EINVAL;
  if (!out || index < 0 || (size_t)index >= b->items.size()) { b->err = "bad index or result"; return PKM_EINVAL; }
  if (!b->ran) { b->err = "batch has not run since its last change"; return PKM_EORDER; }
  BatchItem& it = b->items[index];
  return pkm_internal::finish(it.plan, it.slot->p, it.data.n, it.has_rand ? it.rand.n : 0, out, &b->err);
}

int32_t pkm_batch_size(const pkm_batch* b) { return b ? (int32_t)b->items.size() : 0; }

const char* pkm_batch_last_error(const pkm_batch* b) { return b ? b->err.c_str() : "no batch"; }

void pkm_batch_destroy(pkm_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->origin) (void)hipStreamSynchronize(b->origin);
  drop_graph(b);
  for (hipEvent_t ev : b->joins) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : {b->fork, b->t0, b->t1})
    if (ev) (void)hipEventDestroy(ev);
  b->items.clear();
  if (b->origin) (void)hipStreamDestroy(b->origin);
  delete b;
}

}  // extern "C"

// ===========================================================================================
// Server
// ===========================================================================================
namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t ADMIT_WINDOW = 8;  // queued requests considered for admission, in arrival order
constexpr int MAX_PASSES = 16;      // times the oldest request may be passed before others wait for it

// Plans are interchangeable when these parameters agree (l_max only sizes the buffers).
struct PlanKey {
  pkm_params p;
  bool operator<(const PlanKey& o) const { return std::memcmp(&p, &o.p, sizeof(pkm_params)) < 0; }
};

PlanKey key_of(const pkm_params& p) {
  PlanKey k;
  std::memset(&k.p, 0, sizeof(k.p));
  k.p.nmesh = p.nmesh;
  k.p.box_len = p.box_len;
  for (int a = 0; a < 3; ++a) {
    k.p.box_origin[a] = p.box_origin[a];
    k.p.observer[a] = p.observer[a];
  }
  k.p.window = p.window;
  k.p.interlaced = p.interlaced;
  k.p.compensated = p.compensated;
  k.p.precision = p.precision;
  k.p.max_group = p.max_group;
  k.p.deterministic = p.deterministic;
  return k;  // ell_max_hint excluded: a slot serves any l_max up to its own hint
}
bool same_key(const PlanKey& a, const PlanKey& b) { return !(a < b) && !(b < a); }

// Device memory of the serving loop comes from the device's stream-ordered pool: frees are
// ordered on the slot's stream and do not synchronise the device, so evicting a plan or growing
// a catalog buffer does not wait for the estimates in flight on other streams.  An allocation
// waits for its own stream only (idle when a plan is created or grown), so the memory is ready
// for the plan's table uploads, which are not ordered on that stream.
thread_local hipError_t g_pool_err = hipSuccess;  // the worker's last pool failure

// Hand the free memory the current device's pool keeps back to the device.
void trim_pool() {
  int dev = 0;
  hipMemPool_t pool = nullptr;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool)
    (void)hipMemPoolTrimTo(pool, 0);
  (void)hipGetLastError();
}

void* pool_alloc(size_t bytes, void* stream, void*) {
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, bytes, (hipStream_t)stream);
  if (e == hipErrorOutOfMemory) {  // the pool's kept free blocks may not fit: release them, retry once
    (void)hipGetLastError();
    trim_pool();
    e = hipMallocAsync(&p, bytes, (hipStream_t)stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    g_pool_err = e;
    (void)hipGetLastError();
    if (p) (void)hipFreeAsync(p, (hipStream_t)stream);
    return nullptr;
  }
  return p;
}
void pool_free(void* p, void* stream, void*) { (void)hipFreeAsync(p, (hipStream_t)stream); }

// A catalog registered with the server: device copies of data (and randoms), resident until
// unregistered.
struct RegCat {
  double* dev = nullptr;  // pos, w, nbar of data then of randoms
  int64_t nd = 0, nr = 0;
  bool has_rand = false, dw = false, dn = false, rw = false;
  int64_t bytes = 0;
  int refs = 0;           // queued or running requests that name it
};

// One resident plan with its stream and grow-only staging buffers.
struct Slot {
  pkm_plan* plan = nullptr;
  hipStream_t stream = nullptr;
  PlanKey key;
  int hint = 0;              // largest l_max the plan's field buffers were sized for
  int64_t bytes = 0;         // plan bytes + catalog buffer, as counted in the server's resident bytes
  bool busy = false;
  uint64_t painted_cat = 0;  // registered catalog whose painted field the plan holds (0: none)
  Clock::time_point last_used;
  std::unique_ptr<PinnedBuf> stage;   // host catalog staging
  std::unique_ptr<PinnedBuf> result;  // bin sums of the estimate in flight
  double* dev_cat = nullptr;
  size_t dev_cap = 0;        // doubles
};

struct Request {
  int64_t ticket = 0;
  pkm_params params{};
  int ell_max = 0;
  std::vector<double> edges;
  int64_t nd = 0, nr = 0;
  bool has_rand = false;
  uint64_t cat_id = 0;           // registered catalog, or 0: host catalogs copied at submit
  std::vector<double> host_cat;  // pos, w, nbar of data then randoms
  bool dw = false, dn = false, rw = false;
  int64_t need = 0;              // footprint of a new plan for this request (catalog excluded)
  int passed = 0;                // later requests admitted while this one waited
  bool reused_mesh = false;      // served from the painted field its slot already held
  Slot* slot_plan = nullptr;
  hipEvent_t done = nullptr;
  Clock::time_point t_submit, t_done;
  // result
  pkm_status status = PKM_OK;
  std::string err;
  std::vector<double> poles, kmean;
  std::vector<int64_t> nmodes;
  double alpha = 0, norm_I = 0, shot = 0;
  int n_transforms = 0;
};

}  // namespace

struct pkm_server {
  pkm_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> inflight;
  std::unordered_map<int64_t, std::shared_ptr<Request>> finished;
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<std::unique_ptr<PinnedBuf>> spare_pinned;  // pinned buffers of evicted slots
  std::unordered_map<uint64_t, RegCat> cats;
  uint64_t next_cat = 1;
  int64_t next_ticket = 1;
  int64_t resident = 0, peak_resident = 0;  // plans, their catalog buffers and registered catalogs
  int64_t cat_bytes = 0;                    // of which registered catalogs
  int max_concurrent = 0;
  std::vector<double> latencies_ms, latencies_prec[2];
  int64_t completed = 0, failed = 0, mesh_reuses = 0;
  Clock::time_point t_first_submit, t_last_done;
  bool any_submit = false;
  bool stop = false;
  std::thread worker;
  std::string err;
};

namespace {

// The server's device allocator: the caller's hooks when given, else the stream-ordered pool.
void* dev_alloc(const pkm_server* sv, size_t bytes, hipStream_t s) {
  return sv->cfg.alloc ? sv->cfg.alloc(bytes, s, sv->cfg.alloc_ctx) : pool_alloc(bytes, s, nullptr);
}
void dev_free(const pkm_server* sv, void* p, hipStream_t s) {
  if (!p) return;
  if (sv->cfg.alloc) sv->cfg.free(p, s, sv->cfg.alloc_ctx);
  else pool_free(p, s, nullptr);
}

std::unique_ptr<PinnedBuf> take_pinned(pkm_server* sv) {
  if (!sv->spare_pinned.empty()) {
    std::unique_ptr<PinnedBuf> b = std::move(sv->spare_pinned.back());
    sv->spare_pinned.pop_back();
    return b;
  }
  return std::unique_ptr<PinnedBuf>(new (std::nothrow) PinnedBuf());
}

// The device's pool keeps the blocks of evicted plans for reuse, and reserves fresh memory when
// those do not fit a new plan's buffers.  Its reserved bytes (live plus kept) are held within
// the plan budget (the server budget less the registered catalogs), less `extra` bytes about to
// be allocated, so the device keeps the headroom outside the budget that the runtime itself
// needs (scratch for kernel launches, queues).  Kept blocks are released, live ones never.
void bound_pool(const pkm_server* sv, int64_t extra) {
  if (sv->cfg.alloc) return;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, sv->cfg.device_id) != hipSuccess || !pool) {
    (void)hipGetLastError();
    return;
  }
  uint64_t reserved = 0;
  if (hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &reserved) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  const int64_t bound = std::max<int64_t>(0, sv->cfg.hbm_budget_bytes - sv->cat_bytes - extra);
  if ((int64_t)reserved > bound) (void)hipMemPoolTrimTo(pool, (size_t)bound);
  (void)hipGetLastError();
}

// Whether the device keeps its headroom after `need` more bytes: the pool's reserved blocks
// (live, kept or fragmented) count against the device's free memory, and the runtime allocates
// a queue's kernel scratch from what is left when a kernel that spills first runs there, so a
// pool that fills the device makes that dispatch fail.  The headroom is 2 GiB or 1% of the
// device, whichever is larger; kept blocks are released before the second look.
bool device_room(int64_t need) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // no reading: the budget alone decides
  }
  const int64_t headroom = std::max<int64_t>(int64_t(2) << 30, (int64_t)(tot / 100));
  if ((int64_t)fr - need >= headroom) return true;
  trim_pool();
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return (int64_t)fr - need >= headroom;
}

// Evict an idle slot: its plan and catalog buffer go back to the pool on its own stream (which
// runs nothing else, so waiting for it waits for the frees only and lets any stream reuse the
// blocks at once), its pinned buffers to the server's spares (freeing pinned memory would
// synchronise the device).
void free_slot(pkm_server* sv, Slot* s) {
  pkm_plan_destroy(s->plan);
  dev_free(sv, s->dev_cat, s->stream);
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  if (s->stage) sv->spare_pinned.push_back(std::move(s->stage));
  if (s->result) sv->spare_pinned.push_back(std::move(s->result));
  sv->resident -= s->bytes;
}

// Copy the request's host catalog through the slot's pinned staging to its device buffer.
pkm_status stage_request(const pkm_server* sv, Request* r, Slot* sl) {
  const size_t total = r->host_cat.size();
  if (sl->dev_cap < total) {
    dev_free(sv, sl->dev_cat, sl->stream);
    sl->dev_cap = 0;
    sl->dev_cat = (double*)dev_alloc(sv, total * sizeof(double), sl->stream);
    if (!sl->dev_cat) {
      r->err = "catalog allocation failed";
      return PKM_ENOMEM;
    }
    sl->dev_cap = total;
  }
  if (sl->stage->resize(total) != hipSuccess) { r->err = "pinned staging allocation failed"; return PKM_ENOMEM; }
  std::memcpy(sl->stage->p, r->host_cat.data(), total * sizeof(double));
  const hipError_t e = hipMemcpyAsync(sl->dev_cat, sl->stage->p, total * sizeof(double), hipMemcpyHostToDevice,
                                      sl->stream);
  if (e != hipSuccess) { r->err = hipGetErrorString(e); return PKM_EDEVICE; }
  return PKM_OK;
}

// Device catalogs of a request laid out from `base`: pos, w, nbar of data, then of randoms.
void catalogs_of(const Request* r, const double* base, pkm_catalog* d, pkm_catalog* rr) {
  const double* p = base;
  d->pos = p; p += 3 * r->nd;
  d->w = r->dw ? p : nullptr; if (r->dw) p += r->nd;
  d->nbar = r->dn ? p : nullptr; if (r->dn) p += r->nd;
  d->n = r->nd;
  d->on_device = 1;
  if (r->has_rand) {
    rr->pos = p; p += 3 * r->nr;
    rr->w = r->rw ? p : nullptr; if (r->rw) p += r->nr;
    rr->nbar = p;
    rr->n = r->nr;
    rr->on_device = 1;
  }
}

void complete(pkm_server* sv, std::shared_ptr<Request> r, pkm_status st) {
  r->status = st;
  r->t_done = Clock::now();
  if (r->done) (void)hipEventDestroy(r->done);
  r->done = nullptr;
  std::vector<double>().swap(r->host_cat);
  if (r->slot_plan) {
    Slot* sl = r->slot_plan;
    // the plan now holds the painted field of this request's catalog (none after a failure or
    // for host catalogs, which cannot be named again)
    if (!r->reused_mesh || st != PKM_OK) sl->painted_cat = st == PKM_OK ? r->cat_id : 0;
    sl->busy = false;
    sl->last_used = r->t_done;
    r->slot_plan = nullptr;
  }
  if (r->cat_id) {
    auto it = sv->cats.find(r->cat_id);
    if (it != sv->cats.end()) --it->second.refs;
  }
  if (st == PKM_OK) {
    const double ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    sv->latencies_ms.push_back(ms);
    sv->latencies_prec[r->params.precision == PKM_FP64 ? 1 : 0].push_back(ms);
    if (r->reused_mesh) ++sv->mesh_reuses;
    ++sv->completed;
  } else {
    ++sv->failed;
  }
  sv->t_last_done = r->t_done;
  sv->finished[r->ticket] = r;
}

// Issue request r on slot `sl` (its plan created first when sl->plan is null).  Runs without
// the server lock: only the worker thread touches a busy slot.
pkm_status start_request(pkm_server* sv, Request* r, Slot* sl, const double* reg_base) {
  if (!sl->plan) {
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      sl->stream = nullptr;
      r->err = "stream creation failed";
      return PKM_EDEVICE;
    }
    pkm_device dev{};
    dev.device_id = sv->cfg.device_id;
    dev.hip_stream = sl->stream;
    dev.alloc = sv->cfg.alloc ? sv->cfg.alloc : pool_alloc;
    dev.free = sv->cfg.alloc ? sv->cfg.free : pool_free;
    dev.alloc_ctx = sv->cfg.alloc ? sv->cfg.alloc_ctx : nullptr;
    pkm_params pp = sl->key.p;
    pp.ell_max_hint = sl->hint;
    const pkm_status st = pkm_plan_create(&pp, &dev, &sl->plan);
    if (st != PKM_OK) {
      sl->plan = nullptr;
      r->err = std::string("plan creation failed: ") + pkm_plan_last_error(nullptr);
      if (g_pool_err != hipSuccess) r->err += std::string(" (") + hipGetErrorString(g_pool_err) + ")";
      g_pool_err = hipSuccess;
      return st;
    }
  }
  r->slot_plan = sl;
  pkm_status st = pkm_internal::prepare(sl->plan, r->ell_max, r->edges.data(), (int)r->edges.size(), r->nd + r->nr);
  if (st != PKM_OK) { r->err = pkm_internal::error_of(sl->plan); return st; }
  if (sl->result->resize(pkm_internal::slot_doubles(sl->plan)) != hipSuccess) {
    r->err = "pinned result allocation failed";
    return PKM_ENOMEM;
  }
  if (r->reused_mesh) {
    st = pkm_internal::enqueue_compute_only(sl->plan, sl->result->p);
  } else {
    const double* base = reg_base;
    if (!base) {
      st = stage_request(sv, r, sl);
      base = sl->dev_cat;
    }
    if (st == PKM_OK) {
      pkm_catalog d{}, rr{};
      catalogs_of(r, base, &d, &rr);
      st = pkm_internal::enqueue(sl->plan, &d, r->has_rand ? &rr : nullptr, sl->result->p, false);
    }
  }
  if (st != PKM_OK) {
    if (r->err.empty()) r->err = pkm_internal::error_of(sl->plan);
    return st;
  }
  if (hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r->done, sl->stream) != hipSuccess) {
    r->err = "event failed";
    return PKM_EDEVICE;
  }
  return PKM_OK;
}

// Admit one request from the first ADMIT_WINDOW queued ones, in arrival order: the first that
// fits the budget (after evicting idle plans, least recently used first) while fewer than
// max_inflight estimates run.  A request is served from the painted field a slot already holds
// when it names the catalog that slot painted last.  A request that cannot fit even with nothing
// else running fails with PKM_ENOMEM.  Once the oldest request has been passed MAX_PASSES times,
// nothing is admitted before it.  Returns true when the queue changed.
bool admit_some(pkm_server* sv, std::unique_lock<std::mutex>& lk) {
  if (sv->queue.empty() || (int)sv->inflight.size() >= sv->cfg.max_inflight) return false;
  const size_t window = sv->queue.front()->passed >= MAX_PASSES ? 1 : std::min(sv->queue.size(), ADMIT_WINDOW);
  for (size_t qi = 0; qi < window; ++qi) {
    std::shared_ptr<Request> r = sv->queue[qi];
    const PlanKey key = key_of(r->params);
    // an idle plan of the same key: the one holding this catalog's painted field, else one
    // holding no registered catalog's field, else the least recently used
    Slot* use = nullptr;
    bool hit = false;
    for (auto& s : sv->slots) {
      if (s->busy || s->hint < r->ell_max || !same_key(s->key, key)) continue;
      if (r->cat_id && s->painted_cat == r->cat_id) { use = s.get(); hit = true; break; }
      const bool blank = s->painted_cat == 0;
      if (!use || (blank && use->painted_cat != 0) ||
          (blank == (use->painted_cat == 0) && s->last_used < use->last_used))
        use = s.get();
    }
    const int64_t cat_bytes = r->cat_id ? 0 : (int64_t)r->host_cat.size() * 8;
    // a reused plan grows only by what this request needs beyond its present buffers
    const int64_t need = use ? std::max<int64_t>(0, r->need - pkm_internal::device_bytes(use->plan)) +
                                   std::max<int64_t>(0, cat_bytes - (int64_t)use->dev_cap * 8)
                             : r->need + cat_bytes;
    int64_t evictable = 0;
    bool running = false;
    for (auto& s : sv->slots) {
      if (s->busy) running = true;
      else if (s.get() != use) evictable += s->bytes;
    }
    if (sv->resident - evictable + need > sv->cfg.hbm_budget_bytes) {
      if (!running && qi == 0) {  // cannot fit even with nothing else resident but catalogs
        sv->queue.pop_front();
        r->err = "request footprint above the server's HBM budget";
        complete(sv, r, PKM_ENOMEM);
        sv->cv_done.notify_all();
        return true;
      }
      continue;  // wait for running estimates; look at the next request
    }
    auto evict_lru = [&]() {
      Slot* victim = nullptr;
      for (auto& s : sv->slots)
        if (!s->busy && s.get() != use && (!victim || s->last_used < victim->last_used)) victim = s.get();
      if (!victim) return false;
      free_slot(sv, victim);
      sv->slots.erase(std::find_if(sv->slots.begin(), sv->slots.end(), [&](auto& p) { return p.get() == victim; }));
      return true;
    };
    while (sv->resident + need > sv->cfg.hbm_budget_bytes && evict_lru()) {
    }
    // the device's own free memory (budget or not): evict further idle plans while it lacks the
    // headroom; if it still does, wait for the running estimates, or fail when none runs
    bool room = device_room(need);
    while (!room && evict_lru()) room = device_room(need);
    if (!room) {
      if (!running && qi == 0) {
        sv->queue.pop_front();
        r->err = "device memory below the request's footprint plus the runtime's headroom";
        complete(sv, r, PKM_ENOMEM);
        sv->cv_done.notify_all();
        return true;
      }
      continue;
    }
    for (size_t k = 0; k < qi; ++k) ++sv->queue[k]->passed;
    sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)qi);
    r->reused_mesh = hit;
    const double* reg_base = r->cat_id ? sv->cats[r->cat_id].dev : nullptr;
    Slot* slot = use;
    if (!slot) {  // a new slot, visible to no one else until it is added below
      std::unique_ptr<Slot> fresh(new (std::nothrow) Slot());
      if (fresh) {
        fresh->key = key;
        fresh->hint = std::max(r->ell_max, r->params.ell_max_hint);
        fresh->stage = take_pinned(sv);
        fresh->result = take_pinned(sv);
      }
      if (!fresh || !fresh->stage || !fresh->result) {
        if (fresh && fresh->stage) sv->spare_pinned.push_back(std::move(fresh->stage));
        if (fresh && fresh->result) sv->spare_pinned.push_back(std::move(fresh->result));
        complete(sv, r, PKM_ENOMEM);
        sv->cv_done.notify_all();
        return true;
      }
      fresh->busy = true;
      slot = fresh.get();
      sv->slots.push_back(std::move(fresh));
    }
    slot->busy = true;
    sv->resident += need;  // reserved until the plan's size is known
    sv->peak_resident = std::max(sv->peak_resident, sv->resident);
    bound_pool(sv, need);
    lk.unlock();           // device work below; clients touch only the queue and the results
    pkm_status st = start_request(sv, r.get(), slot, reg_base);
    lk.lock();
    bound_pool(sv, 0);
    sv->resident -= need;
    if (slot->plan) {
      const int64_t b = pkm_internal::device_bytes(slot->plan) + (int64_t)slot->dev_cap * 8;
      sv->resident += b - slot->bytes;
      slot->bytes = b;
    } else {  // the plan could not be created: drop the slot
      r->slot_plan = nullptr;
      if (slot->stream) (void)hipStreamDestroy(slot->stream);
      if (slot->stage) sv->spare_pinned.push_back(std::move(slot->stage));
      if (slot->result) sv->spare_pinned.push_back(std::move(slot->result));
      sv->resident -= slot->bytes;
      sv->slots.erase(std::find_if(sv->slots.begin(), sv->slots.end(), [&](auto& p) { return p.get() == slot; }));
    }
    sv->peak_resident = std::max(sv->peak_resident, sv->resident);
    if (st != PKM_OK) {
      complete(sv, r, st);
      sv->cv_done.notify_all();
      return true;
    }
    sv->inflight.push_back(r);
    sv->max_concurrent = std::max(sv->max_concurrent, (int)sv->inflight.size());
    return true;
  }
  return false;
}

void reap(pkm_server* sv, std::unique_lock<std::mutex>& lk) {
  for (size_t i = 0; i < sv->inflight.size();) {
    std::shared_ptr<Request> r = sv->inflight[i];
    const hipError_t e = hipEventQuery(r->done);
    if (e == hipErrorNotReady) { ++i; continue; }
    sv->inflight.erase(sv->inflight.begin() + i);
    pkm_status st = PKM_OK;
    if (e != hipSuccess) {
      r->err = hipGetErrorString(e);
      st = PKM_EDEVICE;
    } else {
      const int nb = (int)r->edges.size() - 1;
      r->poles.assign((size_t)(r->ell_max / 2 + 1) * nb, 0.0);
      r->kmean.assign(nb, 0.0);
      r->nmodes.assign(nb, 0);
      pkm_result res{};
      res.poles = r->poles.data();
      res.k_mean = r->kmean.data();
      res.n_modes = r->nmodes.data();
      st = pkm_internal::finish(r->slot_plan->plan, r->slot_plan->result->p, r->nd, r->nr, &res, &r->err);
      r->alpha = res.alpha;
      r->norm_I = res.norm_I;
      r->shot = res.shot_noise;
      r->n_transforms = res.n_transforms;
    }
    complete(sv, r, st);
    sv->cv_done.notify_all();
  }
  (void)lk;
}

void worker_loop(pkm_server* sv) {
  (void)hipSetDevice(sv->cfg.device_id);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    if (sv->stop && sv->inflight.empty()) break;
    reap(sv, lk);
    bool progressed = false;
    while (!sv->stop && admit_some(sv, lk)) progressed = true;
    if (sv->inflight.empty() && sv->queue.empty()) {
      if (sv->stop) break;
      sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      continue;
    }
    if (!progressed) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
    }
  }
  // cancel what never started
  while (!sv->queue.empty()) {
    auto r = sv->queue.front();
    sv->queue.pop_front();
    r->err = "server stopped";
    complete(sv, r, PKM_ECANCELLED);
  }
  sv->cv_done.notify_all();
}

pkm_status copy_out(const Request& r, pkm_result* out) {
  if (r.status != PKM_OK) return r.status;
  if (out->poles) std::copy(r.poles.begin(), r.poles.end(), out->poles);
  if (out->k_mean) std::copy(r.kmean.begin(), r.kmean.end(), out->k_mean);
  if (out->n_modes) std::copy(r.nmodes.begin(), r.nmodes.end(), out->n_modes);
  out->alpha = r.alpha;
  out->norm_I = r.norm_I;
  out->shot_noise = r.shot;
  out->n_transforms = r.n_transforms;
  return PKM_OK;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

// Doubles of a catalog pair laid out as catalogs_of reads them.
size_t layout_doubles(const pkm_catalog* d, const pkm_catalog* r) {
  size_t n = (size_t)d->n * (3 + (d->w ? 1 : 0) + (d->nbar ? 1 : 0));
  if (r) n += (size_t)r->n * (4 + (r->w ? 1 : 0));
  return n;
}

}  // namespace

extern "C" {

pkm_status pkm_server_create(const pkm_server_config* cfg, pkm_server** out) {
  if (!cfg || !out) return PKM_EINVAL;
  if (cfg->max_inflight < 1 || cfg->max_inflight > 32) return PKM_EINVAL;
  if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return PKM_EINVAL;
  if (cfg->field_group < 0 || cfg->field_group > 256) return PKM_EINVAL;
  pkm_server* sv = new (std::nothrow) pkm_server();
  if (!sv) return PKM_ENOMEM;
  sv->cfg = *cfg;
  if (hipSetDevice(cfg->device_id) != hipSuccess) {
    delete sv;
    return PKM_EDEVICE;
  }
  if (sv->cfg.hbm_budget_bytes <= 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete sv;
      return PKM_EDEVICE;
    }
    sv->cfg.hbm_budget_bytes = (int64_t)(0.8 * (double)free_b);
  }
  // keep freed plan memory in the device's pool for the next plan instead of returning it,
  // reusable by any stream once its free has completed
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, cfg->device_id) == hipSuccess && pool) {
    uint64_t keep = (uint64_t)sv->cfg.hbm_budget_bytes;  // bound_pool keeps it within the plan budget
    int yes = 1;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    (void)hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowOpportunistic, &yes);
    (void)hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &yes);
  }
  (void)hipGetLastError();
  try {
    sv->worker = std::thread(worker_loop, sv);
  } catch (...) {
    delete sv;
    return PKM_ENOMEM;
  }
  *out = sv;
  return PKM_OK;
}

pkm_status pkm_server_register_catalog(pkm_server* sv, const pkm_catalog* data, const pkm_catalog* randoms,
                                       uint64_t* cat_id) {
  if (!sv || !cat_id) return PKM_EINVAL;
  if (pkm_check_catalogs(data, randoms) != PKM_OK) {
    sv->err = "invalid catalogs (empty, missing positions or n-bar, or above PKM_MAX_PARTICLES)";
    return PKM_EINVAL;
  }
  RegCat rc;
  rc.nd = data->n;
  rc.has_rand = randoms != nullptr;
  rc.nr = randoms ? randoms->n : 0;
  rc.dw = data->w != nullptr;
  rc.dn = data->nbar != nullptr;
  rc.rw = randoms && randoms->w != nullptr;
  const size_t total = layout_doubles(data, randoms);
  rc.bytes = (int64_t)(total * sizeof(double));
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) return PKM_ECANCELLED;
    int64_t evictable = 0;
    for (auto& s : sv->slots)
      if (!s->busy) evictable += s->bytes;
    if (sv->resident - evictable + rc.bytes > sv->cfg.hbm_budget_bytes) {
      sv->err = "catalog does not fit the server's HBM budget";
      return PKM_ENOMEM;
    }
    while (sv->resident + rc.bytes > sv->cfg.hbm_budget_bytes) {
      Slot* victim = nullptr;
      for (auto& s : sv->slots)
        if (!s->busy && (!victim || s->last_used < victim->last_used)) victim = s.get();
      if (!victim) break;
      (void)hipSetDevice(sv->cfg.device_id);
      free_slot(sv, victim);
      sv->slots.erase(std::find_if(sv->slots.begin(), sv->slots.end(), [&](auto& p) { return p.get() == victim; }));
    }
    sv->resident += rc.bytes;  // reserved while the copy runs
    sv->peak_resident = std::max(sv->peak_resident, sv->resident);
  }
  hipError_t e = hipSetDevice(sv->cfg.device_id);
  if (e == hipSuccess) e = hipMalloc((void**)&rc.dev, std::max<size_t>(total, 1) * sizeof(double));
  if (e == hipErrorOutOfMemory) {  // free blocks kept by the plans' pool: release them, retry once
    (void)hipGetLastError();
    trim_pool();
    e = hipMalloc((void**)&rc.dev, std::max<size_t>(total, 1) * sizeof(double));
  }
  if (e == hipSuccess) {
    double* p = rc.dev;
    auto put = [&](const double* src, int64_t count) {
      if (e == hipSuccess) e = hipMemcpy(p, src, (size_t)count * sizeof(double), hipMemcpyDefault);
      p += count;
    };
    put(data->pos, 3 * data->n);
    if (rc.dw) put(data->w, data->n);
    if (rc.dn) put(data->nbar, data->n);
    if (randoms) {
      put(randoms->pos, 3 * randoms->n);
      if (rc.rw) put(randoms->w, randoms->n);
      put(randoms->nbar, randoms->n);
    }
  }
  std::lock_guard<std::mutex> g(sv->mu);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (rc.dev) (void)hipFree(rc.dev);
    sv->resident -= rc.bytes;
    sv->err = std::string("catalog upload failed: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PKM_ENOMEM : PKM_EDEVICE;
  }
  *cat_id = sv->next_cat++;
  sv->cat_bytes += rc.bytes;
  sv->cats[*cat_id] = rc;
  bound_pool(sv, 0);
  return PKM_OK;
}

pkm_status pkm_server_unregister_catalog(pkm_server* sv, uint64_t cat_id) {
  if (!sv) return PKM_EINVAL;
  double* dev = nullptr;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->cats.find(cat_id);
    if (it == sv->cats.end()) { sv->err = "unknown catalog"; return PKM_EINVAL; }
    if (it->second.refs > 0) { sv->err = "catalog named by queued or running requests"; return PKM_EBUSY; }
    dev = it->second.dev;
    sv->resident -= it->second.bytes;
    sv->cat_bytes -= it->second.bytes;
    sv->cats.erase(it);
    for (auto& s : sv->slots)
      if (s->painted_cat == cat_id) s->painted_cat = 0;  // the id is not reused, but no stale hit either
  }
  (void)hipSetDevice(sv->cfg.device_id);
  (void)hipFree(dev);
  return PKM_OK;
}

pkm_status pkm_server_submit(pkm_server* sv, const pkm_request* rq, int64_t* ticket) {
  if (!sv || !rq || !ticket) return PKM_EINVAL;
  if (!rq->k_edges || rq->n_edges < 2 || rq->ell_max < 0 || rq->ell_max > 16 || rq->ell_max % 2) {
    sv->err = "need even ell_max in 0..16 and at least two k edges";
    return PKM_EINVAL;
  }
  for (int i = 0; i < rq->n_edges; ++i)
    if (!(rq->k_edges[i] >= 0.0) || !std::isfinite(rq->k_edges[i]) || (i > 0 && !(rq->k_edges[i] > rq->k_edges[i - 1]))) {
      sv->err = "k edges must be finite, >= 0 and strictly increasing";
      return PKM_EINVAL;
    }
  auto r = std::make_shared<Request>();
  r->params = rq->params;
  if (sv->cfg.field_group > 0 && r->params.max_group == 0) {
    r->params.max_group = sv->cfg.field_group;  // one plan per mesh configuration for every ell_max
    r->params.ell_max_hint = 16;
  }
  r->ell_max = rq->ell_max;
  r->edges.assign(rq->k_edges, rq->k_edges + rq->n_edges);
  r->cat_id = rq->catalog_id;
  if (r->cat_id == 0) {
    // host catalogs, copied now so the caller may release its arrays after submit
    if (!rq->data.pos || rq->data.n <= 0 || rq->data.on_device) {
      sv->err = "requests take a non-empty host data catalog or a registered catalog";
      return PKM_EINVAL;
    }
    if (rq->has_randoms && (!rq->randoms.pos || !rq->randoms.nbar || rq->randoms.n <= 0 || rq->randoms.on_device)) {
      sv->err = "randoms need host positions and nbar and n > 0";
      return PKM_EINVAL;
    }
    if (rq->data.n + (rq->has_randoms ? rq->randoms.n : 0) > PKM_MAX_PARTICLES) {
      sv->err = "data + random objects above PKM_MAX_PARTICLES";
      return PKM_EINVAL;
    }
    r->nd = rq->data.n;
    r->has_rand = rq->has_randoms != 0;
    r->nr = r->has_rand ? rq->randoms.n : 0;
    r->dw = rq->data.w != nullptr;
    r->dn = rq->data.nbar != nullptr;
    r->rw = r->has_rand && rq->randoms.w != nullptr;
    const size_t total = layout_doubles(&rq->data, r->has_rand ? &rq->randoms : nullptr);
    try {
      r->host_cat.resize(total);
    } catch (...) {
      return PKM_ENOMEM;
    }
    double* p = r->host_cat.data();
    auto put = [&](const double* src, size_t count) { std::memcpy(p, src, count * sizeof(double)); p += count; };
    put(rq->data.pos, 3 * (size_t)r->nd);
    if (r->dw) put(rq->data.w, r->nd);
    if (r->dn) put(rq->data.nbar, r->nd);
    if (r->has_rand) {
      put(rq->randoms.pos, 3 * (size_t)r->nr);
      if (r->rw) put(rq->randoms.w, r->nr);
      put(rq->randoms.nbar, r->nr);
    }
  }
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->stop) return PKM_ECANCELLED;
  if (r->cat_id) {
    auto it = sv->cats.find(r->cat_id);
    if (it == sv->cats.end()) { sv->err = "unknown catalog id"; return PKM_EINVAL; }
    const RegCat& rc = it->second;
    r->nd = rc.nd; r->nr = rc.nr; r->has_rand = rc.has_rand;
    r->dw = rc.dw; r->dn = rc.dn; r->rw = rc.rw;
  }
  r->need = pkm_internal::footprint(&r->params, r->ell_max, (int)r->edges.size(), r->nd + r->nr);
  if (r->need < 0) { sv->err = "invalid mesh parameters"; return PKM_EINVAL; }
  if (rq->params.max_group == 0 && r->need > sv->cfg.hbm_budget_bytes / 2) {
    // keep fewer weighted fields resident at once (field groups run one after another)
    for (int gmax = 64; gmax >= 1; gmax /= 2) {
      r->params.max_group = gmax;
      r->need = pkm_internal::footprint(&r->params, r->ell_max, (int)r->edges.size(), r->nd + r->nr);
      if (r->need <= sv->cfg.hbm_budget_bytes / 2) break;
    }
  }
  if (r->cat_id) ++sv->cats[r->cat_id].refs;
  r->ticket = sv->next_ticket++;
  r->t_submit = Clock::now();
  if (!sv->any_submit) { sv->t_first_submit = r->t_submit; sv->any_submit = true; }
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv_work.notify_one();
  return PKM_OK;
}

pkm_status pkm_server_poll(pkm_server* sv, int64_t ticket, pkm_result* out) {
  if (!sv || !out) return PKM_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->finished.find(ticket);
  if (it == sv->finished.end()) {
    if (ticket <= 0 || ticket >= sv->next_ticket) { sv->err = "unknown ticket"; return PKM_EINVAL; }
    return PKM_EBUSY;
  }
  std::shared_ptr<Request> r = it->second;
  sv->finished.erase(it);
  if (r->status != PKM_OK) sv->err = r->err;
  return copy_out(*r, out);
}

pkm_status pkm_server_wait(pkm_server* sv, int64_t ticket, pkm_result* out) {
  if (!sv || !out) return PKM_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (ticket <= 0 || ticket >= sv->next_ticket) { sv->err = "unknown ticket"; return PKM_EINVAL; }
  sv->cv_done.wait(lk, [&] { return sv->finished.count(ticket) > 0 || (sv->stop && sv->inflight.empty() && sv->queue.empty()); });
  auto it = sv->finished.find(ticket);
  if (it == sv->finished.end()) { sv->err = "ticket already collected"; return PKM_EINVAL; }
  std::shared_ptr<Request> r = it->second;
  sv->finished.erase(it);
  if (r->status != PKM_OK) sv->err = r->err;
  return copy_out(*r, out);
}

pkm_status pkm_server_stats(pkm_server* sv, pkm_server_stats_t* out) {
  if (!sv || !out) return PKM_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = sv->completed;
  out->failed = sv->failed;
  out->queued = (int64_t)sv->queue.size();
  out->inflight = (int64_t)sv->inflight.size();
  out->resident_plans = (int64_t)sv->slots.size();
  out->resident_bytes = sv->resident;
  out->peak_bytes = sv->peak_resident;
  out->max_concurrent = sv->max_concurrent;
  out->latency_p50_ms = percentile(sv->latencies_ms, 0.50);
  out->latency_p99_ms = percentile(sv->latencies_ms, 0.99);
  out->latency_mean_ms = 0.0;
  for (double v : sv->latencies_ms) out->latency_mean_ms += v;
  if (!sv->latencies_ms.empty()) out->latency_mean_ms /= (double)sv->latencies_ms.size();
  if (sv->any_submit && sv->completed > 0) {
    const double span = std::chrono::duration<double>(sv->t_last_done - sv->t_first_submit).count();
    out->throughput_per_s = span > 0 ? (double)sv->completed / span : 0.0;
  }
  out->completed_fp32 = (int64_t)sv->latencies_prec[0].size();
  out->completed_fp64 = (int64_t)sv->latencies_prec[1].size();
  out->latency_p50_ms_fp32 = percentile(sv->latencies_prec[0], 0.50);
  out->latency_p99_ms_fp32 = percentile(sv->latencies_prec[0], 0.99);
  out->latency_p50_ms_fp64 = percentile(sv->latencies_prec[1], 0.50);
  out->latency_p99_ms_fp64 = percentile(sv->latencies_prec[1], 0.99);
  out->mesh_reuses = sv->mesh_reuses;
  out->registered_catalogs = (int64_t)sv->cats.size();
  out->registered_bytes = sv->cat_bytes;
  return PKM_OK;
}

pkm_status pkm_server_reset_stats(pkm_server* sv) {
  if (!sv) return PKM_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  sv->latencies_ms.clear();
  sv->latencies_prec[0].clear();
  sv->latencies_prec[1].clear();
  sv->completed = sv->failed = sv->mesh_reuses = 0;
  sv->max_concurrent = (int)sv->inflight.size();
  sv->peak_resident = sv->resident;
  sv->any_submit = false;
  return PKM_OK;
}

const char* pkm_server_last_error(const pkm_server* sv) { return sv ? sv->err.c_str() : "no server"; }

void pkm_server_destroy(pkm_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->cfg.device_id);
  for (auto& s : sv->slots) free_slot(sv, s.get());
  sv->slots.clear();
  for (auto& kv : sv->cats) (void)hipFree(kv.second.dev);
  sv->cats.clear();
  (void)hipDeviceSynchronize();
  sv->spare_pinned.clear();
  delete sv;
}

}  // extern "C"
