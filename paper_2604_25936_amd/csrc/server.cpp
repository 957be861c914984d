// Request loop on one GPU: continuous batching of query requests.
//
// Requests (model, map, host point set) are queued by sand_server_submit.
// A scheduler thread admits them first-in first-out while the device bytes
// they need fit a fixed HBM arena (the budget), and whenever one of the
// n_streams launch slots is free it launches the admitted requests of one
// padded width, in order and up to a total of 2M points (a larger request
// alone), as one batch: the point sets are copied in, one lookup /
// bucketing launch and one persistent T-MLP launch cover all of them (each
// tile knows its query and model), and the results are copied back. A
// request that arrives while batches are running joins the next batch as
// soon as memory and a slot free up, so batches overlap on the device
// (different streams) and with the copies. Host callbacks on the stream
// time-stamp completion, release the request's memory and wake waiters.

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "sand_host.h"
#include "batching.h"

using namespace sand;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kMaxBatchRequests = 1024;
// Points one batch gathers before it closes (a larger request still forms a
// batch of its own): a small request does not wait for the copies and
// evaluation of a multi-million-point one launched with it.
constexpr int64_t kBatchPointCap = int64_t(1) << 21;

// Device bytes one request holds from admission to completion.
struct ReqLayout {
  size_t xyz, sdf, depth, perm, counts, total;
  explicit ReqLayout(int64_t n) {
    const size_t nblk = (size_t)((n + kLookupChunk - 1) / kLookupChunk);
    xyz = 0;
    sdf = al256(12 * (size_t)n);
    depth = sdf + al256(4 * (size_t)n);
    perm = depth + al256((size_t)n);
    counts = perm + al256(4 * (size_t)n);
    total = counts + al256(nblk * kBuckets * 4);
  }
};

struct Req {
  sand_model model = nullptr;
  sand_depthmap map = nullptr;
  const float* xyz_host = nullptr;
  float* sdf_host = nullptr;
  int64_t n = 0;
  size_t bytes = 0, off = 0;
  sand_req_stats st{};
  bool done = false;
  bool waiting = false;   // a sand_server_wait is blocked on this request
  sand_status status = SAND_OK;
};

struct Slot {
  sand_server srv = nullptr;
  hipStream_t stream = nullptr;
  BatchReq* desc_host = nullptr;   // pinned
  BatchReq* desc_dev = nullptr;
  int64_t* total_dev = nullptr;
  std::vector<Req*> reqs;
  bool busy = false;
};

}  // namespace

struct sand_server_s {
  int device = 0, prec = 0, num_cu = 0;
  size_t budget = 0;
  char* arena_dev = nullptr;
  Arena arena;
  std::vector<Slot*> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending, admitted;
  std::map<uint64_t, Req*> tickets;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread sched;
  uint64_t submitted = 0, completed = 0, batches = 0;
  int max_batch = 0;
  // host callbacks enqueued and not yet finished (destroy waits for zero)
  int callbacks = 0;
  void run();
  void launch(Slot* s);
};

namespace {

// Complete a batch: release its requests' memory and wake waiters. The
// notifications are sent while the lock is held, so once a thread that
// takes the lock sees the callback count at zero no callback touches the
// server again (sand_server_destroy relies on it).
void finish_batch(Slot* s, sand_status st, bool callback) {
  sand_server srv = s->srv;
  const double t = now_s();
  std::lock_guard<std::mutex> lk(srv->mu);
  for (Req* r : s->reqs) {
    if (r->st.t_done == 0.0) r->st.t_done = t;
    r->st.t_copied = t;
    r->status = st;
    r->done = true;
    srv->arena.release(r->off, r->bytes);
    ++srv->completed;
  }
  s->reqs.clear();
  s->busy = false;
  if (callback) --srv->callbacks;
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
}

void on_kernels_done(void* p) {
  Slot* s = (Slot*)p;
  const double t = now_s();
  std::lock_guard<std::mutex> lk(s->srv->mu);
  for (Req* r : s->reqs) r->st.t_done = t;
  --s->srv->callbacks;
  s->srv->cv_done.notify_all();
}

void on_copied(void* p) { finish_batch((Slot*)p, SAND_OK, true); }

// Enqueue a host callback, counted until it has run.
hipError_t add_callback(sand_server srv, hipStream_t stream, void (*fn)(void*), void* arg) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    ++srv->callbacks;
  }
  const hipError_t e = hipLaunchHostFunc(stream, fn, arg);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(srv->mu);
    --srv->callbacks;
  }
  return e;
}

}  // namespace

void sand_server_s::launch(Slot* s) {
  const double t = now_s();
  const int nreq = (int)s->reqs.size();
  const int WP = s->reqs[0]->model->WP;
  int64_t nblk = 0;
  for (int i = 0; i < nreq; ++i) {
    Req* r = s->reqs[i];
    const ReqLayout lay(r->n);
    char* base = arena_dev + r->off;
    BatchReq& d = s->desc_host[i];
    std::memset(&d, 0, sizeof(d));
    d.xyz = (const float*)(base + lay.xyz);
    d.sdf = (float*)(base + lay.sdf);
    d.depth = (uint8_t*)(base + lay.depth);
    d.perm = (int32_t*)(base + lay.perm);
    d.counts = (int32_t*)(base + lay.counts);
    d.map = r->map->depth;
    d.far = r->map->far;
    d.oct = r->map->oct;
    d.R = r->map->R;
    d.L = r->model->L;
    d.model = r->model->args_dev[prec];
    d.n = r->n;
    d.blk0 = nblk;
    nblk += (r->n + kLookupChunk - 1) / kLookupChunk;
    r->st.t_launch = t;
    r->st.batch_size = nreq;
  }
  hipError_t e = hipSuccess;
  for (int i = 0; i < nreq && e == hipSuccess; ++i)
    e = hipMemcpyAsync((void*)s->desc_host[i].xyz, s->reqs[i]->xyz_host, 12 * (size_t)s->reqs[i]->n,
                       hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->desc_dev, s->desc_host, nreq * sizeof(BatchReq), hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess)
    e = launch_bucketing_batch(s->desc_dev, nreq, nblk, 0, tmlp_tile_points(prec, WP), s->total_dev,
                               s->stream);
  if (e == hipSuccess) {
    BatchArgs ba{s->desc_dev, nreq, s->total_dev};
    e = launch_tmlp_batch(prec, WP, s->reqs[0]->model->act, ba, num_cu, s->stream);
  }
  if (e == hipSuccess) e = add_callback(this, s->stream, on_kernels_done, s);
  for (int i = 0; i < nreq && e == hipSuccess; ++i)
    e = hipMemcpyAsync(s->reqs[i]->sdf_host, s->desc_host[i].sdf, 4 * (size_t)s->reqs[i]->n,
                       hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = add_callback(this, s->stream, on_copied, s);
  if (e != hipSuccess) {
    // what was enqueued may still run; wait for it before releasing memory
    (void)hipStreamSynchronize(s->stream);
    finish_batch(s, SAND_ERR_DEVICE, false);
  }
}

void sand_server_s::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    const size_t first_new = admitted.size();
    if (admit_fifo(pending, admitted, arena) > 0) {
      const double t = now_s();
      for (size_t i = first_new; i < admitted.size(); ++i) admitted[i]->st.t_admit = t;
    }
    Slot* free_slot = nullptr;
    bool any_busy = false;
    for (Slot* s : slots) {
      if (!s->busy && !free_slot) free_slot = s;
      any_busy |= s->busy;
    }
    if (!admitted.empty() && free_slot) {
      // admitted requests of the head's padded width and activation, in
      // order, up to the point cap (the head always goes)
      free_slot->reqs = take_batch(admitted, kBatchPointCap, kMaxBatchRequests, [](const Req* r) {
        return std::make_pair(r->model->WP, r->model->act);
      });
      free_slot->busy = true;
      ++batches;
      max_batch = std::max(max_batch, (int)free_slot->reqs.size());
      lk.unlock();
      launch(free_slot);
      lk.lock();
      continue;
    }
    if (stopping && pending.empty() && admitted.empty() && !any_busy) break;
    cv_work.wait(lk);
  }
}

extern "C" sand_status sand_server_create(int device, size_t budget, int32_t precision,
                                          int32_t n_streams, sand_server* out) {
  if (!out) return fail(SAND_ERR_INVALID, "sand_server_create: null out");
  *out = nullptr;
  if (precision < 0 || precision > 2)
    return fail(SAND_ERR_INVALID, "sand_server_create: precision %d", precision);
  if (n_streams < 1 || n_streams > 16)
    return fail(SAND_ERR_INVALID, "sand_server_create: n_streams %d not in 1..16", n_streams);
  if (budget < (1u << 20)) return fail(SAND_ERR_INVALID, "sand_server_create: budget below 1 MiB");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(SAND_ERR_INVALID, "sand_server_create: device %d not available", device);
  DeviceGuard guard(device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_server_create: cannot select device");
  sand_server srv = new sand_server_s();
  srv->device = device;
  srv->prec = precision;
  srv->budget = budget;
  hipError_t e = hipDeviceGetAttribute(&srv->num_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess) e = hipMalloc((void**)&srv->arena_dev, budget);
  if (e != hipSuccess) {
    delete srv;
    return fail(SAND_ERR_NOMEM, "sand_server_create: arena of %zu bytes", budget);
  }
  srv->arena.init(budget);
  for (int i = 0; i < n_streams && e == hipSuccess; ++i) {
    Slot* s = new Slot();
    s->srv = srv;
    srv->slots.push_back(s);
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&s->desc_host, kMaxBatchRequests * sizeof(BatchReq), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s->desc_dev, kMaxBatchRequests * sizeof(BatchReq));
    if (e == hipSuccess) e = hipMalloc((void**)&s->total_dev, 256);
  }
  if (e != hipSuccess) {
    for (Slot* s : srv->slots) {
      if (s->stream) (void)hipStreamDestroy(s->stream);
      if (s->desc_host) (void)hipHostFree(s->desc_host);
      if (s->desc_dev) (void)hipFree(s->desc_dev);
      if (s->total_dev) (void)hipFree(s->total_dev);
      delete s;
    }
    (void)hipFree(srv->arena_dev);
    delete srv;
    return device_fail(e, "sand_server_create");
  }
  srv->sched = std::thread([srv] { srv->run(); });
  *out = srv;
  return SAND_OK;
}

extern "C" sand_status sand_server_submit(sand_server srv, sand_model m, sand_depthmap dm,
                                          const float* xyz, int64_t n, float* sdf,
                                          uint64_t* ticket) {
  if (!srv || !m || !dm || !ticket) return fail(SAND_ERR_INVALID, "sand_server_submit: null argument");
  if (n < 0 || n > 2147483647LL) return fail(SAND_ERR_INVALID, "sand_server_submit: n out of range");
  if (n > 0 && (!xyz || !sdf)) return fail(SAND_ERR_INVALID, "sand_server_submit: null buffer");
  if (dm->model != m) return fail(SAND_ERR_INVALID, "sand_server_submit: map of another model");
  if (m->device != srv->device)
    return fail(SAND_ERR_INVALID, "sand_server_submit: model on device %d, server on %d", m->device,
                srv->device);
  Req* r = new Req();
  r->model = m;
  r->map = dm;
  r->xyz_host = xyz;
  r->sdf_host = sdf;
  r->n = n;
  r->bytes = n > 0 ? ReqLayout(n).total : 0;
  r->st.n = n;
  r->st.t_submit = now_s();
  if (r->bytes > srv->budget) {
    delete r;
    return fail(SAND_ERR_BUDGET, "sand_server_submit: %lld points need %zu bytes, budget %zu",
                (long long)n, ReqLayout(n).total, srv->budget);
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) {
      delete r;
      return fail(SAND_ERR_INVALID, "sand_server_submit: server is shutting down");
    }
    *ticket = srv->next_ticket++;
    srv->tickets[*ticket] = r;
    ++srv->submitted;
    if (n == 0) {
      r->done = true;
      r->st.t_admit = r->st.t_launch = r->st.t_done = r->st.t_copied = r->st.t_submit;
      ++srv->completed;
    } else {
      srv->pending.push_back(r);
    }
  }
  srv->cv_work.notify_all();
  return SAND_OK;
}

extern "C" sand_status sand_server_wait(sand_server srv, uint64_t ticket, double timeout_s,
                                        sand_req_stats* stats) {
  if (!srv) return fail(SAND_ERR_INVALID, "sand_server_wait: null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end())
    return fail(SAND_ERR_INVALID, "sand_server_wait: unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second;
  if (r->waiting)
    return fail(SAND_ERR_INVALID, "sand_server_wait: ticket %llu already has a waiter",
                (unsigned long long)ticket);
  auto ready = [r] { return r->done; };
  r->waiting = true;
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    r->waiting = false;
    return fail(SAND_ERR_TIMEOUT, "sand_server_wait: ticket %llu not done after %.3f s",
                (unsigned long long)ticket, timeout_s);
  }
  if (stats) *stats = r->st;
  const sand_status st = r->status;
  srv->tickets.erase(it);
  delete r;
  if (st != SAND_OK) return fail(st, "sand_server_wait: request failed on the device");
  return SAND_OK;
}

extern "C" sand_status sand_server_stats(sand_server srv, sand_server_info* info) {
  if (!srv || !info) return fail(SAND_ERR_INVALID, "sand_server_stats: null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  std::memset(info, 0, sizeof(*info));
  info->budget_bytes = srv->budget;
  info->reserved_bytes = srv->arena.used;
  info->peak_reserved_bytes = srv->arena.peak;
  info->submitted = srv->submitted;
  info->completed = srv->completed;
  info->batches = srv->batches;
  info->max_batch_requests = srv->max_batch;
  int busy = 0;
  for (Slot* s : srv->slots) busy += s->busy;
  info->in_flight_batches = busy;
  return SAND_OK;
}

extern "C" void sand_server_destroy(sand_server srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  if (srv->sched.joinable()) srv->sched.join();
  {
    // every batch is complete and no host callback still reads the server
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [srv] { return srv->callbacks == 0; });
  }
  DeviceGuard guard(srv->device);
  for (Slot* s : srv->slots) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamDestroy(s->stream);
    (void)hipHostFree(s->desc_host);
    (void)hipFree(s->desc_dev);
    (void)hipFree(s->total_dev);
    delete s;
  }
  for (auto& kv : srv->tickets) delete kv.second;
  (void)hipFree(srv->arena_dev);
  delete srv;
}
