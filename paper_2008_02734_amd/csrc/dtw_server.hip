// Serving loop: continuous batching of alignment requests over one device
// memory pool (API and contract in include/dtw.h).  A scheduler thread owns
// the pool allocator, the slots (one stream, one completion event and one
// pinned error word each) and the HIP calls; submitters and pollers only touch
// the queue and the request table under the mutex.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dtw.h"
#include "dtw_pool.h"

namespace dtw {
dtw_status batch_workspace(int32_t B, const int64_t* x_offsets, const int64_t* y_offsets, int32_t d,
                           int32_t in_dtype, const dtw_opts* opts, size_t* bytes);
dtw_status enqueue_batch(int32_t B, const void* X, const int64_t* xo, const void* Y, const int64_t* yo, int32_t d,
                         int32_t in_dtype, const dtw_opts* opts, void* ws, size_t ws_bytes, double* costs,
                         int32_t* paths, const int64_t* path_offsets, int64_t* lens, hipStream_t st,
                         int32_t** device_error_word);
}  // namespace dtw

namespace {

using dtw::PoolAllocator;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  dtw_request r;
  dtw_result res;
  bool done = false;
};

// Layout of one batch inside its pool block.
struct BatchPlan {
  std::vector<uint64_t> tickets;
  std::vector<int64_t> xo, yo, po;  // B+1 frame / path offsets
  size_t ws_bytes = 0, total = 0;
  size_t off_ws = 0, off_x = 0, off_y = 0, off_cost = 0, off_path = 0, off_len = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t* err_host = nullptr;  // pinned
  bool busy = false;
  size_t pool_off = SIZE_MAX;
  BatchPlan plan;
  int32_t status = DTW_OK;
};

size_t elem_bytes(int32_t in_dtype) { return in_dtype == DTW_F64 ? 8 : 4; }

bool same_class(const dtw_request& a, const dtw_request& b) {
  return a.d == b.d && a.in_dtype == b.in_dtype && a.opts.precision == b.opts.precision &&
         a.opts.min_block == b.opts.min_block && a.opts.cost == b.opts.cost &&
         a.opts.tie_exact == b.opts.tie_exact;
}

// Footprint of a batch made of `reqs`; fills the plan's offsets.  Returns
// the status of the workspace query (DTW_OK when the batch is valid).
dtw_status plan_batch(const std::vector<const dtw_request*>& reqs, BatchPlan* bp) {
  const int B = (int)reqs.size();
  bp->xo.assign(B + 1, 0);
  bp->yo.assign(B + 1, 0);
  bp->po.assign(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    bp->xo[b + 1] = bp->xo[b] + reqs[b]->M;
    bp->yo[b + 1] = bp->yo[b] + reqs[b]->N;
    bp->po[b + 1] = bp->po[b] + reqs[b]->M + reqs[b]->N - 1;
  }
  const dtw_request& r0 = *reqs[0];
  dtw_status rc = dtw::batch_workspace(B, bp->xo.data(), bp->yo.data(), r0.d, r0.in_dtype, &r0.opts, &bp->ws_bytes);
  if (rc != DTW_OK) return rc;
  const size_t eb = elem_bytes(r0.in_dtype);
  size_t t = 0;
  auto put = [&](size_t bytes) {
    const size_t off = t;
    t = PoolAllocator::round_up(t + bytes);
    return off;
  };
  bp->off_ws = put(bp->ws_bytes);
  bp->off_x = put(eb * (size_t)bp->xo[B] * r0.d);
  bp->off_y = put(eb * (size_t)bp->yo[B] * r0.d);
  bp->off_cost = put(8 * (size_t)B);
  bp->off_path = put(8 * (size_t)bp->po[B]);
  bp->off_len = put(8 * (size_t)B);
  bp->total = t;
  return DTW_OK;
}

}  // namespace

struct dtw_server {
  dtw_server_opts opts{};
  void* pool = nullptr;
  PoolAllocator alloc;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  int32_t fatal = DTW_OK;
  std::thread thread;

  void run();
  bool collect();
  bool admit();
  void fail_batch(Slot& s, int32_t status);
};

// Mark a finished (or failed) batch's requests done and free its resources.
void dtw_server::fail_batch(Slot& s, int32_t status) {
  const int64_t t = now_ns();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (uint64_t tk : s.plan.tickets) {
      auto it = reqs.find(tk);
      if (it == reqs.end()) continue;
      it->second.res.status = status;
      it->second.res.device_error = (s.err_host && status == DTW_ERR_INTERNAL) ? *s.err_host : 0;
      it->second.res.t_done_ns = t;
      it->second.done = true;
    }
  }
  cv_done.notify_all();
  if (s.pool_off != SIZE_MAX) alloc.release(s.pool_off);
  s.pool_off = SIZE_MAX;
  s.busy = false;
}

// Completed slots: results out, pool block and slot back.  True if any.
bool dtw_server::collect() {
  bool any = false;
  for (Slot& s : slots) {
    if (!s.busy) continue;
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) continue;
    int32_t status = s.status;
    if (q != hipSuccess) status = DTW_ERR_HIP;
    else if (*s.err_host != 0) status = DTW_ERR_INTERNAL;
    fail_batch(s, status);
    any = true;
  }
  return any;
}

// Form and launch batches while a slot is free and the head of the queue
// fits in the pool.  True if any batch was launched.
bool dtw_server::admit() {
  bool any = false;
  for (Slot& s : slots) {
    if (s.busy) continue;
    std::vector<const dtw_request*> cand;
    BatchPlan plan, best;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (queue.empty()) return any;
      const size_t room = alloc.largest_free();
      // the head of the queue, then later requests of its class in
      // submission order, while the batch fits
      for (uint64_t tk : queue) {
        if ((int)cand.size() >= opts.max_batch) break;
        const dtw_request& r = reqs[tk].r;
        if (!cand.empty() && !same_class(*cand[0], r)) continue;
        cand.push_back(&r);
        plan.tickets.push_back(tk);
        if (plan_batch(cand, &plan) != DTW_OK || plan.total > room) {
          cand.pop_back();
          plan.tickets.pop_back();
          break;
        }
        best = plan;
      }
      if (cand.empty()) return any;  // the head waits for memory
      plan_batch(cand, &best);
      const int64_t t = now_ns();
      for (uint64_t tk : best.tickets) {
        for (auto it = queue.begin(); it != queue.end(); ++it)
          if (*it == tk) {
            queue.erase(it);
            break;
          }
        Req& q = reqs[tk];
        q.res.t_admit_ns = t;
        q.res.batch_size = (int32_t)best.tickets.size();
      }
    }
    const size_t off = alloc.alloc(best.total);
    s.plan = best;
    s.pool_off = off;
    s.busy = true;
    s.status = DTW_OK;
    *s.err_host = 0;
    if (off == SIZE_MAX) {  // cannot happen: the plan was sized to the largest free block
      fail_batch(s, DTW_ERR_WORKSPACE);
      continue;
    }
    char* base = static_cast<char*>(pool) + off;
    const dtw_request& r0 = *cand[0];
    const int B = (int)cand.size();
    const size_t eb = elem_bytes(r0.in_dtype);
    hipError_t e = hipSuccess;
    for (int b = 0; b < B && e == hipSuccess; ++b) {
      e = hipMemcpyAsync(base + best.off_x + eb * best.xo[b] * r0.d, cand[b]->X, eb * cand[b]->M * r0.d,
                         hipMemcpyDeviceToDevice, s.stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(base + best.off_y + eb * best.yo[b] * r0.d, cand[b]->Y, eb * cand[b]->N * r0.d,
                           hipMemcpyDeviceToDevice, s.stream);
    }
    int32_t* err_dev = nullptr;
    dtw_status rc = DTW_OK;
    if (e == hipSuccess)
      rc = dtw::enqueue_batch(B, base + best.off_x, best.xo.data(), base + best.off_y, best.yo.data(), r0.d,
                              r0.in_dtype, &r0.opts, base + best.off_ws, best.ws_bytes,
                              reinterpret_cast<double*>(base + best.off_cost),
                              reinterpret_cast<int32_t*>(base + best.off_path), best.po.data(),
                              reinterpret_cast<int64_t*>(base + best.off_len), s.stream, &err_dev);
    for (int b = 0; b < B && e == hipSuccess && rc == DTW_OK; ++b) {
      const dtw_request& r = *cand[b];
      e = hipMemcpyAsync(r.cost_out, base + best.off_cost + 8 * b, 8, hipMemcpyDeviceToDevice, s.stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(r.path_out, base + best.off_path + 8 * best.po[b], 8 * (r.M + r.N - 1),
                           hipMemcpyDeviceToDevice, s.stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(r.path_len_out, base + best.off_len + 8 * b, 8, hipMemcpyDeviceToDevice, s.stream);
    }
    if (e == hipSuccess && rc == DTW_OK && err_dev)
      e = hipMemcpyAsync(s.err_host, err_dev, 4, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess || rc != DTW_OK) {
      (void)hipStreamSynchronize(s.stream);  // nothing of the batch may still run when its block is reused
      *s.err_host = 0;
      fail_batch(s, rc != DTW_OK ? rc : DTW_ERR_HIP);
      continue;
    }
    any = true;
  }
  return any;
}

void dtw_server::run() {
  if (hipSetDevice(opts.device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    fatal = DTW_ERR_HIP;
  }
  for (;;) {
    const bool did = collect() | admit();
    bool busy = false;
    for (const Slot& s : slots) busy |= s.busy;
    std::unique_lock<std::mutex> lk(mu);
    if (stop && queue.empty() && !busy) break;
    if (did) continue;
    if (busy) cv_work.wait_for(lk, std::chrono::microseconds(20));  // poll the running batches
    else if (queue.empty()) cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    else cv_work.wait_for(lk, std::chrono::microseconds(200));       // head waits for memory
  }
}

extern "C" {

void dtw_server_default_opts(dtw_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->pool_bytes = (size_t)8 << 30;
  o->max_slots = 4;
  o->max_batch = 64;
  o->device = 0;
}

dtw_status dtw_server_create(const dtw_server_opts* opts, dtw_server** out) {
  if (!out) return DTW_ERR_INVALID_ARG;
  *out = nullptr;
  dtw_server_opts o;
  dtw_server_default_opts(&o);
  if (opts) o = *opts;
  if (o.max_slots < 1 || o.max_slots > 16 || o.max_batch < 1 || o.pool_bytes < PoolAllocator::kAlign)
    return DTW_ERR_INVALID_ARG;
  for (int i = 0; i < 5; ++i)
    if (o.reserved[i] != 0) return DTW_ERR_INVALID_ARG;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(o.device) != hipSuccess) return DTW_ERR_HIP;
  dtw_server* s = new dtw_server();
  s->opts = o;
  dtw_status rc = DTW_OK;
  if (hipMalloc(&s->pool, o.pool_bytes) != hipSuccess) rc = DTW_ERR_HIP;
  s->alloc.reset(o.pool_bytes);
  s->slots.resize(o.max_slots);
  for (Slot& sl : s->slots) {
    if (rc != DTW_OK) break;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.err_host), 4, hipHostMallocDefault) != hipSuccess)
      rc = DTW_ERR_HIP;
  }
  (void)hipSetDevice(prev);
  if (rc != DTW_OK) {
    for (Slot& sl : s->slots) {
      if (sl.err_host) (void)hipHostFree(sl.err_host);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return rc;
  }
  s->thread = std::thread([s] { s->run(); });
  *out = s;
  return DTW_OK;
}

dtw_status dtw_server_submit(dtw_server* s, const dtw_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket || !r->X || !r->Y || !r->cost_out || !r->path_out || !r->path_len_out) return DTW_ERR_INVALID_ARG;
  if (r->M < 1 || r->N < 1 || r->d < 1 || r->M > INT32_MAX || r->N > INT32_MAX) return DTW_ERR_INVALID_ARG;
  if (r->in_dtype != DTW_F64 && r->in_dtype != DTW_F32) return DTW_ERR_INVALID_ARG;
  if (r->path_cap < r->M + r->N - 1) return DTW_ERR_CAPACITY;
  std::vector<const dtw_request*> one{r};
  BatchPlan bp;
  dtw_status rc = plan_batch(one, &bp);
  if (rc != DTW_OK) return rc;
  if (bp.total > s->alloc.size()) return DTW_ERR_WORKSPACE;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != DTW_OK) return (dtw_status)s->fatal;
    if (s->stop) return DTW_ERR_INVALID_ARG;
    const uint64_t tk = s->next_ticket++;
    Req q;
    q.r = *r;
    std::memset(&q.res, 0, sizeof(q.res));
    q.res.status = DTW_ERR_BUSY;
    q.res.t_submit_ns = now_ns();
    s->reqs[tk] = q;
    s->queue.push_back(tk);
    *ticket = tk;
  }
  s->cv_work.notify_one();
  return DTW_OK;
}

static dtw_status take_result(dtw_server* s, uint64_t ticket, dtw_result* out, bool block) {
  if (!s || !out) return DTW_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DTW_ERR_NOT_FOUND;
  if (block) s->cv_done.wait(lk, [&] { return it->second.done; });
  if (!it->second.done) return DTW_ERR_BUSY;
  *out = it->second.res;
  s->reqs.erase(it);
  return DTW_OK;
}

dtw_status dtw_server_poll(dtw_server* s, uint64_t ticket, dtw_result* out) { return take_result(s, ticket, out, false); }
dtw_status dtw_server_wait(dtw_server* s, uint64_t ticket, dtw_result* out) { return take_result(s, ticket, out, true); }

dtw_status dtw_server_destroy(dtw_server* s) {
  if (!s) return DTW_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->opts.device);
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.err_host) (void)hipHostFree(sl.err_host);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  const hipError_t e = s->pool ? hipFree(s->pool) : hipSuccess;
  (void)hipSetDevice(prev);
  delete s;
  return e == hipSuccess ? DTW_OK : DTW_ERR_HIP;
}

}  // extern "C"
