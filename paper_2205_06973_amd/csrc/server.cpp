// server.cpp -- continuous batching of many circuits on one GPU.
//
// Requests are partitioned and compiled on the submitting thread.  A worker
// thread then admits them in arrival order while the bytes of resident
// states (plus their plans) stay within the budget, allocates each state
// with the stream-ordered allocator on the least loaded stream of a pool,
// enqueues the set-basis kernel and one part-pass per part, and records an
// event.  It keeps polling those events: a finished request frees its slot
// on the stream, keeps its state resident until released, and has its
// latency (submit to observed completion) recorded.  Requests admitted while
// others are running overlap with them on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "hisv_internal.h"

using namespace hisv;

namespace {

using Clock = std::chrono::steady_clock;

enum ReqStatus { RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_FAILED, RQ_RELEASED };

struct Request {
  uint64_t ticket = 0;
  int n = 0;
  hs_dtype dtype = HS_C64;
  uint64_t init = 0;
  std::unique_ptr<Plan> plan;
  size_t bytes = 0;  // state + plan descriptors
  State st;
  int stream = -1;
  double work = 0;  // estimated device work: part-passes x state bytes
  hipEvent_t done = nullptr;
  Clock::time_point t_submit, t_done;
  ReqStatus status = RQ_QUEUED;
  hs_status err = HS_OK;
  std::string err_msg;
};

}  // namespace

struct hs_server_ {
  int device = 0;
  size_t budget = 0;
  size_t cur_bytes = 0, peak_bytes = 0;
  int peak_inflight = 0;
  uint64_t completed = 0;
  uint64_t next_ticket = 1;
  std::vector<hipStream_t> streams;
  std::vector<double> load;  // estimated outstanding work per stream
  hipStream_t read_stream = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::vector<Request*> running;
  std::map<uint64_t, Request*> reqs;
  bool stop = false;
  std::thread worker;
};

namespace {

size_t plan_bytes(const Plan& p, hs_dtype dt) {
  size_t b = 0;
  for (const CompiledPart& cp : p.comp[dt])
    b += sizeof(IPart) + cp.stages.size() * sizeof(IStage) +
         cp.ops.size() * (dt == HS_C64 ? sizeof(OpDesc<float>) : sizeof(OpDesc<double>));
  return b;
}

// Launch everything for an admitted request (called with the lock held) on
// the stream with the least outstanding work, so that small requests do not
// queue behind large ones when another stream is nearly idle.
hs_status launch(hs_server_* sv, Request* r) {
  int best = 0;
  for (int i = 1; i < (int)sv->streams.size(); ++i)
    if (sv->load[i] < sv->load[best]) best = i;
  r->stream = best;
  hipStream_t s = sv->streams[best];
  r->st.n = r->n;
  r->st.dtype = r->dtype;
  r->st.bytes = (size_t(1) << r->n) * amp_bytes(r->dtype);
  r->st.device = sv->device;
  r->st.stream = s;
  r->st.owned = true;
  hipError_t e = hipMallocAsync(&r->st.ptr, r->st.bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HS_E_NOMEM, "hipMallocAsync(%zu): %s", r->st.bytes, hipGetErrorString(e));
  }
  if (hs_status rc = dev_set_basis(&r->st, r->init)) return rc;
  for (int i = 0; i < (int)r->plan->parts.size(); ++i)
    if (hs_status rc = dev_run_part(&r->st, r->plan.get(), i)) return rc;
  e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(r->done, s);
  if (e != hipSuccess) return fail(HS_E_HIP, "event: %s", hipGetErrorString(e));
  sv->load[best] += r->work;
  return HS_OK;
}

void worker_main(hs_server_* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    bool progress = false;
    // retire finished requests
    for (size_t i = 0; i < sv->running.size();) {
      Request* r = sv->running[i];
      if (hipEventQuery(r->done) == hipSuccess) {
        r->t_done = Clock::now();
        r->status = RQ_DONE;
        sv->load[r->stream] -= r->work;
        sv->completed++;
        sv->running[i] = sv->running.back();
        sv->running.pop_back();
        progress = true;
      } else {
        ++i;
      }
    }
    // admit in arrival order while the budget allows
    while (!sv->queue.empty()) {
      Request* r = sv->queue.front();
      if (sv->cur_bytes + r->bytes > sv->budget) break;
      sv->queue.pop_front();
      sv->cur_bytes += r->bytes;
      sv->peak_bytes = std::max(sv->peak_bytes, sv->cur_bytes);
      hs_status rc = launch(sv, r);
      if (rc != HS_OK) {
        r->status = RQ_FAILED;
        r->err = rc;
        r->err_msg = hs_last_error();
        if (r->st.ptr) (void)hipFreeAsync(r->st.ptr, (hipStream_t)r->st.stream);
        r->st.ptr = nullptr;
        sv->cur_bytes -= r->bytes;
        r->t_done = Clock::now();
      } else {
        r->status = RQ_RUNNING;
        sv->running.push_back(r);
        sv->peak_inflight = std::max(sv->peak_inflight, (int)sv->running.size());
      }
      progress = true;
    }
    if (progress) sv->cv.notify_all();
    if (sv->stop && sv->queue.empty() && sv->running.empty()) break;
    if (!progress)
      sv->cv.wait_for(lk, std::chrono::microseconds(sv->running.empty() ? 2000 : 20));
  }
  sv->cv.notify_all();
}

Request* find(hs_server_* sv, uint64_t t) {
  auto it = sv->reqs.find(t);
  return it == sv->reqs.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

hs_status hs_server_create(size_t budget_bytes, int num_streams, hs_server* out) {
  if (!out) return fail(HS_E_ARG, "null output");
  if (num_streams < 1 || num_streams > 64) return fail(HS_E_ARG, "num_streams %d", num_streams);
  auto sv = std::make_unique<hs_server_>();
  if (hipGetDevice(&sv->device) != hipSuccess) return fail(HS_E_HIP, "no HIP device");
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(HS_E_HIP, "hipMemGetInfo failed");
  const size_t reserve = size_t(4) << 30;
  sv->budget = budget_bytes ? budget_bytes : (free_b > reserve ? free_b - reserve : free_b / 2);
  for (int i = 0; i < num_streams; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
      return fail(HS_E_HIP, "hipStreamCreate failed");
    sv->streams.push_back(s);
    sv->load.push_back(0);
  }
  if (hipStreamCreateWithFlags(&sv->read_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(HS_E_HIP, "hipStreamCreate failed");
  hs_server_* raw = sv.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return HS_OK;
}

hs_status hs_server_submit(hs_server sv, int n, const hs_gate* gates, size_t count, hs_dtype dtype,
                           uint64_t init_basis, int k, hs_strategy strategy, uint64_t* ticket) {
  if (!sv || !ticket || (!gates && count)) return fail(HS_E_ARG, "null argument");
  if (n < 1 || n > 40) return fail(HS_E_ARG, "n = %d outside [1, 40]", n);
  if (dtype != HS_C64 && dtype != HS_C128) return fail(HS_E_ARG, "bad dtype");
  if (init_basis >= (uint64_t(1) << n)) return fail(HS_E_ARG, "basis index outside the state");
  if (k < 1) return fail(HS_E_ARG, "k = %d < 1", k);
  auto r = std::make_unique<Request>();
  r->n = n;
  r->dtype = dtype;
  r->init = init_basis;
  std::vector<Gate> gs;
  gs.reserve(count);
  for (size_t i = 0; i < count; ++i)
    if (hs_status rc = expand_gate(n, gates[i], &gs)) return rc;
  for (const Gate& g : gs)
    if (g.arity() > k) return fail(HS_E_ARITY_GT_K, "gate wider than k = %d", k);
  std::vector<int32_t> part;
  const Dag dag = build_dag(gs);
  switch (strategy) {
    case HS_PART_NAT: partition_nat(gs, k, &part); break;
    case HS_PART_DFS: partition_dfs(gs, dag, k, 0x5eed + count, 16, &part); break;
    case HS_PART_DAGP: partition_dagp(gs, dag, n, k, 0x5eed + count, &part); break;
    case HS_PART_GREEDY: partition_greedy(gs, dag, k, 0x5eed + count, 16, &part); break;
    default: return fail(HS_E_ARG, "unknown strategy %d", (int)strategy);
  }
  r->plan = std::make_unique<Plan>();
  if (hs_status rc = plan_build(n, gs, k, part, r->plan.get())) return rc;
  if (hs_status rc = plan_compile(r->plan.get(), dtype)) return rc;
  r->bytes = (size_t(1) << n) * amp_bytes(dtype) + plan_bytes(*r->plan, dtype);
  r->work = (double)r->plan->parts.size() * (double)((size_t(1) << n) * amp_bytes(dtype));
  if (r->bytes > sv->budget)
    return fail(HS_E_ADMISSION, "request needs %zu bytes, budget is %zu", r->bytes, sv->budget);
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  r->ticket = sv->next_ticket++;
  *ticket = r->ticket;
  sv->reqs[r->ticket] = r.get();
  sv->queue.push_back(r.release());
  sv->cv.notify_all();
  return HS_OK;
}

hs_status hs_server_wait(hs_server sv, uint64_t ticket, int64_t timeout_ms) {
  if (!sv) return fail(HS_E_ARG, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  Request* r = find(sv, ticket);
  if (!r) return fail(HS_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  auto ready = [&] { return r->status == RQ_DONE || r->status == RQ_FAILED || r->status == RQ_RELEASED; };
  if (timeout_ms < 0) sv->cv.wait(lk, ready);
  else if (!sv->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return fail(HS_E_STATE, "ticket %llu not finished", (unsigned long long)ticket);
  if (r->status == RQ_FAILED) return fail(r->err, "request failed: %s", r->err_msg.c_str());
  return HS_OK;
}

hs_status hs_server_poll(hs_server sv, uint64_t ticket, int* done) {
  if (!sv || !done) return fail(HS_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  Request* r = find(sv, ticket);
  if (!r) return fail(HS_E_ARG, "unknown ticket");
  *done = (r->status == RQ_DONE || r->status == RQ_FAILED) ? 1 : 0;
  return HS_OK;
}

hs_status hs_server_read(hs_server sv, uint64_t ticket, uint64_t first, uint64_t count, double* out) {
  if (!sv || (!out && count)) return fail(HS_E_ARG, "null argument");
  State view;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    Request* r = find(sv, ticket);
    if (!r) return fail(HS_E_ARG, "unknown ticket");
    if (r->status != RQ_DONE) return fail(HS_E_STATE, "ticket is not finished");
    const uint64_t N = uint64_t(1) << r->n;
    if (first > N || count > N - first) return fail(HS_E_ARG, "range outside the state");
    view = r->st;
  }
  // read on a stream of its own, ordered after the request's kernels
  view.stream = sv->read_stream;
  view.owned = false;
  view.scratch = nullptr;
  view.scratch_bytes = 0;
  hs_status rc = count ? dev_read(&view, first, count, out, false) : HS_OK;
  if (view.scratch) (void)hipFree(view.scratch);
  return rc;
}

hs_status hs_server_latency(hs_server sv, uint64_t ticket, double* seconds) {
  if (!sv || !seconds) return fail(HS_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  Request* r = find(sv, ticket);
  if (!r) return fail(HS_E_ARG, "unknown ticket");
  if (r->status != RQ_DONE && r->status != RQ_RELEASED) return fail(HS_E_STATE, "ticket is not finished");
  *seconds = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  return HS_OK;
}

hs_status hs_server_release(hs_server sv, uint64_t ticket) {
  if (!sv) return fail(HS_E_ARG, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  Request* r = find(sv, ticket);
  if (!r) return fail(HS_E_ARG, "unknown ticket");
  if (r->status == RQ_RELEASED) return HS_OK;
  if (r->status != RQ_DONE && r->status != RQ_FAILED) return fail(HS_E_STATE, "ticket is not finished");
  if (r->status == RQ_DONE) {
    // the read stream may still hold copies of this state
    (void)hipStreamSynchronize(sv->read_stream);
    (void)hipFreeAsync(r->st.ptr, (hipStream_t)r->st.stream);
    r->st.ptr = nullptr;
    sv->cur_bytes -= r->bytes;
  }
  if (r->done) (void)hipEventDestroy(r->done);
  r->done = nullptr;
  r->plan.reset();
  r->status = RQ_RELEASED;
  sv->cv.notify_all();
  return HS_OK;
}

hs_status hs_server_stats(hs_server sv, uint64_t* completed, uint64_t* peak_bytes, uint64_t* cur_bytes,
                          int* peak_inflight) {
  if (!sv) return fail(HS_E_ARG, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (completed) *completed = sv->completed;
  if (peak_bytes) *peak_bytes = sv->peak_bytes;
  if (cur_bytes) *cur_bytes = sv->cur_bytes;
  if (peak_inflight) *peak_inflight = sv->peak_inflight;
  return HS_OK;
}

hs_status hs_server_destroy(hs_server sv) {
  if (!sv) return HS_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->device);
  for (auto& kv : sv->reqs) {
    Request* r = kv.second;
    if (r->st.ptr) (void)hipFreeAsync(r->st.ptr, (hipStream_t)r->st.stream);
    if (r->done) (void)hipEventDestroy(r->done);
    delete r;
  }
  for (hipStream_t s : sv->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  (void)hipStreamSynchronize(sv->read_stream);
  (void)hipStreamDestroy(sv->read_stream);
  delete sv;
  return HS_OK;
}

}  // extern "C"
