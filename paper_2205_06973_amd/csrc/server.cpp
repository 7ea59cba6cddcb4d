// server.cpp -- continuous batching of many circuits on one GPU.
//
// A request's life:
//   submit    the caller's thread copies and validates the gate list, checks
//             that the state could ever fit the byte budget, and queues the
//             request; nothing else happens on that thread, so an arrival
//             loop keeps its schedule.  The latency clock starts at the
//             request's arrival time (given by the caller on the server
//             clock, or the time of the call).
//   prepare   one of a pool of host threads partitions the circuit, compiles
//             the interpreter descriptors and queues their upload with the
//             stream-ordered allocator on its own stream -- all without the
//             server lock, and without waiting for the copies: a preparing
//             stream can share a hardware queue with long part kernels, and
//             a host wait there held small requests behind large ones.
//   admit     the worker thread admits prepared requests strictly in ticket
//             order while the bytes of resident states (plus their
//             descriptors) stay within the budget, allocates the state on the
//             stream of a pool with the least unfinished work, makes that
//             stream wait (on the device) for the descriptor copies, and
//             enqueues set-basis and the part-passes -- a chunk of parts at a
//             time, at most two chunks queued, refilled as chunks finish, so
//             a request admitted behind a large one on the same hardware
//             queue waits for two chunks, not for the large one's whole
//             circuit.  An event follows the last part.
//             Requests admitted while others run overlap with them on the
//             device.  (Preparation finishes out of order on the host
//             threads; admitting in that order could let later requests
//             fill the budget and hold it until released, while a client
//             releasing in submission order waits for an earlier one that
//             no longer fits.)
//   retire    the worker polls the events; a finished request keeps its state
//             resident until it is read and released.
//   release   state and descriptors go back with hipFreeAsync (no device-wide
//             wait), outside the server lock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "hisv_internal.h"

using namespace hisv;

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

enum ReqStatus { RQ_QUEUED, RQ_PREPARING, RQ_READY, RQ_RUNNING, RQ_DONE, RQ_FAILED, RQ_RELEASED };

struct Request {
  uint64_t ticket = 0;
  int n = 0, k = 0;
  hs_dtype dtype = HS_C64;
  hs_strategy strategy = HS_PART_GREEDY;
  uint64_t init = 0;
  std::vector<Gate> gates;
  std::unique_ptr<Plan> plan;
  size_t bytes = 0;  // state + plan descriptors
  State st;
  int stream = -1;
  hipEvent_t done = nullptr;  // recorded after the last part
  // parts go to the device a chunk at a time, at most two chunks queued
  int next_part = 0;                           // first part not yet enqueued
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // recorded after each chunk
  double chunk_work[2] = {0, 0};
  int chunk_old = 0;                           // slot of the oldest queued chunk
  int chunks_out = 0;                          // chunks queued, not seen finished
  int chunk_parts = 8;                         // parts a chunk
  double remaining = 0;                        // its work not seen finished (stream load)
  bool launched = false;                       // work was queued on its stream
  int readers = 0;                             // hs_server_read calls copying its state
  // server clock (seconds): arrival, preparation start and end, launch, done
  double t_arrival = 0, t_prep0 = 0, t_prep1 = 0, t_launch = 0, t_done = 0;
  ReqStatus status = RQ_QUEUED;
  hs_status err = HS_OK;
  std::string err_msg;
};

constexpr int kPrepThreads = 4;
constexpr size_t kReadScratch = size_t(64) << 20;  // covers dev_read's largest chunk
constexpr size_t kPinnedStaging = size_t(8) << 20;  // descriptor staging per preparing thread
// Parts a request enqueues at a time (hs_tune "serve_chunk", default 8,
// read at launch).  A hardware queue runs its commands in order, so a
// request admitted behind a large one waits for what the large one has
// queued: at most two chunks, a few milliseconds, instead of hundreds of
// part-passes.

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
  std::vector<hipStream_t> prep_streams;
  std::vector<PinnedStaging> pins;  // one per preparing thread
  hipStream_t read_stream = nullptr;
  void* read_scratch = nullptr;  // persistent staging of hs_server_read
  std::mutex read_mu;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> prep_queue;
  std::map<uint64_t, Request*> ready;  // prepared, waiting for admission (ticket order)
  uint64_t next_admit = 1;              // the lowest ticket not yet admitted or failed
  std::vector<Request*> running;
  std::map<uint64_t, Request*> reqs;
  bool stop = false;
  std::thread worker;
  std::vector<std::thread> preppers;
};

namespace {

size_t plan_bytes(const Plan& p, hs_dtype dt) {
  size_t b = 0;
  for (const CompiledPart& cp : p.comp[dt])
    b += sizeof(IPart) + cp.stages.size() * sizeof(IStage) +
         cp.ops.size() * (dt == HS_C64 ? sizeof(OpDesc<float>) : sizeof(OpDesc<double>));
  return b;
}

// Partition, compile and upload one request (no server lock held).
hs_status prepare(hs_server_* sv, Request* r, hipStream_t stream, const PinnedStaging* pin) {
  const std::vector<Gate>& gs = r->gates;
  std::vector<int32_t> part;
  const Dag dag = build_dag(gs);
  const uint64_t seed = 0x5eed + gs.size();
  switch (r->strategy) {
    case HS_PART_NAT: partition_nat(gs, r->k, &part); break;
    case HS_PART_DFS: partition_dfs(gs, dag, r->k, seed, 16, &part); break;
    case HS_PART_DAGP: partition_dagp(gs, dag, r->n, r->k, seed, &part); break;
    case HS_PART_GREEDY: partition_greedy(gs, dag, r->k, seed, 16, &part); break;
    case HS_PART_CLOSURE: partition_closure(gs, dag, r->k, 1, &part); break;
    default: return fail(HS_E_ARG, "unknown strategy %d", (int)r->strategy);
  }
  auto plan = std::make_unique<Plan>();
  if (hs_status rc = plan_build(r->n, gs, r->k, part, plan.get())) return rc;
  if (hs_status rc = plan_compile(plan.get(), r->dtype)) return rc;
  r->bytes = (size_t(1) << r->n) * amp_bytes(r->dtype) + plan_bytes(*plan, r->dtype);
  if (r->bytes > sv->budget)
    return fail(HS_E_ADMISSION, "request needs %zu bytes, budget is %zu", r->bytes, sv->budget);
  if (hs_status rc = dev_plan_upload_async(plan.get(), r->dtype, sv->device, stream, pin)) return rc;
  r->plan = std::move(plan);
  r->gates.clear();
  r->gates.shrink_to_fit();
  return HS_OK;
}

void prep_main(hs_server_* sv, int idx) {
  (void)hipSetDevice(sv->device);
  hipStream_t stream = sv->prep_streams[idx];
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    sv->cv.wait(lk, [&] { return sv->stop || !sv->prep_queue.empty(); });
    if (sv->prep_queue.empty()) break;  // stopping and nothing left
    Request* r = sv->prep_queue.front();
    sv->prep_queue.pop_front();
    r->status = RQ_PREPARING;
    lk.unlock();
    r->t_prep0 = now_s();
    hs_status rc = guarded([&] { return prepare(sv, r, stream, &sv->pins[idx]); });
    r->t_prep1 = now_s();
    lk.lock();
    if (rc == HS_OK) rc = guarded([&] {
      sv->ready.emplace(r->ticket, r);
      return HS_OK;
    });
    if (rc) {
      r->status = RQ_FAILED;
      r->err = rc;
      r->err_msg = hs_last_error();  // this thread's message
      r->t_done = r->t_prep1;
    } else {
      r->status = RQ_READY;
    }
    sv->cv.notify_all();
  }
}

Request* find(hs_server_* sv, uint64_t t) {
  auto it = sv->reqs.find(t);
  return it == sv->reqs.end() ? nullptr : it->second;
}

// Enqueue the request's next chunk of parts (lock held; nothing waits on the
// device) and, after the last part, its done event.
hs_status enqueue_chunk(hs_server_* sv, Request* r) {
  hipStream_t s = sv->streams[r->stream];
  const int P = (int)r->plan->parts.size();
  const int first = r->next_part, last = std::min(P, first + r->chunk_parts);
  for (int i = first; i < last; ++i)
    if (hs_status rc = dev_run_part(&r->st, r->plan.get(), i)) return rc;
  r->next_part = last;
  const int slot = (r->chunk_old + r->chunks_out) & 1;
  if (hipEventRecord(r->chunk_ev[slot], s) != hipSuccess) return fail(HS_E_HIP, "event record failed");
  r->chunk_work[slot] = (double)(last - first) * (double)r->st.bytes;
  r->chunks_out++;
  if (last == P) {
    hipError_t e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->done, s);
    if (e != hipSuccess) return fail(HS_E_HIP, "event: %s", hipGetErrorString(e));
  }
  return HS_OK;
}

// Chunks of a running request that have finished leave the stream's load;
// new ones are queued while fewer than two are outstanding.
hs_status feed(hs_server_* sv, Request* r, bool* progress) {
  while (r->chunks_out > 0 && hipEventQuery(r->chunk_ev[r->chunk_old]) == hipSuccess) {
    sv->load[r->stream] -= r->chunk_work[r->chunk_old];
    r->remaining -= r->chunk_work[r->chunk_old];
    r->chunk_old ^= 1;
    r->chunks_out--;
    *progress = true;
  }
  while (r->next_part < (int)r->plan->parts.size() && r->chunks_out < 2) {
    if (hs_status rc = enqueue_chunk(sv, r)) return rc;
    *progress = true;
  }
  return HS_OK;
}

// Start an admitted request (called with the lock held; nothing here waits
// on the device) on the stream with the least unfinished work (all parts of
// its requests, queued or not), so that requests spread over the streams:
// the state, a wait for the descriptor copies, set-basis and the first
// chunks of parts.
hs_status launch(hs_server_* sv, Request* r) {
  int best = 0;
  for (int i = 1; i < (int)sv->streams.size(); ++i)
    if (sv->load[i] < sv->load[best]) best = i;
  r->stream = best;
  r->chunk_parts = serve_chunk_parts();
  r->remaining = (double)r->plan->parts.size() * (double)((size_t(1) << r->n) * amp_bytes(r->dtype));
  sv->load[best] += r->remaining;
  hipStream_t s = sv->streams[best];
  r->st.n = r->n;
  r->st.dtype = r->dtype;
  r->st.bytes = (size_t(1) << r->n) * amp_bytes(r->dtype);
  r->st.device = sv->device;
  r->st.stream = s;
  r->st.owned = true;
  r->launched = true;
  hipError_t e = hipMallocAsync(&r->st.ptr, r->st.bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    r->st.ptr = nullptr;
    return fail(HS_E_NOMEM, "hipMallocAsync(%zu): %s", r->st.bytes, hipGetErrorString(e));
  }
  for (hipEvent_t& ev : r->chunk_ev)
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
      return fail(HS_E_HIP, "event create failed");
  // the descriptors were copied on a preparing stream: wait for them here,
  // on the device
  if (hs_status rc = dev_plan_stream_wait(r->plan.get(), r->dtype, sv->device, s)) return rc;
  if (hs_status rc = dev_set_basis(&r->st, r->init)) return rc;
  if (r->plan->parts.empty()) {  // no gates: set-basis is the whole request
    hipError_t e2 = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
    if (e2 == hipSuccess) e2 = hipEventRecord(r->done, s);
    if (e2 != hipSuccess) return fail(HS_E_HIP, "event: %s", hipGetErrorString(e2));
    return HS_OK;
  }
  bool progress = false;
  return feed(sv, r, &progress);
}

// Give back what a failed running request holds (lock held).
void fail_running(hs_server_* sv, Request* r, hs_status rc) {
  r->status = RQ_FAILED;
  r->err = rc;
  r->err_msg = hs_last_error();
  if (r->stream >= 0) sv->load[r->stream] -= r->remaining;
  r->remaining = 0;
  r->chunks_out = 0;
  if (r->st.ptr) (void)hipFreeAsync(r->st.ptr, (hipStream_t)r->st.stream);  // after its queued kernels
  r->st.ptr = nullptr;
  sv->cur_bytes -= r->bytes;
  r->t_done = now_s();
}

void worker_main(hs_server_* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    bool progress = false;
    // feed running requests their next chunks; retire finished ones
    for (size_t i = 0; i < sv->running.size();) {
      Request* r = sv->running[i];
      if (hs_status rc = guarded([&] { return feed(sv, r, &progress); })) {
        fail_running(sv, r, rc);
        sv->running[i] = sv->running.back();
        sv->running.pop_back();
        progress = true;
        continue;
      }
      if (r->done && hipEventQuery(r->done) == hipSuccess) {
        r->t_done = now_s();
        r->status = RQ_DONE;
        sv->load[r->stream] -= r->remaining;
        r->remaining = 0;
        r->chunks_out = 0;
        sv->completed++;
        sv->running[i] = sv->running.back();
        sv->running.pop_back();
        progress = true;
      } else {
        ++i;
      }
    }
    // admit prepared requests strictly in ticket order while the budget
    // allows: skip tickets that failed in preparation, stop at one still
    // being prepared or one that does not fit yet
    while (sv->next_admit < sv->next_ticket) {
      Request* nr = find(sv, sv->next_admit);
      if (!nr || nr->status == RQ_FAILED || nr->status == RQ_RELEASED) {
        ++sv->next_admit;
        continue;
      }
      if (nr->status != RQ_READY) break;
      Request* r = nr;
      if (sv->cur_bytes + r->bytes > sv->budget) break;
      sv->ready.erase(r->ticket);
      ++sv->next_admit;
      sv->cur_bytes += r->bytes;
      sv->peak_bytes = std::max(sv->peak_bytes, sv->cur_bytes);
      r->t_launch = now_s();
      hs_status rc = guarded([&] { return launch(sv, r); });
      if (rc == HS_OK) rc = guarded([&] {
        sv->running.push_back(r);
        return HS_OK;
      });
      if (rc != HS_OK) {
        fail_running(sv, r, rc);
      } else {
        r->status = RQ_RUNNING;
        sv->peak_inflight = std::max(sv->peak_inflight, (int)sv->running.size());
      }
      progress = true;
    }
    if (progress) sv->cv.notify_all();
    if (sv->stop && sv->prep_queue.empty() && sv->running.empty()) {
      bool preparing = false;
      for (auto& kv : sv->reqs) preparing |= kv.second->status == RQ_PREPARING;
      if (!preparing) {
        // nothing runs and nothing more will be released: whatever is still
        // waiting did not fit above and never will
        for (auto& kv : sv->ready) {
          Request* r = kv.second;
          r->status = RQ_FAILED;
          r->err = HS_E_ADMISSION;
          r->err_msg = "server stopped before the request could be admitted";
          r->t_done = now_s();
        }
        sv->ready.clear();
        break;
      }
    }
    if (!progress)
      sv->cv.wait_for(lk, std::chrono::microseconds(sv->running.empty() ? 2000 : 20));
  }
  sv->cv.notify_all();
}

// Free a request's device memory and handles; no lock held.
void drop_request_memory(hs_server_* sv, std::unique_ptr<Plan> plan, void* state,
                         hipStream_t stream, const std::vector<hipEvent_t>& events, bool drain) {
  (void)hipSetDevice(sv->device);
  // a request that failed with parts queued: they may still read the
  // descriptors, which are freed on another stream (rare; waits here)
  if (drain && stream) (void)hipStreamSynchronize(stream);
  if (state) (void)hipFreeAsync(state, stream);
  plan.reset();  // descriptors: hipFreeAsync on the preparing stream
  for (hipEvent_t ev : events)
    if (ev) (void)hipEventDestroy(ev);
}

}  // namespace

extern "C" {

hs_status hs_server_create(size_t budget_bytes, int num_streams, hs_server* out) {
  return guarded([&]() -> hs_status {
    if (!out) return fail(HS_E_ARG, "null output");
    if (num_streams < 1 || num_streams > 64) return fail(HS_E_ARG, "num_streams %d", num_streams);
    auto sv = std::make_unique<hs_server_>();
    if (hipGetDevice(&sv->device) != hipSuccess) return fail(HS_E_HIP, "no HIP device");
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(HS_E_HIP, "hipMemGetInfo failed");
    const size_t reserve = size_t(4) << 30;
    sv->budget = budget_bytes ? budget_bytes : (free_b > reserve ? free_b - reserve : free_b / 2);
    auto new_stream = [](hipStream_t* s) {
      return hipStreamCreateWithFlags(s, hipStreamNonBlocking) == hipSuccess;
    };
    auto cleanup = [&]() {
      for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
      for (hipStream_t s : sv->prep_streams) (void)hipStreamDestroy(s);
      for (PinnedStaging& p : sv->pins) {
        if (p.ptr) (void)hipHostFree(p.ptr);
        if (p.busy) (void)hipEventDestroy((hipEvent_t)p.busy);
      }
      if (sv->read_stream) (void)hipStreamDestroy(sv->read_stream);
      if (sv->read_scratch) (void)hipFree(sv->read_scratch);
    };
    for (int i = 0; i < num_streams; ++i) {
      hipStream_t s;
      if (!new_stream(&s)) {
        cleanup();
        return fail(HS_E_HIP, "hipStreamCreate failed");
      }
      sv->streams.push_back(s);
      sv->load.push_back(0);
    }
    for (int i = 0; i < kPrepThreads; ++i) {
      hipStream_t s;
      if (!new_stream(&s)) {
        cleanup();
        return fail(HS_E_HIP, "hipStreamCreate failed");
      }
      sv->prep_streams.push_back(s);
      // pinned staging for its descriptor copies (without it, copies go from
      // pageable memory)
      PinnedStaging p;
      hipEvent_t ev = nullptr;
      if (hipHostMalloc(&p.ptr, kPinnedStaging, hipHostMallocDefault) == hipSuccess &&
          hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
        p.bytes = kPinnedStaging;
        p.busy = ev;
      } else {
        (void)hipGetLastError();
        if (p.ptr) (void)hipHostFree(p.ptr);
        p = PinnedStaging{};
      }
      sv->pins.push_back(p);
    }
    if (!new_stream(&sv->read_stream)) {
      cleanup();
      return fail(HS_E_HIP, "hipStreamCreate failed");
    }
    if (hipMalloc(&sv->read_scratch, kReadScratch) != hipSuccess) {
      (void)hipGetLastError();
      sv->read_scratch = nullptr;
      cleanup();
      return fail(HS_E_NOMEM, "read staging buffer of %zu bytes", kReadScratch);
    }
    hs_server_* raw = sv.get();
    try {
      raw->worker = std::thread(worker_main, raw);
      for (int i = 0; i < kPrepThreads; ++i) raw->preppers.emplace_back(prep_main, raw, i);
    } catch (const std::exception& e) {  // a thread could not be started: stop the others
      {
        std::lock_guard<std::mutex> lk(raw->mu);
        raw->stop = true;
        raw->cv.notify_all();
      }
      for (auto& t : raw->preppers)
        if (t.joinable()) t.join();
      if (raw->worker.joinable()) raw->worker.join();
      cleanup();
      return fail(HS_E_INTERNAL, "server threads: %s", e.what());
    }
    *out = sv.release();
    return HS_OK;
  });
}

hs_status hs_server_clock(hs_server sv, double* seconds) {
  return guarded([&]() -> hs_status {
    if (!sv || !seconds) return fail(HS_E_ARG, "null argument");
    *seconds = now_s();
    return HS_OK;
  });
}

hs_status hs_server_submit(hs_server sv, int n, const hs_gate* gates, size_t count, hs_dtype dtype,
                           uint64_t init_basis, int k, hs_strategy strategy, double arrival_s,
                           uint64_t* ticket) {
  return guarded([&]() -> hs_status {
    const double t_call = now_s();
    if (!sv || !ticket || (!gates && count)) return fail(HS_E_ARG, "null argument");
    if (n < 1 || n > 40) return fail(HS_E_ARG, "n = %d outside [1, 40]", n);
    if (dtype != HS_C64 && dtype != HS_C128) return fail(HS_E_ARG, "bad dtype");
    if (init_basis >= (uint64_t(1) << n)) return fail(HS_E_ARG, "basis index outside the state");
    if (k < 1) return fail(HS_E_ARG, "k = %d < 1", k);
    if (strategy < HS_PART_NAT || strategy > HS_PART_CLOSURE)
      return fail(HS_E_ARG, "unknown strategy %d", (int)strategy);
    if (arrival_s > t_call) return fail(HS_E_ARG, "arrival time lies in the future");
    auto r = std::make_unique<Request>();
    r->n = n;
    r->k = k;
    r->dtype = dtype;
    r->strategy = strategy;
    r->init = init_basis;
    r->t_arrival = arrival_s >= 0 ? arrival_s : t_call;
    r->gates.reserve(count);
    for (size_t i = 0; i < count; ++i)
      if (hs_status rc = expand_gate(n, gates[i], &r->gates)) return rc;
    for (const Gate& g : r->gates)
      if (g.arity() > k) return fail(HS_E_ARITY_GT_K, "gate wider than k = %d", k);
    const size_t state_bytes = (size_t(1) << n) * amp_bytes(dtype);
    if (state_bytes > sv->budget)
      return fail(HS_E_ADMISSION, "state needs %zu bytes, budget is %zu", state_bytes, sv->budget);
    std::lock_guard<std::mutex> lk(sv->mu);
    r->ticket = sv->next_ticket++;  // a ticket lost to a failed insert is skipped at admission
    sv->reqs[r->ticket] = r.get();
    try {
      sv->prep_queue.push_back(r.get());
    } catch (...) {
      sv->reqs.erase(r->ticket);
      throw;
    }
    *ticket = r.release()->ticket;
    sv->cv.notify_all();
    return HS_OK;
  });
}

hs_status hs_server_wait(hs_server sv, uint64_t ticket, int64_t timeout_ms) {
  return guarded([&]() -> hs_status {
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
  });
}

hs_status hs_server_poll(hs_server sv, uint64_t ticket, int* done) {
  return guarded([&]() -> hs_status {
    if (!sv || !done) return fail(HS_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    Request* r = find(sv, ticket);
    if (!r) return fail(HS_E_ARG, "unknown ticket");
    *done = (r->status == RQ_DONE || r->status == RQ_FAILED) ? 1 : 0;
    return HS_OK;
  });
}

hs_status hs_server_read(hs_server sv, uint64_t ticket, uint64_t first, uint64_t count, double* out) {
  return guarded([&]() -> hs_status {
    if (!sv || (!out && count)) return fail(HS_E_ARG, "null argument");
    State view;
    Request* reader = nullptr;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      Request* r = find(sv, ticket);
      if (!r) return fail(HS_E_ARG, "unknown ticket");
      if (r->status == RQ_RELEASED) return fail(HS_E_STATE, "ticket was released");
      if (r->status != RQ_DONE) return fail(HS_E_STATE, "ticket is not finished");
      const uint64_t N = uint64_t(1) << r->n;
      if (first > N || count > N - first) return fail(HS_E_ARG, "range outside the state");
      if (!count) return HS_OK;
      view = r->st;
      reader = r;
      r->readers++;  // hs_server_release waits for this read before freeing the state
    }
    hs_status rc;
    {
      // read on a stream of its own (the request's kernels have finished),
      // staged through the server's persistent buffer
      std::lock_guard<std::mutex> rl(sv->read_mu);
      view.stream = sv->read_stream;
      view.owned = false;
      view.scratch = sv->read_scratch;
      view.scratch_bytes = kReadScratch;
      rc = dev_read(&view, first, count, out, false);
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (--reader->readers == 0) sv->cv.notify_all();
    return rc;
  });
}

hs_status hs_server_latency(hs_server sv, uint64_t ticket, double* seconds) {
  return guarded([&]() -> hs_status {
    if (!sv || !seconds) return fail(HS_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    Request* r = find(sv, ticket);
    if (!r) return fail(HS_E_ARG, "unknown ticket");
    if (r->status != RQ_DONE && r->status != RQ_RELEASED) return fail(HS_E_STATE, "ticket is not finished");
    *seconds = r->t_done - r->t_arrival;
    return HS_OK;
  });
}

hs_status hs_server_timing(hs_server sv, uint64_t ticket, double* out4) {
  return guarded([&]() -> hs_status {
    if (!sv || !out4) return fail(HS_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    Request* r = find(sv, ticket);
    if (!r) return fail(HS_E_ARG, "unknown ticket");
    if (r->status != RQ_DONE && r->status != RQ_RELEASED) return fail(HS_E_STATE, "ticket is not finished");
    out4[0] = r->t_prep0 - r->t_arrival;
    out4[1] = r->t_prep1 - r->t_prep0;
    out4[2] = r->t_launch - r->t_prep1;
    out4[3] = r->t_done - r->t_launch;
    return HS_OK;
  });
}

hs_status hs_server_release(hs_server sv, uint64_t ticket) {
  return guarded([&]() -> hs_status {
    if (!sv) return fail(HS_E_ARG, "null server");
    std::unique_ptr<Plan> plan;
    void* state = nullptr;
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> events;
    bool drain = false;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      Request* r = find(sv, ticket);
      if (!r) return fail(HS_E_ARG, "unknown ticket");
      // reads of its state still copying finish first (a read that starts
      // later finds the ticket released)
      sv->cv.wait(lk, [&] { return r->readers == 0; });
      if (r->status == RQ_RELEASED) return HS_OK;
      if (r->status != RQ_DONE && r->status != RQ_FAILED) return fail(HS_E_STATE, "ticket is not finished");
      if (r->status == RQ_DONE) {
        state = r->st.ptr;
        stream = (hipStream_t)r->st.stream;
        r->st.ptr = nullptr;
        sv->cur_bytes -= r->bytes;
      }
      if (r->status == RQ_FAILED && r->launched) {
        drain = true;
        stream = (hipStream_t)r->st.stream;
      }
      events = {r->done, r->chunk_ev[0], r->chunk_ev[1]};
      r->done = r->chunk_ev[0] = r->chunk_ev[1] = nullptr;
      plan = std::move(r->plan);
      r->status = RQ_RELEASED;
      sv->cv.notify_all();
    }
    // a finished request's kernels are complete: the frees are stream-ordered
    // and wait for nothing on the device
    drop_request_memory(sv, std::move(plan), state, stream, events, drain);
    return HS_OK;
  });
}

hs_status hs_server_stats(hs_server sv, uint64_t* completed, uint64_t* peak_bytes, uint64_t* cur_bytes,
                          int* peak_inflight) {
  return guarded([&]() -> hs_status {
    if (!sv) return fail(HS_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (completed) *completed = sv->completed;
    if (peak_bytes) *peak_bytes = sv->peak_bytes;
    if (cur_bytes) *cur_bytes = sv->cur_bytes;
    if (peak_inflight) *peak_inflight = sv->peak_inflight;
    return HS_OK;
  });
}

hs_status hs_server_destroy(hs_server sv) {
  return guarded([&]() -> hs_status {
    if (!sv) return HS_OK;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
      sv->cv.notify_all();
    }
    for (auto& t : sv->preppers)
      if (t.joinable()) t.join();
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipSetDevice(sv->device);
    for (auto& kv : sv->reqs) {
      Request* r = kv.second;
      if (r->st.ptr) (void)hipFreeAsync(r->st.ptr, (hipStream_t)r->st.stream);
      for (hipEvent_t ev : {r->done, r->chunk_ev[0], r->chunk_ev[1]})
        if (ev) (void)hipEventDestroy(ev);
      delete r;  // plan descriptors: hipFreeAsync on the preparing stream
    }
    for (hipStream_t s : sv->streams) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    for (hipStream_t s : sv->prep_streams) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    (void)hipStreamSynchronize(sv->read_stream);
    (void)hipStreamDestroy(sv->read_stream);
    if (sv->read_scratch) (void)hipFree(sv->read_scratch);
    for (PinnedStaging& p : sv->pins) {  // every copy from them has run
      if (p.ptr) (void)hipHostFree(p.ptr);
      if (p.busy) (void)hipEventDestroy((hipEvent_t)p.busy);
    }
    delete sv;
    return HS_OK;
  });
}

}  // extern "C"
