// Serving loop for dynamic updates (host runtime).
//
// Each registered graph is a katz_state (device-resident graph, walk history,
// bounds and active set).  Requests are edge-update batches.  An update runs
// in two halves (prepare_batch / apply_batch): the host half validates the
// batch on its own and groups its arcs by row, reading no graph state; the
// device half checks the batch against the graph, merges it, re-walks and
// re-certifies (Algorithm 2).  The device halves of one graph's requests run
// in arrival order, one at a time, so request j's result reflects exactly that
// graph's batches up to j; host halves run ahead on idle slots, so the host
// work of request j+1 overlaps the device work of request j of the same graph.
// A pool of worker slots, each with its own HIP stream, takes, in this order:
// the oldest prepared request at the head of an idle graph's queue whose
// estimated device memory fits the remaining budget (its device half); the
// oldest request not yet prepared (its host half, and then its device half at
// once if it heads an idle graph's queue and fits).  Requests of different
// graphs overlap on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "katz_internal.h"

#define KATZ_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

using Clock = std::chrono::steady_clock;

enum Phase { QUEUED, PREPARING, PREPARED, RUNNING, DONE };

struct Request {
  int64_t ticket = 0;
  int32_t graph = 0;
  std::vector<int32_t> iu, iv, du, dv;
  int64_t bytes = 0;              // admission estimate of the device half
  Clock::time_point arrival;
  Phase phase = QUEUED;
  int prep_rc = KATZ_OK;
  katz::PreparedBatch pb;
  double prepare_ms = 0.0;
  // completion
  int status = 0;
  std::vector<int32_t> ids;
  std::vector<double> lo, up;
  katz_result res{};
  double latency_ms = 0.0;
  double service_ms = 0.0;
};

struct GraphEntry {
  katz_state* st = nullptr;
  int32_t k = 0;
  int64_t n = 0;
  int mode = 0;                                  // how update pairs read (katz::PairMode)
  std::deque<std::shared_ptr<Request>> queue;   // arrival order, not yet on the device
  bool busy = false;                             // a device half of this graph runs
};

}  // namespace

struct katz_server {
  std::mutex mu;
  std::condition_variable cv_work;   // workers wait for work
  std::condition_variable cv_done;   // callers wait for completions; destroy waits for callers
  // A deque: add_graph appends while workers hold pointers to other entries,
  // and push_back on a deque never moves the elements already in it.
  std::deque<GraphEntry> graphs;
  std::map<int64_t, std::shared_ptr<Request>> tickets;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;  // one per worker, created with the server
  int64_t next_ticket = 1;
  int64_t budget = 0;                // bytes; 0 = unlimited
  int64_t in_use = 0;
  int waiters = 0;                   // threads inside katz_server_wait
  bool stopping = false;
  int device = 0;
  std::atomic<int64_t> completed{0};
};

namespace {

// Device bytes the device half of a request may allocate beyond the state's
// resident memory: the batch arrays and per-touched-row tables, the row-merge
// scratch, one more level of the walk history (8 n bytes) should the
// re-certification need another iteration, and the slack-pool growth its
// insertions can force (the pool at most doubles: bounded here by the
// relocated rows' arcs, twice per inserted pair, with the slack factor).
int64_t estimate_bytes(int64_t pairs, int64_t n) {
  const int64_t batch = 4096 + pairs * (2 * 4 + 4 * (8 + 8 + 4 * 5 + 8));
  const int64_t level = 8 * n;
  const int64_t pool = pairs * 2 * 4 * 9 / 8 * 2;
  return batch + level + pool;
}

bool fits(const katz_server* sv, const Request& rq) {
  return sv->budget <= 0 || sv->in_use == 0 || sv->in_use + rq.bytes <= sv->budget;
}

// The oldest prepared request heading the queue of an idle graph that fits.
std::shared_ptr<Request> pick_run(katz_server* sv) {
  std::shared_ptr<Request> best;
  for (GraphEntry& ge : sv->graphs) {
    if (ge.busy || ge.queue.empty()) continue;
    const auto& head = ge.queue.front();
    if (head->phase != PREPARED || !fits(sv, *head)) continue;
    if (!best || head->ticket < best->ticket) best = head;
  }
  return best;
}

// The oldest request whose host half has not started.
std::shared_ptr<Request> pick_prepare(katz_server* sv) {
  std::shared_ptr<Request> best;
  for (GraphEntry& ge : sv->graphs)
    for (const auto& rq : ge.queue)
      if (rq->phase == QUEUED) {
        if (!best || rq->ticket < best->ticket) best = rq;
        break;   // later requests of this graph are younger
      }
  return best;
}

// Completes a request (lock held).
void finish(katz_server* sv, Request& rq, int status, Clock::time_point t_end) {
  rq.status = status;
  rq.latency_ms = std::chrono::duration<double, std::milli>(t_end - rq.arrival).count();
  rq.phase = DONE;
  sv->completed++;
}

// Device half of the request at the head of its idle graph's queue (called
// with the lock held; returns with it held).
void run_device_half(katz_server* sv, std::unique_lock<std::mutex>& lk, const std::shared_ptr<Request>& rq,
                     hipStream_t s) {
  GraphEntry& ge = sv->graphs[rq->graph];
  ge.queue.pop_front();
  ge.busy = true;
  rq->phase = RUNNING;
  sv->in_use += rq->bytes;
  lk.unlock();
  rq->ids.resize(ge.k);
  rq->lo.resize(ge.k);
  rq->up.resize(ge.k);
  rq->res = katz_result{};
  rq->res.topk_ids = rq->ids.data();
  rq->res.lower = rq->lo.data();
  rq->res.upper = rq->up.data();
  const auto t0 = Clock::now();
  int rc = rq->prep_rc;
  if (rc >= 0) rc = katz::apply_batch(ge.st, rq->pb, &rq->res, s);
  const auto t1 = Clock::now();
  rq->pb = katz::PreparedBatch{};
  lk.lock();
  rq->service_ms = rq->prepare_ms + std::chrono::duration<double, std::milli>(t1 - t0).count();
  finish(sv, *rq, rc, t1);
  ge.busy = false;
  sv->in_use -= rq->bytes;
  sv->cv_done.notify_all();
  sv->cv_work.notify_all();
}

void worker_main(katz_server* sv, hipStream_t s) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    if (sv->stopping) break;
    if (auto rq = pick_run(sv)) {
      run_device_half(sv, lk, rq, s);
      continue;
    }
    if (auto rq = pick_prepare(sv)) {
      rq->phase = PREPARING;
      const int64_t n = sv->graphs[rq->graph].n;
      const int mode = sv->graphs[rq->graph].mode;
      lk.unlock();
      const auto t0 = Clock::now();
      const int rc = katz::prepare_batch(n, mode, rq->iu.data(), rq->iv.data(), (int64_t)rq->iu.size(), rq->du.data(),
                                         rq->dv.data(), (int64_t)rq->du.size(), rq->pb);
      const auto t1 = Clock::now();
      lk.lock();
      if (sv->stopping) break;
      // katz_server_cancel may have ended the request meanwhile (phase DONE).
      if (rq->phase != PREPARING) continue;
      rq->prepare_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      rq->prep_rc = rc;
      rq->phase = PREPARED;
      sv->cv_work.notify_all();
      GraphEntry& ge = sv->graphs[rq->graph];
      if (!ge.busy && !ge.queue.empty() && ge.queue.front() == rq && fits(sv, *rq)) run_device_half(sv, lk, rq, s);
      continue;
    }
    sv->cv_work.wait(lk);
  }
}

}  // namespace

KATZ_EXPORT int katz_server_create(int32_t slots, int64_t memory_budget, katz_server** out) {
  if (!out || slots < 1 || slots > 64 || memory_budget < 0) return KATZ_E_INVALID_ARG;
  katz_server* sv = new katz_server;
  sv->budget = memory_budget;
  bool ok = hipGetDevice(&sv->device) == hipSuccess;
  for (int i = 0; ok && i < slots; ++i) {
    hipStream_t s = nullptr;
    ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    if (ok) sv->streams.push_back(s);
  }
  if (!ok) {
    for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    delete sv;
    return KATZ_E_HIP;
  }
  for (hipStream_t s : sv->streams) sv->workers.emplace_back(worker_main, sv, s);
  *out = sv;
  return KATZ_OK;
}

KATZ_EXPORT int katz_server_add_graph(katz_server* sv, const katz_csr* g, const katz_params* p, katz_result* out,
                                      int32_t* graph_id) {
  if (!sv || !graph_id) return KATZ_E_INVALID_ARG;
  katz_state* st = nullptr;
  const int rc = katz_rank_static(1, g, p, out, &st, nullptr);
  if (rc < 0) return rc;
  std::lock_guard<std::mutex> lk(sv->mu);
  GraphEntry ge;
  ge.st = st;
  ge.k = p->k;
  ge.n = katz::state_nodes(st);
  ge.mode = katz::state_pair_mode(st);
  sv->graphs.push_back(std::move(ge));
  *graph_id = (int32_t)sv->graphs.size() - 1;
  return rc;
}

KATZ_EXPORT int katz_server_submit(katz_server* sv, int32_t graph_id, const int32_t* ins_u, const int32_t* ins_v,
                                   int64_t n_ins, const int32_t* del_u, const int32_t* del_v, int64_t n_del,
                                   int64_t* ticket) {
  if (!sv || !ticket || n_ins < 0 || n_del < 0) return KATZ_E_INVALID_ARG;
  if ((n_ins > 0 && (!ins_u || !ins_v)) || (n_del > 0 && (!del_u || !del_v))) return KATZ_E_INVALID_ARG;
  auto rq = std::make_shared<Request>();
  rq->arrival = Clock::now();
  rq->iu.assign(ins_u, ins_u + n_ins);
  rq->iv.assign(ins_v, ins_v + n_ins);
  rq->du.assign(del_u, del_u + n_del);
  rq->dv.assign(del_v, del_v + n_del);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (graph_id < 0 || graph_id >= (int32_t)sv->graphs.size() || sv->stopping) return KATZ_E_INVALID_ARG;
    rq->graph = graph_id;
    rq->bytes = estimate_bytes(n_ins + n_del, sv->graphs[graph_id].n);
    rq->ticket = sv->next_ticket++;
    sv->graphs[graph_id].queue.push_back(rq);
    sv->tickets[rq->ticket] = rq;
    *ticket = rq->ticket;
  }
  sv->cv_work.notify_one();
  return KATZ_OK;
}

namespace {

// Waits for a request (timeout_ms < 0: without a limit); on completion the
// ticket is consumed and the result copied out.
int wait_request(katz_server* sv, int64_t ticket, int64_t timeout_ms, katz_result* out, double* latency_ms,
                 double* service_ms) {
  if (!sv || !out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  std::shared_ptr<Request> rq;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return KATZ_E_INVALID_ARG;
    rq = it->second;
    ++sv->waiters;
    const auto done = [&] { return rq->phase == DONE; };
    bool finished = true;
    if (timeout_ms < 0) sv->cv_done.wait(lk, done);
    else finished = sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
    if (finished) sv->tickets.erase(ticket);
    --sv->waiters;
    sv->cv_done.notify_all();   // destroy may be waiting for the last waiter
    if (!finished) return KATZ_E_TIMEOUT;
  }
  const int k = (int)rq->ids.size();
  if (rq->status >= 0) {
    std::memcpy(out->topk_ids, rq->ids.data(), sizeof(int32_t) * k);
    std::memcpy(out->lower, rq->lo.data(), sizeof(double) * k);
    std::memcpy(out->upper, rq->up.data(), sizeof(double) * k);
  }
  out->rest_upper_max = rq->res.rest_upper_max;
  out->alpha_used = rq->res.alpha_used;
  out->eta = rq->res.eta;
  out->active_final = rq->res.active_final;
  out->iterations = rq->res.iterations;
  out->status = rq->status;
  if (latency_ms) *latency_ms = rq->latency_ms;
  if (service_ms) *service_ms = rq->service_ms;
  return rq->status;
}

}  // namespace

KATZ_EXPORT int katz_server_wait(katz_server* sv, int64_t ticket, katz_result* out, double* latency_ms,
                                 double* service_ms) {
  return wait_request(sv, ticket, -1, out, latency_ms, service_ms);
}

KATZ_EXPORT int katz_server_wait_for(katz_server* sv, int64_t ticket, int64_t timeout_ms, katz_result* out,
                                     double* latency_ms, double* service_ms) {
  if (timeout_ms < 0) return KATZ_E_INVALID_ARG;
  return wait_request(sv, ticket, timeout_ms, out, latency_ms, service_ms);
}

KATZ_EXPORT int katz_server_cancel(katz_server* sv, int64_t ticket) {
  if (!sv) return KATZ_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return KATZ_E_INVALID_ARG;
    const std::shared_ptr<Request> rq = it->second;
    if (rq->phase == RUNNING || rq->phase == DONE) return KATZ_E_BUSY;
    // Not on the device yet: out of its graph's queue, ended for its waiter.
    // Later requests of the graph run without its batch.  A host half being
    // prepared meanwhile is dropped by its worker.
    auto& q = sv->graphs[rq->graph].queue;
    q.erase(std::remove(q.begin(), q.end(), rq), q.end());
    finish(sv, *rq, KATZ_E_CANCELLED, Clock::now());
  }
  sv->cv_done.notify_all();
  sv->cv_work.notify_all();
  return KATZ_OK;
}

KATZ_EXPORT void katz_server_destroy(katz_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
    // Requests that have not reached the device end now; a waiter wakes with
    // E_CANCELLED.  Those on the device finish before the workers stop.
    const auto now = Clock::now();
    for (GraphEntry& ge : sv->graphs) {
      for (auto& rq : ge.queue)
        if (rq->phase != DONE) finish(sv, *rq, KATZ_E_CANCELLED, now);
      ge.queue.clear();
    }
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  for (std::thread& t : sv->workers) t.join();
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->waiters == 0; });
  }
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  for (GraphEntry& ge : sv->graphs) katz_state_free(ge.st);
  delete sv;
}
