// Serving loop for dynamic updates (host runtime).
//
// Each registered graph is a katz_state (device-resident graph, walk history,
// bounds and active set).  Requests are edge-update batches; every graph keeps
// its requests in arrival order and runs at most one at a time, so the result
// of request j reflects exactly the batches of that graph up to j.  A pool of
// worker slots, each with its own HIP stream, takes the oldest request of any
// idle graph whose estimated device memory fits the remaining budget: requests
// that arrive while others run are admitted as soon as a slot and memory free
// up, and updates of different graphs overlap on the device.
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

struct Request {
  int64_t ticket = 0;
  int32_t graph = 0;
  std::vector<int32_t> iu, iv, du, dv;
  int64_t bytes = 0;              // admission estimate
  Clock::time_point arrival;
  // completion
  bool done = false;
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
  std::deque<std::shared_ptr<Request>> queue;
  bool busy = false;
};

}  // namespace

struct katz_server {
  std::mutex mu;
  std::condition_variable cv_work;   // workers wait for admissible requests
  std::condition_variable cv_done;   // callers wait for completions
  // A deque: add_graph appends while workers hold pointers to other entries,
  // and push_back on a deque never moves the elements already in it.
  std::deque<GraphEntry> graphs;
  std::map<int64_t, std::shared_ptr<Request>> tickets;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;  // one per worker, created with the server
  int64_t next_ticket = 1;
  int64_t budget = 0;                // bytes; 0 = unlimited
  int64_t in_use = 0;
  bool stopping = false;
  int device = 0;
  std::atomic<int64_t> completed{0};
};

namespace {

// Device bytes a request may need beyond the state's resident memory: the
// batch arrays, the per-row merge scratch and the per-touched-row tables.
int64_t estimate_bytes(int64_t pairs) { return 4096 + pairs * (2 * 4 + 4 * (8 + 8 + 4 * 5 + 8)); }

// Oldest request of an idle graph that fits the memory budget.
std::shared_ptr<Request> pick(katz_server* sv) {
  std::shared_ptr<Request> best;
  for (GraphEntry& ge : sv->graphs) {
    if (ge.busy || ge.queue.empty()) continue;
    const auto& head = ge.queue.front();
    if (sv->budget > 0 && sv->in_use + head->bytes > sv->budget && sv->in_use > 0) continue;
    if (!best || head->ticket < best->ticket) best = head;
  }
  return best;
}

void worker_main(katz_server* sv, hipStream_t s) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    std::shared_ptr<Request> rq;
    GraphEntry* gep = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] { return sv->stopping || (rq = pick(sv)) != nullptr; });
      if (!rq) break;
      gep = &sv->graphs[rq->graph];
      gep->queue.pop_front();
      gep->busy = true;
      sv->in_use += rq->bytes;
    }
    GraphEntry& ge = *gep;  // st and k never change once registered
    rq->ids.resize(ge.k);
    rq->lo.resize(ge.k);
    rq->up.resize(ge.k);
    rq->res = katz_result{};
    rq->res.topk_ids = rq->ids.data();
    rq->res.lower = rq->lo.data();
    rq->res.upper = rq->up.data();
    const auto t0 = Clock::now();
    const int rc = katz_rank_update(ge.st, rq->iu.data(), rq->iv.data(), (int64_t)rq->iu.size(), rq->du.data(),
                                    rq->dv.data(), (int64_t)rq->du.size(), &rq->res, s);
    const auto t1 = Clock::now();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      rq->status = rc;
      rq->service_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      rq->latency_ms = std::chrono::duration<double, std::milli>(t1 - rq->arrival).count();
      rq->done = true;
      ge.busy = false;
      sv->in_use -= rq->bytes;
      sv->completed++;
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
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
  rq->bytes = estimate_bytes(n_ins + n_del);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (graph_id < 0 || graph_id >= (int32_t)sv->graphs.size() || sv->stopping) return KATZ_E_INVALID_ARG;
    rq->graph = graph_id;
    rq->ticket = sv->next_ticket++;
    sv->graphs[graph_id].queue.push_back(rq);
    sv->tickets[rq->ticket] = rq;
    *ticket = rq->ticket;
  }
  sv->cv_work.notify_one();
  return KATZ_OK;
}

KATZ_EXPORT int katz_server_wait(katz_server* sv, int64_t ticket, katz_result* out, double* latency_ms,
                                 double* service_ms) {
  if (!sv || !out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  std::shared_ptr<Request> rq;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return KATZ_E_INVALID_ARG;
    rq = it->second;
    sv->cv_done.wait(lk, [&] { return rq->done; });
    sv->tickets.erase(it);
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

KATZ_EXPORT void katz_server_destroy(katz_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  for (std::thread& t : sv->workers) t.join();
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  for (GraphEntry& ge : sv->graphs) katz_state_free(ge.st);
  delete sv;
}
