// Host runtime of the C ABI declared in include/katz.h.
//
// A ranking call validates its arguments on the host, stages host inputs to the
// device, bins the rows (prep), then enqueues iterations of Algorithm 1
// (walk step + selection + converged()) and reads the device stop flag one
// iteration behind.  Static calls take their workspace from a per-device pool
// of grow-only arenas; a dynamic state (Algorithm 2) owns its memory: the graph
// as a CSR with per-row slack, the walk history x_1..x_r, c_r and M.
#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <dlfcn.h>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "katz_internal.h"

#define KATZ_EXPORT extern "C" __attribute__((visibility("default")))

#define KATZ_HIP(call)                    \
  do {                                    \
    if ((call) != hipSuccess) {           \
      (void)hipGetLastError();            \
      return KATZ_E_HIP;                  \
    }                                     \
  } while (0)

#define KATZ_TRY(expr)          \
  do {                          \
    const int rc_ = (expr);     \
    if (rc_ < 0) return rc_;    \
  } while (0)

namespace katz {
namespace {

constexpr double kU64 = 0x1p-53;   // unit roundoff of FP64
constexpr double kU32 = 0x1p-24;   // unit roundoff of FP32

// ---------------------------------------------------------------------------
// Pinned host mirrors used to read the device flags.
// ---------------------------------------------------------------------------
struct HostSync {
  RunScalars* sc = nullptr;        // final read-back
  RunScalars* ring = nullptr;      // 2 slots: per-pass copies of the flags
  hipEvent_t ev[2] = {nullptr, nullptr};   // null: each pass synchronises the stream
  unsigned long long* bits = nullptr;   // 8 words of scalar read-backs
  bool borrowed = false;           // the mirrors are static host memory, not owned

  int init() {
    if (sc) return KATZ_OK;
    if (hipHostMalloc((void**)&sc, sizeof(RunScalars)) != hipSuccess) return KATZ_E_OOM;
    if (hipHostMalloc((void**)&ring, 2 * sizeof(RunScalars)) != hipSuccess) return KATZ_E_OOM;
    if (hipHostMalloc((void**)&bits, 8 * sizeof(unsigned long long)) != hipSuccess) return KATZ_E_OOM;
    for (hipEvent_t& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return KATZ_E_HIP;
    return KATZ_OK;
  }
  ~HostSync() {
    if (borrowed) return;
    if (sc) (void)hipHostFree(sc);
    if (ring) (void)hipHostFree(ring);
    if (bits) (void)hipHostFree(bits);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------------------
// Workspace arenas for static calls.
// ---------------------------------------------------------------------------
struct Arena {
  int device = -1;
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool measuring = false;
  bool fixed = false;   // base is the library's static scratch: never grown or freed
  HostSync hs;
  // The last call's work on this workspace: an event recorded on its stream
  // when the call returned (a stream-ordered call may still be running).
  hipEvent_t last = nullptr;
  hipStream_t last_stream = nullptr;
  bool recorded = false;
  // Batched calls: the stream their hipGraph replays on, and the instantiated
  // graph of the last batch with the bytes of every argument it captured (a
  // call whose arguments are byte-identical replays it without re-capturing).
  hipStream_t graph_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<unsigned char> graph_key;

  ~Arena() {
    if (recorded) (void)hipEventSynchronize(last);
    if (last) (void)hipEventDestroy(last);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph_stream) (void)hipStreamDestroy(graph_stream);
    if (base && !fixed) (void)hipFree(base);
  }
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    graph_key.clear();
  }
  // A call on stream s that takes over the workspace orders its work after
  // the previous call's.
  int order_after(hipStream_t s) {
    if (recorded && last_stream != s) KATZ_HIP(hipStreamWaitEvent(s, last, 0));
    return KATZ_OK;
  }
  void mark_used(hipStream_t s) {
    if (!last && hipEventCreateWithFlags(&last, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      last = nullptr;
      return;
    }
    if (hipEventRecord(last, s) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);   // no event: the work is finished instead
      recorded = false;
      return;
    }
    recorded = true;
    last_stream = s;
  }
  template <class T>
  T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = measuring ? nullptr : reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
  int grow(size_t bytes) {
    KATZ_TRY(hs.init());
    if (bytes <= cap) return KATZ_OK;
    if (fixed) return KATZ_E_SCRATCH;
    if (recorded) KATZ_HIP(hipEventSynchronize(last));   // a stream-ordered call may still use it
    drop_graph();                                          // its captured arguments point into the old buffer
    if (base) (void)hipFree(base);
    base = nullptr;
    cap = 0;
    if (hipMalloc((void**)&base, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return KATZ_E_OOM;
    }
    cap = bytes;
    return KATZ_OK;
  }
};

std::mutex g_pool_mu;
std::vector<Arena*> g_pool;

Arena* acquire_arena(int device) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (size_t i = 0; i < g_pool.size(); ++i) {
    if (g_pool[i]->device == device) {
      Arena* a = g_pool[i];
      g_pool.erase(g_pool.begin() + i);
      return a;
    }
  }
  Arena* a = new Arena;
  a->device = device;
  return a;
}

void release_arena(Arena* a) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pool.push_back(a);
}

// A static call's hold on a workspace: the call's stream is ordered after the
// workspace's previous user, and the workspace records the call's work when
// it goes back to the pool.
struct ArenaLease {
  Arena* a;
  hipStream_t s;
  int rc;
  ArenaLease(int dev, hipStream_t stream) : a(acquire_arena(dev)), s(stream), rc(a->order_after(stream)) {}
  ~ArenaLease() {
    a->mark_used(s);
    release_arena(a);
  }
};

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// ---------------------------------------------------------------------------
// Optional device timing of the phases of every call (hipEvent pairs recorded
// on the call's stream; summed when the call has synchronised).
// ---------------------------------------------------------------------------
enum TimedKind { T_PREP = 0, T_FIRST, T_STEP, T_SELECT, T_RESULT, T_RENUM, T_KINDS };

struct TimingState {
  std::mutex mu;
  bool on = false;
  katz_timing acc{};
};
TimingState g_timing;

// Launch tuning of the walk step (katz_tuning_set); read once per call.
struct TuningState {
  std::mutex mu;
  katz_tuning t{};
};
TuningState g_tuning;

katz_tuning current_tuning() {
  std::lock_guard<std::mutex> lk(g_tuning.mu);
  return g_tuning.t;
}

int tuning_valid(const katz_tuning& t) {
  if (t.walk_groups != 0 && t.walk_groups != 1 && t.walk_groups != kWalkGroups) return KATZ_E_INVALID_ARG;
  const int hub_max = t.walk_groups == kWalkGroups ? 162816 : 65536;
  if (t.hub_bytes < 0 || t.hub_bytes > hub_max || (t.hub_bytes & 15)) return KATZ_E_INVALID_ARG;
  if (t.blocks_per_cu < 0 || t.blocks_per_cu > 32) return KATZ_E_INVALID_ARG;
  if (t.batch_blocks_per_cu < 0 || t.batch_blocks_per_cu > 32) return KATZ_E_INVALID_ARG;
  if (t.batch_tile < 0 || t.batch_tile > 16) return KATZ_E_INVALID_ARG;
  if (t.batch_xcd != 0 && t.batch_xcd != 1) return KATZ_E_INVALID_ARG;
  if (t.hub_bytes > 0 && t.blocks_per_cu == 0) return KATZ_E_INVALID_ARG;
  if (t.split_hot_bytes < 0 || t.split_hot_bytes > (64 << 20) || (t.split_hot_bytes > 0 && (t.split_hot_bytes & 15)))
    return KATZ_E_INVALID_ARG;
  if (t.reserved != 0) return KATZ_E_INVALID_ARG;
  // bin_bounds: all 0 (the default classes), or strictly increasing from 1,
  // the last below kBlockRowMax (the one-workgroup class keeps its end).
  bool any = false;
  for (int v : t.bin_bounds) any = any || v != 0;
  if (any) {
    int prev = 0;
    for (int v : t.bin_bounds) {
      if (v <= prev) return KATZ_E_INVALID_ARG;
      prev = v;
    }
    if (prev >= kBlockRowMax) return KATZ_E_INVALID_ARG;
  }
  return KATZ_OK;
}

BinBounds bounds_of(const katz_tuning& t) {
  BinBounds bb;
  if (t.bin_bounds[0] == 0) return bb;
  bb.g4 = t.bin_bounds[0];
  bb.g8 = t.bin_bounds[1];
  bb.g16 = t.bin_bounds[2];
  bb.g32 = t.bin_bounds[3];
  bb.w16 = t.bin_bounds[4];
  bb.w64 = t.bin_bounds[5];
  return bb;
}

int cu_count(int dev) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    v = 256;
  }
  cache[dev] = v;
  return v;
}

// ---------------------------------------------------------------------------
// roctx ranges for rocprofv3's marker trace (host side: each call, the enqueue
// of each iteration, the two halves of an update).  KATZ_ROCTX=1 turns them
// on: the range functions are then looked up in the ROCm roctx library at run
// time (no link dependency); without the variable, or without the library,
// a range costs one test of a null pointer.
// ---------------------------------------------------------------------------
struct RoctxApi {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};

const RoctxApi& roctx_api() {
  static const RoctxApi api = [] {
    RoctxApi a;
    const char* e = std::getenv("KATZ_ROCTX");
    if (!e || std::strcmp(e, "1") != 0) return a;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    if (!h) return a;
    a.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    a.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!a.push || !a.pop) a = RoctxApi{};
    return a;
  }();
  return api;
}

struct Range {
  bool on;
  explicit Range(const char* name) : on(roctx_api().push != nullptr) {
    if (on) roctx_api().push(name);
  }
  Range(const char* name, int v) : on(roctx_api().push != nullptr) {
    if (!on) return;
    char buf[96];
    std::snprintf(buf, sizeof(buf), "%s %d", name, v);
    roctx_api().push(buf);
  }
  ~Range() {
    if (on) roctx_api().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct CallTimer {
  bool on = false;
  std::vector<int> kind;
  std::vector<hipEvent_t> ev;   // start, stop pairs
  hipEvent_t call0 = nullptr, call1 = nullptr;

  explicit CallTimer(bool allow = true) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    on = allow && g_timing.on;
  }
  ~CallTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (call0) (void)hipEventDestroy(call0);
    if (call1) (void)hipEventDestroy(call1);
  }
  void call_begin(hipStream_t s) {
    if (!on) return;
    (void)hipEventCreate(&call0);
    (void)hipEventCreate(&call1);
    (void)hipEventRecord(call0, s);
  }
  int start(int k, hipStream_t s) {
    if (!on) return -1;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
    ev.push_back(a);
    ev.push_back(b);
    kind.push_back(k);
    return (int)kind.size() - 1;
  }
  void stop(int i, hipStream_t s) {
    if (i >= 0) (void)hipEventRecord(ev[2 * i + 1], s);
  }
  // Call after the stream has been synchronised.
  void commit(hipStream_t s) {
    if (!on) return;
    (void)hipEventRecord(call1, s);
    (void)hipEventSynchronize(call1);
    double sum[T_KINDS] = {};
    long long cnt[T_KINDS] = {};
    for (size_t i = 0; i < kind.size(); ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
        sum[kind[i]] += ms;
        cnt[kind[i]] += 1;
      } else {
        (void)hipGetLastError();
      }
    }
    float call_ms = 0.f;
    if (hipEventElapsedTime(&call_ms, call0, call1) != hipSuccess) (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(g_timing.mu);
    katz_timing& t = g_timing.acc;
    t.prep_ms += sum[T_PREP];
    t.walk_first_ms += sum[T_FIRST];
    t.walk_first_launches += cnt[T_FIRST];
    t.walk_step_ms += sum[T_STEP];
    t.walk_step_launches += cnt[T_STEP];
    t.renumber_step_ms += sum[T_RENUM];
    t.renumber_step_launches += cnt[T_RENUM];
    t.select_ms += sum[T_SELECT];
    t.select_iterations += cnt[T_SELECT];
    t.result_ms += sum[T_RESULT];
    t.call_ms += call_ms;
    t.calls += 1;
  }
};

int clog2(long long d) {
  int e = 0;
  while ((1ll << e) < d) ++e;
  return e;
}

// ---------------------------------------------------------------------------
// Argument checks (before any device work).
// ---------------------------------------------------------------------------
int check_graph(const katz_csr* g) {
  if (!g) return KATZ_E_INVALID_ARG;
  if (g->n < 1 || g->n > INT32_MAX || g->nnz < 0) return KATZ_E_INVALID_ARG;
  if (!g->row_ptr || (g->nnz > 0 && !g->col)) return KATZ_E_INVALID_ARG;
  if (g->row_ptr_64 != 0 && g->row_ptr_64 != 1) return KATZ_E_INVALID_ARG;
  if (!g->row_ptr_64 && g->nnz > INT32_MAX) return KATZ_E_INVALID_ARG;
  if (g->undirected != 0 && g->undirected != 1) return KATZ_E_INVALID_ARG;
  return KATZ_OK;
}

int check_params(const katz_params* p, long long n, bool need_k) {
  if (!p) return KATZ_E_INVALID_ARG;
  if (p->precision != KATZ_FP64 && p->precision != KATZ_FP32_MARGIN) return KATZ_E_INVALID_ARG;
  if (p->validate < 0 || p->validate > 2 ||
      (p->flags & ~(KATZ_FLAG_NO_REORDER | KATZ_FLAG_REORDER | KATZ_FLAG_INBOUND)) || p->max_iter < 0)
    return KATZ_E_INVALID_ARG;
  if (p->degree_cap < 0) return KATZ_E_INVALID_ARG;
  if (std::isnan(p->alpha) || p->alpha < 0.0 || std::isinf(p->alpha)) return KATZ_E_ALPHA;
  if (need_k) {
    if (p->criterion < KATZ_TOPK || p->criterion > KATZ_PAIR) return KATZ_E_INVALID_ARG;
    if (p->criterion == KATZ_TOPK && (p->k < 1 || p->k > n)) return KATZ_E_INVALID_ARG;
    if (p->criterion == KATZ_PAIR &&
        (p->pair_u < 0 || p->pair_u >= n || p->pair_v < 0 || p->pair_v >= n || p->pair_u == p->pair_v))
      return KATZ_E_INVALID_ARG;
    if (!(p->epsilon >= 0.0) || std::isinf(p->epsilon)) return KATZ_E_INVALID_ARG;
  }
  return KATZ_OK;
}

// Length of the ranked output list: k for top-k, every node for the ranking
// and score criteria, the two nodes for the pair criterion.
int output_len(const katz_params* p, long long n) {
  switch (p->criterion) {
    case KATZ_RANKING:
    case KATZ_SCORE: return (int)n;
    case KATZ_PAIR: return 2;
    default: return p->k;
  }
}

// Batched graphs and dynamic states select with one workgroup's LDS sort.
int check_lds_criterion(const katz_params* p) {
  return (p->criterion != KATZ_TOPK || p->k > kMaxK) ? KATZ_E_UNSUPPORTED : KATZ_OK;
}

// ---------------------------------------------------------------------------
// Bins of one graph (or of one list of affected rows).
// ---------------------------------------------------------------------------
struct Bins {
  RowDesc* desc = nullptr;
  SegDesc* segs = nullptr;
  HugeRow* huge = nullptr;
  long long* blk = nullptr;
  long long* scan_sums = nullptr;    // scratch of the device-wide scans
  long long* scan_totals = nullptr;  // [2]
  int nblocks = 0;
  long long seg_cap = 0, huge_cap = 0;
  long long count = 0;   // rows binned
  long long bin_count[NUM_BINS] = {};
  long long bin_base[NUM_BINS] = {};
  long long seg_total = 0;
  int dmax = 0;
  BinBounds bb;   // the length classes the rows are binned by

  void read_back(const RunScalars& h, long long rows) {
    std::memcpy(bin_count, h.bin_count, sizeof(bin_count));
    std::memcpy(bin_base, h.bin_base, sizeof(bin_base));
    seg_total = h.seg_total;
    dmax = h.dmax;
    count = rows;
  }
};

// Capacities for binning up to `rows` rows that hold at most `arcs` arcs.
void bins_caps(Bins& b, long long rows, long long arcs) {
  b.nblocks = (int)std::max<long long>(1, (rows + kWG - 1) / kWG);
  b.seg_cap = 2 * (arcs / kSeg) + 2;
  b.huge_cap = arcs / (kBlockRowMax + 1) + 1;
}

// ---------------------------------------------------------------------------
// Per-run buffers.
// ---------------------------------------------------------------------------
struct Work {
  void* x[2] = {nullptr, nullptr};
  double* c = nullptr;
  float* e = nullptr;
  void* partial = nullptr;
  void* blkmax = nullptr;          // per-workgroup maxima of one walk launch
  int32_t* act[2] = {nullptr, nullptr};
  unsigned long long* keys = nullptr;
  unsigned long long* cand_key[2] = {nullptr, nullptr};
  int32_t* cand_v[2] = {nullptr, nullptr};
  unsigned* hist = nullptr;
  unsigned* xmax32 = nullptr;
  unsigned long long* xmax64 = nullptr;
  double* sigma = nullptr;
  double* sigma_sum = nullptr;
  int32_t* top_sorted = nullptr;
  double* top_lo = nullptr;
  double* top_up = nullptr;
  uint8_t* mark = nullptr;
  unsigned long long* rest_bits = nullptr;
  unsigned long long* sep_count = nullptr;   // separated pairs (ranking and score criteria)
  unsigned long long* sort_key = nullptr;    // device-wide sort of the ranked list
  int32_t* sort_ext = nullptr;
  void* hot_part = nullptr;                  // two-pass walk step: per-row pass-1 sums
  RunScalars* sc = nullptr;
};

struct Scalars {
  double alpha = 0, gamma = 0, beta = 0, beta_hi = 0;
  double rho = 0;
  std::vector<double> eta, etap;   // [max_iter + 1]
};

// gamma and beta exactly as the plain FP64 method evaluates them (Theorem 1);
// beta_hi rounded upward for the FP32 form: 1 - alpha d with one rounding
// (fma), each of the three operations at most one ulp, then 8 ulps of slack.
void set_gamma(Scalars& S, int dmax) {
  S.gamma = (double)dmax / (1.0 - S.alpha * (double)dmax);
  S.beta = S.alpha * S.gamma;
  const double den = std::fma(-S.alpha, (double)dmax, 1.0);
  S.beta_hi = S.alpha * ((double)dmax / den) * (1.0 + 8.0 * kU64);
}

int resolve_alpha(double alpha_in, int dmax, Scalars& S) {
  const double alpha = alpha_in == 0.0 ? 1.0 / (1.0 + (double)dmax) : alpha_in;
  if (!(alpha > 0.0) || !(alpha * (double)dmax < 1.0)) return KATZ_E_ALPHA;
  S.alpha = alpha;
  set_gamma(S, dmax);
  return KATZ_OK;
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Deepest rounding chain of a row sum under the bin schedule: a row of
// length L summed by G lanes takes ceil(L/G) - 1 serial adds per lane, then
// log2(G) combining levels (butterflies, and for a workgroup the two levels
// over its four wave sums); a segmented row adds the combine of its segment
// sums.  Every class up to the longest row's counts at its longest row.
int reduction_depth(long long dmax, const BinBounds& bb) {
  if (dmax <= 0) return 0;
  const long long caps[] = {bb.g4, bb.g8, bb.g16, bb.g32, bb.w16, bb.w64, kBlockRowMax};
  const int bins[] = {BIN_G4, BIN_G8, BIN_G16, BIN_G32, BIN_W16, BIN_W64, BIN_B256};
  int depth = 0;
  for (int i = 0; i < 7; ++i) {
    const long long first = i == 0 ? 1 : caps[i - 1] + 1;
    if (dmax < first) break;
    const int lanes = kBinLanes[bins[i]];
    depth = std::max(depth, (int)((caps[i] + lanes - 1) / lanes - 1) + ilog2(lanes));
  }
  if (dmax > kBlockRowMax) {
    const long long max_seg = (dmax + kSeg - 1) / kSeg;
    const long long q = (max_seg + kWave - 1) / kWave;
    depth = std::max(depth, (int)((kPerLane - 1) + 8 + (q - 1) + 6));
  }
  return depth;
}

// FP32 form: eta_r bounds the relative error of every entry of x~_r; eta_1 = 0
// because the first walk step sums exact ones; later steps multiply by (1 + rho),
// rho = gamma_m = m u / (1 - m u) for the deepest reduction chain m.
// extra: rounding levels added to every row sum (1 for the two-pass walk step,
// whose second pass adds the first pass's sum).
void fp32_tables(Scalars& S, long long dmax, int max_iter, const BinBounds& bb, int extra = 0) {
  const int m = reduction_depth(dmax, bb) + extra;
  S.rho = (m * kU32) / (1.0 - m * kU32) * (1.0 + 0x1p-40);
  S.eta.assign(max_iter + 1, 0.0);
  S.etap.assign(max_iter + 1, 0.0);
  const double up = 1.0 + 0x1p-50;
  S.eta[1] = dmax < (1 << 24) ? 0.0 : kU32;
  for (int r = 2; r <= max_iter; ++r) S.eta[r] = ((1.0 + S.eta[r - 1]) * (1.0 + S.rho) - 1.0) * up;
  for (int r = 1; r <= max_iter; ++r) S.etap[r] = S.eta[r] / (1.0 - S.eta[r]) * up;
}

}  // namespace
}  // namespace katz

namespace katz {
// Device scratch of one update batch; grows to the largest batch seen.
struct UpdateBufs {
  int32_t* pairs = nullptr; size_t pairs_cap = 0;       // a[...] then b[...]
  int32_t* rows = nullptr; size_t rows_cap = 0;
  long long* ll = nullptr; size_t ll_cap = 0;           // ins_off | del_off | new_len | sbase | dest_off
  int* ints = nullptr; size_t ints_cap = 0;             // ins_cnt | del_cnt | delta | dest_cap | caps
  int32_t* dst = nullptr; size_t dst_cap = 0;           // ins_dst | del_dst
  int32_t* scratch = nullptr; size_t scratch_cap = 0;
};
}  // namespace katz

// ---------------------------------------------------------------------------
// Dynamic state (opaque in the C ABI).
// ---------------------------------------------------------------------------
struct katz_state {
  int device = 0;
  long long n = 0, nnz = 0;
  double alpha = 0, eps = 0;
  int k = 1, max_iter = 1000;
  long long degree_cap = 0;
  int r = 0;       // iterations reached
  int cur = 0;     // active-list buffer holding M
  // Slack CSR.
  long long* row_off = nullptr;
  int* row_len = nullptr;
  int* row_cap = nullptr;
  int32_t* pool = nullptr;
  long long pool_cap = 0, pool_used = 0;
  // Directed states: the reverse graph as a second slack CSR (row v lists the
  // sources of the arcs into v, as stored ids in caller-id order), which
  // Algorithm 2's breadth-first search follows.  Unused in undirected states,
  // which are their own reverse.
  long long* rrow_off = nullptr;
  int* rrow_len = nullptr;
  int* rrow_cap = nullptr;
  int32_t* rpool = nullptr;
  long long rpool_cap = 0, rpool_used = 0;
  int directed = 0;   // the graph is directed: lower bound c_r, reverse CSR kept
  int inbound = 0;    // the state holds (and ranks) the reverse of the caller's graph
  // Internal renumbering (as in static calls): row i of the slack CSR is the
  // caller's node ext_of[i]; entries are internal ids, each row kept in the
  // caller-id order of its entries.  Null: the state is in caller order.
  int32_t* ext_of = nullptr;
  int32_t* int_of = nullptr;
  katz::Bins bins;    // whole graph
  bool bins_stale = false;   // rows changed length since the bins were built
  katz::Bins lbins;   // one re-walk level
  katz::Work w;
  katz::Scalars S;
  std::vector<void*> X;            // X[1..]: walk history (X[0] unused); double, or float x~ (FP32)
  void** X_dev = nullptr;          // device copy of the pointer table
  int X_dev_cap = 0;
  // FP32 form (Section 3.3): level i keeps the scale it was first computed
  // with (from the stored maximum of level i - 1 and the degree cap), so a
  // re-walk reproduces the history's arithmetic; eta'_i on the device for the
  // recomputed margins.
  int fp32 = 0;
  double* etap_dev = nullptr;
  // Re-walk scratch.
  int* level_of = nullptr;
  int32_t* clist = nullptr;
  int* counter = nullptr;
  unsigned long long* frontier_arcs = nullptr;   // arcs of the last expansion's new frontier
  long long* foff = nullptr;       // frontier row offsets of an expansion (n), scan scratch, total
  long long* fsums = nullptr;
  long long* ftotal = nullptr;
  int* dmax_dev = nullptr;
  int* err_dev = nullptr;
  unsigned long long* min_bits = nullptr;
  uint8_t* tmark = nullptr;        // touched rows
  katz::RunScalars* sc2 = nullptr;       // prep of one level
  int32_t* out_ids = nullptr;      // [k] staging for outputs in host memory
  double* out_lo = nullptr;
  double* out_up = nullptr;
  katz::UpdateBufs ub;
  katz::UpdateBufs rub;            // the same for the reverse graph of a directed state
  int X_dev_synced = 0;            // entries of X already copied to X_dev
  katz::HostSync hs;
  std::vector<void*> owned;

  ~katz_state() {
    for (void* p : owned) (void)hipFree(p);
    for (void* p : X)
      if (p) (void)hipFree(p);
  }
};

namespace katz {
namespace {

template <class T>
T* dalloc(katz_state* st, size_t count) {
  T* p = nullptr;
  if (hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  st->owned.push_back(p);
  return p;
}

void dfree(katz_state* st, void* p) {
  auto it = std::find(st->owned.begin(), st->owned.end(), p);
  if (it != st->owned.end()) {
    st->owned.erase(it);
    (void)hipFree(p);
  }
}

// ---------------------------------------------------------------------------
// A run: the graph view, its bins, the buffers and the parameters.
// ---------------------------------------------------------------------------
struct Run {
  long long n = 0, nnz = 0;
  int undirected = 1;
  int fp32 = 0;
  int validate = 0;
  const int32_t* col = nullptr;
  Bins* bins = nullptr;
  Work* w = nullptr;
  katz_state* st = nullptr;   // history mode when set
  // FP32 states: the deg_max bound that fixes the scales and the underflow
  // term (the degree cap, so that they hold for every graph the state may
  // reach); 0: the bins' deg_max.
  long long scale_dmax = 0;
  const int32_t* ext_of = nullptr;   // internal -> caller id (nullptr: identity)
  const int32_t* int_of = nullptr;
  Scalars* S = nullptr;
  double eps = 0;
  int criterion = KATZ_TOPK;
  int pair_u = 0, pair_v = 0;  // caller ids (pair criterion)
  int k = 1;                   // length of the ranked list
  int max_iter = 1000;
  int cur = 0;
  bool first_select = true;
  int grid = 1;
  int hub_n = 0;               // walk entries copied to LDS (renumbered static runs)
  long long walk_grid = 0;     // persistent walk grid (0: one workgroup per work item)
  int walk_groups = 1;         // 256-thread groups per walk workgroup (1 or kWalkGroups)
  int split_n = 0;             // two-pass walk steps: hot entries are ids below split_n (0: one pass)
  // Renumbered static runs: walk step 2 also renames the caller's column ids
  // into col (walk_step<F32, true>).
  bool renumber = false;
  const int32_t* col_src = nullptr;
  const long long* coff = nullptr;
  const IdLen* pmap = nullptr;
  int32_t* ncol = nullptr;
};

void* x_at(const Run& run, int r) { return run.st ? run.st->X[r] : run.w->x[r & 1]; }

long long scale_dmax_of(const Run& run) { return run.scale_dmax ? run.scale_dmax : run.bins->dmax; }

void fill_blocks(IterArgs& ia, const Bins& b, bool write_empty, long long& total) {
  long long blocks[NUM_BINS] = {};
  blocks[BIN_HUGE] = b.seg_total;
  blocks[BIN_B256] = b.bin_count[BIN_B256];
  for (int i = BIN_W64; i <= BIN_G4; ++i)
    blocks[i] = (b.bin_count[i] + bin_rows_per_group(i) - 1) / bin_rows_per_group(i);
  blocks[BIN_EMPTY] = write_empty ? (b.bin_count[BIN_EMPTY] + kWG - 1) / kWG : 0;
  ia.first_block[0] = 0;
  for (int i = 0; i < NUM_BINS; ++i) ia.first_block[i + 1] = ia.first_block[i] + blocks[i];
  total = ia.first_block[NUM_BINS];
}

IterArgs iter_args(const Run& run, const Bins& b, int r, bool rewalk, long long& total_blocks) {
  IterArgs ia{};
  ia.desc = b.desc;
  ia.col = run.col;
  ia.segs = b.segs;
  ia.huge = b.huge;
  for (int i = 0; i < NUM_BINS; ++i) {
    ia.bin_base[i] = b.bin_base[i];
    ia.bin_count[i] = b.bin_count[i];
  }
  fill_blocks(ia, b, rewalk || r == 2, total_blocks);
  ia.x_in = r >= 2 ? x_at(run, r - 1) : nullptr;
  ia.x_out = x_at(run, r);
  ia.c = run.w->c;
  ia.e = run.w->e;
  ia.partial = run.w->partial;
  ia.blkmax = run.w->blkmax;
  ia.xmax32 = run.w->xmax32;
  ia.xmax64 = run.w->xmax64;
  ia.sigma = run.w->sigma;
  ia.sigma_sum = run.w->sigma_sum;
  ia.sc = run.w->sc;
  ia.n = (int)run.n;
  ia.r = r;
  ia.count_first = (int)b.count;
  ia.clog2_dmax = clog2((int)std::max<long long>(scale_dmax_of(run), 1));
  ia.rewalk = rewalk ? 1 : 0;
  ia.hub_n = rewalk ? 0 : run.hub_n;
  ia.alpha = run.S->alpha;
  ia.etap = run.fp32 ? run.S->etap[r] : 0.0;
  return ia;
}

BoundArgs bound_args(const Run& run, int r) {
  const Scalars& S = *run.S;
  BoundArgs b{};
  b.c = run.w->c;
  b.x = x_at(run, r);
  b.e = run.w->e;
  b.sigma = run.w->sigma;
  b.sigma_sum = run.w->sigma_sum;
  b.r = r;
  b.fp32 = run.fp32;
  b.undirected = run.undirected;
  b.alpha = S.alpha;
  b.eps = run.eps;
  if (!run.fp32) {
    b.beta = S.beta;
  } else {
    // kappa covers the FP64 roundings of sigma_r (r products), of s~ (one),
    // of c~ (r sums) and of the bound expressions themselves.
    const double kap = (2.0 * r + 32.0) * kU64;
    const double ep = S.etap[r];
    b.beta = S.beta_hi;
    b.kappa = kap;
    b.f_lo_c = 1.0 - kap;
    b.f_hi_c = 1.0 + kap;
    b.f_e = 1.0 + kap;
    b.f_lo_s = run.undirected ? S.alpha * (1.0 - ep) * (1.0 - kap) * (1.0 - 8.0 * kU64) : 0.0;
    b.f_hi_s = S.beta_hi * (1.0 + ep) * (1.0 + kap) * (1.0 + 8.0 * kU64);
    // Underflow of x~ entries: at most (deg_max + 1) 2^-126 per entry and level
    // in units of sigma_i, carried through c (r levels) and the bounds (beta).
    b.tau_coef = 4.0 * (r + S.beta_hi + 2.0) * ((double)scale_dmax_of(run) + 2.0) * 0x1p-126;
  }
  return b;
}

SelArgs sel_args(const Run& run, int r) {
  SelArgs sa{};
  sa.b = bound_args(run, r);
  sa.act_in = run.w->act[run.cur];
  sa.act_out = run.w->act[run.cur ^ 1];
  sa.act_out_idx = run.cur ^ 1;
  sa.keys = run.w->keys;
  sa.cand_key[0] = run.w->cand_key[0];
  sa.cand_key[1] = run.w->cand_key[1];
  sa.cand_v[0] = run.w->cand_v[0];
  sa.cand_v[1] = run.w->cand_v[1];
  sa.hist = run.w->hist;
  sa.top_sorted = run.w->top_sorted;
  sa.top_lo = run.w->top_lo;
  sa.top_up = run.w->top_up;
  sa.xmax32 = run.w->xmax32;
  sa.xmax64 = run.w->xmax64;
  sa.sc = run.w->sc;
  sa.identity_in = run.first_select ? 1 : 0;
  sa.ext_of = run.ext_of;
  sa.int_of = run.int_of;
  sa.k = run.k;
  sa.n = (int)run.n;
  sa.max_iter = run.max_iter;
  return sa;
}

int ensure_levels(katz_state* st, int r);

int refresh_bins(katz_state* st, hipStream_t s);

int enqueue_walk(Run& run, int r, hipStream_t s, CallTimer& T) {
  // A dynamic state re-bins its rows lazily, before the first whole-graph walk
  // after the updates that changed row lengths.
  if (run.st) KATZ_TRY(refresh_bins(run.st, s));
  long long tb = 0;
  IterArgs ia = iter_args(run, *run.bins, r, false, tb);
  const bool renum = run.renumber && r == 2;
  if (run.split_n > 0 && r >= 3) {
    ia.hot_n = run.split_n;
    ia.hot_part = run.w->hot_part;
  }
  if (renum) {
    ia.col_src = run.col_src;
    ia.coff = run.coff;
    ia.pmap = run.pmap;
    ia.ncol = run.ncol;
    ia.hub_n = 0;
  }
  const int tw = T.start(r == 1 ? T_FIRST : renum ? T_RENUM : T_STEP, s);
  if (r == 1) KATZ_HIP(launch_walk_first(ia, run.fp32, run.n, run.nnz, run.validate >= KATZ_VALIDATE_BASIC, s));
  long long grid = 1;
  // The renumbering step runs 256-thread workgroups: as many of them as the
  // tuned grid has groups.
  if (r >= 2)
    KATZ_HIP(launch_walk_step(ia, run.fp32, tb, renum ? run.walk_grid * run.walk_groups : run.walk_grid, &grid, s,
                              renum, renum ? 1 : run.walk_groups));
  T.stop(tw, s);
  const long long nb = r == 1 ? std::max<long long>(1, (run.bins->count + kWG - 1) / kWG) : grid;
  KATZ_HIP(launch_reduce_blkmax(run.w->blkmax, nb, run.fp32, run.w->xmax32, run.w->xmax64, r, run.w->sc, s));
  return KATZ_OK;
}

// small_m: the active set is known to hold at most kSmallActive nodes, so one
// workgroup runs the whole of converged().
int enqueue_select(Run& run, int r, hipStream_t s, CallTimer& T, bool small_m) {
  const int ts = T.start(T_SELECT, s);
  if (run.criterion == KATZ_SCORE) {
    KATZ_HIP(launch_score_check(sel_args(run, r), s));
  } else if (run.criterion == KATZ_PAIR) {
    KATZ_HIP(launch_pair_check(sel_args(run, r), run.pair_u, run.pair_v, s));
  } else if (small_m && run.k <= kMaxK) {
    GraphSel gs{};
    gs.b = bound_args(run, r);
    gs.act[0] = run.w->act[0];
    gs.act[1] = run.w->act[1];
    gs.keys = run.w->keys;
    gs.cand_key = run.w->cand_key[0];
    gs.cand_v = run.w->cand_v[0];
    gs.top_sorted = run.w->top_sorted;
    gs.top_lo = run.w->top_lo;
    gs.top_up = run.w->top_up;
    gs.sc = run.w->sc;
    gs.xmax32 = run.w->xmax32;
    gs.xmax64 = run.w->xmax64;
    gs.base = 0;
    gs.n = (int)run.n;
    gs.k = run.k;
    gs.max_iter = run.max_iter;
    gs.identity_in = run.first_select ? 1 : 0;
    gs.cur = run.cur;
    gs.ext_of = run.ext_of;
    gs.int_of = run.int_of;
    KATZ_HIP(launch_select_wg_one(gs, s));
  } else {
    const SelArgs sa = sel_args(run, r);
    const bool large = run.k > kMaxK;
    KATZ_HIP(launch_select_iteration(sa, run.grid, s, large ? run.w->sort_key : nullptr,
                                     large ? run.w->sort_ext : nullptr));
  }
  T.stop(ts, s);
  run.cur ^= 1;
  run.first_select = false;
  return KATZ_OK;
}

// Iterates until the device stop flag: walk step r_next, selection,
// converged(); then r_next + 1, ...  With check_first, the first pass is only a
// selection at r_next - 1 (after a dynamic update).  Pass p is enqueued before
// the host waits for the flags of pass p - 1; passes enqueued after the stop
// return at once on the device.  On return hs.sc holds the final flags.
int iterate(Run& run, HostSync& hs, int r_next, bool check_first, hipStream_t s, CallTimer& T) {
  bool stopped = false;
  int pass = 0;
  int r = r_next;
  // Upper bound of |M| from the latest flags read back; M never grows inside
  // this loop, so a bound read one pass behind stays valid.
  long long m_known = check_first ? LLONG_MAX : run.n;
  while (!stopped) {
    const Range range("katz iteration", r);
    const bool small_m = m_known <= kSmallActive;
    if (pass == 0 && check_first) {
      KATZ_TRY(enqueue_select(run, r - 1, s, T, false));
    } else if (r <= run.max_iter) {
      if (run.st) KATZ_TRY(ensure_levels(run.st, r));
      KATZ_TRY(enqueue_walk(run, r, s, T));
      KATZ_TRY(enqueue_select(run, r, s, T, small_m));
      ++r;
    } else {
      break;
    }
    KATZ_HIP(hipMemcpyAsync(&hs.ring[pass & 1], run.w->sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    if (hs.ev[0]) KATZ_HIP(hipEventRecord(hs.ev[pass & 1], s));
    if (pass >= 1) {
      if (hs.ev[0]) KATZ_HIP(hipEventSynchronize(hs.ev[(pass - 1) & 1]));
      else KATZ_HIP(hipStreamSynchronize(s));
      const RunScalars& prev = hs.ring[(pass - 1) & 1];
      if (prev.err || prev.done) stopped = true;
      m_known = prev.m;
    }
    ++pass;
  }
  KATZ_HIP(hipMemcpyAsync(hs.sc, run.w->sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (hs.sc->err) return hs.sc->err == 2 ? KATZ_E_HIP : KATZ_E_CSR;
  return KATZ_OK;
}

// Writes ids and bounds of the ranked nodes and the scalar outputs.
int write_result(Run& run, HostSync& hs, katz_result* out, int32_t* stage_ids, double* stage_lo,
                 double* stage_up, hipStream_t s, CallTimer& T) {
  const int rf = hs.sc->iterations;
  const int status = hs.sc->status;
  const long long m_final = hs.sc->m;
  const bool ids_dev = is_device_ptr(out->topk_ids), lo_dev = is_device_ptr(out->lower),
             up_dev = is_device_ptr(out->upper);
  const bool direct = ids_dev && lo_dev && up_dev;
  SelArgs fa{};
  fa.b = bound_args(run, rf);
  fa.top_sorted = run.w->top_sorted;
  fa.top_lo = run.w->top_lo;
  fa.top_up = run.w->top_up;
  fa.ext_of = run.ext_of;
  fa.int_of = run.int_of;
  fa.k = run.k;
  fa.n = (int)run.n;
  int32_t* ids = direct ? out->topk_ids : stage_ids;
  double* lo = direct ? out->lower : stage_lo;
  double* up = direct ? out->upper : stage_up;
  if (!ids || !lo || !up) return KATZ_E_INVALID_ARG;
  const int tr = T.start(T_RESULT, s);
  // Score criterion: the output is every node in ranking order.
  if (run.criterion == KATZ_SCORE) KATZ_HIP(launch_score_output(fa, run.w->sort_key, run.w->sort_ext, s));
  KATZ_HIP(hipMemsetAsync(run.w->mark, 0, (size_t)run.n, s));
  KATZ_HIP(hipMemsetAsync(run.w->rest_bits, 0, sizeof(unsigned long long), s));
  KATZ_HIP(launch_write_result(fa, run.w->mark, ids, lo, up, run.w->rest_bits, run.grid, s));
  // Ranking and score criteria: the sorted lower bounds of every node give the
  // separated pairs.
  const bool all_ranked = run.criterion == KATZ_RANKING || run.criterion == KATZ_SCORE;
  if (all_ranked) {
    KATZ_HIP(hipMemsetAsync(run.w->sep_count, 0, sizeof(unsigned long long), s));
    KATZ_HIP(launch_separated_count(run.w->top_lo, run.w->top_up, run.n, run.w->sep_count, s));
    KATZ_HIP(hipMemcpyAsync(hs.bits + 1, run.w->sep_count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  }
  T.stop(tr, s);
  KATZ_HIP(hipMemcpyAsync(hs.bits, run.w->rest_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (!direct) {
    KATZ_HIP(hipMemcpyAsync(out->topk_ids, ids, sizeof(int32_t) * run.k, hipMemcpyDefault, s));
    KATZ_HIP(hipMemcpyAsync(out->lower, lo, sizeof(double) * run.k, hipMemcpyDefault, s));
    KATZ_HIP(hipMemcpyAsync(out->upper, up, sizeof(double) * run.k, hipMemcpyDefault, s));
  }
  KATZ_HIP(hipStreamSynchronize(s));
  T.commit(s);
  double rest;
  std::memcpy(&rest, hs.bits, sizeof(double));
  out->rest_upper_max = (run.k == run.n) ? -std::numeric_limits<double>::infinity() : rest;
  out->separated_fraction = std::numeric_limits<double>::quiet_NaN();
  if (all_ranked)
    out->separated_fraction = run.n < 2 ? 1.0 : (double)hs.bits[1] / ((double)run.n * (double)(run.n - 1) / 2.0);
  out->alpha_used = run.S->alpha;
  out->eta = run.fp32 ? run.S->eta[rf] : 0.0;
  out->active_final = m_final;
  out->iterations = rf;
  out->status = status;
  return status;
}

// ---------------------------------------------------------------------------
// Static calls: workspace layout in an arena (measure pass, then real pass).
// ---------------------------------------------------------------------------
struct Plan {
  const katz_csr* g;
  int fp32;
  int k;
  int max_iter;
  int validate;
  bool rp_host, col_host, out_host, select;
  bool reorder;   // renumber nodes by degree class (internal)
  size_t out_n;   // elements per output array (k for ranking, n for bounds)
  size_t sort_n;  // records of the device-wide sort of the ranked list (0: none)
  bool check_columns_first = false;   // range-check the column ids during preparation
  int solve_vectors = 0;              // katz_solve: extra n-vectors (FP64) and reduction slots
  int split_n = 0;                    // two-pass walk steps (hot ids below split_n)
};

struct Staging {
  const void* row_ptr = nullptr;
  const int32_t* col = nullptr;
  // Internal renumbering (Plan::reorder).
  int32_t* ncol = nullptr;
  long long* noff = nullptr;
  long long* len_ll = nullptr;
  int* len32 = nullptr;
  int32_t* ext_of = nullptr;
  int32_t* int_of = nullptr;
  long long* coff = nullptr;      // internal id -> caller row offset
  IdLen* pmap = nullptr;          // caller id -> {internal id, length}
  long long* sums = nullptr;
  long long* total = nullptr;
  long long* row_off = nullptr;   // strict symmetry check
  int* row_len = nullptr;
  int32_t* out_ids = nullptr;
  double* out_lo = nullptr;
  double* out_up = nullptr;
  double* vec = nullptr;          // katz_solve: solve_vectors n-vectors
  double* slots = nullptr;        // katz_solve: reduction slots, results and scalars
};

void layout(Arena& ar, const Plan& pl, Bins& b, Work& w, Staging& stg) {
  const long long n = pl.g->n, nnz = pl.g->nnz;
  ar.used = 0;
  bins_caps(b, n, nnz);
  w.sc = ar.take<RunScalars>(1);
  b.blk = ar.take<long long>((size_t)(NUM_BINS + 2) * b.nblocks);
  b.scan_sums = ar.take<long long>(scan_sums_capacity((long long)NUM_BINS * b.nblocks));
  b.scan_totals = ar.take<long long>(2);
  b.desc = ar.take<RowDesc>(n);
  b.segs = ar.take<SegDesc>(b.seg_cap);
  b.huge = ar.take<HugeRow>(b.huge_cap);
  if (pl.rp_host) stg.row_ptr = ar.take<char>((size_t)(n + 1) * (pl.g->row_ptr_64 ? 8 : 4));
  if (pl.col_host) stg.col = ar.take<int32_t>(std::max<long long>(nnz, 1));
  if (pl.validate == KATZ_VALIDATE_STRICT && pl.g->undirected) {
    stg.row_off = ar.take<long long>(n);
    stg.row_len = ar.take<int>(n);
  }
  if (pl.reorder) {
    stg.ncol = ar.take<int32_t>(std::max<long long>(nnz, 1));
    stg.noff = ar.take<long long>(n);
    stg.len_ll = ar.take<long long>(n);
    stg.len32 = ar.take<int>(n);
    stg.ext_of = ar.take<int32_t>(n);
    stg.int_of = ar.take<int32_t>(n);
    stg.coff = ar.take<long long>(n);
    stg.pmap = ar.take<IdLen>(n);
    stg.sums = ar.take<long long>(scan_sums_capacity(n));
    stg.total = ar.take<long long>(1);
  }
  const size_t xs = pl.fp32 ? 4 : 8;
  w.x[0] = ar.take<char>(n * xs);
  w.x[1] = ar.take<char>(n * xs);
  w.c = ar.take<double>(n);
  if (pl.fp32) w.e = ar.take<float>(n);
  if (pl.split_n) w.hot_part = ar.take<char>(n * xs);
  w.partial = ar.take<char>(b.seg_cap * xs);
  w.blkmax = ar.take<double>(n + 2 * b.seg_cap + 16);
  w.xmax32 = ar.take<unsigned>(pl.max_iter + 1);
  w.xmax64 = ar.take<unsigned long long>(pl.max_iter + 1);
  w.sigma = ar.take<double>(pl.max_iter + 1);
  w.sigma_sum = ar.take<double>(pl.max_iter + 1);
  w.hist = ar.take<unsigned>(2 * kDigits);
  if (pl.select) {
    w.act[0] = ar.take<int32_t>(n);
    w.act[1] = ar.take<int32_t>(n);
    w.keys = ar.take<unsigned long long>(n);
    w.cand_key[0] = ar.take<unsigned long long>(n);
    w.cand_key[1] = ar.take<unsigned long long>(n);
    w.cand_v[0] = ar.take<int32_t>(n);
    w.cand_v[1] = ar.take<int32_t>(n);
    w.top_sorted = ar.take<int32_t>(pl.k);
    w.top_lo = ar.take<double>(pl.k);
    w.top_up = ar.take<double>(pl.k);
    w.mark = ar.take<uint8_t>(n);
    w.rest_bits = ar.take<unsigned long long>(1);
    w.sep_count = ar.take<unsigned long long>(1);
    if (pl.sort_n) {
      w.sort_key = ar.take<unsigned long long>(pl.sort_n);
      w.sort_ext = ar.take<int32_t>(pl.sort_n);
    }
  }
  if (pl.solve_vectors) {
    stg.vec = ar.take<double>((size_t)pl.solve_vectors * n);
    stg.slots = ar.take<double>(linear_reduce_slots() + 16);
  }
  if (pl.out_host) {
    stg.out_ids = ar.take<int32_t>(pl.out_n);
    stg.out_lo = ar.take<double>(pl.out_n);
    stg.out_up = ar.take<double>(pl.out_n);
  }
}

int plan_and_allocate(Arena& ar, const Plan& pl, Bins& b, Work& w, Staging& stg) {
  ar.measuring = true;
  layout(ar, pl, b, w, stg);
  ar.measuring = false;
  KATZ_TRY(ar.grow(ar.used));
  layout(ar, pl, b, w, stg);
  return KATZ_OK;
}

// Renumbered runs that reach walk step 2 rename the column ids there; with
// basic validation that step also range-checks them.
bool renumber_in_walk(const Plan& pl) { return pl.reorder && pl.max_iter >= 2; }

// Range check of the caller's column ids for a renumbered run that stopped
// before walk step 2 read them.
int check_columns_if_unread(const Plan& pl, const Staging& stg, const Work& w, HostSync& hs, hipStream_t s) {
  if (!renumber_in_walk(pl) || pl.validate != KATZ_VALIDATE_BASIC || hs.sc->iterations >= 2) return KATZ_OK;
  KATZ_HIP(launch_check_col_range(stg.col, pl.g->nnz, pl.g->n, w.sc, s));
  KATZ_HIP(hipMemcpyAsync(hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  return hs.sc->err ? KATZ_E_CSR : KATZ_OK;
}

// Stages host inputs, bins the rows, reads back d_max and the bin sizes.
int prepare(HostSync& hs, const Plan& pl, Bins& b, Work& w, Staging& stg, hipStream_t s) {
  const katz_csr* g = pl.g;
  if (pl.rp_host)
    KATZ_HIP(hipMemcpyAsync((void*)stg.row_ptr, g->row_ptr, (size_t)(g->n + 1) * (g->row_ptr_64 ? 8 : 4),
                            hipMemcpyHostToDevice, s));
  else
    stg.row_ptr = g->row_ptr;
  if (pl.col_host) {
    if (g->nnz > 0)
      KATZ_HIP(hipMemcpyAsync((void*)stg.col, g->col, (size_t)g->nnz * 4, hipMemcpyHostToDevice, s));
  } else {
    stg.col = g->col;
  }
  KATZ_HIP(launch_init_run(w.sc, g->n, w.sigma, w.sigma_sum, w.xmax32, w.xmax64, pl.max_iter, w.hist, s));
  KATZ_HIP(launch_prep_count(stg.row_ptr, g->row_ptr_64, g->n, g->nnz, b.blk, b.nblocks, w.sc, b.bb, s));
  KATZ_HIP(launch_prep_scan(b.blk, b.nblocks, b.scan_sums, b.scan_totals, w.sc, s));
  KATZ_HIP(launch_prep_scatter(stg.row_ptr, g->row_ptr_64, g->n, b.blk, b.nblocks, b.desc, b.segs, b.huge, w.sc, b.bb,
                               s));
  // Column ids are range-checked before any gather uses them: here, or, when
  // the graph is renumbered with basic validation, in walk step 2, which reads
  // every caller column id to rename it and never indexes with a bad one (no
  // step before it reads a column id; a run that stops before step 2 is
  // checked by check_columns_if_unread).
  const bool check_in_walk = renumber_in_walk(pl) && !pl.check_columns_first;
  if (pl.validate >= KATZ_VALIDATE_BASIC && !check_in_walk)
    KATZ_HIP(launch_check_col_range(stg.col, g->nnz, g->n, w.sc, s));
  KATZ_HIP(hipMemcpyAsync(hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (hs.sc->err) return KATZ_E_CSR;
  b.read_back(*hs.sc, g->n);
  if (pl.validate == KATZ_VALIDATE_STRICT) {
    KATZ_HIP(launch_validate_strict(b.desc, g->n, b.segs, b.seg_total, b.huge, stg.col, g->undirected, stg.row_off,
                                    stg.row_len, w.sc, s));
    KATZ_HIP(hipMemcpyAsync(hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (hs.sc->err) return KATZ_E_CSR;
  }
  if (pl.reorder) {
    // Renumber by the binned order and rebuild the bins on the renumbered rows
    // (now contiguous per bin).
    KATZ_HIP(launch_relabel(b.desc, g->n, stg.ext_of, stg.int_of, stg.coff, stg.pmap, stg.len_ll, stg.len32,
                            stg.noff, stg.sums, stg.total, s));
    KATZ_HIP(launch_prep_rows(nullptr, g->n, stg.noff, stg.len32, b.blk, b.nblocks, b.scan_sums, b.scan_totals,
                              b.desc, b.segs, b.huge, w.sc, b.bb, s));
    KATZ_HIP(hipMemcpyAsync(hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (hs.sc->err) return hs.sc->err == 1 ? KATZ_E_CSR : KATZ_E_HIP;
    b.read_back(*hs.sc, g->n);
  }
  return KATZ_OK;
}

// Two-pass walk steps (katz_tuning.split_hot_bytes): hot ids below the
// returned count; 0 = one pass (the default: on R-MAT 27 the split made the
// walk step 9-17% slower for hot sets of 1-4 MiB).  Renumbered runs only (the
// hot nodes are the first ids, the longest rows).
int split_count(const katz_tuning& tu, const Plan& pl) {
  if (!pl.reorder || tu.split_hot_bytes <= 0) return 0;
  const long long xs = pl.fp32 ? 4 : 8;
  return (int)std::min<long long>(pl.g->n, tu.split_hot_bytes / xs);
}

int check_rank_args(const katz_csr* g, const katz_params* p, const katz_result* out) {
  KATZ_TRY(check_graph(g));
  KATZ_TRY(check_params(p, g->n, true));
  if (!out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  return KATZ_OK;
}

// One static ranking in the workspace of `ar` (grown as needed unless fixed).
// timing: whether the call may record the phase timers (events are created).
int rank_in_arena(Arena& ar, const katz_csr* g, const katz_params* p, katz_result* out, hipStream_t s,
                  bool timing) {
  const Range range_call("katz_rank_static");
  const int dev = ar.device;
  Plan pl{};
  pl.g = g;
  pl.fp32 = p->precision == KATZ_FP32_MARGIN;
  pl.k = p->k;
  pl.max_iter = p->max_iter ? p->max_iter : 1000;
  pl.validate = p->validate;
  pl.rp_host = !is_device_ptr(g->row_ptr);
  pl.col_host = g->nnz > 0 && !is_device_ptr(g->col);
  pl.out_host = !(is_device_ptr(out->topk_ids) && is_device_ptr(out->lower) && is_device_ptr(out->upper));
  pl.select = true;
  pl.reorder = !(p->flags & KATZ_FLAG_NO_REORDER);
  const int klen = output_len(p, g->n);
  pl.k = klen;
  pl.out_n = (size_t)klen;
  pl.sort_n = p->criterion == KATZ_SCORE ? (size_t)g->n : klen > kMaxK ? (size_t)klen : 0;
  const katz_tuning tu = current_tuning();   // one setting for the whole call
  pl.split_n = split_count(tu, pl);

  Bins b;
  b.bb = bounds_of(tu);
  Work w;
  Staging stg;
  KATZ_TRY(plan_and_allocate(ar, pl, b, w, stg));
  CallTimer T(timing);
  T.call_begin(s);
  const int tp = T.start(T_PREP, s);
  const int prc = prepare(ar.hs, pl, b, w, stg, s);
  T.stop(tp, s);
  KATZ_TRY(prc);

  Scalars S;
  KATZ_TRY(resolve_alpha(p->alpha, b.dmax, S));
  if (pl.fp32) fp32_tables(S, b.dmax, pl.max_iter, b.bb, pl.split_n > 0 ? 1 : 0);

  Run run;
  run.n = g->n;
  run.nnz = g->nnz;
  run.undirected = g->undirected;
  run.fp32 = pl.fp32;
  run.validate = KATZ_VALIDATE_NONE;   // columns are checked in prepare() or in walk step 2
  run.col = pl.reorder ? stg.ncol : stg.col;
  run.ext_of = pl.reorder ? stg.ext_of : nullptr;
  run.int_of = pl.reorder ? stg.int_of : nullptr;
  run.renumber = renumber_in_walk(pl);
  run.col_src = stg.col;
  run.coff = stg.coff;
  run.pmap = stg.pmap;
  run.ncol = stg.ncol;
  run.walk_grid = (long long)tu.blocks_per_cu * cu_count(dev);
  run.walk_groups = tu.walk_groups == kWalkGroups ? kWalkGroups : 1;
  run.hub_n = pl.reorder ? (int)std::min<long long>(g->n, tu.hub_bytes / (pl.fp32 ? 4 : 8)) : 0;
  run.split_n = pl.split_n;
  run.bins = &b;
  run.w = &w;
  run.S = &S;
  run.eps = p->epsilon;
  run.criterion = p->criterion;
  run.pair_u = p->pair_u;
  run.pair_v = p->pair_v;
  run.k = klen;
  run.max_iter = pl.max_iter;
  run.grid = (int)std::min<long long>((g->n + kWG - 1) / kWG, 2048);
  KATZ_TRY(iterate(run, ar.hs, 1, false, s, T));
  KATZ_TRY(check_columns_if_unread(pl, stg, w, ar.hs, s));
  return write_result(run, ar.hs, out, stg.out_ids, stg.out_lo, stg.out_up, s, T);
}

// ---------------------------------------------------------------------------
// Inbound form (KATZ_FLAG_INBOUND): inbound Katz centrality of a directed
// graph is the outbound centrality of its reverse graph (Section 2.1), which
// the call builds on the device and ranks in place of g.
// ---------------------------------------------------------------------------
bool wants_reverse(const katz_csr* g, const katz_params* p) {
  return (p->flags & KATZ_FLAG_INBOUND) && !g->undirected;
}

// Checks the offsets and column ids of g (always: the transpose places arcs by
// them) and writes its reverse graph into `ar`.  gt describes the reverse graph
// (device memory, int64 offsets); p2 holds the parameters for the run on it
// (the basic checks are done; strict validation, if asked for, runs on gt,
// which has the same repeated arcs and self-loops as g).
int reverse_graphs(Arena& ar, int count, const katz_csr* g, const katz_params* p, std::vector<katz_csr>& gt,
                   std::vector<katz_params>& p2, hipStream_t s) {
  gt.assign(g, g + count);
  p2.assign(p, p + count);
  // One workspace: per reversed graph its staging and its reverse; the check
  // flags, bin counts and transpose scratch are shared (used one graph at a time).
  long long n_max = 1, nnz_max = 0;
  for (int i = 0; i < count; ++i)
    if (wants_reverse(&g[i], &p[i])) {
      n_max = std::max<long long>(n_max, g[i].n);
      nnz_max = std::max<long long>(nnz_max, g[i].nnz);
    }
  Bins tmp;
  bins_caps(tmp, n_max, nnz_max);
  struct Place {
    char* rp_dev = nullptr;
    int32_t* col_dev = nullptr;
    long long* rt_ptr = nullptr;
    int32_t* rt_col = nullptr;
  };
  std::vector<Place> pl(count);
  RunScalars* sc = nullptr;
  long long* blk = nullptr;
  char* scratch = nullptr;
  auto place = [&]() {
    ar.used = 0;
    sc = ar.take<RunScalars>(1);
    blk = ar.take<long long>((size_t)(NUM_BINS + 2) * tmp.nblocks);
    scratch = ar.take<char>(transpose_scratch_bytes(n_max, nnz_max));
    for (int i = 0; i < count; ++i) {
      if (!wants_reverse(&g[i], &p[i])) continue;
      const long long n = g[i].n, nnz = g[i].nnz;
      if (!is_device_ptr(g[i].row_ptr)) pl[i].rp_dev = ar.take<char>((size_t)(n + 1) * (g[i].row_ptr_64 ? 8 : 4));
      if (nnz > 0 && !is_device_ptr(g[i].col)) pl[i].col_dev = ar.take<int32_t>(nnz);
      pl[i].rt_ptr = ar.take<long long>(n + 1);
      pl[i].rt_col = ar.take<int32_t>(std::max<long long>(nnz, 1));
    }
  };
  ar.measuring = true;
  place();
  ar.measuring = false;
  KATZ_TRY(ar.grow(ar.used));
  place();
  for (int i = 0; i < count; ++i) {
    if (!wants_reverse(&g[i], &p[i])) continue;
    const long long n = g[i].n, nnz = g[i].nnz;
    const void* rp = g[i].row_ptr;
    const int32_t* col = g[i].col;
    if (pl[i].rp_dev) {
      KATZ_HIP(hipMemcpyAsync(pl[i].rp_dev, g[i].row_ptr, (size_t)(n + 1) * (g[i].row_ptr_64 ? 8 : 4),
                              hipMemcpyHostToDevice, s));
      rp = pl[i].rp_dev;
    }
    if (pl[i].col_dev) {
      KATZ_HIP(hipMemcpyAsync(pl[i].col_dev, g[i].col, (size_t)nnz * 4, hipMemcpyHostToDevice, s));
      col = pl[i].col_dev;
    }
    Bins bi;
    bins_caps(bi, n, nnz);
    KATZ_HIP(launch_reset_flags(sc, s));
    KATZ_HIP(launch_prep_count(rp, g[i].row_ptr_64, n, nnz, blk, bi.nblocks, sc, BinBounds{}, s));
    KATZ_HIP(launch_check_col_range(col, nnz, n, sc, s));
    KATZ_HIP(hipMemcpyAsync(ar.hs.sc, sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (ar.hs.sc->err) return KATZ_E_CSR;
    KATZ_HIP(launch_transpose(rp, g[i].row_ptr_64, col, n, nnz, scratch, pl[i].rt_ptr, pl[i].rt_col, s));
    katz_csr& t = gt[i];
    t = katz_csr{};
    t.n = n;
    t.nnz = nnz;
    t.row_ptr = pl[i].rt_ptr;
    t.col = pl[i].rt_col;
    t.row_ptr_64 = 1;
    t.undirected = 0;
    p2[i].flags &= ~KATZ_FLAG_INBOUND;
    if (p2[i].validate == KATZ_VALIDATE_BASIC) p2[i].validate = KATZ_VALIDATE_NONE;
  }
  return KATZ_OK;
}

int reverse_graph(Arena& ar, const katz_csr* g, const katz_params* p, katz_csr& gt, katz_params& p2, hipStream_t s) {
  std::vector<katz_csr> gv;
  std::vector<katz_params> pv;
  KATZ_TRY(reverse_graphs(ar, 1, g, p, gv, pv, s));
  gt = gv[0];
  p2 = pv[0];
  return KATZ_OK;
}

// body(graph, params) on the reverse graph when the call asks for the inbound
// form of a directed graph, else on g itself.  The reverse graph's workspace
// is held until body returns (and ordered after its stream's work).
template <class F>
int on_call_graph(const katz_csr* g, const katz_params* p, hipStream_t s, F&& body) {
  if (!wants_reverse(g, p)) return body(g, p);
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ArenaLease rl(dev, s);
  KATZ_TRY(rl.rc);
  katz_csr gt{};
  katz_params p2{};
  KATZ_TRY(reverse_graph(*rl.a, g, p, gt, p2, s));
  return body(&gt, &p2);
}

int rank_one(const katz_csr* g0, const katz_params* p0, katz_result* out, hipStream_t s) {
  KATZ_TRY(check_rank_args(g0, p0, out));
  return on_call_graph(g0, p0, s, [&](const katz_csr* g, const katz_params* p) {
    int dev = 0;
    KATZ_HIP(hipGetDevice(&dev));
    ArenaLease lease(dev, s);
    KATZ_TRY(lease.rc);
    return rank_in_arena(*lease.a, g, p, out, s, true);
  });
}

int bounds_on(const katz_csr* g, const katz_params* p, int r_target, double* lower, double* upper, hipStream_t s);

int bounds_one(const katz_csr* g, const katz_params* p, int r_target, double* lower, double* upper,
               hipStream_t s) {
  KATZ_TRY(check_graph(g));
  KATZ_TRY(check_params(p, g->n, false));
  if (r_target < 1 || !lower || !upper) return KATZ_E_INVALID_ARG;
  return on_call_graph(g, p, s, [&](const katz_csr* g2, const katz_params* p2) {
    return bounds_on(g2, p2, r_target, lower, upper, s);
  });
}

int bounds_on(const katz_csr* g, const katz_params* p, int r_target, double* lower, double* upper, hipStream_t s) {
  const Range range_call("katz_bounds");
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ArenaLease lease(dev, s);
  KATZ_TRY(lease.rc);
  Arena& ar = *lease.a;
  Plan pl{};
  pl.g = g;
  pl.fp32 = p->precision == KATZ_FP32_MARGIN;
  pl.k = 1;
  pl.max_iter = r_target;
  pl.validate = p->validate;
  pl.rp_host = !is_device_ptr(g->row_ptr);
  pl.col_host = g->nnz > 0 && !is_device_ptr(g->col);
  const bool lo_dev = is_device_ptr(lower), up_dev = is_device_ptr(upper);
  pl.out_host = !(lo_dev && up_dev);
  // Device outputs: the call is stream-ordered and returns once its work is
  // enqueued.  Every error must then be known before that, so the column ids
  // are range-checked in the preparation (a renumbered walk step 2 would
  // otherwise find a bad id only on the device).
  const bool async = !pl.out_host;
  pl.check_columns_first = async;
  pl.select = false;
  pl.reorder = !(p->flags & KATZ_FLAG_NO_REORDER);
  pl.out_n = (size_t)g->n;
  const katz_tuning tu = current_tuning();   // one setting for the whole call
  pl.split_n = split_count(tu, pl);
  Bins b;
  b.bb = bounds_of(tu);
  Work w;
  Staging stg;
  KATZ_TRY(plan_and_allocate(ar, pl, b, w, stg));
  KATZ_TRY(prepare(ar.hs, pl, b, w, stg, s));
  Scalars S;
  KATZ_TRY(resolve_alpha(p->alpha, b.dmax, S));
  if (pl.fp32) fp32_tables(S, b.dmax, pl.max_iter, b.bb, pl.split_n > 0 ? 1 : 0);
  Run run;
  run.n = g->n;
  run.nnz = g->nnz;
  run.undirected = g->undirected;
  run.fp32 = pl.fp32;
  run.validate = KATZ_VALIDATE_NONE;   // columns are checked in prepare() or in walk step 2
  run.col = pl.reorder ? stg.ncol : stg.col;
  run.ext_of = pl.reorder ? stg.ext_of : nullptr;
  run.int_of = pl.reorder ? stg.int_of : nullptr;
  run.renumber = renumber_in_walk(pl);
  run.col_src = stg.col;
  run.coff = stg.coff;
  run.pmap = stg.pmap;
  run.ncol = stg.ncol;
  run.walk_grid = (long long)tu.blocks_per_cu * cu_count(dev);
  run.walk_groups = tu.walk_groups == kWalkGroups ? kWalkGroups : 1;
  run.hub_n = pl.reorder ? (int)std::min<long long>(g->n, tu.hub_bytes / (pl.fp32 ? 4 : 8)) : 0;
  run.split_n = pl.split_n;
  run.bins = &b;
  run.w = &w;
  run.S = &S;
  CallTimer T;
  T.call_begin(s);
  for (int r = 1; r <= r_target; ++r) KATZ_TRY(enqueue_walk(run, r, s, T));
  if (!async) {
    KATZ_HIP(hipMemcpyAsync(ar.hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (ar.hs.sc->err) return KATZ_E_CSR;
  }
  const BoundArgs bd = bound_args(run, r_target);
  double* lo = pl.out_host ? stg.out_lo : lower;
  double* up = pl.out_host ? stg.out_up : upper;
  KATZ_HIP(launch_all_bounds(bd, g->n, run.ext_of, lo, up, s));
  if (pl.out_host) {
    KATZ_HIP(hipMemcpyAsync(lower, lo, sizeof(double) * g->n, hipMemcpyDefault, s));
    KATZ_HIP(hipMemcpyAsync(upper, up, sizeof(double) * g->n, hipMemcpyDefault, s));
    KATZ_HIP(hipStreamSynchronize(s));
  }
  T.commit(s);   // with the timers on this waits for the stream
  return KATZ_OK;
}

// ---------------------------------------------------------------------------
// The paper's comparison methods (katz_solve): Foster's heuristic and
// conjugate gradients on Eq. (la), on the walk kernels' SpMV.
// ---------------------------------------------------------------------------
// y = alpha A v: one walk launch in re-walk mode (row sums times alpha only).
int spmv(const Run& run, const double* v, double* y, hipStream_t s) {
  long long tb = 0;
  IterArgs ia = iter_args(run, *run.bins, 2, true, tb);
  ia.x_in = v;
  ia.x_out = y;
  ia.hub_n = 0;
  long long grid = 0;
  KATZ_HIP(launch_walk_step(ia, 0, tb, run.walk_grid, &grid, s, false, run.walk_groups));
  return KATZ_OK;
}

int read_scalar(const double* dev, double* host, hipStream_t s) {
  KATZ_HIP(hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  return KATZ_OK;
}

int solve_on(const katz_csr* g, const katz_params* p, int method, double tol, double* scores, katz_solve_info* info,
             hipStream_t s);

int solve_one(const katz_csr* g, const katz_params* p, int method, double tol, double* scores,
              katz_solve_info* info, hipStream_t s) {
  KATZ_TRY(check_graph(g));
  KATZ_TRY(check_params(p, g->n, false));
  if (!scores || !(tol > 0.0) || std::isinf(tol)) return KATZ_E_INVALID_ARG;
  if (method != KATZ_SOLVE_FOSTER && method != KATZ_SOLVE_CG) return KATZ_E_INVALID_ARG;
  // CG needs the symmetric matrix of an undirected graph.
  if (method == KATZ_SOLVE_CG && !g->undirected) return KATZ_E_UNSUPPORTED;
  return on_call_graph(g, p, s, [&](const katz_csr* g2, const katz_params* p2) {
    return solve_on(g2, p2, method, tol, scores, info, s);
  });
}

int solve_on(const katz_csr* g, const katz_params* p, int method, double tol, double* scores, katz_solve_info* info,
             hipStream_t s) {
  const Range range_call("katz_solve");
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ArenaLease lease(dev, s);
  KATZ_TRY(lease.rc);
  Arena& ar = *lease.a;
  const long long n = g->n;
  Plan pl{};
  pl.g = g;
  pl.fp32 = 0;
  pl.k = 1;
  pl.max_iter = 2;
  pl.validate = p->validate;
  pl.rp_host = !is_device_ptr(g->row_ptr);
  pl.col_host = g->nnz > 0 && !is_device_ptr(g->col);
  pl.out_host = !is_device_ptr(scores);
  pl.select = false;
  pl.reorder = false;   // caller order: the SpMV reads the caller's column ids
  pl.out_n = (size_t)n;
  pl.solve_vectors = 3;
  Bins b;
  b.bb = bounds_of(current_tuning());
  Work w;
  Staging stg;
  KATZ_TRY(plan_and_allocate(ar, pl, b, w, stg));
  KATZ_TRY(prepare(ar.hs, pl, b, w, stg, s));
  Scalars S;
  KATZ_TRY(resolve_alpha(p->alpha, b.dmax, S));
  Run run;
  run.n = n;
  run.nnz = g->nnz;
  run.undirected = g->undirected;
  run.fp32 = 0;
  run.col = stg.col;
  run.bins = &b;
  run.w = &w;
  run.S = &S;
  {
    const katz_tuning tu = current_tuning();
    run.walk_grid = (long long)tu.blocks_per_cu * cu_count(dev);
    run.walk_groups = tu.walk_groups == kWalkGroups ? kWalkGroups : 1;
  }
  const int max_iter = p->max_iter ? p->max_iter : 1000;
  double* x0 = static_cast<double*>(w.x[0]);
  double* x1 = static_cast<double*>(w.x[1]);
  double* y = w.c;
  double* v0 = stg.vec;
  double* v1 = stg.vec + n;
  double* slots = stg.slots;
  double* res_dev = slots + linear_reduce_slots();   // [0] p.q / max change, [1] r.r
  double* scal = res_dev + 4;                         // [0] r.r, [1] a, [2] b
  double* out = pl.out_host ? stg.out_lo : scores;
  int it = 0;
  bool conv = false;
  double resid = 0.0;
  if (method == KATZ_SOLVE_FOSTER) {
    // f_0 = 1; f_{i+1} = alpha A f_i + 1; the Katz vector is f - 1.
    double* f = x0;
    double* fn = x1;
    KATZ_HIP(launch_fill_value(f, n, 1.0, s));
    while (it < max_iter) {
      KATZ_TRY(spmv(run, f, y, s));
      KATZ_HIP(launch_foster_step(y, f, fn, n, slots, res_dev, s));
      ++it;
      std::swap(f, fn);
      KATZ_TRY(read_scalar(res_dev, &resid, s));
      if (resid < tol) {
        conv = true;
        break;
      }
    }
    KATZ_HIP(launch_write_scores(f, -1.0, n, nullptr, out, s));
  } else {
    // (I - alpha A) z = 1 from z = 0: r = p = 1, r.r = n.
    double* z = x0;
    double* r = x1;
    double* pv = v0;
    double* q = v1;
    KATZ_HIP(launch_fill_value(z, n, 0.0, s));
    KATZ_HIP(launch_fill_value(r, n, 1.0, s));
    KATZ_HIP(launch_fill_value(pv, n, 1.0, s));
    KATZ_HIP(launch_fill_value(scal, 1, (double)n, s));
    const double bnorm = std::sqrt((double)n);
    while (it < max_iter) {
      KATZ_TRY(spmv(run, pv, y, s));
      KATZ_HIP(launch_cg_apply(pv, y, q, n, slots, res_dev, scal, s));
      KATZ_HIP(launch_cg_update(z, r, pv, q, n, slots, res_dev + 1, scal, s));
      ++it;
      double rr = 0.0;
      KATZ_TRY(read_scalar(res_dev + 1, &rr, s));
      resid = std::sqrt(rr) / bnorm;
      if (resid < tol) {
        conv = true;
        break;
      }
      KATZ_HIP(launch_cg_direction(pv, r, scal, n, s));
    }
    // The Katz vector alpha A z.
    KATZ_TRY(spmv(run, z, y, s));
    KATZ_HIP(launch_write_scores(y, 0.0, n, nullptr, out, s));
  }
  if (pl.out_host) KATZ_HIP(hipMemcpyAsync(scores, out, sizeof(double) * n, hipMemcpyDefault, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iterations = it;
    info->converged = conv ? 1 : 0;
    info->residual = resid;
    info->alpha_used = S.alpha;
  }
  return conv ? KATZ_OK : KATZ_W_ITER_LIMIT;
}

// ---------------------------------------------------------------------------
// Batched form: many graphs in one sequence of launches (katz_batch.hip).
// ---------------------------------------------------------------------------
constexpr int kItersPerGraph = 4;   // iterations captured in one hipGraph

int rank_batch(int count, const katz_csr* g, const katz_params* p, katz_result* out, hipStream_t s) {
  const Range range_call("katz_rank_static batch");
  const katz_tuning tu_b = current_tuning();   // one setting for the whole call
  const int xcd_groups = tu_b.batch_xcd ? kXcds : 1;
  const int fp32 = p[0].precision == KATZ_FP32_MARGIN;
  long long total_n = 0, total_nnz = 0, max_n = 0, sum_k = 0;
  int max_iter = 1;
  for (int i = 0; i < count; ++i) {
    if ((p[i].precision == KATZ_FP32_MARGIN) != (fp32 != 0)) return KATZ_E_UNSUPPORTED;
    if (wants_reverse(&g[i], &p[i])) return KATZ_E_UNSUPPORTED;
    total_n += g[i].n;
    total_nnz += g[i].nnz;
    max_n = std::max<long long>(max_n, g[i].n);
    sum_k += p[i].k;
    max_iter = std::max(max_iter, p[i].max_iter ? p[i].max_iter : 1000);
  }
  // Renumbering pays where a walk vector outgrows one XCD's L2 (4 MiB).
  bool reorder = false, no_reorder = false;
  for (int i = 0; i < count; ++i) {
    if (p[i].flags & KATZ_FLAG_NO_REORDER) no_reorder = true;
    if ((p[i].flags & KATZ_FLAG_REORDER) || g[i].n * (fp32 ? 4 : 8) > (4ll << 20)) reorder = true;
  }
  if (no_reorder) reorder = false;
  if (total_n > INT32_MAX) return KATZ_E_UNSUPPORTED;
  const int stride = max_iter + 1;
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ArenaLease lease(dev, s);
  KATZ_TRY(lease.rc);
  Arena& ar = *lease.a;

  // ---- layout ----
  std::vector<bool> rp_host(count), col_host(count);
  bool out_host = false;
  for (int i = 0; i < count; ++i) {
    rp_host[i] = !is_device_ptr(g[i].row_ptr);
    col_host[i] = g[i].nnz > 0 && !is_device_ptr(g[i].col);
    out_host = out_host || !(is_device_ptr(out[i].topk_ids) && is_device_ptr(out[i].lower) &&
                             is_device_ptr(out[i].upper));
  }
  Bins b;
  b.bb = bounds_of(tu_b);
  Work w;
  RunScalars* gsc = nullptr;
  long long* gbase = nullptr;
  long long* gabase = nullptr;   // arc bases: graph g's arcs are gabase[g] .. gabase[g+1]-1 of the batch
  // Internal renumbering of the batch (unless a graph sets KATZ_FLAG_NO_REORDER).
  long long *run_first = nullptr, *run_last = nullptr, *run_start = nullptr;
  int32_t *ext_of = nullptr, *int_of = nullptr, *ncol = nullptr;
  long long *coff = nullptr, *len_ll = nullptr, *noff = nullptr, *rsums = nullptr, *rtot = nullptr;
  int* len32 = nullptr;
  IdLen* pmap = nullptr;
  const int32_t** gcol_walk = nullptr;   // column array of every graph as the walk reads it
  const void** grp = nullptr;
  int* grp64 = nullptr;
  long long* gnnz = nullptr;
  const int32_t** gcol = nullptr;
  double* galpha = nullptr;
  int* gclog2 = nullptr;
  int* gdmax = nullptr;
  double *gsigma = nullptr, *gsigsum = nullptr, *etap = nullptr;
  unsigned long long* rest = nullptr;
  int* gexp = nullptr;
  unsigned* gxmax32 = nullptr;
  unsigned long long* gxmax64 = nullptr;
  int* gid_of = nullptr;
  GraphSel* gsel = nullptr;
  int* blk_g = nullptr;
  double* blk_m = nullptr;
  int* item_g = nullptr;
  int* items = nullptr;
  int* n_items = nullptr;
  int* xcd_of = nullptr;
  long long blk_cap = 0;
  int* r_dev = nullptr;
  int* ndone = nullptr;
  int32_t** o_ids = nullptr;
  double** o_lo = nullptr;
  double** o_up = nullptr;
  std::vector<void*> stage_rp(count, nullptr), stage_col(count, nullptr);
  int32_t* st_ids = nullptr;
  double *st_lo = nullptr, *st_up = nullptr;
  auto lay = [&]() {
    ar.used = 0;
    bins_caps(b, total_n, total_nnz + count);
    w.sc = ar.take<RunScalars>(1);
    gsc = ar.take<RunScalars>(count);
    gbase = ar.take<long long>(count + 1);
    gabase = ar.take<long long>(count + 1);
    gcol_walk = ar.take<const int32_t*>(count);
    if (reorder) {
      run_first = ar.take<long long>((size_t)count * NUM_BINS);
      run_last = ar.take<long long>((size_t)count * NUM_BINS);
      run_start = ar.take<long long>((size_t)count * NUM_BINS);
      ext_of = ar.take<int32_t>(total_n);
      int_of = ar.take<int32_t>(total_n);
      coff = ar.take<long long>(total_n);
      len_ll = ar.take<long long>(total_n);
      noff = ar.take<long long>(total_n);
      len32 = ar.take<int>(total_n);
      pmap = ar.take<IdLen>(total_n);
      ncol = ar.take<int32_t>(std::max<long long>(total_nnz, 1));
      rsums = ar.take<long long>(scan_sums_capacity(total_n));
      rtot = ar.take<long long>(2);
    }
    grp = ar.take<const void*>(count);
    grp64 = ar.take<int>(count);
    gnnz = ar.take<long long>(count);
    gcol = ar.take<const int32_t*>(count);
    galpha = ar.take<double>(count);
    gclog2 = ar.take<int>(count);
    gdmax = ar.take<int>(count);
    gsigma = ar.take<double>((size_t)count * stride);
    gsigsum = ar.take<double>((size_t)count * stride);
    gexp = ar.take<int>((size_t)count * stride);
    gxmax32 = ar.take<unsigned>((size_t)count * stride);
    gxmax64 = ar.take<unsigned long long>((size_t)count * stride);
    etap = ar.take<double>((size_t)count * stride);
    rest = ar.take<unsigned long long>(count);
    gid_of = ar.take<int>(total_n);
    gsel = ar.take<GraphSel>(count);
    // Workgroup slots of one walk step: at most one per 4 rows of up to 1024
    // arcs, one per longer row or segment, one per long row's combine wave group.
    blk_cap = total_n / 4 + total_nnz / 1025 + 2 * b.seg_cap + 64;
    blk_g = ar.take<int>(blk_cap);
    blk_m = ar.take<double>(blk_cap);
    item_g = ar.take<int>(blk_cap);
    items = ar.take<int>(blk_cap * xcd_groups);
    n_items = ar.take<int>(kXcds);
    xcd_of = ar.take<int>(count);
    r_dev = ar.take<int>(1);
    ndone = ar.take<int>(1);
    o_ids = ar.take<int32_t*>(count);
    o_lo = ar.take<double*>(count);
    o_up = ar.take<double*>(count);
    b.blk = ar.take<long long>((size_t)(NUM_BINS + 2) * b.nblocks);
    b.scan_sums = ar.take<long long>(scan_sums_capacity((long long)NUM_BINS * b.nblocks));
    b.scan_totals = ar.take<long long>(2);
    b.desc = ar.take<RowDesc>(total_n);
    b.segs = ar.take<SegDesc>(b.seg_cap);
    b.huge = ar.take<HugeRow>(b.huge_cap);
    const size_t xs = fp32 ? 4 : 8;
    w.x[0] = ar.take<char>(total_n * xs);
    w.x[1] = ar.take<char>(total_n * xs);
    w.c = ar.take<double>(total_n);
    if (fp32) w.e = ar.take<float>(total_n);
    w.partial = ar.take<char>(b.seg_cap * xs);
    w.act[0] = ar.take<int32_t>(total_n);
    w.act[1] = ar.take<int32_t>(total_n);
    w.keys = ar.take<unsigned long long>(total_n);
    w.cand_key[0] = ar.take<unsigned long long>(total_n);
    w.cand_v[0] = ar.take<int32_t>(total_n);
    w.top_sorted = ar.take<int32_t>(sum_k);
    w.top_lo = ar.take<double>(sum_k);
    w.top_up = ar.take<double>(sum_k);
    w.mark = ar.take<uint8_t>(total_n);
    for (int i = 0; i < count; ++i) {
      if (rp_host[i]) stage_rp[i] = ar.take<char>((size_t)(g[i].n + 1) * (g[i].row_ptr_64 ? 8 : 4));
      if (col_host[i]) stage_col[i] = ar.take<int32_t>(g[i].nnz);
    }
    if (out_host) {
      st_ids = ar.take<int32_t>(sum_k);
      st_lo = ar.take<double>(sum_k);
      st_up = ar.take<double>(sum_k);
    }
  };
  ar.measuring = true;
  lay();
  ar.measuring = false;
  KATZ_TRY(ar.grow(ar.used));
  lay();

  CallTimer T;
  T.call_begin(s);
  const int tp = T.start(T_PREP, s);
  // ---- per-graph tables ----
  std::vector<long long> h_base(count + 1, 0), h_abase(count + 1, 0), h_nnz(count);
  std::vector<const void*> h_rp(count);
  std::vector<const int32_t*> h_col(count);
  std::vector<int> h_rp64(count);
  for (int i = 0; i < count; ++i) {
    h_base[i + 1] = h_base[i] + g[i].n;
    h_abase[i + 1] = h_abase[i] + g[i].nnz;
    h_nnz[i] = g[i].nnz;
    h_rp64[i] = g[i].row_ptr_64;
    h_rp[i] = rp_host[i] ? stage_rp[i] : g[i].row_ptr;
    h_col[i] = col_host[i] ? (const int32_t*)stage_col[i] : g[i].col;
    if (rp_host[i])
      KATZ_HIP(hipMemcpyAsync(stage_rp[i], g[i].row_ptr, (size_t)(g[i].n + 1) * (g[i].row_ptr_64 ? 8 : 4),
                              hipMemcpyHostToDevice, s));
    if (col_host[i])
      KATZ_HIP(hipMemcpyAsync(stage_col[i], g[i].col, (size_t)g[i].nnz * 4, hipMemcpyHostToDevice, s));
  }
  KATZ_HIP(hipMemcpyAsync(gbase, h_base.data(), sizeof(long long) * (count + 1), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gnnz, h_nnz.data(), sizeof(long long) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gabase, h_abase.data(), sizeof(long long) * (count + 1), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(grp, h_rp.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(grp64, h_rp64.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gcol, h_col.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(launch_reset_flags(w.sc, s));
  KATZ_HIP(hipMemsetAsync(gdmax, 0, sizeof(int) * count, s));
  int validate = 0;
  for (int i = 0; i < count; ++i) validate = std::max(validate, p[i].validate);
  KATZ_HIP(launch_batch_prep(gbase, grp, grp64, gnnz, gabase, gcol, count, total_n, total_nnz, gid_of, b.blk,
                             b.nblocks, b.scan_sums, b.scan_totals, b.desc, b.segs, b.huge, w.sc, validate, b.bb, s));
  KATZ_HIP(launch_batch_dmax(grp, grp64, gbase, count, total_n, gdmax, s));
  std::vector<int> h_dmax(count);
  KATZ_HIP(hipMemcpyAsync(h_dmax.data(), gdmax, sizeof(int) * count, hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipMemcpyAsync(ar.hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (ar.hs.sc->err) return KATZ_E_CSR;
  b.read_back(*ar.hs.sc, total_n);
  if (reorder && total_n > 0) {
    // Rename every graph's nodes by its binned order, bin the renamed rows
    // again, then write the renamed column ids (graph-local) into ncol.
    KATZ_HIP(hipMemsetAsync(run_first, 0xFF, sizeof(long long) * (size_t)count * NUM_BINS, s));
    KATZ_HIP(hipMemsetAsync(run_last, 0xFF, sizeof(long long) * (size_t)count * NUM_BINS, s));
    KATZ_HIP(launch_batch_relabel(b.desc, total_n, gbase, count, w.sc, run_first, run_last, run_start, ext_of, int_of,
                                  coff, pmap, len_ll, len32, noff, rsums, rtot, s));
    KATZ_HIP(launch_prep_rows(nullptr, total_n, noff, len32, b.blk, b.nblocks, b.scan_sums, b.scan_totals, b.desc,
                              b.segs, b.huge, w.sc, b.bb, s));
    KATZ_HIP(hipMemcpyAsync(ar.hs.sc, w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (ar.hs.sc->err) return ar.hs.sc->err == 1 ? KATZ_E_CSR : KATZ_E_HIP;
    b.read_back(*ar.hs.sc, total_n);
    KATZ_HIP(launch_batch_rename(b.desc, b.bin_base, b.bin_count, b.segs, b.seg_total, b.huge, noff, gid_of, gbase,
                                 gcol, coff, pmap, ncol, s));
  }
  std::vector<const int32_t*> h_cw(count);
  for (int i = 0; i < count; ++i) h_cw[i] = reorder ? ncol : h_col[i];
  KATZ_HIP(hipMemcpyAsync(gcol_walk, h_cw.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));

  // ---- per-graph scalars, selection views, initial state ----
  std::vector<Scalars> S(count);
  for (int i = 0; i < count; ++i) KATZ_TRY(resolve_alpha(p[i].alpha, h_dmax[i], S[i]));
  // FP32 eta tables per graph, from the graph's own longest row (the same
  // tables a single-graph call builds, so results match it bitwise).
  if (fp32)
    for (int i = 0; i < count; ++i) fp32_tables(S[i], h_dmax[i], max_iter, b.bb);
  std::vector<double> h_alpha(count), h_sigma((size_t)count * stride, 0.0), h_sigsum((size_t)count * stride, 0.0);
  std::vector<int> h_clog2(count), h_exp((size_t)count * stride, 0);
  std::vector<RunScalars> h_sc(count);
  std::vector<GraphSel> h_sel(count);
  std::vector<int32_t*> h_oids(count);
  std::vector<double*> h_olo(count), h_oup(count);
  long long koff = 0;
  for (int i = 0; i < count; ++i) {
    h_alpha[i] = S[i].alpha;
    h_clog2[i] = clog2(std::max(h_dmax[i], 1));
    h_sigma[(size_t)i * stride] = 1.0;
    if (fp32) {
      // x_0 = 1, so the first scale exponent is 1 + ceil(log2 d_max).
      const int e1 = 1 + h_clog2[i];
      h_exp[(size_t)i * stride + 1] = e1;
      h_sigma[(size_t)i * stride + 1] = std::ldexp(S[i].alpha, e1);
      h_sigsum[(size_t)i * stride + 1] = h_sigma[(size_t)i * stride + 1];
    }
    RunScalars z{};
    z.m = (int)g[i].n;
    h_sc[i] = z;
    GraphSel& gs = h_sel[i];
    gs = GraphSel{};
    BoundArgs& bd = gs.b;
    bd.c = w.c;
    bd.e = w.e;
    bd.sigma = gsigma + (size_t)i * stride;
    bd.sigma_sum = gsigsum + (size_t)i * stride;
    bd.fp32 = fp32;
    bd.undirected = g[i].undirected;
    bd.alpha = S[i].alpha;
    bd.beta = fp32 ? S[i].beta_hi : S[i].beta;
    bd.eps = p[i].epsilon;
    // Underflow slack with r at its largest (it grows with r).
    bd.tau_coef = 4.0 * (stride + S[i].beta_hi + 2.0) * (h_dmax[i] + 2.0) * 0x1p-126;
    gs.xbuf[0] = w.x[0];
    gs.xbuf[1] = w.x[1];
    gs.etap = etap + (size_t)i * stride;
    gs.act[0] = w.act[0] + h_base[i];
    gs.act[1] = w.act[1] + h_base[i];
    gs.keys = w.keys + h_base[i];
    gs.cand_key = w.cand_key[0] + h_base[i];
    gs.cand_v = w.cand_v[0] + h_base[i];
    gs.top_sorted = w.top_sorted + koff;
    gs.top_lo = w.top_lo + koff;
    gs.top_up = w.top_up + koff;
    gs.sc = gsc + i;
    gs.xmax32 = gxmax32 + (size_t)i * stride;
    gs.xmax64 = gxmax64 + (size_t)i * stride;
    gs.base = (int)h_base[i];
    gs.n = (int)g[i].n;
    gs.ext_of = reorder ? ext_of : nullptr;
    gs.int_of = reorder ? int_of : nullptr;
    gs.k = p[i].k;
    gs.max_iter = p[i].max_iter ? p[i].max_iter : 1000;
    h_oids[i] = out_host ? st_ids + koff : out[i].topk_ids;
    h_olo[i] = out_host ? st_lo + koff : out[i].lower;
    h_oup[i] = out_host ? st_up + koff : out[i].upper;
    koff += p[i].k;
  }
  std::vector<double> h_etap((size_t)count * stride, 0.0);
  if (fp32)
    for (int i = 0; i < count; ++i)
      for (int r = 0; r <= max_iter; ++r) h_etap[(size_t)i * stride + r] = S[i].etap[r];
  KATZ_HIP(hipMemcpyAsync(galpha, h_alpha.data(), sizeof(double) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gclog2, h_clog2.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gsigma, h_sigma.data(), sizeof(double) * h_sigma.size(), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gsigsum, h_sigsum.data(), sizeof(double) * h_sigsum.size(), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gexp, h_exp.data(), sizeof(int) * h_exp.size(), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(etap, h_etap.data(), sizeof(double) * h_etap.size(), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gsc, h_sc.data(), sizeof(RunScalars) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(gsel, h_sel.data(), sizeof(GraphSel) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(o_ids, h_oids.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(o_lo, h_olo.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(o_up, h_oup.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemsetAsync(gxmax32, 0, sizeof(unsigned) * (size_t)count * stride, s));
  KATZ_HIP(hipMemsetAsync(gxmax64, 0, sizeof(unsigned long long) * (size_t)count * stride, s));
  KATZ_HIP(launch_fill_ones(w.x[0], total_n, fp32, s));
  const int one = 1;
  KATZ_HIP(hipMemcpyAsync(r_dev, &one, sizeof(int), hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemsetAsync(ndone, 0, sizeof(int), s));
  T.stop(tp, s);

  // ---- the iteration, captured once and replayed ----
  BatchWalk bw;
  std::memset(&bw, 0, sizeof(bw));   // padding too: the bytes key the cached hipGraph
  bw.desc = b.desc;
  bw.segs = b.segs;
  bw.huge = b.huge;
  const int tile = std::max(1, tu_b.batch_tile);
  {
    // Work items per bin: one per segment / long row, `tile` row groups
    // otherwise (a row group is one workgroup's worth of rows).
    long long per[NUM_BINS];
    for (int i = 0; i < NUM_BINS; ++i) per[i] = bin_rows_per_group(i);
    long long items[NUM_BINS] = {};
    items[BIN_HUGE] = b.seg_total;
    items[BIN_B256] = b.bin_count[BIN_B256];
    for (int i = BIN_W64; i < NUM_BINS; ++i) items[i] = (b.bin_count[i] + per[i] * tile - 1) / (per[i] * tile);
    bw.first_block[0] = 0;
    for (int i = 0; i < NUM_BINS; ++i) bw.first_block[i + 1] = bw.first_block[i] + items[i];
  }
  bw.tile = tile;
  for (int i = 0; i < NUM_BINS; ++i) {
    bw.bin_base[i] = b.bin_base[i];
    bw.bin_count[i] = b.bin_count[i];
  }
  bw.gid_of = gid_of;
  bw.gcol = gcol_walk;
  bw.gbase = gbase;
  bw.galpha = galpha;
  bw.gsc = gsc;
  bw.gsigma = gsigma;
  bw.gexp = gexp;
  bw.gxmax32 = gxmax32;
  bw.gxmax64 = gxmax64;
  bw.xbuf[0] = w.x[0];
  bw.xbuf[1] = w.x[1];
  bw.c = w.c;
  bw.e = w.e;
  bw.partial = w.partial;
  bw.etap = etap;
  bw.r_dev = r_dev;
  bw.stride = stride;
  bw.blk_g = blk_g;
  bw.blk_m = blk_m;
  bw.count = count;
  bw.direct_max = count > kBatchMaxLdsGraphs ? 1 : 0;
  bw.item_g = item_g;
  bw.items = items;
  bw.n_items = n_items;
  bw.xcd_groups = xcd_groups;
  bw.item_cap = blk_cap;
  bw.xcd_of = xcd_of;
  std::vector<int> h_xcd(count, 0);
  if (xcd_groups > 1) {
    // Graphs to XCDs, largest first, each to the least loaded (by arcs).
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) { return g[a2].nnz > g[b2].nnz; });
    long long load[kXcds] = {};
    for (int i : order) {
      int best = 0;
      for (int x = 1; x < kXcds; ++x)
        if (load[x] < load[best]) best = x;
      h_xcd[i] = best;
      load[best] += g[i].nnz + g[i].n;
    }
  }
  KATZ_HIP(hipMemcpyAsync(xcd_of, h_xcd.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
  bw.fp32 = fp32;
  const long long total_blocks = bw.first_block[NUM_BINS];
  long long walk_grid = (long long)tu_b.batch_blocks_per_cu * cu_count(dev);
  if (walk_grid > 0) walk_grid = std::min(walk_grid, batch_walk_resident(fp32));
  {
    const long long nh = b.bin_count[BIN_HUGE];
    if (total_blocks + (nh + kWG / kWave - 1) / (kWG / kWave) > blk_cap) return KATZ_E_HIP;   // sizing bound broken
  }

  if (!ar.graph_stream) KATZ_HIP(hipStreamCreateWithFlags(&ar.graph_stream, hipStreamNonBlocking));
  hipStream_t cs = ar.graph_stream;
  KATZ_HIP(launch_batch_item_graphs(bw, total_blocks, item_g, s));
  KATZ_HIP(hipMemsetAsync(n_items, 0, sizeof(int) * kXcds, s));
  KATZ_HIP(hipStreamSynchronize(s));
  // The captured launches and every value they take; all pointers lie in this
  // call's workspace or its per-graph tables, so a batch of the same shape in
  // the same workspace captures the same bytes.
  std::vector<unsigned char> key;
  auto put = [&key](const void* v, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(v);
    key.insert(key.end(), c, c + bytes);
  };
  const long long n_huge = b.bin_count[BIN_HUGE];
  const void* ptrs[] = {gsel, r_dev, gsc, gxmax32, gsigma, gsigsum, gexp, galpha, gclog2, ndone, n_items, items};
  put(&bw, sizeof(bw));
  put(ptrs, sizeof(ptrs));
  put(&count, sizeof(count));
  put(&stride, sizeof(stride));
  put(&fp32, sizeof(fp32));
  put(&total_blocks, sizeof(total_blocks));
  put(&walk_grid, sizeof(walk_grid));
  put(&n_huge, sizeof(n_huge));
  if (!ar.graph_exec || key != ar.graph_key) {
    ar.drop_graph();
    hipGraph_t gr = nullptr;
    KATZ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int it = 0; it < kItersPerGraph && ce == hipSuccess; ++it) {
      ce = launch_batch_live_items(bw, total_blocks, items, n_items, cs);
      if (ce == hipSuccess) ce = launch_walk_batch(bw, total_blocks, walk_grid, n_huge, cs);
      if (ce == hipSuccess) ce = launch_select_wg(gsel, count, r_dev, cs);
      if (ce == hipSuccess)
        ce = launch_batch_advance(r_dev, count, gsc, gxmax32, gsigma, gsigsum, gexp, galpha, gclog2, stride, fp32,
                                  ndone, n_items, cs);
    }
    const hipError_t ee = hipStreamEndCapture(cs, &gr);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
      return KATZ_E_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&ar.graph_exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ie != hipSuccess) {
      ar.graph_exec = nullptr;
      (void)hipGetLastError();
      return KATZ_E_HIP;
    }
    ar.graph_key = std::move(key);
  }
  const int ts = T.start(T_STEP, cs);
  const int max_replays = (max_iter + kItersPerGraph - 1) / kItersPerGraph + 1;
  int replay = 0;
  bool finished = false;
  int* h_done = reinterpret_cast<int*>(ar.hs.bits);
  while (!finished && replay < max_replays) {
    KATZ_HIP(hipGraphLaunch(ar.graph_exec, cs));
    KATZ_HIP(hipMemcpyAsync(&h_done[replay & 1], ndone, sizeof(int), hipMemcpyDeviceToHost, cs));
    KATZ_HIP(hipEventRecord(ar.hs.ev[replay & 1], cs));
    if (replay >= 1) {
      KATZ_HIP(hipEventSynchronize(ar.hs.ev[(replay - 1) & 1]));
      if (h_done[(replay - 1) & 1] >= count) finished = true;
    }
    ++replay;
  }
  T.stop(ts, cs);
  KATZ_HIP(hipStreamSynchronize(cs));

  // ---- outputs ----
  std::vector<RunScalars> fin(count);
  KATZ_HIP(hipMemcpyAsync(fin.data(), gsc, sizeof(RunScalars) * count, hipMemcpyDeviceToHost, cs));
  KATZ_HIP(hipStreamSynchronize(cs));
  for (int i = 0; i < count; ++i)
    if (fin[i].err) return fin[i].err == 2 ? KATZ_E_HIP : KATZ_E_CSR;
  const int tr = T.start(T_RESULT, cs);
  KATZ_HIP(hipMemsetAsync(w.mark, 0, (size_t)total_n, cs));
  KATZ_HIP(hipMemsetAsync(rest, 0, sizeof(unsigned long long) * count, cs));
  KATZ_HIP(launch_batch_write(gsel, count, max_n, o_ids, o_lo, o_up, w.mark, rest, cs));
  T.stop(tr, cs);
  std::vector<unsigned long long> h_rest(count);
  KATZ_HIP(hipMemcpyAsync(h_rest.data(), rest, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, cs));
  if (out_host) {
    koff = 0;
    for (int i = 0; i < count; ++i) {
      KATZ_HIP(hipMemcpyAsync(out[i].topk_ids, st_ids + koff, sizeof(int32_t) * p[i].k, hipMemcpyDefault, cs));
      KATZ_HIP(hipMemcpyAsync(out[i].lower, st_lo + koff, sizeof(double) * p[i].k, hipMemcpyDefault, cs));
      KATZ_HIP(hipMemcpyAsync(out[i].upper, st_up + koff, sizeof(double) * p[i].k, hipMemcpyDefault, cs));
      koff += p[i].k;
    }
  }
  KATZ_HIP(hipStreamSynchronize(cs));
  T.commit(cs);
  int worst = KATZ_OK;
  for (int i = 0; i < count; ++i) {
    double rest_i;
    std::memcpy(&rest_i, &h_rest[i], sizeof(double));
    out[i].iterations = fin[i].iterations;
    out[i].status = fin[i].done ? fin[i].status : KATZ_W_ITER_LIMIT;
    out[i].active_final = fin[i].m;
    out[i].alpha_used = S[i].alpha;
    out[i].eta = fp32 ? S[i].eta[std::max(1, fin[i].iterations)] : 0.0;
    out[i].rest_upper_max = (p[i].k == g[i].n) ? -std::numeric_limits<double>::infinity() : rest_i;
    worst = std::max(worst, out[i].status);
  }
  return worst;
}

// ---------------------------------------------------------------------------
// Dynamic state.
// ---------------------------------------------------------------------------
long long slack_cap_host(long long len) { return len + std::max(2ll, len >> 3); }

// Walk history levels 1..r exist (zero-initialised, so rows that are empty from
// the start read as 0 without ever being written).
int ensure_levels(katz_state* st, int r) {
  if ((int)st->X.size() <= r) {
    const int want = std::max(r + 1, (int)st->X.size() + 8);
    const size_t xs = st->fp32 ? sizeof(float) : sizeof(double);
    while ((int)st->X.size() < want) {
      void* p = nullptr;
      if (st->X.empty()) {
        st->X.push_back(nullptr);   // level 0 is the implicit all-ones vector
        continue;
      }
      if (hipMalloc(&p, xs * st->n) != hipSuccess) {
        (void)hipGetLastError();
        return KATZ_E_OOM;
      }
      if (hipMemset(p, 0, xs * st->n) != hipSuccess) return KATZ_E_HIP;
      st->X.push_back(p);
    }
  }
  if (st->X_dev_synced == (int)st->X.size()) return KATZ_OK;
  if (st->X_dev_cap < (int)st->X.size()) {
    if (st->X_dev) dfree(st, st->X_dev);
    st->X_dev_cap = (int)st->X.size() + 8;
    st->X_dev = dalloc<void*>(st, st->X_dev_cap);
    if (!st->X_dev) return KATZ_E_OOM;
  }
  KATZ_HIP(hipMemcpy(st->X_dev, st->X.data(), sizeof(void*) * st->X.size(), hipMemcpyHostToDevice));
  st->X_dev_synced = (int)st->X.size();
  return KATZ_OK;
}

// Bins sized for the pool capacity (an upper bound of the arc count).
int alloc_bins(katz_state* st, Bins& b) {
  if (b.desc) {
    dfree(st, b.desc);
    dfree(st, b.segs);
    dfree(st, b.huge);
    dfree(st, b.blk);
    dfree(st, b.scan_sums);
    dfree(st, b.scan_totals);
  }
  bins_caps(b, st->n, st->pool_cap);
  b.desc = dalloc<RowDesc>(st, st->n);
  b.segs = dalloc<SegDesc>(st, b.seg_cap);
  b.huge = dalloc<HugeRow>(st, b.huge_cap);
  b.blk = dalloc<long long>(st, (size_t)(NUM_BINS + 2) * b.nblocks);
  b.scan_sums = dalloc<long long>(st, scan_sums_capacity((long long)NUM_BINS * b.nblocks));
  b.scan_totals = dalloc<long long>(st, 2);
  if (!b.desc || !b.segs || !b.huge || !b.blk || !b.scan_sums || !b.scan_totals) return KATZ_E_OOM;
  return KATZ_OK;
}

int alloc_partial(katz_state* st) {
  if (st->w.partial) dfree(st, st->w.partial);
  if (st->w.blkmax) dfree(st, st->w.blkmax);
  st->w.partial = dalloc<double>(st, st->bins.seg_cap);
  st->w.blkmax = dalloc<double>(st, st->n + 2 * st->bins.seg_cap + 16);
  return st->w.partial && st->w.blkmax ? KATZ_OK : KATZ_E_OOM;
}

// Bins the rows `ids[0..count)` (or every row when ids is null) of the slack CSR.
int bin_rows(katz_state* st, Bins& b, RunScalars* sc, const int32_t* ids, long long count, hipStream_t s) {
  KATZ_HIP(launch_reset_flags(sc, s));
  b.nblocks = (int)std::max<long long>(1, (count + kWG - 1) / kWG);
  KATZ_HIP(launch_prep_rows(ids, count, st->row_off, st->row_len, b.blk, b.nblocks, b.scan_sums, b.scan_totals,
                            b.desc, b.segs, b.huge, sc, b.bb, s));
  KATZ_HIP(hipMemcpyAsync(st->hs.sc, sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (st->hs.sc->err) return KATZ_E_HIP;
  b.read_back(*st->hs.sc, count);
  return KATZ_OK;
}

// The whole-graph bins, rebuilt if an update changed row lengths since they
// were built (the maximum row length is tracked by the updates themselves).
int refresh_bins(katz_state* st, hipStream_t s) {
  if (!st->bins_stale) return KATZ_OK;
  const int dmax = st->bins.dmax;
  KATZ_TRY(bin_rows(st, st->bins, st->sc2, nullptr, st->n, s));
  st->bins.dmax = dmax;
  st->bins_stale = false;
  return KATZ_OK;
}

// The deg_max bound of an FP32 state's scales and error tables: its degree
// cap, or n - 1 when that is smaller (rows hold no repeated neighbour and no
// loop, so no row grows past it).
long long scale_cap(const katz_state* st) {
  return std::max<long long>(1, std::min<long long>(st->degree_cap, std::max<long long>(st->n - 1, 1)));
}

Run state_run(katz_state* st) {
  Run run;
  run.n = st->n;
  run.nnz = st->nnz;
  run.undirected = st->directed ? 0 : 1;
  run.fp32 = st->fp32;
  run.scale_dmax = st->fp32 ? scale_cap(st) : 0;
  run.validate = 0;
  run.col = st->pool;
  run.bins = &st->bins;
  run.w = &st->w;
  run.st = st;
  run.S = &st->S;
  run.eps = st->eps;
  run.k = st->k;
  run.max_iter = st->max_iter;
  run.cur = st->cur;
  run.first_select = false;
  run.grid = (int)std::min<long long>((st->n + kWG - 1) / kWG, 2048);
  run.ext_of = st->ext_of;
  run.int_of = st->int_of;
  if (st->ext_of) {
    // Renumbered: whole-graph walks take the tuned launch shape with the LDS
    // copy of the hottest entries, as static calls do.
    const katz_tuning tu = current_tuning();
    run.walk_grid = (long long)tu.blocks_per_cu * cu_count(st->device);
    run.walk_groups = tu.walk_groups == kWalkGroups ? kWalkGroups : 1;
    run.hub_n = run.walk_grid > 0 ? (int)std::min<long long>(st->n, tu.hub_bytes / (st->fp32 ? 4 : 8)) : 0;
  }
  return run;
}

// Algorithm 1 from level 1 on the state's current graph, in history mode.
int run_from_start(katz_state* st, katz_result* out, hipStream_t s, CallTimer& T) {
  Run run = state_run(st);
  run.first_select = true;
  run.cur = 0;
  KATZ_TRY(iterate(run, st->hs, 1, false, s, T));
  st->r = st->hs.sc->iterations;
  st->cur = st->hs.sc->cur;
  return write_result(run, st->hs, out, st->out_ids, st->out_lo, st->out_up, s, T);
}

// An FP32 state whose re-walk left the range of its stored scales: the whole
// history is recomputed from level 1 with fresh scales (levels cleared, so
// rows that are empty now read as 0 at every level).
int rerun_state(katz_state* st, katz_result* out, hipStream_t s, CallTimer& T) {
  const Range range("katz state re-run");
  Work& w = st->w;
  const size_t xs = st->fp32 ? sizeof(float) : sizeof(double);
  for (size_t i = 1; i < st->X.size(); ++i) KATZ_HIP(hipMemsetAsync(st->X[i], 0, xs * st->n, s));
  KATZ_HIP(hipMemsetAsync(w.mark, 0, st->n, s));
  KATZ_HIP(launch_init_run(w.sc, st->n, w.sigma, w.sigma_sum, w.xmax32, w.xmax64, st->max_iter, w.hist, s));
  return run_from_start(st, out, s, T);
}

// Creates a state from a caller CSR and runs Algorithm 1 on it in history mode.
// One slack CSR of a state: its graph, or a directed state's reverse graph.
struct SlackRef {
  long long*& row_off;
  int*& row_len;
  int*& row_cap;
  int32_t*& pool;
  long long& pool_cap;
  long long& pool_used;
  bool forward;   // the graph the walks read (its pool size sizes the bins)
};

SlackRef fwd_csr(katz_state* st) {
  return SlackRef{st->row_off, st->row_len, st->row_cap, st->pool, st->pool_cap, st->pool_used, true};
}

SlackRef rev_csr(katz_state* st) {
  return SlackRef{st->rrow_off, st->rrow_len, st->rrow_cap, st->rpool, st->rpool_cap, st->rpool_used, false};
}

// A slack CSR from a device CSR: per-row capacities with room to grow, their
// offsets, the rows copied in.
// The layout of a slack CSR (lengths, capacities with room to grow, their
// offsets, the pool size) without its rows.
int slack_layout(katz_state* st, SlackRef c, const void* rp, int rp64, long long n, hipStream_t s) {
  c.row_off = dalloc<long long>(st, n);
  c.row_len = dalloc<int>(st, n);
  c.row_cap = dalloc<int>(st, n);
  long long* cap_ll = dalloc<long long>(st, n);
  long long* sums = dalloc<long long>(st, scan_sums_capacity(n));
  long long* total = dalloc<long long>(st, 1);
  if (!c.row_off || !c.row_len || !c.row_cap || !cap_ll || !sums || !total) return KATZ_E_OOM;
  KATZ_HIP(launch_slack_caps(rp, rp64, n, c.row_len, c.row_cap, cap_ll, s));
  KATZ_HIP(launch_scan_ll(cap_ll, n, c.row_off, sums, total, s));
  long long pool_need = 0;
  KATZ_HIP(hipMemcpyAsync(&pool_need, total, sizeof(long long), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  dfree(st, cap_ll);
  dfree(st, sums);
  dfree(st, total);
  c.pool_used = pool_need;
  c.pool_cap = pool_need + pool_need / 8 + 4096;
  return KATZ_OK;
}

// A slack CSR from a device CSR: the layout, then the rows copied in.
int build_slack(katz_state* st, SlackRef c, const void* rp, int rp64, const int32_t* col, long long n, long long nnz,
                hipStream_t s) {
  KATZ_TRY(slack_layout(st, c, rp, rp64, n, s));
  c.pool = dalloc<int32_t>(st, c.pool_cap);
  if (!c.pool) return KATZ_E_OOM;
  KATZ_HIP(launch_copy_rows_to_pool(rp, rp64, col, n, nnz, c.row_off, c.pool, s));
  return KATZ_OK;
}

// Renames a directed state's reverse CSR by the state's renumbering (rows in
// internal order, entries internal ids kept in caller-id order), as the
// forward CSR was renamed.
int rename_slack(katz_state* st, SlackRef c, hipStream_t s) {
  const long long n = st->n;
  long long* cap_ll = dalloc<long long>(st, n);
  long long* sums = dalloc<long long>(st, scan_sums_capacity(n));
  long long* total = dalloc<long long>(st, 1);
  long long* off_new = dalloc<long long>(st, n);
  int* len_new = dalloc<int>(st, n);
  int* cap_new = dalloc<int>(st, n);
  if (!cap_ll || !sums || !total || !off_new || !len_new || !cap_new) return KATZ_E_OOM;
  // The relabelling kernel rewrites ext_of / int_of from the same bins (the
  // same values) and lists this CSR's capacities in internal order.
  KATZ_HIP(launch_state_relabel(st->bins.desc, n, c.row_cap, st->ext_of, st->int_of, cap_ll, s));
  KATZ_HIP(launch_scan_ll(cap_ll, n, off_new, sums, total, s));
  long long used = 0;
  KATZ_HIP(hipMemcpyAsync(&used, total, sizeof(long long), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  const long long cap = used + used / 8 + 4096;
  int32_t* pool_new = dalloc<int32_t>(st, cap);
  if (!pool_new) return KATZ_E_OOM;
  KATZ_HIP(launch_state_rename_rows(st->ext_of, st->int_of, n, c.row_off, 1, c.row_len, c.row_cap, c.pool, off_new,
                                    used, len_new, cap_new, pool_new, cap_ll, s));
  KATZ_HIP(hipStreamSynchronize(s));
  dfree(st, c.pool);
  dfree(st, c.row_off);
  dfree(st, c.row_len);
  dfree(st, c.row_cap);
  dfree(st, cap_ll);
  dfree(st, sums);
  dfree(st, total);
  c.pool = pool_new;
  c.pool_cap = cap;
  c.pool_used = used;
  c.row_off = off_new;
  c.row_len = len_new;
  c.row_cap = cap_new;
  return KATZ_OK;
}

// The buffers of a state's runs (bound arguments, active lists, selection,
// re-walk scratch, output staging), zeroed where a run expects zeros.  The
// bins must exist (the partial sums are sized by them).
int alloc_run_buffers(katz_state* st, hipStream_t s) {
  Work& w = st->w;
  const long long n = st->n;
  KATZ_TRY(alloc_partial(st));
  w.c = dalloc<double>(st, n);
  w.act[0] = dalloc<int32_t>(st, n);
  w.act[1] = dalloc<int32_t>(st, n);
  w.keys = dalloc<unsigned long long>(st, n);
  w.cand_key[0] = dalloc<unsigned long long>(st, n);
  w.cand_key[1] = dalloc<unsigned long long>(st, n);
  w.cand_v[0] = dalloc<int32_t>(st, n);
  w.cand_v[1] = dalloc<int32_t>(st, n);
  w.hist = dalloc<unsigned>(st, 2 * kDigits);
  w.xmax32 = dalloc<unsigned>(st, st->max_iter + 1);
  w.xmax64 = dalloc<unsigned long long>(st, st->max_iter + 1);
  w.sigma = dalloc<double>(st, st->max_iter + 1);
  w.sigma_sum = dalloc<double>(st, st->max_iter + 1);
  w.top_sorted = dalloc<int32_t>(st, st->k);
  w.top_lo = dalloc<double>(st, st->k);
  w.top_up = dalloc<double>(st, st->k);
  w.mark = dalloc<uint8_t>(st, n);
  w.rest_bits = dalloc<unsigned long long>(st, 1);
  st->level_of = dalloc<int>(st, n);
  st->clist = dalloc<int32_t>(st, n);
  st->counter = dalloc<int>(st, 1);
  st->frontier_arcs = dalloc<unsigned long long>(st, 1);
  st->foff = dalloc<long long>(st, n);
  st->fsums = dalloc<long long>(st, scan_sums_capacity(n));
  st->ftotal = dalloc<long long>(st, 1);
  st->dmax_dev = dalloc<int>(st, 1);
  st->err_dev = dalloc<int>(st, 1);
  st->min_bits = dalloc<unsigned long long>(st, 1);
  st->tmark = dalloc<uint8_t>(st, n);
  st->out_ids = dalloc<int32_t>(st, st->k);
  st->out_lo = dalloc<double>(st, st->k);
  st->out_up = dalloc<double>(st, st->k);
  if (st->fp32) {
    w.e = dalloc<float>(st, n);
    st->etap_dev = dalloc<double>(st, st->max_iter + 1);
    if (!w.e || !st->etap_dev) return KATZ_E_OOM;
    KATZ_HIP(hipMemcpy(st->etap_dev, st->S.etap.data(), sizeof(double) * (st->max_iter + 1), hipMemcpyHostToDevice));
  }
  if (!w.c || !w.act[0] || !w.act[1] || !w.keys || !w.cand_key[0] || !w.cand_key[1] || !w.cand_v[0] ||
      !w.cand_v[1] || !w.hist || !w.xmax32 || !w.xmax64 || !w.sigma || !w.sigma_sum || !w.top_sorted ||
      !w.top_lo || !w.top_up || !w.mark || !w.rest_bits || !st->level_of || !st->clist || !st->counter || !st->frontier_arcs ||
      !st->foff || !st->fsums || !st->ftotal ||
      !st->dmax_dev || !st->err_dev || !st->min_bits || !st->tmark || !st->out_ids || !st->out_lo || !st->out_up)
    return KATZ_E_OOM;
  KATZ_HIP(hipMemsetAsync(w.mark, 0, n, s));
  KATZ_HIP(hipMemsetAsync(st->tmark, 0, n, s));
  KATZ_HIP(hipMemsetAsync(st->level_of, 0, sizeof(int) * n, s));
  KATZ_HIP(launch_init_run(w.sc, n, w.sigma, w.sigma_sum, w.xmax32, w.xmax64, st->max_iter, w.hist, s));
  return KATZ_OK;
}

int create_state(const katz_csr* g, const katz_params* p, katz_result* out, katz_state** stp, hipStream_t s) {
  const Range range_call("katz_rank_static state");
  KATZ_TRY(check_graph(g));
  KATZ_TRY(check_params(p, g->n, true));
  if (!out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  katz_state* st = new katz_state;
  struct Guard {
    katz_state*& p;
    bool keep = false;
    ~Guard() {
      if (!keep) delete p;
    }
  } guard{st};
  st->device = dev;
  st->n = g->n;
  st->nnz = g->nnz;
  st->directed = g->undirected ? 0 : 1;
  st->inbound = wants_reverse(g, p) ? 1 : 0;
  st->fp32 = p->precision == KATZ_FP32_MARGIN ? 1 : 0;
  st->eps = p->epsilon;
  st->k = p->k;
  st->max_iter = p->max_iter ? p->max_iter : 1000;
  KATZ_TRY(st->hs.init());
  const long long n = g->n;

  // Stage a host CSR.
  const void* rp = g->row_ptr;
  const int32_t* col = g->col;
  void* rp_tmp = nullptr;
  int32_t* col_tmp = nullptr;
  if (!is_device_ptr(g->row_ptr)) {
    rp_tmp = dalloc<char>(st, (size_t)(n + 1) * (g->row_ptr_64 ? 8 : 4));
    if (!rp_tmp) return KATZ_E_OOM;
    KATZ_HIP(hipMemcpyAsync(rp_tmp, g->row_ptr, (size_t)(n + 1) * (g->row_ptr_64 ? 8 : 4), hipMemcpyHostToDevice,
                            s));
    rp = rp_tmp;
  }
  if (g->nnz > 0 && !is_device_ptr(g->col)) {
    col_tmp = dalloc<int32_t>(st, g->nnz);
    if (!col_tmp) return KATZ_E_OOM;
    KATZ_HIP(hipMemcpyAsync(col_tmp, g->col, (size_t)g->nnz * 4, hipMemcpyHostToDevice, s));
    col = col_tmp;
  }

  // Validate the input CSR (offsets, column range) before converting it.
  st->w.sc = dalloc<RunScalars>(st, 1);
  st->sc2 = dalloc<RunScalars>(st, 1);
  if (!st->w.sc || !st->sc2) return KATZ_E_OOM;
  {
    Bins tmp;
    bins_caps(tmp, n, g->nnz);
    long long* blk = dalloc<long long>(st, (size_t)(NUM_BINS + 2) * tmp.nblocks);
    if (!blk) return KATZ_E_OOM;
    KATZ_HIP(launch_reset_flags(st->w.sc, s));
    KATZ_HIP(launch_prep_count(rp, g->row_ptr_64, n, g->nnz, blk, tmp.nblocks, st->w.sc, BinBounds{}, s));
    KATZ_HIP(launch_check_col_range(col, g->nnz, n, st->w.sc, s));
    KATZ_HIP(hipMemcpyAsync(st->hs.sc, st->w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    dfree(st, blk);
    if (st->hs.sc->err) return KATZ_E_CSR;
  }

  // Every state transposes its graph once on the device (reversed rows list
  // their sources in ascending order).  An undirected graph must equal its
  // transpose: that is the symmetry check (one pass over the arcs instead of a
  // search per arc).  A directed state keeps the transpose as the reverse
  // graph for Algorithm 2's search; an inbound state ranks the reverse of the
  // caller's graph (Section 2.1) and keeps the caller's graph, rows sorted by
  // a second transpose, as that reverse: fwd = g or T(g), rev = T(g) or T(T(g)).
  const void* fwd_rp = rp;
  int fwd_rp64 = g->row_ptr_64;
  const int32_t* fwd_col = col;
  const void* rev_rp = nullptr;
  const int32_t* rev_col = nullptr;
  std::vector<void*> temps;
  {
    const long long nnz = g->nnz;
    char* scratch = dalloc<char>(st, transpose_scratch_bytes(n, nnz));
    long long* t1_ptr = dalloc<long long>(st, n + 1);
    int32_t* t1_col = dalloc<int32_t>(st, std::max<long long>(nnz, 1));
    if (!scratch || !t1_ptr || !t1_col) return KATZ_E_OOM;
    temps.insert(temps.end(), {scratch, t1_ptr, t1_col});
    KATZ_HIP(launch_transpose(rp, g->row_ptr_64, col, n, nnz, scratch, t1_ptr, t1_col, s));
    if (!st->directed) {
      KATZ_HIP(launch_reset_flags(st->w.sc, s));
      KATZ_HIP(launch_csr_equal(rp, g->row_ptr_64, col, t1_ptr, t1_col, n, nnz, st->w.sc, s));
    } else if (!st->inbound) {
      rev_rp = t1_ptr;
      rev_col = t1_col;
    } else {
      long long* t2_ptr = dalloc<long long>(st, n + 1);
      int32_t* t2_col = dalloc<int32_t>(st, std::max<long long>(nnz, 1));
      if (!t2_ptr || !t2_col) return KATZ_E_OOM;
      temps.insert(temps.end(), {t2_ptr, t2_col});
      KATZ_HIP(launch_transpose(t1_ptr, 1, t1_col, n, nnz, scratch, t2_ptr, t2_col, s));
      fwd_rp = t1_ptr;
      fwd_rp64 = 1;
      fwd_col = t1_col;
      rev_rp = t2_ptr;
      rev_col = t2_col;
    }
    // Strict checks of the graph the state ranks: no self-loop, rows strictly
    // ascending (sorted, no neighbour twice).  With the symmetry check above
    // (an undirected graph), one read-back.
    KATZ_HIP(launch_check_rows_strict(fwd_rp, fwd_rp64, fwd_col, n, nnz, st->w.sc, s));
    KATZ_HIP(hipMemcpyAsync(st->hs.sc, st->w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (st->hs.sc->err) return KATZ_E_CSR;
  }

  // Slack CSRs: capacities and offsets, then the rows copied in; a renumbered
  // state's graph takes its rows renamed straight from the CSR below instead.
  const bool reorder = !(p->flags & KATZ_FLAG_NO_REORDER);
  if (reorder) KATZ_TRY(slack_layout(st, fwd_csr(st), fwd_rp, fwd_rp64, n, s));
  else KATZ_TRY(build_slack(st, fwd_csr(st), fwd_rp, fwd_rp64, fwd_col, n, g->nnz, s));
  if (st->directed) KATZ_TRY(build_slack(st, rev_csr(st), rev_rp, 1, rev_col, n, g->nnz, s));

  // Bins of the whole graph.  The state keeps the length classes of its
  // creation for every later binning, so its re-walks sum rows as a static
  // run with that tuning does.
  st->bins.bb = st->lbins.bb = bounds_of(current_tuning());
  KATZ_TRY(alloc_bins(st, st->bins));
  KATZ_TRY(alloc_bins(st, st->lbins));
  KATZ_TRY(bin_rows(st, st->bins, st->w.sc, nullptr, n, s));

  if (reorder) {
    // Renumber by the binned order (longest rows first), as static calls do, so
    // the walk's most gathered entries share cache lines and the LDS copy.
    st->ext_of = dalloc<int32_t>(st, n);
    st->int_of = dalloc<int32_t>(st, n);
    long long* cap_ll = dalloc<long long>(st, n);
    long long* sums = dalloc<long long>(st, scan_sums_capacity(n));
    long long* total = dalloc<long long>(st, 1);
    long long* off_new = dalloc<long long>(st, n);
    int* len_new = dalloc<int>(st, n);
    int* cap_new = dalloc<int>(st, n);
    if (!st->ext_of || !st->int_of || !cap_ll || !sums || !total || !off_new || !len_new || !cap_new)
      return KATZ_E_OOM;
    KATZ_HIP(launch_state_relabel(st->bins.desc, n, st->row_cap, st->ext_of, st->int_of, cap_ll, s));
    KATZ_HIP(launch_scan_ll(cap_ll, n, off_new, sums, total, s));
    long long used = 0;
    KATZ_HIP(hipMemcpyAsync(&used, total, sizeof(long long), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    const long long cap = used + used / 8 + 4096;
    int32_t* pool_new = dalloc<int32_t>(st, cap);
    if (!pool_new) return KATZ_E_OOM;
    KATZ_HIP(launch_state_rename_rows(st->ext_of, st->int_of, n, fwd_rp, fwd_rp64, st->row_len, st->row_cap, fwd_col,
                                      off_new, used, len_new, cap_new, pool_new, cap_ll, s));
    KATZ_HIP(hipStreamSynchronize(s));
    dfree(st, st->row_off);
    dfree(st, st->row_len);
    dfree(st, st->row_cap);
    dfree(st, cap_ll);
    dfree(st, sums);
    dfree(st, total);
    st->pool = pool_new;
    st->pool_cap = cap;
    st->pool_used = used;
    st->row_off = off_new;
    st->row_len = len_new;
    st->row_cap = cap_new;
    if (st->directed) KATZ_TRY(rename_slack(st, rev_csr(st), s));
    KATZ_TRY(bin_rows(st, st->bins, st->w.sc, nullptr, n, s));
  }
  KATZ_HIP(hipStreamSynchronize(s));
  for (void* t : temps) dfree(st, t);
  if (rp_tmp) dfree(st, rp_tmp);
  if (col_tmp) dfree(st, col_tmp);

  const int dmax = st->bins.dmax;
  KATZ_TRY(resolve_alpha(p->alpha, dmax, st->S));
  st->alpha = st->S.alpha;
  st->degree_cap = p->degree_cap ? p->degree_cap : dmax;
  if (st->degree_cap < dmax) return KATZ_E_INVALID_ARG;
  if (!(st->alpha * (double)st->degree_cap < 1.0)) return KATZ_E_ALPHA;
  // FP32 form: error tables for every graph up to the degree cap.
  if (st->fp32) fp32_tables(st->S, scale_cap(st), st->max_iter, st->bins.bb);

  // Run buffers.
  KATZ_TRY(alloc_run_buffers(st, s));

  CallTimer T;
  T.call_begin(s);
  const int status = run_from_start(st, out, s, T);
  if (status < 0) return status;
  guard.keep = true;
  *stp = st;
  return status;
}

struct Arc {
  int32_t src, dst;
  bool operator<(const Arc& o) const { return src != o.src ? src < o.src : dst < o.dst; }
};

// Copies `count` ids from host or device memory into a host vector.
// Host arrays are copied without a HIP call, so preparing a batch never waits
// on device work.
int fetch_ids(const int32_t* p, long long count, std::vector<int32_t>& out) {
  out.resize(count);
  if (count == 0) return KATZ_OK;
  if (!is_device_ptr(p)) {
    std::memcpy(out.data(), p, sizeof(int32_t) * count);
    return KATZ_OK;
  }
  KATZ_HIP(hipMemcpy(out.data(), p, sizeof(int32_t) * count, hipMemcpyDefault));
  return KATZ_OK;
}

// A device buffer owned by the state that grows on demand.
template <class T>
int grow_buf(katz_state* st, T*& p, size_t& cap, size_t count) {
  if (count <= cap && p) return KATZ_OK;
  if (p) dfree(st, p);
  cap = std::max<size_t>(count, 1024);
  p = dalloc<T>(st, cap);
  return p ? KATZ_OK : KATZ_E_OOM;
}


// Moves the pool to a larger allocation.
int grow_pool(katz_state* st, SlackRef c, long long need, hipStream_t s) {
  if (c.pool_used + need <= c.pool_cap) return KATZ_OK;
  const long long cap = std::max(c.pool_cap * 2, c.pool_used + need + 4096);
  int32_t* np = dalloc<int32_t>(st, cap);
  if (!np) return KATZ_E_OOM;
  KATZ_HIP(hipMemcpyAsync(np, c.pool, sizeof(int32_t) * c.pool_used, hipMemcpyDeviceToDevice, s));
  KATZ_HIP(hipStreamSynchronize(s));
  dfree(st, c.pool);
  c.pool = np;
  c.pool_cap = cap;
  if (c.forward) {
    KATZ_TRY(alloc_bins(st, st->bins));
    KATZ_TRY(alloc_bins(st, st->lbins));
    KATZ_TRY(alloc_partial(st));
  }
  return KATZ_OK;
}

// The touched rows of one slack CSR, read before anything changes.
struct Touched {
  long long t = 0;
  std::vector<long long> new_len, offs;
  std::vector<int> caps;
};

// Uploads one set of row groups into ub (rows in internal ids) and reads back
// each touched row's new length, capacity and offset.  The touched rows are
// left marked in st->tmark.
int stage_groups(katz_state* st, UpdateBufs& ub, SlackRef c, const RowGroups& g, Touched& tt, hipStream_t s) {
  const long long t = (long long)g.rows.size();
  tt.t = t;
  if (t == 0) return KATZ_OK;
  KATZ_TRY(grow_buf(st, ub.rows, ub.rows_cap, t));
  KATZ_TRY(grow_buf(st, ub.ll, ub.ll_cap, 5 * t));
  KATZ_TRY(grow_buf(st, ub.ints, ub.ints_cap, 5 * t));
  KATZ_TRY(grow_buf(st, ub.dst, ub.dst_cap, g.ins_dst.size() + g.del_dst.size()));
  long long* d_ins_off = ub.ll;
  long long* d_del_off = ub.ll + t;
  long long* d_new_len = ub.ll + 2 * t;
  long long* d_offs = ub.ll + 4 * t;
  int* d_ins_cnt = ub.ints;
  int* d_del_cnt = ub.ints + t;
  int* d_delta = ub.ints + 2 * t;
  int* d_caps = ub.ints + 4 * t;
  int32_t* d_ins_dst = ub.dst;
  int32_t* d_del_dst = ub.dst + g.ins_dst.size();
  KATZ_HIP(hipMemcpyAsync(ub.rows, g.rows.data(), sizeof(int32_t) * t, hipMemcpyHostToDevice, s));
  if (st->int_of) KATZ_HIP(launch_map_ids(ub.rows, t, st->int_of, s));   // touched rows, internal ids
  KATZ_HIP(hipMemcpyAsync(d_ins_off, g.ins_off.data(), sizeof(long long) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(d_del_off, g.del_off.data(), sizeof(long long) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(d_ins_cnt, g.ins_cnt.data(), sizeof(int) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(d_del_cnt, g.del_cnt.data(), sizeof(int) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(d_delta, g.delta.data(), sizeof(int) * t, hipMemcpyHostToDevice, s));
  if (!g.ins_dst.empty())
    KATZ_HIP(hipMemcpyAsync(d_ins_dst, g.ins_dst.data(), sizeof(int32_t) * g.ins_dst.size(), hipMemcpyHostToDevice,
                            s));
  if (!g.del_dst.empty())
    KATZ_HIP(hipMemcpyAsync(d_del_dst, g.del_dst.data(), sizeof(int32_t) * g.del_dst.size(), hipMemcpyHostToDevice,
                            s));
  KATZ_HIP(launch_touched_lengths(ub.rows, t, d_delta, c.row_len, d_new_len, st->tmark, s));
  KATZ_HIP(launch_gather_int(ub.rows, t, c.row_cap, d_caps, s));
  KATZ_HIP(launch_gather_ll(ub.rows, t, c.row_off, d_offs, s));
  tt.new_len.resize(t);
  tt.caps.resize(t);
  tt.offs.resize(t);
  KATZ_HIP(hipMemcpyAsync(tt.new_len.data(), d_new_len, sizeof(long long) * t, hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipMemcpyAsync(tt.caps.data(), d_caps, sizeof(int) * t, hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipMemcpyAsync(tt.offs.data(), d_offs, sizeof(long long) * t, hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  return KATZ_OK;
}

// Pool entries the touched rows that outgrow their capacity will take.
long long growth_need(const Touched& tt) {
  long long need = 0;
  for (long long i = 0; i < tt.t; ++i)
    if (tt.new_len[i] > tt.caps[i]) need += slack_cap_host(tt.new_len[i]);
  return need;
}

// Merges every touched row (old row without the deletions, with the
// insertions, in caller-id order) into scratch, then places it in place when
// it fits its capacity, else in a fresh region at the pool's end (the pool
// has grown already).  ub holds what stage_groups uploaded.
int merge_groups(katz_state* st, UpdateBufs& ub, SlackRef c, const RowGroups& g, const Touched& tt, hipStream_t s) {
  const long long t = tt.t;
  if (t == 0) return KATZ_OK;
  std::vector<long long> sbase(t), dest_off(t);
  std::vector<int> dest_cap(t);
  long long scratch_total = 0;
  for (long long i = 0; i < t; ++i) {
    sbase[i] = scratch_total;
    scratch_total += tt.new_len[i];
    if (tt.new_len[i] <= tt.caps[i]) {
      dest_off[i] = tt.offs[i];
      dest_cap[i] = tt.caps[i];
    } else {
      dest_cap[i] = (int)slack_cap_host(tt.new_len[i]);
      dest_off[i] = c.pool_used;
      c.pool_used += dest_cap[i];
    }
  }
  KATZ_TRY(grow_buf(st, ub.scratch, ub.scratch_cap, (size_t)scratch_total));
  long long* d_ins_off = ub.ll;
  long long* d_del_off = ub.ll + t;
  long long* d_new_len = ub.ll + 2 * t;
  long long* d_sbase = ub.ll + 3 * t;
  long long* d_dest_off = ub.ll + 4 * t;
  int* d_ins_cnt = ub.ints;
  int* d_del_cnt = ub.ints + t;
  int* d_dest_cap = ub.ints + 3 * t;
  int32_t* d_ins_dst = ub.dst;
  int32_t* d_del_dst = ub.dst + g.ins_dst.size();
  KATZ_HIP(hipMemcpyAsync(d_sbase, sbase.data(), sizeof(long long) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(d_dest_off, dest_off.data(), sizeof(long long) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(hipMemcpyAsync(d_dest_cap, dest_cap.data(), sizeof(int) * t, hipMemcpyHostToDevice, s));
  KATZ_HIP(launch_merge_rows(ub.rows, t, d_ins_off, d_ins_cnt, d_ins_dst, d_del_off, d_del_cnt, d_del_dst, d_sbase,
                             c.row_off, c.row_len, c.pool, st->ext_of, st->int_of, ub.scratch, s));
  KATZ_HIP(launch_copy_back_rows(ub.rows, t, d_sbase, d_new_len, d_dest_off, d_dest_cap, ub.scratch, c.row_off,
                                 c.row_len, c.row_cap, c.pool, s));
  // The host vectors above are read by the copies: wait before they go.
  KATZ_HIP(hipStreamSynchronize(s));
  return KATZ_OK;
}

// Arcs grouped by the row that stores them (sorted by row, then entry).
void group_arcs(std::vector<Arc>& ia, std::vector<Arc>& da, RowGroups& g) {
  std::sort(ia.begin(), ia.end());
  std::sort(da.begin(), da.end());
  std::vector<int32_t>& rows = g.rows;
  for (const Arc& a : ia) rows.push_back(a.src);
  for (const Arc& a : da) rows.push_back(a.src);
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  const long long t = (long long)rows.size();
  g.ins_off.assign(t, 0);
  g.del_off.assign(t, 0);
  g.ins_cnt.assign(t, 0);
  g.del_cnt.assign(t, 0);
  g.delta.assign(t, 0);
  size_t pi = 0, pd = 0;
  for (long long i = 0; i < t; ++i) {
    g.ins_off[i] = (long long)g.ins_dst.size();
    while (pi < ia.size() && ia[pi].src == rows[i]) g.ins_dst.push_back(ia[pi++].dst);
    g.ins_cnt[i] = (int)(g.ins_dst.size() - g.ins_off[i]);
    g.del_off[i] = (long long)g.del_dst.size();
    while (pd < da.size() && da[pd].src == rows[i]) g.del_dst.push_back(da[pd++].dst);
    g.del_cnt[i] = (int)(g.del_dst.size() - g.del_off[i]);
    g.delta[i] = g.ins_cnt[i] - g.del_cnt[i];
  }
}

}  // namespace

// Host-side half of an update: the batch on its own (ids, loops, repeats,
// I n D) and its arcs grouped by stored row.  It reads no graph state, so a
// server may prepare a request while an earlier request of the same graph is
// still running.
int prepare_batch(long long n, int mode, const int32_t* ins_u, const int32_t* ins_v, long long n_ins,
                  const int32_t* del_u, const int32_t* del_v, long long n_del, PreparedBatch& pb) {
  const Range range_call("katz_rank_update host half");
  if (n_ins < 0 || n_del < 0) return KATZ_E_INVALID_ARG;
  if (mode < PAIRS_UNDIRECTED || mode > PAIRS_REVERSED) return KATZ_E_INVALID_ARG;
  if ((n_ins > 0 && (!ins_u || !ins_v)) || (n_del > 0 && (!del_u || !del_v))) return KATZ_E_INVALID_ARG;
  pb = PreparedBatch{};
  pb.n = n;
  pb.mode = mode;
  pb.n_ins = n_ins;
  pb.n_del = n_del;
  std::vector<int32_t> iu, iv, du, dv;
  KATZ_TRY(fetch_ids(ins_u, n_ins, iu));
  KATZ_TRY(fetch_ids(ins_v, n_ins, iv));
  KATZ_TRY(fetch_ids(del_u, n_del, du));
  KATZ_TRY(fetch_ids(del_v, n_del, dv));
  // An inbound state stores the caller's arc u -> v as v -> u.
  if (mode == PAIRS_REVERSED) {
    std::swap(iu, iv);
    std::swap(du, dv);
  }
  const bool und = mode == PAIRS_UNDIRECTED;
  // Keys of the stored arcs (an undirected edge by its ordered ends).
  auto key = [&](int32_t a, int32_t b) {
    return und ? (long long)std::min(a, b) * n + std::max(a, b) : (long long)a * n + b;
  };
  std::vector<long long> ki, kd;
  ki.reserve(n_ins);
  kd.reserve(n_del);
  for (long long j = 0; j < n_ins; ++j) {
    if (iu[j] < 0 || iu[j] >= n || iv[j] < 0 || iv[j] >= n || iu[j] == iv[j]) return KATZ_E_UPDATE;
    ki.push_back(key(iu[j], iv[j]));
  }
  for (long long j = 0; j < n_del; ++j) {
    if (du[j] < 0 || du[j] >= n || dv[j] < 0 || dv[j] >= n || du[j] == dv[j]) return KATZ_E_UPDATE;
    kd.push_back(key(du[j], dv[j]));
  }
  std::sort(ki.begin(), ki.end());
  std::sort(kd.begin(), kd.end());
  if (std::adjacent_find(ki.begin(), ki.end()) != ki.end()) return KATZ_E_UPDATE;
  if (std::adjacent_find(kd.begin(), kd.end()) != kd.end()) return KATZ_E_UPDATE;
  {
    std::vector<long long> both;
    std::set_intersection(ki.begin(), ki.end(), kd.begin(), kd.end(), std::back_inserter(both));
    if (!both.empty()) return KATZ_E_UPDATE;
  }
  // Arcs for the existence check: a-ends then b-ends, insertions first (an
  // undirected edge is checked by one of its arcs).
  const long long np = n_ins + n_del;
  pb.pa.resize(2 * np);
  for (long long j = 0; j < n_ins; ++j) {
    pb.pa[j] = iu[j];
    pb.pa[np + j] = iv[j];
  }
  for (long long j = 0; j < n_del; ++j) {
    pb.pa[n_ins + j] = du[j];
    pb.pa[np + n_ins + j] = dv[j];
  }
  // Stored arcs by source row; a directed state also keeps the reverse arcs by
  // target row (its reverse graph).
  std::vector<Arc> ia, da, ra, rd;
  ia.reserve(2 * n_ins);
  da.reserve(2 * n_del);
  for (long long j = 0; j < n_ins; ++j) {
    ia.push_back({iu[j], iv[j]});
    if (und) ia.push_back({iv[j], iu[j]});
    else ra.push_back({iv[j], iu[j]});
  }
  for (long long j = 0; j < n_del; ++j) {
    da.push_back({du[j], dv[j]});
    if (und) da.push_back({dv[j], du[j]});
    else rd.push_back({dv[j], du[j]});
  }
  group_arcs(ia, da, pb.fwd);
  if (!und) group_arcs(ra, rd, pb.rev);
  return KATZ_OK;
}

int state_pair_mode(const katz_state* st) {
  return !st->directed ? PAIRS_UNDIRECTED : (st->inbound ? PAIRS_REVERSED : PAIRS_DIRECTED);
}

long long state_nodes(const katz_state* st) { return st->n; }

// Device-side half of an update: existence checks against the state's graph,
// the merge into the slack CSR, the re-walk and the re-certification.
int apply_batch(katz_state* st, const PreparedBatch& pb, katz_result* out, hipStream_t s) {
  const Range range_call("katz_rank_update device half");
  if (!out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  if (pb.n != st->n || pb.mode != state_pair_mode(st)) return KATZ_E_INVALID_ARG;
  const long long n = st->n;
  const long long n_ins = pb.n_ins, n_del = pb.n_del;
  UpdateBufs& ub = st->ub;

  // ---- existence checks against the graph (device) ----
  const long long np = n_ins + n_del;
  if (np > 0) {
    KATZ_TRY(grow_buf(st, ub.pairs, ub.pairs_cap, 2 * np));
    KATZ_HIP(hipMemcpyAsync(ub.pairs, pb.pa.data(), sizeof(int32_t) * 2 * np, hipMemcpyHostToDevice, s));
    KATZ_HIP(hipMemsetAsync(st->err_dev, 0, sizeof(int), s));
    KATZ_HIP(launch_batch_exist(ub.pairs, ub.pairs + np, n_ins, np, st->row_off, st->row_len, st->pool, st->ext_of,
                                st->int_of, st->err_dev, s));
    int err = 0;
    KATZ_HIP(hipMemcpyAsync(&err, st->err_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (err) return KATZ_E_UPDATE;
  }
  const long long t = (long long)pb.fwd.rows.size();

  CallTimer T;
  T.call_begin(s);
  Run run = state_run(st);
  int new_dmax = st->bins.dmax;
  if (t > 0) {
    // ---- candidate degrees and the degree cap (Theorem 1 needs alpha d < 1) ----
    Touched ft, rt;
    KATZ_TRY(stage_groups(st, ub, fwd_csr(st), pb.fwd, ft, s));
    // The new deg_max: the old one raised by the touched rows, unless a row of
    // the old maximum length shrank, when every untouched row is scanned too.
    bool shrank_max = false;
    new_dmax = st->bins.dmax;
    for (long long i = 0; i < t; ++i) {
      const long long old_len = ft.new_len[i] - pb.fwd.delta[i];
      if (old_len == st->bins.dmax && ft.new_len[i] < old_len) shrank_max = true;
      new_dmax = (int)std::max<long long>(new_dmax, ft.new_len[i]);
    }
    if (shrank_max) {
      KATZ_HIP(hipMemsetAsync(st->dmax_dev, 0, sizeof(int), s));
      KATZ_HIP(launch_max_len_after(st->row_len, st->tmark, n, ub.ll + 2 * t, t, st->dmax_dev, s));
      KATZ_HIP(hipMemcpyAsync(&new_dmax, st->dmax_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    }
    KATZ_HIP(launch_unmark_rows(ub.rows, t, st->tmark, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (!(st->alpha * (double)new_dmax < 1.0) || new_dmax > st->degree_cap) return KATZ_E_DEGREE_CAP;
    if (st->directed) {
      KATZ_TRY(stage_groups(st, st->rub, rev_csr(st), pb.rev, rt, s));
      if (rt.t) KATZ_HIP(launch_unmark_rows(st->rub.rows, rt.t, st->tmark, s));
    }

    // ---- apply: pools grown first (a failed allocation leaves the state as
    // it was), then every touched row merged into scratch and placed ----
    KATZ_TRY(grow_pool(st, fwd_csr(st), growth_need(ft), s));
    if (st->directed) KATZ_TRY(grow_pool(st, rev_csr(st), growth_need(rt), s));
    KATZ_TRY(merge_groups(st, ub, fwd_csr(st), pb.fwd, ft, s));
    if (st->directed) KATZ_TRY(merge_groups(st, st->rub, rev_csr(st), pb.rev, rt, s));
    st->nnz += (st->directed ? 1 : 2) * (n_ins - n_del);

    // ---- bins of the new graph: rebuilt before the next whole-graph walk ----
    run = state_run(st);
    st->bins_stale = true;
    st->bins.dmax = new_dmax;

    // ---- re-walk levels 1..r over the affected set (Algorithm 2) ----
    // The walk kernels return at once while the run's stop flag is set; the
    // previous run left it set.
    KATZ_HIP(launch_reset_flags(st->w.sc, s));
    // Dense re-walk (every row) once C covers a quarter of the nodes, or once
    // the frontier to expand is large or has many arcs: expanding it would
    // scan about as many arcs as re-walking every row does.
    const long long dense_at = std::max<long long>(1, n / 4);
    const long long dense_frontier = std::max<long long>(4096, n / 64);
    const unsigned long long dense_arcs = std::max<unsigned long long>(1ull << 16, (unsigned long long)st->nnz / 16);
    unsigned long long f_arcs = 0;   // arcs of the frontier about to be expanded (0: not known)
    KATZ_HIP(hipMemcpyAsync(st->clist, ub.rows, sizeof(int32_t) * t, hipMemcpyDeviceToDevice, s));
    KATZ_HIP(launch_set_levels(ub.rows, t, st->level_of, 1, s));
    long long csize = t, fbeg = 0;
    bool dense = csize > dense_at;
    for (int i = 1; i <= st->r; ++i) {
      if (i >= 2 && !dense && (csize - fbeg > dense_frontier || f_arcs > dense_arcs)) dense = true;
      if (i >= 2 && !dense) {
        // C_i = C_{i-1} u in-neighbours(F_{i-1}); F_{i-1} = C[fbeg .. csize).
        KATZ_HIP(hipMemcpyAsync(st->counter, &csize, sizeof(int), hipMemcpyHostToDevice, s));
        KATZ_HIP(hipMemsetAsync(st->frontier_arcs, 0, sizeof(unsigned long long), s));
        // In-neighbours: the reverse graph's rows (an undirected graph's own).
        const SlackRef in = st->directed ? rev_csr(st) : fwd_csr(st);
        KATZ_HIP(launch_frontier_expand(st->clist + fbeg, csize - fbeg, in.row_off, in.row_len, in.pool,
                                        st->level_of, i, st->clist, st->counter, st->frontier_arcs, st->foff,
                                        st->fsums, st->ftotal, f_arcs, s));
        int c2 = 0;
        KATZ_HIP(hipMemcpyAsync(&c2, st->counter, sizeof(int), hipMemcpyDeviceToHost, s));
        KATZ_HIP(hipMemcpyAsync(&f_arcs, st->frontier_arcs, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        KATZ_HIP(hipStreamSynchronize(s));
        fbeg = csize;
        csize = c2;
        if (csize > dense_at) dense = true;
      }
      long long tb = 0;
      if (dense) {
        // A whole-graph re-walk level: the tuned launch shape (LDS copy of the
        // hottest entries of x_{i-1} in a renumbered state).
        KATZ_TRY(refresh_bins(st, s));
        IterArgs ia2 = iter_args(run, st->bins, i, true, tb);
        ia2.hub_n = run.hub_n;
        long long g_used = 0;
        if (i == 1) KATZ_HIP(launch_walk_first(ia2, run.fp32, n, st->nnz, 0, s));
        else KATZ_HIP(launch_walk_step(ia2, run.fp32, tb, run.walk_grid, &g_used, s, false, run.walk_groups));
      } else {
        KATZ_TRY(bin_rows(st, st->lbins, st->sc2, st->clist, csize, s));
        const IterArgs ia2 = iter_args(run, st->lbins, i, true, tb);
        long long g_used = 0;
        if (i == 1) KATZ_HIP(launch_walk_first(ia2, run.fp32, n, st->nnz, 0, s));
        else KATZ_HIP(launch_walk_step(ia2, run.fp32, tb, 0, &g_used, s));
      }
    }
    // c_r(w) = sum_i x_i(w) for every recomputed w, in the static order (FP32
    // form: sum_i sigma_i x~_i and the margin e_r).
    const int32_t* rows = dense ? nullptr : st->clist;
    const long long count = dense ? n : csize;
    if (!st->fp32) {
      KATZ_HIP(launch_c_from_history(rows, count, reinterpret_cast<double* const*>(st->X_dev), st->r, st->w.c, s));
    } else {
      KATZ_HIP(launch_c_from_history_f32(rows, count, reinterpret_cast<float* const*>(st->X_dev), st->w.sigma,
                                         st->etap_dev, st->r, st->w.c, st->w.e, s));
    }
    KATZ_HIP(launch_clear_levels(st->clist, csize, st->level_of, s));
    if (st->fp32) {
      int rescale = 0;
      KATZ_HIP(hipMemcpyAsync(&rescale, &st->w.sc->rescale, sizeof(int), hipMemcpyDeviceToHost, s));
      KATZ_HIP(hipStreamSynchronize(s));
      if (rescale) {
        set_gamma(st->S, new_dmax);
        return rerun_state(st, out, s, T);
      }
    }
  }

  // ---- gamma from the new deg_max; bounds, reactivation, resume ----
  // The top level's maximum is recomputed (FP32 form: it also sets the scale
  // of the next level); the lower levels keep theirs, which fixed the scales
  // of the levels above them.
  set_gamma(st->S, new_dmax);
  if (!st->fp32) {
    KATZ_HIP(hipMemsetAsync(&st->w.xmax64[st->r], 0, sizeof(unsigned long long), s));
    KATZ_HIP(launch_max_of_vector(static_cast<const double*>(st->X[st->r]), n, &st->w.xmax64[st->r], s));
  } else {
    KATZ_HIP(hipMemsetAsync(&st->w.xmax32[st->r], 0, sizeof(unsigned), s));
    KATZ_HIP(launch_max_of_vector_f32(static_cast<const float*>(st->X[st->r]), n, &st->w.xmax32[st->r], s));
  }
  KATZ_HIP(launch_reset_flags(st->w.sc, s));
  run = state_run(st);
  const BoundArgs b = bound_args(run, st->r);
  KATZ_HIP(hipMemsetAsync(st->min_bits, 0xff, sizeof(unsigned long long), s));
  KATZ_HIP(launch_min_lower_active(b, st->w.act[st->cur], &st->w.sc->m, st->min_bits, st->w.mark, n, s));
  KATZ_HIP(hipMemsetAsync(&st->w.sc->m, 0, sizeof(int), s));
  KATZ_HIP(launch_reactivate_all(b, n, st->min_bits, st->w.mark, st->w.act[st->cur ^ 1], &st->w.sc->m, s));
  run.cur = st->cur ^ 1;
  KATZ_TRY(iterate(run, st->hs, st->r + 1, true, s, T));
  st->r = st->hs.sc->iterations;
  st->cur = st->hs.sc->cur;
  return write_result(run, st->hs, out, st->out_ids, st->out_lo, st->out_up, s, T);
}

// ---------------------------------------------------------------------------
// Saving and restoring a state (Algorithm 2 resumes from Algorithm 1's walk
// counts, bounds and active set: a restored state continues exactly where the
// saved one stood).  The file holds a header of sizes and scalars, then the
// arrays: the slack CSR (and a directed state's reverse CSR) as offsets,
// lengths, capacities and the used part of the pool, the renumbering maps,
// the walk history x_1..x_r, c_r, the active set M, the per-level maxima and
// the run's device flags; an FP32 state adds its margins e_r, the scales
// sigma_i and their sums, and the FP32 level maxima (last in the file).  A
// file records the library's layout version and
// the size of the flag block, and is refused by a library that differs.
// ---------------------------------------------------------------------------
constexpr char kStateMagic[8] = {'K', 'A', 'T', 'Z', 'S', 'T', 'A', 'T'};
constexpr int64_t kStateVersion = 2;

struct StateHeader {
  char magic[8];
  int64_t version, sc_bytes;
  int64_t n, nnz, k, max_iter, degree_cap, r, cur, directed, inbound, renumbered, dmax, m;
  int64_t pool_used, rpool_used;
  double alpha, eps;
  int32_t bb[6];
  int32_t fp32;
};

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

// Device array <-> file through a host buffer.
template <class T>
int write_dev(FILE* f, const T* dev, size_t count) {
  if (count == 0) return KATZ_OK;
  std::vector<T> h(count);
  KATZ_HIP(hipMemcpy(h.data(), dev, sizeof(T) * count, hipMemcpyDeviceToHost));
  return std::fwrite(h.data(), sizeof(T), count, f) == count ? KATZ_OK : KATZ_E_INVALID_ARG;
}

template <class T>
int read_dev(FILE* f, T* dev, size_t count) {
  if (count == 0) return KATZ_OK;
  std::vector<T> h(count);
  if (std::fread(h.data(), sizeof(T), count, f) != count) return KATZ_E_INVALID_ARG;
  KATZ_HIP(hipMemcpy(dev, h.data(), sizeof(T) * count, hipMemcpyHostToDevice));
  return KATZ_OK;
}

int write_slack(FILE* f, const katz_state* st, bool rev) {
  const long long n = st->n;
  KATZ_TRY(write_dev(f, rev ? st->rrow_off : st->row_off, n));
  KATZ_TRY(write_dev(f, rev ? st->rrow_len : st->row_len, n));
  KATZ_TRY(write_dev(f, rev ? st->rrow_cap : st->row_cap, n));
  return write_dev(f, rev ? st->rpool : st->pool, (size_t)(rev ? st->rpool_used : st->pool_used));
}

int read_slack(FILE* f, katz_state* st, SlackRef c, long long used) {
  const long long n = st->n;
  c.row_off = dalloc<long long>(st, n);
  c.row_len = dalloc<int>(st, n);
  c.row_cap = dalloc<int>(st, n);
  c.pool_used = used;
  c.pool_cap = used + used / 8 + 4096;
  c.pool = dalloc<int32_t>(st, c.pool_cap);
  if (!c.row_off || !c.row_len || !c.row_cap || !c.pool) return KATZ_E_OOM;
  KATZ_TRY(read_dev(f, c.row_off, n));
  KATZ_TRY(read_dev(f, c.row_len, n));
  KATZ_TRY(read_dev(f, c.row_cap, n));
  return read_dev(f, c.pool, (size_t)used);
}

int save_state(katz_state* st, const char* path) {
  if (!st || !path) return KATZ_E_INVALID_ARG;
  KATZ_HIP(hipSetDevice(st->device));
  KATZ_HIP(hipDeviceSynchronize());
  RunScalars sc{};
  KATZ_HIP(hipMemcpy(&sc, st->w.sc, sizeof(RunScalars), hipMemcpyDeviceToHost));
  StateHeader h{};
  std::memcpy(h.magic, kStateMagic, sizeof(h.magic));
  h.version = kStateVersion;
  h.sc_bytes = sizeof(RunScalars);
  h.n = st->n;
  h.nnz = st->nnz;
  h.k = st->k;
  h.max_iter = st->max_iter;
  h.degree_cap = st->degree_cap;
  h.r = st->r;
  h.cur = st->cur;
  h.directed = st->directed;
  h.inbound = st->inbound;
  h.renumbered = st->ext_of ? 1 : 0;
  h.dmax = st->bins.dmax;
  h.m = sc.m;
  h.pool_used = st->pool_used;
  h.rpool_used = st->directed ? st->rpool_used : 0;
  h.alpha = st->alpha;
  h.eps = st->eps;
  h.fp32 = st->fp32;
  const BinBounds& bb = st->bins.bb;
  const int32_t bbv[6] = {bb.g4, bb.g8, bb.g16, bb.g32, bb.w16, bb.w64};
  std::memcpy(h.bb, bbv, sizeof(bbv));
  File file;
  file.f = std::fopen(path, "wb");
  if (!file.f) return KATZ_E_INVALID_ARG;
  if (std::fwrite(&h, sizeof(h), 1, file.f) != 1) return KATZ_E_INVALID_ARG;
  if (std::fwrite(&sc, sizeof(sc), 1, file.f) != 1) return KATZ_E_INVALID_ARG;
  KATZ_TRY(write_slack(file.f, st, false));
  if (st->directed) KATZ_TRY(write_slack(file.f, st, true));
  if (st->ext_of) {
    KATZ_TRY(write_dev(file.f, st->ext_of, st->n));
    KATZ_TRY(write_dev(file.f, st->int_of, st->n));
  }
  const size_t xs = st->fp32 ? sizeof(float) : sizeof(double);
  for (long long i = 1; i <= st->r; ++i)
    KATZ_TRY(write_dev(file.f, static_cast<const char*>(st->X[i]), xs * st->n));
  KATZ_TRY(write_dev(file.f, st->w.c, st->n));
  KATZ_TRY(write_dev(file.f, st->w.act[st->cur], (size_t)std::max(sc.m, 0)));
  KATZ_TRY(write_dev(file.f, st->w.xmax64, (size_t)st->max_iter + 1));
  if (st->fp32) {
    KATZ_TRY(write_dev(file.f, st->w.e, st->n));
    KATZ_TRY(write_dev(file.f, st->w.sigma, (size_t)st->max_iter + 1));
    KATZ_TRY(write_dev(file.f, st->w.sigma_sum, (size_t)st->max_iter + 1));
    KATZ_TRY(write_dev(file.f, st->w.xmax32, (size_t)st->max_iter + 1));
  }
  return std::fflush(file.f) == 0 ? KATZ_OK : KATZ_E_INVALID_ARG;
}

int load_state(const char* path, katz_state** stp, hipStream_t s) {
  if (!path || !stp) return KATZ_E_INVALID_ARG;
  File file;
  file.f = std::fopen(path, "rb");
  if (!file.f) return KATZ_E_INVALID_ARG;
  StateHeader h{};
  if (std::fread(&h, sizeof(h), 1, file.f) != 1) return KATZ_E_INVALID_ARG;
  if (std::memcmp(h.magic, kStateMagic, sizeof(h.magic)) != 0 || h.version != kStateVersion ||
      h.sc_bytes != (int64_t)sizeof(RunScalars))
    return KATZ_E_INVALID_ARG;
  if (h.n < 1 || h.n > INT32_MAX || h.k < 1 || h.k > h.n || h.max_iter < 1 || h.r < 1 || h.r > h.max_iter ||
      h.m < 0 || h.m > h.n || (h.cur != 0 && h.cur != 1) || h.pool_used < 0 || h.rpool_used < 0 ||
      (h.fp32 != 0 && h.fp32 != 1) || h.degree_cap < h.dmax)
    return KATZ_E_INVALID_ARG;
  RunScalars sc{};
  if (std::fread(&sc, sizeof(sc), 1, file.f) != 1) return KATZ_E_INVALID_ARG;
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  katz_state* st = new katz_state;
  struct Guard {
    katz_state*& p;
    bool keep = false;
    ~Guard() {
      if (!keep) delete p;
    }
  } guard{st};
  st->device = dev;
  st->n = h.n;
  st->nnz = h.nnz;
  st->k = (int)h.k;
  st->max_iter = (int)h.max_iter;
  st->degree_cap = h.degree_cap;
  st->r = (int)h.r;
  st->cur = (int)h.cur;
  st->directed = (int)h.directed;
  st->inbound = (int)h.inbound;
  st->fp32 = h.fp32;
  st->alpha = h.alpha;
  st->eps = h.eps;
  KATZ_TRY(st->hs.init());
  const long long n = st->n;
  st->w.sc = dalloc<RunScalars>(st, 1);
  st->sc2 = dalloc<RunScalars>(st, 1);
  if (!st->w.sc || !st->sc2) return KATZ_E_OOM;
  KATZ_TRY(read_slack(file.f, st, fwd_csr(st), h.pool_used));
  if (st->directed) KATZ_TRY(read_slack(file.f, st, rev_csr(st), h.rpool_used));
  if (h.renumbered) {
    st->ext_of = dalloc<int32_t>(st, n);
    st->int_of = dalloc<int32_t>(st, n);
    if (!st->ext_of || !st->int_of) return KATZ_E_OOM;
    KATZ_TRY(read_dev(file.f, st->ext_of, n));
    KATZ_TRY(read_dev(file.f, st->int_of, n));
  }
  BinBounds bb;
  bb.g4 = h.bb[0];
  bb.g8 = h.bb[1];
  bb.g16 = h.bb[2];
  bb.g32 = h.bb[3];
  bb.w16 = h.bb[4];
  bb.w64 = h.bb[5];
  st->bins.bb = st->lbins.bb = bb;
  KATZ_TRY(alloc_bins(st, st->bins));
  KATZ_TRY(alloc_bins(st, st->lbins));
  st->bins.dmax = (int)h.dmax;
  st->bins_stale = true;   // binned before the first whole-graph walk
  st->S.alpha = st->alpha;
  set_gamma(st->S, (int)h.dmax);
  if (st->fp32) fp32_tables(st->S, scale_cap(st), st->max_iter, bb);
  KATZ_TRY(alloc_run_buffers(st, s));
  // The flag initialisation runs on s; the copies below must follow it.
  KATZ_HIP(hipStreamSynchronize(s));
  KATZ_TRY(ensure_levels(st, st->r));
  const size_t xs = st->fp32 ? sizeof(float) : sizeof(double);
  for (long long i = 1; i <= st->r; ++i) KATZ_TRY(read_dev(file.f, static_cast<char*>(st->X[i]), xs * n));
  KATZ_TRY(read_dev(file.f, st->w.c, n));
  KATZ_TRY(read_dev(file.f, st->w.act[st->cur], (size_t)h.m));
  KATZ_TRY(read_dev(file.f, st->w.xmax64, (size_t)st->max_iter + 1));
  if (st->fp32) {
    KATZ_TRY(read_dev(file.f, st->w.e, n));
    KATZ_TRY(read_dev(file.f, st->w.sigma, (size_t)st->max_iter + 1));
    KATZ_TRY(read_dev(file.f, st->w.sigma_sum, (size_t)st->max_iter + 1));
    KATZ_TRY(read_dev(file.f, st->w.xmax32, (size_t)st->max_iter + 1));
  }
  KATZ_HIP(hipStreamSynchronize(s));   // alloc_run_buffers initialised the flags on s
  KATZ_HIP(hipMemcpy(st->w.sc, &sc, sizeof(RunScalars), hipMemcpyHostToDevice));
  *st->hs.sc = sc;
  guard.keep = true;
  *stp = st;
  return KATZ_OK;
}

int update_state(katz_state* st, const int32_t* ins_u, const int32_t* ins_v, long long n_ins, const int32_t* del_u,
                 const int32_t* del_v, long long n_del, katz_result* out, hipStream_t s) {
  if (!out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  PreparedBatch pb;
  KATZ_TRY(prepare_batch(st->n, state_pair_mode(st), ins_u, ins_v, n_ins, del_u, del_v, n_del, pb));
  return apply_batch(st, pb, out, s);
}

}  // namespace katz

// ---------------------------------------------------------------------------
// Allocation-free ranking: the workspace is a static device array of fixed
// size (each device that loads the library holds its own copy until the
// process ends), and the flag read-backs go to static host memory.
// ---------------------------------------------------------------------------
namespace katz {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// Device-side only: host code reaches it through the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
  std::once_flag once;
  int rc = KATZ_E_HIP;
  unsigned char* ptr = nullptr;   // device address of `scratch` on this device
  RunScalars sc;                  // static host mirrors of the flags
  RunScalars ring[2];
  unsigned long long bits[8];
};
ScratchSlot g_scratch[kMaxDevices];

// Set-up, once per device with that device current: look up the address of
// the device's copy of the scratch array.
ScratchSlot* scratch_slot(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  ScratchSlot& sl = g_scratch[dev];
  std::call_once(sl.once, [&sl] {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) {
      sl.ptr = static_cast<unsigned char*>(p);
      sl.rc = KATZ_OK;
    } else {
      (void)hipGetLastError();
    }
  });
  return sl.rc == KATZ_OK ? &sl : nullptr;
}

int rank_noalloc(const katz_csr* g, const katz_params* p, katz_result* out, hipStream_t s) {
  KATZ_TRY(check_rank_args(g, p, out));
  if (wants_reverse(g, p)) return KATZ_E_UNSUPPORTED;   // the reverse graph needs its own workspace
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ScratchSlot* sl = scratch_slot(dev);
  if (!sl) return KATZ_E_HIP;
  Arena ar;
  ar.device = dev;
  ar.base = reinterpret_cast<char*>(sl->ptr);
  ar.cap = kScratchBytes;
  ar.fixed = true;
  ar.hs.borrowed = true;
  ar.hs.sc = &sl->sc;
  ar.hs.ring = sl->ring;
  ar.hs.bits = sl->bits;
  return rank_in_arena(ar, g, p, out, s, false);
}

}  // namespace
}  // namespace katz

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
KATZ_EXPORT int katz_rank_static_noalloc(const katz_csr* g, const katz_params* p, katz_result* out, void* stream) {
  return katz::rank_noalloc(g, p, out, (hipStream_t)stream);
}

KATZ_EXPORT int katz_rank_static(int32_t count, const katz_csr* g, const katz_params* p, katz_result* out,
                                 katz_state** states, void* stream) {
  if (count < 1 || !g || !p || !out) return KATZ_E_INVALID_ARG;
  for (int32_t i = 0; i < count; ++i) {
    int rc = katz::check_graph(&g[i]);
    if (!rc) rc = katz::check_params(&p[i], g[i].n, true);
    if (!rc && (!out[i].topk_ids || !out[i].lower || !out[i].upper)) rc = KATZ_E_INVALID_ARG;
    if (!rc && (states || count > 1)) rc = katz::check_lds_criterion(&p[i]);
    if (rc) return rc;
  }
  if (count > 1 && !states) {
    bool any_inbound = false;
    for (int32_t i = 0; i < count; ++i) any_inbound = any_inbound || katz::wants_reverse(&g[i], &p[i]);
    if (!any_inbound) return katz::rank_batch(count, g, p, out, (hipStream_t)stream);
    // Inbound graphs of the batch are ranked on their reverse graphs, built in
    // one workspace held for the call.
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KATZ_E_HIP;
    katz::ArenaLease rl(dev, (hipStream_t)stream);
    if (rl.rc < 0) return rl.rc;
    std::vector<katz_csr> g2;
    std::vector<katz_params> p2;
    const int rc = katz::reverse_graphs(*rl.a, count, g, p, g2, p2, (hipStream_t)stream);
    if (rc < 0) return rc;
    return katz::rank_batch(count, g2.data(), p2.data(), out, (hipStream_t)stream);
  }
  int worst = KATZ_OK;
  for (int32_t i = 0; i < count; ++i) {
    int rc;
    if (states) {
      states[i] = nullptr;
      rc = katz::create_state(&g[i], &p[i], &out[i], &states[i], (hipStream_t)stream);
      if (rc < 0) {
        for (int32_t j = 0; j < i; ++j) {
          delete states[j];
          states[j] = nullptr;
        }
      }
    } else {
      rc = katz::rank_one(&g[i], &p[i], &out[i], (hipStream_t)stream);
    }
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
  }
  return worst;
}

KATZ_EXPORT int katz_rank_update(katz_state* st, const int32_t* ins_u, const int32_t* ins_v, int64_t n_ins,
                                 const int32_t* del_u, const int32_t* del_v, int64_t n_del, katz_result* out,
                                 void* stream) {
  if (!st) return KATZ_E_INVALID_ARG;
  return katz::update_state(st, ins_u, ins_v, n_ins, del_u, del_v, n_del, out, (hipStream_t)stream);
}

KATZ_EXPORT int katz_bounds(const katz_csr* g, const katz_params* p, int32_t r, double* lower, double* upper,
                            void* stream) {
  return katz::bounds_one(g, p, r, lower, upper, (hipStream_t)stream);
}

KATZ_EXPORT int katz_solve(const katz_csr* g, const katz_params* p, int32_t method, double tol, double* scores,
                           katz_solve_info* info, void* stream) {
  return katz::solve_one(g, p, method, tol, scores, info, (hipStream_t)stream);
}

KATZ_EXPORT void katz_state_free(katz_state* st) { delete st; }

KATZ_EXPORT int katz_state_save(katz_state* st, const char* path) { return katz::save_state(st, path); }

KATZ_EXPORT int katz_state_load(const char* path, katz_state** out, void* stream) {
  if (out) *out = nullptr;
  return katz::load_state(path, out, (hipStream_t)stream);
}

KATZ_EXPORT int katz_state_size(const katz_state* st, int64_t* n, int32_t* k) {
  if (!st) return KATZ_E_INVALID_ARG;
  if (n) *n = st->n;
  if (k) *k = st->k;
  return KATZ_OK;
}

KATZ_EXPORT void katz_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(katz::g_timing.mu);
  katz::g_timing.on = on != 0;
  katz::g_timing.acc = katz_timing{};
}

KATZ_EXPORT int katz_timing_read(katz_timing* out) {
  if (!out) return KATZ_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(katz::g_timing.mu);
  *out = katz::g_timing.acc;
  return KATZ_OK;
}

KATZ_EXPORT int katz_tuning_get(katz_tuning* t) {
  if (!t) return KATZ_E_INVALID_ARG;
  *t = katz::current_tuning();
  return KATZ_OK;
}

KATZ_EXPORT int katz_tuning_set(const katz_tuning* t) {
  if (!t) return KATZ_E_INVALID_ARG;
  KATZ_TRY(katz::tuning_valid(*t));
  std::lock_guard<std::mutex> lk(katz::g_tuning.mu);
  katz::g_tuning.t = *t;
  return KATZ_OK;
}

// ---------------------------------------------------------------------------
// Autotuner cache: one text line per tuned workload, "<key>\t<13 integers>"
// (the katz_tuning fields in declaration order, reserved left out).  The key
// names the device (architecture and compute units) and the workload (graph
// count, total nodes and arcs, precision, criterion, flags).  The last valid
// line of a key wins; lines that do not parse or hold an invalid setting are
// skipped.
// ---------------------------------------------------------------------------
namespace katz {
namespace {

struct TuneCache {
  std::mutex mu;
  std::string path;
} g_tune_cache;

std::string tune_key(int32_t count, const katz_csr* g, const katz_params* p) {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return std::string();
  }
  long long n = 0, nnz = 0;
  for (int32_t i = 0; i < count; ++i) {
    n += g[i].n;
    nnz += g[i].nnz;
  }
  char buf[320];
  std::snprintf(buf, sizeof(buf), "%s/%d/count=%d/n=%lld/nnz=%lld/prec=%d/crit=%d/flags=%d/und=%d",
                prop.gcnArchName, prop.multiProcessorCount, (int)count, n, nnz, (int)p[0].precision,
                (int)p[0].criterion, (int)p[0].flags, (int)g[0].undirected);
  for (char* c = buf; *c; ++c)
    if (*c == '\t' || *c == '\n') *c = ' ';
  return std::string(buf);
}

bool cache_lookup(const std::string& path, const std::string& key, katz_tuning& out) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  bool found = false;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    char* tab = std::strchr(line, '\t');
    if (!tab || (size_t)(tab - line) != key.size() || std::strncmp(line, key.c_str(), key.size()) != 0) continue;
    katz_tuning t{};
    int32_t* v[13] = {&t.hub_bytes, &t.blocks_per_cu, &t.batch_blocks_per_cu, &t.batch_tile, &t.batch_xcd,
                      &t.walk_groups, &t.split_hot_bytes, &t.bin_bounds[0], &t.bin_bounds[1], &t.bin_bounds[2],
                      &t.bin_bounds[3], &t.bin_bounds[4], &t.bin_bounds[5]};
    char* s = tab + 1;
    bool ok = true;
    for (int i = 0; i < 13 && ok; ++i) {
      char* e = nullptr;
      const long x = std::strtol(s, &e, 10);
      ok = e != s && x >= INT32_MIN && x <= INT32_MAX;
      *v[i] = (int32_t)x;
      s = e;
    }
    while (ok && (*s == ' ' || *s == '\r' || *s == '\n')) ++s;
    if (ok && *s == '\0' && tuning_valid(t) == KATZ_OK) {
      out = t;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& path, const std::string& key, const katz_tuning& t) {
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s\t%d %d %d %d %d %d %d %d %d %d %d %d %d\n", key.c_str(), t.hub_bytes, t.blocks_per_cu,
               t.batch_blocks_per_cu, t.batch_tile, t.batch_xcd, t.walk_groups, t.split_hot_bytes, t.bin_bounds[0],
               t.bin_bounds[1], t.bin_bounds[2], t.bin_bounds[3], t.bin_bounds[4], t.bin_bounds[5]);
  std::fclose(f);
}

}  // namespace
}  // namespace katz

KATZ_EXPORT int katz_autotune_cache(const char* path) {
  std::lock_guard<std::mutex> lk(katz::g_tune_cache.mu);
  katz::g_tune_cache.path = path ? path : "";
  return KATZ_OK;
}

// Candidate launch shapes, timed on the caller's graph(s); the fastest is kept.
KATZ_EXPORT int katz_autotune(int32_t count, const katz_csr* g, const katz_params* p, katz_tuning* best,
                              void* stream) {
  if (count < 1 || !g || !p) return KATZ_E_INVALID_ARG;
  long long sum_k = 0;
  for (int32_t i = 0; i < count; ++i) {
    KATZ_TRY(katz::check_graph(&g[i]));
    KATZ_TRY(katz::check_params(&p[i], g[i].n, true));
    sum_k += katz::output_len(&p[i], g[i].n);
  }
  std::string cache_path, cache_key;
  {
    std::lock_guard<std::mutex> lk(katz::g_tune_cache.mu);
    cache_path = katz::g_tune_cache.path;
  }
  if (!cache_path.empty()) {
    cache_key = katz::tune_key(count, g, p);
    katz_tuning hit{};
    if (!cache_key.empty() && katz::cache_lookup(cache_path, cache_key, hit)) {
      std::lock_guard<std::mutex> lk(katz::g_tuning.mu);
      katz::g_tuning.t = hit;
      if (best) *best = hit;
      return KATZ_OK;
    }
  }
  // {hub_bytes, blocks_per_cu, walk_groups}: hub copies sized so that 3..8
  // workgroups fill the 160 KiB of LDS of a CU (with the kernel's own few bytes
  // of static LDS), and one 1024-thread workgroup with a copy of 64..156 KiB.
  static const int kSingle[][3] = {{0, 0, 0},      {0, 4, 0},      {0, 8, 0},       {0, 16, 0},      {16384, 4, 0},
                                   {20416, 8, 0},  {24512, 6, 0},  {32704, 5, 0},   {32768, 4, 0},   {40896, 4, 0},
                                   {54208, 3, 0},  {65536, 2, 0},  {65536, 1, 4},   {98304, 1, 4},   {131072, 1, 4},
                                   {159744, 1, 4}};
  static const int kBatch[][3] = {{0, 1, 0}, {4, 1, 0},  {16, 1, 0}, {4, 2, 0}, {16, 2, 0}, {4, 4, 0}, {16, 4, 0},
                                  {16, 8, 0}, {0, 1, 1},  {16, 1, 1}, {4, 4, 1}, {16, 4, 1}, {16, 8, 1}};
  const katz_tuning saved = katz::current_tuning();
  int32_t* ids = nullptr;
  double *lo = nullptr, *up = nullptr;
  if (hipMalloc((void**)&ids, sizeof(int32_t) * sum_k) != hipSuccess ||
      hipMalloc((void**)&lo, sizeof(double) * sum_k) != hipSuccess ||
      hipMalloc((void**)&up, sizeof(double) * sum_k) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(ids);
    (void)hipFree(lo);
    (void)hipFree(up);
    return KATZ_E_OOM;
  }
  std::vector<katz_tuning> cand;
  if (count == 1) {
    for (const auto& c : kSingle) {
      katz_tuning t = saved;
      t.hub_bytes = c[0];
      t.blocks_per_cu = c[1];
      t.walk_groups = c[2];
      cand.push_back(t);
    }
  } else {
    for (const auto& c : kBatch) {
      katz_tuning t = saved;
      t.batch_blocks_per_cu = c[0];
      t.batch_tile = c[1];
      t.batch_xcd = c[2];
      cand.push_back(t);
    }
  }
  std::vector<katz_result> out(count);
  long long koff = 0;
  for (int32_t i = 0; i < count; ++i) {
    out[i] = katz_result{};
    out[i].topk_ids = ids + koff;
    out[i].lower = lo + koff;
    out[i].upper = up + koff;
    koff += katz::output_len(&p[i], g[i].n);
  }
  katz_tuning pick = saved;
  double pick_ms = 1e300;
  int rc = KATZ_OK;
  auto trial = [&](const katz_tuning& t) {
    {
      std::lock_guard<std::mutex> lk(katz::g_tuning.mu);
      katz::g_tuning.t = t;
    }
    double ms = 0.0;
    for (int rep = 0; rep < 2 && rc >= 0; ++rep) {
      const auto t0 = std::chrono::steady_clock::now();
      rc = katz_rank_static(count, g, p, out.data(), nullptr, stream);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc >= 0 && ms < pick_ms) {
      pick_ms = ms;
      pick = t;
    }
  };
  // Stage 1: launch shapes with the caller's row-length classes.
  for (const katz_tuning& t : cand) {
    trial(t);
    if (rc < 0) break;
  }
  // Stage 2: row-length classes (bin_bounds) with the chosen shape: the
  // defaults, fewer lanes per row (longer classes), more lanes per row.
  static const int kBins[][6] = {{0, 0, 0, 0, 0, 0},
                                 {4, 8, 16, 64, 256, 2048},
                                 {2, 4, 8, 16, 64, 512},
                                 {4, 8, 24, 48, 192, 1536}};
  const katz_tuning shape = pick;
  for (int i = 0; i < (int)(sizeof(kBins) / sizeof(kBins[0])) && rc >= 0; ++i) {
    katz_tuning t = shape;
    for (int j = 0; j < 6; ++j) t.bin_bounds[j] = kBins[i][j];
    if (std::equal(t.bin_bounds, t.bin_bounds + 6, shape.bin_bounds)) continue;   // timed in stage 1
    trial(t);
  }
  (void)hipFree(ids);
  (void)hipFree(lo);
  (void)hipFree(up);
  if (rc >= 0 && !cache_key.empty()) katz::cache_store(cache_path, cache_key, pick);
  std::lock_guard<std::mutex> lk(katz::g_tuning.mu);
  katz::g_tuning.t = rc < 0 ? saved : pick;
  if (best) *best = katz::g_tuning.t;
  return rc < 0 ? rc : KATZ_OK;
}

KATZ_EXPORT const char* katz_strerror(int code) {
  switch (code) {
    case KATZ_OK: return "ok: ranking certified";
    case KATZ_W_ITER_LIMIT: return "warning: iteration limit reached before certification";
    case KATZ_W_PRECISION_LIMIT: return "warning: FP32 rounding margin stops further separation";
    case KATZ_W_EXACT_TIES: return "warning: walks died out; remaining pairs are exact ties";
    case KATZ_E_INVALID_ARG: return "error: invalid argument";
    case KATZ_E_ALPHA: return "error: alpha must satisfy 0 < alpha < 1/deg_max";
    case KATZ_E_CSR: return "error: malformed CSR graph";
    case KATZ_E_UPDATE: return "error: invalid edge-update batch";
    case KATZ_E_DEGREE_CAP: return "error: update exceeds the degree cap";
    case KATZ_E_OOM: return "error: device memory allocation failed";
    case KATZ_E_HIP: return "error: HIP runtime failure";
    case KATZ_E_UNSUPPORTED: return "error: unsupported request";
    case KATZ_E_SCRATCH: return "error: the problem needs more workspace than the fixed scratch array holds";
    case KATZ_E_CANCELLED: return "error: the request was cancelled before it ran";
    case KATZ_E_TIMEOUT: return "error: the request did not finish within the time limit";
    case KATZ_E_BUSY: return "error: the request is already on the device or finished";
    default: return "unknown status code";
  }
}
