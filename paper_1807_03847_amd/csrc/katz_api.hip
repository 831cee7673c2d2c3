// Host runtime of the C ABI declared in include/katz.h.
//
// A call validates its arguments on the host, stages host inputs to the
// device, bins the rows (prep), then enqueues iterations of Algorithm 1
// (walk step + selection + converged()) and reads the device stop flag.
// Workspace comes from a per-device pool of grow-only arenas, so repeated calls
// on graphs of similar size do not call hipMalloc.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "katz_internal.h"

#define KATZ_EXPORT extern "C" __attribute__((visibility("default")))

namespace katz {

namespace {

constexpr double kU64 = 0x1p-53;   // unit roundoff of FP64
constexpr double kU32 = 0x1p-24;   // unit roundoff of FP32

// ---------------------------------------------------------------------------
// Workspace arenas.
// ---------------------------------------------------------------------------
struct Arena {
  int device = -1;
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool measuring = false;
  RunScalars* host_sc = nullptr;          // pinned
  unsigned long long* host_bits = nullptr;  // pinned, 8 words

  ~Arena() {
    if (base) (void)hipFree(base);
    if (host_sc) (void)hipHostFree(host_sc);
    if (host_bits) (void)hipHostFree(host_bits);
  }
  template <class T>
  T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = measuring ? nullptr : reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
  int grow(size_t bytes) {
    if (!host_sc) {
      if (hipHostMalloc((void**)&host_sc, sizeof(RunScalars)) != hipSuccess) return KATZ_E_OOM;
      if (hipHostMalloc((void**)&host_bits, 8 * sizeof(unsigned long long)) != hipSuccess) return KATZ_E_OOM;
    }
    if (bytes <= cap) return KATZ_OK;
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

struct ArenaLease {
  Arena* a;
  explicit ArenaLease(int dev) : a(acquire_arena(dev)) {}
  ~ArenaLease() { release_arena(a); }
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
enum TimedKind { T_PREP = 0, T_FIRST, T_STEP, T_SELECT, T_RESULT, T_KINDS };

struct TimingState {
  std::mutex mu;
  bool on = false;
  katz_timing acc{};
};
TimingState g_timing;

struct CallTimer {
  bool on = false;
  std::vector<int> kind;
  std::vector<hipEvent_t> ev;   // start, stop pairs
  hipEvent_t call0 = nullptr, call1 = nullptr;

  CallTimer() {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    on = g_timing.on;
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
    t.select_ms += sum[T_SELECT];
    t.select_iterations += cnt[T_SELECT];
    t.result_ms += sum[T_RESULT];
    t.call_ms += call_ms;
    t.calls += 1;
  }
};

#define KATZ_HIP(call)                    \
  do {                                    \
    if ((call) != hipSuccess) {           \
      (void)hipGetLastError();            \
      return KATZ_E_HIP;                  \
    }                                     \
  } while (0)

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
  if (p->validate < 0 || p->validate > 2 || p->reserved != 0 || p->max_iter < 0) return KATZ_E_INVALID_ARG;
  if (std::isnan(p->alpha) || p->alpha < 0.0 || std::isinf(p->alpha)) return KATZ_E_ALPHA;
  if (need_k) {
    if (p->criterion != KATZ_TOPK) return KATZ_E_UNSUPPORTED;
    if (p->k < 1 || p->k > n) return KATZ_E_INVALID_ARG;
    if (!(p->epsilon >= 0.0) || std::isinf(p->epsilon)) return KATZ_E_INVALID_ARG;
    if (p->k > kMaxK) return KATZ_E_UNSUPPORTED;
  }
  return KATZ_OK;
}

// ---------------------------------------------------------------------------
// One prepared graph on the device.
// ---------------------------------------------------------------------------
struct Prepared {
  const void* row_ptr = nullptr;
  const int32_t* col = nullptr;
  RowDesc* desc = nullptr;
  SegDesc* segs = nullptr;
  HugeRow* huge = nullptr;
  long long* blk = nullptr;
  long long* row_off = nullptr;
  int* row_len = nullptr;
  int* seg_done = nullptr;
  RunScalars* sc = nullptr;
  int nblocks = 0;
  long long seg_cap = 0, huge_cap = 0;
  // read back after prep
  long long bin_count[NUM_BINS] = {};
  long long bin_base[NUM_BINS] = {};
  long long seg_total = 0;
  int dmax = 0;
};

struct RunBuffers {
  void* x[2] = {nullptr, nullptr};
  double* c = nullptr;
  float* e = nullptr;
  void* partial = nullptr;
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
  int32_t* out_ids = nullptr;
  double* out_lo = nullptr;
  double* out_up = nullptr;
};

// Lays out every buffer of one call in the arena (measure pass, then real pass).
struct Plan {
  const katz_csr* g;
  int fp32;
  int k;
  int max_iter;
  int validate;
  bool rp_host, col_host, out_host, select;
  size_t out_n;   // elements per output array (k for ranking, n for bounds)
};

void layout(Arena& ar, const Plan& pl, Prepared& pr, RunBuffers& rb) {
  const long long n = pl.g->n, nnz = pl.g->nnz;
  ar.used = 0;
  pr.nblocks = (int)((n + kWG - 1) / kWG);
  pr.seg_cap = 2 * (nnz / kSeg) + 2;
  pr.huge_cap = nnz / (kBlockRowMax + 1) + 1;
  pr.sc = ar.take<RunScalars>(1);
  pr.blk = ar.take<long long>((size_t)(NUM_BINS + 1) * pr.nblocks);
  pr.desc = ar.take<RowDesc>(n);
  pr.segs = ar.take<SegDesc>(pr.seg_cap);
  pr.huge = ar.take<HugeRow>(pr.huge_cap);
  pr.seg_done = ar.take<int>(pr.huge_cap);
  if (pl.rp_host) pr.row_ptr = ar.take<char>((size_t)(n + 1) * (pl.g->row_ptr_64 ? 8 : 4));
  if (pl.col_host) pr.col = ar.take<int32_t>(std::max<long long>(nnz, 1));
  if (pl.validate == KATZ_VALIDATE_STRICT && pl.g->undirected) {
    pr.row_off = ar.take<long long>(n);
    pr.row_len = ar.take<int>(n);
  }
  const size_t xs = pl.fp32 ? 4 : 8;
  rb.x[0] = ar.take<char>(n * xs);
  rb.x[1] = ar.take<char>(n * xs);
  rb.c = ar.take<double>(n);
  if (pl.fp32) rb.e = ar.take<float>(n);
  rb.partial = ar.take<char>(pr.seg_cap * xs);
  rb.xmax32 = ar.take<unsigned>(pl.max_iter + 1);
  rb.xmax64 = ar.take<unsigned long long>(pl.max_iter + 1);
  rb.sigma = ar.take<double>(pl.max_iter + 1);
  rb.sigma_sum = ar.take<double>(pl.max_iter + 1);
  rb.hist = ar.take<unsigned>(2 * kDigits);
  if (pl.select) {
    rb.act[0] = ar.take<int32_t>(n);
    rb.act[1] = ar.take<int32_t>(n);
    rb.keys = ar.take<unsigned long long>(n);
    rb.cand_key[0] = ar.take<unsigned long long>(n);
    rb.cand_key[1] = ar.take<unsigned long long>(n);
    rb.cand_v[0] = ar.take<int32_t>(n);
    rb.cand_v[1] = ar.take<int32_t>(n);
    rb.top_sorted = ar.take<int32_t>(pl.k);
    rb.top_lo = ar.take<double>(pl.k);
    rb.top_up = ar.take<double>(pl.k);
    rb.mark = ar.take<uint8_t>(n);
    rb.rest_bits = ar.take<unsigned long long>(1);
  }
  if (pl.out_host) {
    rb.out_ids = ar.take<int32_t>(pl.out_n);
    rb.out_lo = ar.take<double>(pl.out_n);
    rb.out_up = ar.take<double>(pl.out_n);
  }
}

int plan_and_allocate(Arena& ar, const Plan& pl, Prepared& pr, RunBuffers& rb) {
  ar.measuring = true;
  layout(ar, pl, pr, rb);
  ar.measuring = false;
  const int rc = ar.grow(ar.used);
  if (rc) return rc;
  layout(ar, pl, pr, rb);
  return KATZ_OK;
}

// Stages host inputs, bins the rows, reads back d_max and the bin sizes.
int prepare(Arena& ar, const Plan& pl, Prepared& pr, int max_iter, RunBuffers& rb, hipStream_t s) {
  const katz_csr* g = pl.g;
  if (pl.rp_host) {
    KATZ_HIP(hipMemcpyAsync((void*)pr.row_ptr, g->row_ptr, (size_t)(g->n + 1) * (g->row_ptr_64 ? 8 : 4),
                            hipMemcpyHostToDevice, s));
  } else {
    pr.row_ptr = g->row_ptr;
  }
  if (pl.col_host) {
    if (g->nnz > 0)
      KATZ_HIP(hipMemcpyAsync((void*)pr.col, g->col, (size_t)g->nnz * 4, hipMemcpyHostToDevice, s));
  } else {
    pr.col = g->col;
  }
  KATZ_HIP(launch_init_run(pr.sc, g->n, rb.sigma, rb.sigma_sum, rb.xmax32, rb.xmax64, max_iter, rb.hist, s));
  KATZ_HIP(hipMemsetAsync(pr.seg_done, 0, sizeof(int) * pr.huge_cap, s));
  KATZ_HIP(launch_prep_count(pr.row_ptr, g->row_ptr_64, g->n, g->nnz, pr.blk, pr.nblocks, pr.sc, s));
  KATZ_HIP(launch_prep_scan(pr.blk, pr.nblocks, pr.sc, s));
  KATZ_HIP(launch_prep_scatter(pr.row_ptr, g->row_ptr_64, g->n, pr.blk, pr.nblocks, pr.desc, pr.segs, pr.huge,
                               pr.sc, s));
  KATZ_HIP(hipMemcpyAsync(ar.host_sc, pr.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (ar.host_sc->err) return KATZ_E_CSR;
  std::memcpy(pr.bin_count, ar.host_sc->bin_count, sizeof(pr.bin_count));
  std::memcpy(pr.bin_base, ar.host_sc->bin_base, sizeof(pr.bin_base));
  pr.seg_total = ar.host_sc->seg_total;
  pr.dmax = ar.host_sc->dmax;
  if (pl.validate == KATZ_VALIDATE_STRICT) {
    KATZ_HIP(launch_validate_strict(pr.desc, g->n, pr.col, g->undirected, pr.row_off, pr.row_len, pr.sc, s));
    KATZ_HIP(hipMemcpyAsync(ar.host_sc, pr.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipStreamSynchronize(s));
    if (ar.host_sc->err) return KATZ_E_CSR;
  }
  return KATZ_OK;
}

// Deepest rounding chain of any row sum under the bin schedule: serial adds per
// lane, then the butterfly levels (and the segment combine for huge rows).
int max_reduction_depth(const Prepared& pr) {
  int m = 0;
  auto upd = [&](int bin, int d) {
    if (pr.bin_count[bin] > 0) m = std::max(m, d);
  };
  upd(BIN_G4, 2);
  upd(BIN_G8, 3);
  upd(BIN_G16, 4);
  upd(BIN_G32, 5);
  upd(BIN_W64, (kPerLane - 1) + 6);
  upd(BIN_B256, (kPerLane - 1) + 8);
  if (pr.bin_count[BIN_HUGE] > 0) {
    const long long max_seg = (pr.dmax + kSeg - 1) / kSeg;
    const long long q = (max_seg + kWave - 1) / kWave;
    m = std::max<long long>(m, (kPerLane - 1) + 8 + (q - 1) + 6);
  }
  return m;
}

struct Scalars {
  double alpha, gamma, beta, beta_hi;
  double rho;
  std::vector<double> eta, etap;   // [max_iter + 1]
  double tau_coef0;
};

// FP32 form: eta_r bounds the relative error of every entry of x~_r; eta_1 = 0
// because the first walk step sums exact ones; later steps multiply by (1 + rho),
// rho = gamma_m = m u / (1 - m u) for the deepest reduction chain m.
void fp32_tables(Scalars& S, const Prepared& pr, int max_iter) {
  const int m = max_reduction_depth(pr);
  S.rho = (m * kU32) / (1.0 - m * kU32) * (1.0 + 0x1p-40);
  S.eta.assign(max_iter + 1, 0.0);
  S.etap.assign(max_iter + 1, 0.0);
  const double up = 1.0 + 0x1p-50;
  S.eta[1] = pr.dmax < (1 << 24) ? 0.0 : kU32;
  for (int r = 2; r <= max_iter; ++r) S.eta[r] = ((1.0 + S.eta[r - 1]) * (1.0 + S.rho) - 1.0) * up;
  for (int r = 1; r <= max_iter; ++r) S.etap[r] = S.eta[r] / (1.0 - S.eta[r]) * up;
}

BoundArgs bound_args(const Plan& pl, const Prepared& pr, const RunBuffers& rb, const Scalars& S, int r,
                     double eps, int undirected) {
  BoundArgs b{};
  b.c = rb.c;
  b.x = rb.x[r & 1];
  b.e = rb.e;
  b.sigma = rb.sigma;
  b.sigma_sum = rb.sigma_sum;
  b.r = r;
  b.fp32 = pl.fp32;
  b.undirected = undirected;
  b.alpha = S.alpha;
  b.eps = eps;
  if (!pl.fp32) {
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
    b.f_lo_s = undirected ? S.alpha * (1.0 - ep) * (1.0 - kap) * (1.0 - 8.0 * kU64) : 0.0;
    b.f_hi_s = S.beta_hi * (1.0 + ep) * (1.0 + kap) * (1.0 + 8.0 * kU64);
    // Underflow of x~ entries: at most (deg_max + 1) 2^-126 per entry and level
    // in units of sigma_i, carried through c (r levels) and the bounds (beta).
    b.tau_coef = 4.0 * (r + S.beta_hi + 2.0) * (pr.dmax + 2.0) * 0x1p-126;
  }
  return b;
}

void fill_blocks(IterArgs& ia, const Prepared& pr, bool write_empty, long long& total) {
  long long blocks[NUM_BINS] = {};
  blocks[BIN_HUGE] = pr.seg_total;
  blocks[BIN_B256] = pr.bin_count[BIN_B256];
  blocks[BIN_W64] = (pr.bin_count[BIN_W64] + 3) / 4;
  blocks[BIN_G32] = (pr.bin_count[BIN_G32] + 7) / 8;
  blocks[BIN_G16] = (pr.bin_count[BIN_G16] + 15) / 16;
  blocks[BIN_G8] = (pr.bin_count[BIN_G8] + 31) / 32;
  blocks[BIN_G4] = (pr.bin_count[BIN_G4] + 63) / 64;
  blocks[BIN_EMPTY] = write_empty ? (pr.bin_count[BIN_EMPTY] + kWG - 1) / kWG : 0;
  ia.first_block[0] = 0;
  for (int b = 0; b < NUM_BINS; ++b) ia.first_block[b + 1] = ia.first_block[b] + blocks[b];
  total = ia.first_block[NUM_BINS];
}

IterArgs iter_args(const Plan& pl, const Prepared& pr, const RunBuffers& rb, const Scalars& S, int r,
                   long long& total_blocks) {
  IterArgs ia{};
  ia.desc = pr.desc;
  ia.col = pr.col;
  ia.segs = pr.segs;
  ia.huge = pr.huge;
  for (int b = 0; b < NUM_BINS; ++b) {
    ia.bin_base[b] = pr.bin_base[b];
    ia.bin_count[b] = pr.bin_count[b];
  }
  fill_blocks(ia, pr, r == 2, total_blocks);
  ia.x_in = rb.x[(r + 1) & 1];
  ia.x_out = rb.x[r & 1];
  ia.c = rb.c;
  ia.e = rb.e;
  ia.partial = rb.partial;
  ia.seg_done = pr.seg_done;
  ia.xmax32 = rb.xmax32;
  ia.xmax64 = rb.xmax64;
  ia.sigma = rb.sigma;
  ia.sigma_sum = rb.sigma_sum;
  ia.sc = pr.sc;
  ia.n = (int)pl.g->n;
  ia.r = r;
  ia.validate_cols = (r == 1 && pl.validate >= KATZ_VALIDATE_BASIC) ? 1 : 0;
  ia.write_empty = r == 2;
  ia.clog2_dmax = clog2(std::max(pr.dmax, 1));
  ia.alpha = S.alpha;
  ia.etap = pl.fp32 ? S.etap[r] : 0.0;
  return ia;
}

int resolve_alpha(const katz_params* p, int dmax, Scalars& S) {
  const double alpha = p->alpha == 0.0 ? 1.0 / (1.0 + (double)dmax) : p->alpha;
  if (!(alpha > 0.0) || !(alpha * (double)dmax < 1.0)) return KATZ_E_ALPHA;
  S.alpha = alpha;
  // gamma and beta exactly as the plain FP64 method evaluates them (Theorem 1).
  S.gamma = (double)dmax / (1.0 - alpha * (double)dmax);
  S.beta = alpha * S.gamma;
  // Upward-rounded beta for the FP32 form: 1 - alpha d with one rounding (fma),
  // each of the three operations at most one ulp, then 8 ulps of slack.
  const double den = std::fma(-alpha, (double)dmax, 1.0);
  S.beta_hi = alpha * ((double)dmax / den) * (1.0 + 8.0 * kU64);
  return KATZ_OK;
}

int sync_every_default() { return 1; }

// ---------------------------------------------------------------------------
// Static ranking of one graph.
// ---------------------------------------------------------------------------
int rank_one(const katz_csr* g, const katz_params* p, katz_result* out, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  rc = check_params(p, g->n, true);
  if (rc) return rc;
  if (!out || !out->topk_ids || !out->lower || !out->upper) return KATZ_E_INVALID_ARG;
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ArenaLease lease(dev);
  Arena& ar = *lease.a;

  Plan pl{};
  pl.g = g;
  pl.fp32 = p->precision == KATZ_FP32_MARGIN;
  pl.k = p->k;
  pl.max_iter = p->max_iter ? p->max_iter : 1000;
  pl.validate = p->validate;
  pl.rp_host = !is_device_ptr(g->row_ptr);
  pl.col_host = g->nnz > 0 && !is_device_ptr(g->col);
  const bool ids_dev = is_device_ptr(out->topk_ids), lo_dev = is_device_ptr(out->lower),
             up_dev = is_device_ptr(out->upper);
  pl.out_host = !(ids_dev && lo_dev && up_dev);
  pl.select = true;
  pl.out_n = (size_t)p->k;

  Prepared pr;
  RunBuffers rb;
  rc = plan_and_allocate(ar, pl, pr, rb);
  if (rc) return rc;
  CallTimer T;
  T.call_begin(s);
  const int tp = T.start(T_PREP, s);
  rc = prepare(ar, pl, pr, pl.max_iter, rb, s);
  T.stop(tp, s);
  if (rc) return rc;

  Scalars S{};
  rc = resolve_alpha(p, pr.dmax, S);
  if (rc) return rc;
  if (pl.fp32) fp32_tables(S, pr, pl.max_iter);

  const long long n = g->n;
  const int grid = (int)std::min<long long>((n + kWG - 1) / kWG, 2048);
  const int sync_every = sync_every_default();
  int r = 0;
  for (r = 1; r <= pl.max_iter; ++r) {
    long long total_blocks = 0;
    const IterArgs ia = iter_args(pl, pr, rb, S, r, total_blocks);
    const int tw = T.start(r == 1 ? T_FIRST : T_STEP, s);
    if (r == 1) KATZ_HIP(launch_walk_first(ia, pl.fp32, n, g->nnz, pl.validate >= KATZ_VALIDATE_BASIC, s));
    else KATZ_HIP(launch_walk_step(ia, pl.fp32, total_blocks, s));
    T.stop(tw, s);
    SelArgs sa{};
    sa.b = bound_args(pl, pr, rb, S, r, p->epsilon, g->undirected);
    sa.act_in = rb.act[(r + 1) & 1];
    sa.act_out = rb.act[r & 1];
    sa.keys = rb.keys;
    sa.cand_key[0] = rb.cand_key[0];
    sa.cand_key[1] = rb.cand_key[1];
    sa.cand_v[0] = rb.cand_v[0];
    sa.cand_v[1] = rb.cand_v[1];
    sa.hist = rb.hist;
    sa.top_sorted = rb.top_sorted;
    sa.top_lo = rb.top_lo;
    sa.top_up = rb.top_up;
    sa.xmax32 = rb.xmax32;
    sa.xmax64 = rb.xmax64;
    sa.sc = pr.sc;
    sa.identity_in = r == 1;
    sa.k = p->k;
    sa.n = (int)n;
    sa.max_iter = pl.max_iter;
    const int ts = T.start(T_SELECT, s);
    KATZ_HIP(launch_select_iteration(sa, grid, s));
    T.stop(ts, s);
    if (r % sync_every == 0 || r == pl.max_iter) {
      KATZ_HIP(hipMemcpyAsync(ar.host_sc, pr.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
      KATZ_HIP(hipStreamSynchronize(s));
      if (ar.host_sc->err) return KATZ_E_CSR;
      if (ar.host_sc->done) break;
    }
  }
  const int rf = ar.host_sc->iterations;
  const int status = ar.host_sc->status;
  const long long m_final = ar.host_sc->m;

  SelArgs fa{};
  fa.b = bound_args(pl, pr, rb, S, rf, p->epsilon, g->undirected);
  fa.top_sorted = rb.top_sorted;
  fa.top_lo = rb.top_lo;
  fa.top_up = rb.top_up;
  fa.k = p->k;
  fa.n = (int)n;
  int32_t* ids = pl.out_host ? rb.out_ids : out->topk_ids;
  double* lo = pl.out_host ? rb.out_lo : out->lower;
  double* up = pl.out_host ? rb.out_up : out->upper;
  const int tr = T.start(T_RESULT, s);
  KATZ_HIP(hipMemsetAsync(rb.mark, 0, (size_t)n, s));
  KATZ_HIP(hipMemsetAsync(rb.rest_bits, 0, sizeof(unsigned long long), s));
  KATZ_HIP(launch_write_result(fa, rb.mark, ids, lo, up, rb.rest_bits, grid, s));
  T.stop(tr, s);
  KATZ_HIP(hipMemcpyAsync(ar.host_bits, rb.rest_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (pl.out_host) {
    KATZ_HIP(hipMemcpyAsync(out->topk_ids, ids, sizeof(int32_t) * p->k,
                            ids_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipMemcpyAsync(out->lower, lo, sizeof(double) * p->k,
                            lo_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipMemcpyAsync(out->upper, up, sizeof(double) * p->k,
                            up_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  }
  KATZ_HIP(hipStreamSynchronize(s));
  T.commit(s);
  double rest;
  std::memcpy(&rest, ar.host_bits, sizeof(double));
  out->rest_upper_max = (p->k == n) ? -std::numeric_limits<double>::infinity() : rest;
  out->alpha_used = S.alpha;
  out->eta = pl.fp32 ? S.eta[rf] : 0.0;
  out->active_final = m_final;
  out->iterations = rf;
  out->status = status;
  return status;
}

int bounds_one(const katz_csr* g, const katz_params* p, int r_target, double* lower, double* upper,
               hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  rc = check_params(p, g->n, false);
  if (rc) return rc;
  if (r_target < 1 || !lower || !upper) return KATZ_E_INVALID_ARG;
  int dev = 0;
  KATZ_HIP(hipGetDevice(&dev));
  ArenaLease lease(dev);
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
  pl.select = false;
  pl.out_n = (size_t)g->n;
  Prepared pr;
  RunBuffers rb;
  rc = plan_and_allocate(ar, pl, pr, rb);
  if (rc) return rc;
  rc = prepare(ar, pl, pr, pl.max_iter, rb, s);
  if (rc) return rc;
  Scalars S{};
  rc = resolve_alpha(p, pr.dmax, S);
  if (rc) return rc;
  if (pl.fp32) fp32_tables(S, pr, pl.max_iter);
  for (int r = 1; r <= r_target; ++r) {
    long long total_blocks = 0;
    const IterArgs ia = iter_args(pl, pr, rb, S, r, total_blocks);
    if (r == 1) KATZ_HIP(launch_walk_first(ia, pl.fp32, g->n, g->nnz, pl.validate >= KATZ_VALIDATE_BASIC, s));
    else KATZ_HIP(launch_walk_step(ia, pl.fp32, total_blocks, s));
  }
  KATZ_HIP(hipMemcpyAsync(ar.host_sc, pr.sc, sizeof(RunScalars), hipMemcpyDeviceToHost, s));
  KATZ_HIP(hipStreamSynchronize(s));
  if (ar.host_sc->err) return KATZ_E_CSR;
  const BoundArgs b = bound_args(pl, pr, rb, S, r_target, 0.0, g->undirected);
  double* lo = pl.out_host ? rb.out_lo : lower;
  double* up = pl.out_host ? rb.out_up : upper;
  KATZ_HIP(launch_all_bounds(b, g->n, nullptr, lo, up, s));
  if (pl.out_host) {
    KATZ_HIP(hipMemcpyAsync(lower, lo, sizeof(double) * g->n,
                            lo_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    KATZ_HIP(hipMemcpyAsync(upper, up, sizeof(double) * g->n,
                            up_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  }
  KATZ_HIP(hipStreamSynchronize(s));
  return KATZ_OK;
}

}  // namespace
}  // namespace katz

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
struct katz_state {
  int unused;
};

KATZ_EXPORT int katz_rank_static(int32_t count, const katz_csr* g, const katz_params* p, katz_result* out,
                                 katz_state** states, void* stream) {
  if (count < 1 || !g || !p || !out) return KATZ_E_INVALID_ARG;
  if (states) return KATZ_E_UNSUPPORTED;
  for (int32_t i = 0; i < count; ++i) {
    int rc = katz::check_graph(&g[i]);
    if (!rc) rc = katz::check_params(&p[i], g[i].n, true);
    if (!rc && (!out[i].topk_ids || !out[i].lower || !out[i].upper)) rc = KATZ_E_INVALID_ARG;
    if (rc) return rc;
  }
  int worst = KATZ_OK;
  for (int32_t i = 0; i < count; ++i) {
    const int rc = katz::rank_one(&g[i], &p[i], &out[i], (hipStream_t)stream);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
  }
  return worst;
}

KATZ_EXPORT int katz_rank_update(katz_state* st, const int32_t* ins_u, const int32_t* ins_v, int64_t n_ins,
                                 const int32_t* del_u, const int32_t* del_v, int64_t n_del, katz_result* out,
                                 void* stream) {
  (void)ins_u; (void)ins_v; (void)n_ins; (void)del_u; (void)del_v; (void)n_del; (void)out; (void)stream;
  if (!st) return KATZ_E_INVALID_ARG;
  return KATZ_E_UNSUPPORTED;
}

KATZ_EXPORT int katz_bounds(const katz_csr* g, const katz_params* p, int32_t r, double* lower, double* upper,
                            void* stream) {
  return katz::bounds_one(g, p, r, lower, upper, (hipStream_t)stream);
}

KATZ_EXPORT void katz_state_free(katz_state* st) { delete st; }

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
    default: return "unknown status code";
  }
}
