// Stopping criteria of Section 3.1 beyond the LDS-sized top-k test, and the
// separated-pairs measure of Table 1.
//
//   * Top-k with k larger than one workgroup's LDS sort (k > kMaxK), and the
//     ranking criterion, which is the top-k criterion with k = n: after the
//     radix selection and the deactivation pass (sel_apply) the k top nodes
//     are sorted device-wide by (lower bound desc, caller id asc) and every
//     adjacent pair is tested for eps-separation, u(M[i]) - eps < l(M[i-1]).
//   * Score criterion: every node's interval is narrower than eps,
//     u - l < eps; the final list holds every node in ranking order.
//   * Pair criterion: the two given nodes are eps-separated, l(w) > u(v) - eps
//     with w the one ahead by (lower desc, id asc).
//   * Separated pairs (Table 1): the fraction of the n(n-1)/2 unordered pairs
//     {w, v} with l(w) > u(v) or l(v) > u(w); with the lower bounds sorted
//     descending, node v contributes the number of lower bounds above u(v).
//
// The device-wide sort is a bitonic network in its direction-free form: for
// every block size s = 2, 4, ..., P (P the power of two >= count) first the
// mirrored pairs (i, i ^ (s - 1)) and then the half-cleaner pairs (i, i + d),
// d = s/4, ..., 1, each compare-exchange putting the smaller record at the
// lower index.  Indices at or past `count` hold virtual +infinity records:
// every pair that reaches one is already in order, so those pairs are skipped
// and no padding is stored.  Pairs inside a 2048-record tile run in LDS (one
// launch covers every stage up to s = 2048, and one launch the strides below
// 2048 of each later stage); longer strides run one global pass each.
#include <climits>
#include <cstdint>

#include "katz_device.h"

namespace katz {
namespace {

constexpr int kTile = 2 * kFinishThreads;   // records per LDS tile (2048)

__device__ __forceinline__ bool halted(const RunScalars* sc) { return sc->err || sc->done; }
__device__ __forceinline__ int to_ext(const SelArgs& a, int v) { return a.ext_of ? a.ext_of[v] : v; }
__device__ __forceinline__ int to_int(const SelArgs& a, int e) { return a.int_of ? a.int_of[e] : e; }

// A record orders before another when its key is smaller, then its id.  Keys
// are the complemented bit patterns of non-negative lower bounds, so ascending
// keys are descending lower bounds.
__device__ __forceinline__ bool rec_less(unsigned long long ka, int ea, unsigned long long kb, int eb) {
  return ka < kb || (ka == kb && ea < eb);
}

__device__ __forceinline__ void cmp_swap(unsigned long long* key, int32_t* ext, long long i, long long j) {
  const unsigned long long ki = key[i], kj = key[j];
  const int ei = ext[i], ej = ext[j];
  if (rec_less(kj, ej, ki, ei)) {
    key[i] = kj;
    key[j] = ki;
    ext[i] = ej;
    ext[j] = ei;
  }
}

// Whether the top list is sorted and tested in this iteration (the same rule
// as the LDS check): when no node outside the top-k survived, or when the run
// stops here for another reason and the sorted list is the output.
__device__ __forceinline__ bool sort_needed(const SelArgs& a) {
  const RunScalars* sc = a.sc;
  const bool walk_zero = a.b.fp32 ? (a.xmax32[a.b.r] == 0u) : (a.xmax64[a.b.r] == 0ull);
  return sc->kept_count == 0 || walk_zero || (a.b.fp32 && !sc->progress) || a.b.r >= a.max_iter;
}

// Sort records of the top list: key = ~bits(l), id = caller id.  list = null
// takes the identity list 0..count-1 (every node, score criterion output).
__global__ void __launch_bounds__(kWG) lk_fill(SelArgs a, const int32_t* list, long long count, int gate,
                                               unsigned long long* key, int32_t* ext) {
  if (gate) {
    if (halted(a.sc)) return;
    if (a.sc->top_count != a.k) {
      // The selection must hand over exactly k top nodes; anything else is an
      // internal inconsistency and stops the run before ids are used.
      if (blockIdx.x == 0 && threadIdx.x == 0) a.sc->err = 2;
      return;
    }
    if (!sort_needed(a)) return;
  }
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < count; i += (long long)gridDim.x * kWG) {
    const int v = list ? list[i] : (int)i;
    double lo, up;
    bound_eval(a.b, v, lo, up);
    key[i] = ~key_of(lo);
    ext[i] = to_ext(a, v);
  }
}

// Tile pass in LDS.  full = 1: every stage s = 2 .. kTile; full = 0: the
// half-cleaner strides kTile/2 .. 1 of a later stage.
__global__ void __launch_bounds__(kFinishThreads) lk_tile(SelArgs a, long long count, int gate, int full,
                                                          unsigned long long* key, int32_t* ext) {
  if (gate && (halted(a.sc) || !sort_needed(a))) return;
  __shared__ unsigned long long sk[kTile];
  __shared__ int32_t se[kTile];
  const long long base = (long long)blockIdx.x * kTile;
  for (int t = threadIdx.x; t < kTile; t += kFinishThreads) {
    const long long i = base + t;
    sk[t] = i < count ? key[i] : ~0ull;
    se[t] = i < count ? ext[i] : INT_MAX;
  }
  __syncthreads();
  const int t = threadIdx.x;   // one pair per thread and step
  if (full) {
    for (int s = 2; s <= kTile; s <<= 1) {
      {
        const int h = s >> 1;
        const int i = (t / h) * s + (t % h);
        cmp_swap(sk, se, i, i ^ (s - 1));
      }
      __syncthreads();
      for (int d = s >> 2; d >= 1; d >>= 1) {
        const int i = (t / d) * 2 * d + (t % d);
        cmp_swap(sk, se, i, i + d);
        __syncthreads();
      }
    }
  } else {
    for (int d = kTile >> 1; d >= 1; d >>= 1) {
      const int i = (t / d) * 2 * d + (t % d);
      cmp_swap(sk, se, i, i + d);
      __syncthreads();
    }
  }
  for (int u = threadIdx.x; u < kTile; u += kFinishThreads) {
    const long long i = base + u;
    if (i < count) {
      key[i] = sk[u];
      ext[i] = se[u];
    }
  }
}

// One global pass: mirror = 1 pairs (i, i ^ (s - 1)) of stage s; mirror = 0
// pairs (i, i + d).
__global__ void __launch_bounds__(kWG) lk_pass(SelArgs a, long long count, long long half_pairs, int gate,
                                               int mirror, long long s, long long d, unsigned long long* key,
                                               int32_t* ext) {
  if (gate && (halted(a.sc) || !sort_needed(a))) return;
  for (long long t = (long long)blockIdx.x * kWG + threadIdx.x; t < half_pairs;
       t += (long long)gridDim.x * kWG) {
    long long i, j;
    if (mirror) {
      const long long h = s >> 1;
      i = (t / h) * s + (t % h);
      j = i ^ (s - 1);
    } else {
      i = (t / d) * 2 * d + (t % d);
      j = i + d;
    }
    if (j < count) cmp_swap(key, ext, i, j);
  }
}

// The sorted list becomes the ranking output; with test = 1 every adjacent
// pair is tested for eps-separation (the check of converged()).
__global__ void __launch_bounds__(kWG) lk_emit(SelArgs a, long long count, int gate, int test,
                                               const unsigned long long* key, const int32_t* ext) {
  if (gate && (halted(a.sc) || !sort_needed(a))) return;
  bool fail = false;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < count; i += (long long)gridDim.x * kWG) {
    const int v = to_int(a, ext[i]);
    double lo, up;
    bound_eval(a.b, v, lo, up);
    a.top_sorted[i] = v;
    a.top_lo[i] = lo;
    a.top_up[i] = up;
    if (test && i > 0 && up - a.b.eps >= __longlong_as_double((long long)~key[i - 1])) fail = true;
  }
  if (test && __ballot(fail) && lane_id() == 0) atomicOr(&a.sc->fail, 1);
}

// converged(), decision: the same rule as the LDS check.
__global__ void lk_finish(SelArgs a) {
  RunScalars* sc = a.sc;
  if (halted(sc)) return;
  const bool walk_zero = a.b.fp32 ? (a.xmax32[a.b.r] == 0u) : (a.xmax64[a.b.r] == 0ull);
  const bool sorted = sort_needed(a);
  const int kept = sc->kept_count;
  const bool certified = kept == 0 && sorted && !sc->fail;
  int status = -1;
  if (certified) status = KATZ_OK;
  else if (walk_zero) status = KATZ_W_EXACT_TIES;
  else if (a.b.fp32 && !sc->progress) status = KATZ_W_PRECISION_LIMIT;
  else if (a.b.r >= a.max_iter) status = KATZ_W_ITER_LIMIT;
  sc->iterations = a.b.r;
  sc->cur = a.act_out_idx;
  sc->m = a.k + kept;
  sc->top_count = 0;
  sc->kept_count = 0;
  sc->cand_count[0] = 0;
  sc->cand_count[1] = 0;
  sc->progress = 0;
  sc->fail = 0;
  if (status >= 0) {
    sc->status = status;
    sc->done = 1;
  }
}

// Score criterion, test: some node has u - l >= eps (fail); FP32 form: some
// such node can still narrow (progress).
__global__ void __launch_bounds__(kWG) score_test(SelArgs a) {
  if (halted(a.sc)) return;
  bool fail = false, prog = false;
  for (long long v = (long long)blockIdx.x * kWG + threadIdx.x; v < a.n; v += (long long)gridDim.x * kWG) {
    double lo, up;
    bound_eval(a.b, (int)v, lo, up);
    if (!(up - lo < a.b.eps)) {
      fail = true;
      if (!prog && can_progress(a.b, (int)v)) prog = true;
    }
  }
  const unsigned long long bf = __ballot(fail), bp = __ballot(prog);
  if (lane_id() == 0) {
    if (bf) atomicOr(&a.sc->fail, 1);
    if (bp) atomicOr(&a.sc->progress, 1);
  }
}

__global__ void score_finish(SelArgs a) {
  RunScalars* sc = a.sc;
  if (halted(sc)) return;
  const bool walk_zero = a.b.fp32 ? (a.xmax32[a.b.r] == 0u) : (a.xmax64[a.b.r] == 0ull);
  int status = -1;
  if (!sc->fail) status = KATZ_OK;
  else if (walk_zero) status = KATZ_W_EXACT_TIES;
  else if (a.b.fp32 && !sc->progress) status = KATZ_W_PRECISION_LIMIT;
  else if (a.b.r >= a.max_iter) status = KATZ_W_ITER_LIMIT;
  sc->iterations = a.b.r;
  sc->m = a.n;
  sc->fail = 0;
  sc->progress = 0;
  if (status >= 0) {
    sc->status = status;
    sc->done = 1;
  }
}

// Pair criterion: test and output (both nodes in ranking order).  ea, eb are
// caller ids.
__global__ void pair_test(SelArgs a, int ea, int eb) {
  RunScalars* sc = a.sc;
  if (halted(sc)) return;
  const int va = to_int(a, ea), vb = to_int(a, eb);
  double la, ua, lb, ub;
  bound_eval(a.b, va, la, ua);
  bound_eval(a.b, vb, lb, ub);
  const bool a_first = la > lb || (la == lb && ea < eb);
  const int w = a_first ? va : vb, v = a_first ? vb : va;
  const double lw = a_first ? la : lb, uw = a_first ? ua : ub;
  const double lv = a_first ? lb : la, uv = a_first ? ub : ua;
  a.top_sorted[0] = w;
  a.top_lo[0] = lw;
  a.top_up[0] = uw;
  a.top_sorted[1] = v;
  a.top_lo[1] = lv;
  a.top_up[1] = uv;
  const bool separated = lw > uv - a.b.eps;
  const bool walk_zero = a.b.fp32 ? (a.xmax32[a.b.r] == 0u) : (a.xmax64[a.b.r] == 0ull);
  int status = -1;
  if (separated) status = KATZ_OK;
  else if (walk_zero) status = KATZ_W_EXACT_TIES;
  else if (a.b.fp32 && !can_progress(a.b, w) && !can_progress(a.b, v)) status = KATZ_W_PRECISION_LIMIT;
  else if (a.b.r >= a.max_iter) status = KATZ_W_ITER_LIMIT;
  sc->iterations = a.b.r;
  sc->m = 2;
  if (status >= 0) {
    sc->status = status;
    sc->done = 1;
  }
}

// Separated pairs: lo holds the n lower bounds in descending order, up the
// upper bounds (any order); adds #{w : lo(w) > up(v)} over v to *count.
__global__ void __launch_bounds__(kWG) separated_count(const double* lo, const double* up, long long n,
                                                       unsigned long long* count) {
  unsigned long long acc = 0;
  for (long long v = (long long)blockIdx.x * kWG + threadIdx.x; v < n; v += (long long)gridDim.x * kWG) {
    const double u = up[v];
    // First position whose lower bound is not above u (lo is non-increasing).
    long long a0 = 0, b0 = n;
    while (a0 < b0) {
      const long long mid = a0 + ((b0 - a0) >> 1);
      if (lo[mid] > u) a0 = mid + 1;
      else b0 = mid;
    }
    acc += (unsigned long long)a0;
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane_id() == 0 && acc) atomicAdd(count, acc);
}

unsigned grid_for(long long items, long long cap) {
  const long long g = (items + kWG - 1) / kWG;
  return (unsigned)std::max<long long>(1, std::min<long long>(g, cap));
}

// The whole sort of `count` records already filled into key / ext.
void enqueue_sort(const SelArgs& a, long long count, int gate, unsigned long long* key, int32_t* ext,
                  hipStream_t s) {
  const long long tiles = (count + kTile - 1) / kTile;
  hipLaunchKernelGGL(lk_tile, dim3((unsigned)tiles), dim3(kFinishThreads), 0, s, a, count, gate, 1, key, ext);
  long long P = kTile;
  while (P < count) P <<= 1;
  const long long half = P / 2;
  const unsigned g = grid_for(half, 1 << 16);
  for (long long sz = 2 * (long long)kTile; sz <= P; sz <<= 1) {
    hipLaunchKernelGGL(lk_pass, dim3(g), dim3(kWG), 0, s, a, count, half, gate, 1, sz, 0ll, key, ext);
    for (long long d = sz >> 2; d >= kTile; d >>= 1)
      hipLaunchKernelGGL(lk_pass, dim3(g), dim3(kWG), 0, s, a, count, half, gate, 0, 0ll, d, key, ext);
    hipLaunchKernelGGL(lk_tile, dim3((unsigned)tiles), dim3(kFinishThreads), 0, s, a, count, gate, 0, key, ext);
  }
}

}  // namespace

hipError_t launch_large_check(const SelArgs& a, unsigned long long* key, int32_t* ext, hipStream_t s) {
  const long long k = a.k;
  const unsigned g = grid_for(k, 1 << 14);
  hipLaunchKernelGGL(lk_fill, dim3(g), dim3(kWG), 0, s, a, (const int32_t*)a.act_out, k, 1, key, ext);
  enqueue_sort(a, k, 1, key, ext, s);
  hipLaunchKernelGGL(lk_emit, dim3(g), dim3(kWG), 0, s, a, k, 1, 1, (const unsigned long long*)key,
                     (const int32_t*)ext);
  hipLaunchKernelGGL(lk_finish, dim3(1), dim3(1), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_score_check(const SelArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(score_test, dim3(grid_for(a.n, 1 << 14)), dim3(kWG), 0, s, a);
  hipLaunchKernelGGL(score_finish, dim3(1), dim3(1), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_score_output(const SelArgs& a, unsigned long long* key, int32_t* ext, hipStream_t s) {
  const long long n = a.n;
  const unsigned g = grid_for(n, 1 << 14);
  hipLaunchKernelGGL(lk_fill, dim3(g), dim3(kWG), 0, s, a, (const int32_t*)nullptr, n, 0, key, ext);
  enqueue_sort(a, n, 0, key, ext, s);
  hipLaunchKernelGGL(lk_emit, dim3(g), dim3(kWG), 0, s, a, n, 0, 0, (const unsigned long long*)key,
                     (const int32_t*)ext);
  return hipGetLastError();
}

hipError_t launch_pair_check(const SelArgs& a, int ea, int eb, hipStream_t s) {
  hipLaunchKernelGGL(pair_test, dim3(1), dim3(1), 0, s, a, ea, eb);
  return hipGetLastError();
}

hipError_t launch_separated_count(const double* lo_desc, const double* up, long long n, unsigned long long* count,
                                  hipStream_t s) {
  hipLaunchKernelGGL(separated_count, dim3(grid_for(n, 1 << 14)), dim3(kWG), 0, s, lo_desc, up, n, count);
  return hipGetLastError();
}

}  // namespace katz
