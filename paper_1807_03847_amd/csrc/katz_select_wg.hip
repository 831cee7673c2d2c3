// converged() of Algorithm 1 for one graph in one 1024-thread workgroup: the
// radix select of the k-th largest lower bound over M, the deactivation pass
// (u - eps < l(M[k])), the LDS sort of the top-k and the adjacent-pair
// eps-separation test.  A launch handles one graph per workgroup: the batched
// form runs every graph of a batch in one launch, and a single graph uses it
// once its active set is small.
#include <algorithm>

#include "katz_device.h"

namespace katz {
namespace {

// The bound factors of iteration r, recomputed on the device when r comes from
// a device counter (same expressions as the host-side bound arguments).
__device__ void refresh_bounds(BoundArgs& b, const GraphSel& gs, int r) {
  b.r = r;
  b.x = (r & 1) ? gs.xbuf[1] : gs.xbuf[0];
  if (b.fp32) {
    const double u64 = 0x1p-53;
    const double kap = (2.0 * r + 32.0) * u64;
    const double ep = gs.etap[r];
    b.kappa = kap;
    b.f_lo_c = 1.0 - kap;
    b.f_hi_c = 1.0 + kap;
    b.f_e = 1.0 + kap;
    b.f_lo_s = b.undirected ? b.alpha * (1.0 - ep) * (1.0 - kap) * (1.0 - 8.0 * u64) : 0.0;
    b.f_hi_s = b.beta * (1.0 + ep) * (1.0 + kap) * (1.0 + 8.0 * u64);
  }
}


constexpr int kSelIlp = 4;   // nodes per thread and pass of the key and deactivation passes

struct SortArea {
  unsigned long long key[kMaxK];
  int ext[kMaxK];
};

// Two kernels share the body, so that each reads its GraphSel from one address
// space (global memory or the kernel arguments) and needs no private copy.
__device__ __forceinline__ void select_graph(const GraphSel& gs, const int* r_dev) {
  RunScalars* sc = gs.sc;
  if (sc->done || sc->err) return;
  BoundArgs b = gs.b;
  if (r_dev) refresh_bounds(b, gs, *r_dev);
  const int cur = r_dev ? sc->cur : gs.cur;
  const int32_t* act_in = cur ? gs.act[1] : gs.act[0];
  int32_t* act_out = const_cast<int32_t*>(cur ? gs.act[0] : gs.act[1]);
  const bool identity = r_dev ? (b.r == 1) : gs.identity_in;
  const int m = identity ? gs.n : sc->m;
  const int k = gs.k;
  // The graph's arrays and sizes as locals: read from gs once, not again after
  // every store (gs may sit in global memory, which the stores could alias).
  const int base_id = gs.base;
  const int n_g = gs.n;
  unsigned long long* const keys = gs.keys;
  unsigned long long* const cand_key = gs.cand_key;
  int32_t* const cand_v = gs.cand_v;
  const int32_t* const ext_of = gs.ext_of;
  const int32_t* const int_of = gs.int_of;
  int32_t* const top_sorted = gs.top_sorted;
  double* const top_lo = gs.top_lo;
  double* const top_up = gs.top_up;
  auto ext = [ext_of](int v) { return ext_of ? ext_of[v] : v; };
  const int t = threadIdx.x;

  __shared__ union {
    unsigned h[kDigits];
    SortArea srt;
  } sm;
  __shared__ unsigned long long s_prefix, s_kmin, s_kmax;
  __shared__ int s_need, s_count, s_cnt, s_top, s_kept, s_fail, s_prog, s_idpre, s_idneed;

  // Keys of M, with their minimum and maximum: the bits above the highest bit
  // in which two keys differ are common to all keys, so the radix digits start
  // right below them (the keys of one graph often share their exponent, and a
  // digit inside it would leave every node a candidate).  Every digit choice
  // finds the same k-th key.
  if (t == 0) {
    s_cnt = 0;
    s_top = 0;
    s_kept = 0;
    s_fail = 0;
    s_prog = 0;
    s_kmin = ~0ull;
    s_kmax = 0ull;
  }
  __syncthreads();
  {
    unsigned long long kmin = ~0ull, kmax = 0ull;
    // Four nodes per thread and pass, their loads issued together (a slot past
    // the end evaluates node base, a valid index, and is dropped).
    for (int b0 = 0; b0 < m; b0 += kSelIlp * kFinishThreads) {   // same trip count for every thread
      unsigned long long kk[kSelIlp];
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = b0 + u * kFinishThreads + t;
        const int v = i < m ? (identity ? base_id + i : act_in[i]) : base_id;
        double lo, up;
        bound_eval(b, v, lo, up);
        kk[u] = key_of(lo);
      }
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = b0 + u * kFinishThreads + t;
        if (i < m) {
          keys[i] = kk[u];
          kmin = kk[u] < kmin ? kk[u] : kmin;
          kmax = kk[u] > kmax ? kk[u] : kmax;
        }
      }
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const unsigned long long a = __shfl_xor(kmin, o), c = __shfl_xor(kmax, o);
      kmin = a < kmin ? a : kmin;
      kmax = c > kmax ? c : kmax;
    }
    if (lane_id() == 0) {
      atomicMin(&s_kmin, kmin);
      atomicMax(&s_kmax, kmax);
    }
  }
  __syncthreads();
  const unsigned long long kdiff = s_kmin ^ s_kmax;
  int rem = kdiff ? 64 - __clzll((long long)kdiff) : 0;   // low bits still to resolve
  if (rem > 63) rem = 63;                                   // keys of non-negative bounds are below 2^63
  unsigned long long pre = m > 0 ? (s_kmin >> rem) : 0ull;  // resolved high bits of the k-th key
  // Level 0 over M: histogram of the first digit below the common bits, then
  // the candidates, the nodes in the k-th key's bucket.
  {
    const int w = min(kDigitBits, rem);
    const int shift = rem - w;
    for (int d = t; d < kDigits; d += kFinishThreads) sm.h[d] = 0u;
    __syncthreads();
    for (int b0 = 0; b0 < m; b0 += kSelIlp * kFinishThreads) {
      unsigned long long kk[kSelIlp];
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = b0 + u * kFinishThreads + t;
        kk[u] = i < m ? keys[i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u)
        wave_hist_add(sm.h, (unsigned)((kk[u] >> shift) & ((1u << w) - 1u)), b0 + u * kFinishThreads + t < m);
    }
    __syncthreads();
    const Bucket bk = find_bucket(sm.h, 1 << w, k, true);
    if (t == 0) {
      s_prefix = (pre << w) | (unsigned)bk.b;
      s_need = bk.need;
      s_count = bk.count;
    }
    __syncthreads();
    pre = s_prefix;
    rem = shift;
    for (int b0 = 0; b0 < m; b0 += kSelIlp * kFinishThreads) {
      unsigned long long kk[kSelIlp];
      int vv[kSelIlp];
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = b0 + u * kFinishThreads + t;
        kk[u] = i < m ? keys[i] : 0ull;
        vv[u] = i < m ? (identity ? base_id + i : act_in[i]) : 0;
      }
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const bool pred = b0 + u * kFinishThreads + t < m && (kk[u] >> rem) == pre;
        const int pos = wave_append(&s_cnt, pred);
        if (pred) {
          cand_key[pos] = kk[u];
          cand_v[pos] = vv[u];
        }
      }
    }
  }
  __syncthreads();
  const int cnt = s_cnt;
  // Remaining digits over the candidates, at most 12 bits each.
  while (rem > 0) {
    const int w = min(kDigitBits, rem);
    const int shift = rem - w;
    for (int d = t; d < kDigits; d += kFinishThreads) sm.h[d] = 0u;
    __syncthreads();
    for (int i0 = 0; i0 < cnt; i0 += kSelIlp * kFinishThreads) {
      unsigned long long kk[kSelIlp];
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = i0 + u * kFinishThreads + t;
        kk[u] = i < cnt ? cand_key[i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = i0 + u * kFinishThreads + t;
        wave_hist_add(sm.h, (unsigned)((kk[u] >> shift) & ((1u << w) - 1u)), i < cnt && (kk[u] >> rem) == pre);
      }
    }
    __syncthreads();
    const Bucket bk = find_bucket(sm.h, 1 << w, s_need, true);
    if (t == 0) {
      s_prefix = (pre << w) | (unsigned)bk.b;
      s_need = bk.need;
      s_count = bk.count;
    }
    __syncthreads();
    pre = s_prefix;
    rem = shift;
  }
  const unsigned long long theta_key = s_prefix;
  const double theta = __longlong_as_double((long long)theta_key);
  const int need = s_need;
  const int ties = s_count;
  int cut = INT_MAX;
  if (need < ties) {
    // The need-th smallest id among the ties (ids are 31-bit: 11 + 11 + 9 bits).
    if (t == 0) {
      s_idpre = 0;
      s_idneed = need;
    }
    __syncthreads();
    int shift = 31;
    for (int L = 0; L < 3; ++L) {
      const int width = L < 2 ? 11 : 9;
      const int hishift = shift;
      shift -= width;
      for (int d = t; d < kDigits; d += kFinishThreads) sm.h[d] = 0u;
      __syncthreads();
      const int idpre = s_idpre;
      // Tied ids share their high digits (all of them at the first level when
      // the ids are below 2^20), so the counts go through the wave-aggregated
      // add; the loop has the same trip count for every thread.
      for (int i0 = 0; i0 < cnt; i0 += kFinishThreads) {
        const int i = i0 + t;
        const bool tie = i < cnt && cand_key[i] == theta_key;
        const int e = tie ? ext(cand_v[i]) : 0;
        const bool in = tie && (hishift >= 31 ? 0 : (e >> hishift)) == idpre;
        wave_hist_add(sm.h, (unsigned)((e >> shift) & ((1 << width) - 1)), in);
      }
      __syncthreads();
      const Bucket ib = find_bucket(sm.h, 1 << width, s_idneed, false);
      if (t == 0) {
        s_idpre = (idpre << width) | ib.b;
        s_idneed = ib.need;
      }
      __syncthreads();
    }
    cut = s_idpre;
  }
  // Deactivation: nodes past position k leave M when u - eps < l(M[k]).
  // Four nodes per thread and pass as above (the order of M does not matter).
  {
    bool prog = false;
    for (int base = 0; base < m; base += kSelIlp * kFinishThreads) {
      bool top[kSelIlp], keep[kSelIlp];
      int vv[kSelIlp];
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int i = base + u * kFinishThreads + t;
        const bool valid = i < m;
        const int v = valid ? (identity ? base_id + i : act_in[i]) : base_id;
        const unsigned long long key = valid ? keys[i] : 0ull;
        double lo, up;
        bound_eval(b, v, lo, up);
        top[u] = valid && (key > theta_key || (key == theta_key && ext(v) <= cut));
        keep[u] = valid && !top[u] && !(up - b.eps < theta);
        if ((top[u] || keep[u]) && can_progress(b, v)) prog = true;
        vv[u] = v;
      }
#pragma unroll
      for (int u = 0; u < kSelIlp; ++u) {
        const int pt = wave_append(&s_top, top[u]);
        if (top[u] && pt < k) act_out[pt] = vv[u];
        const int pk = wave_append(&s_kept, keep[u]);
        if (keep[u] && k + pk < n_g) act_out[k + pk] = vv[u];
      }
    }
    if (prog) s_prog = 1;
  }
  __syncthreads();
  if (s_top != k) {
    if (t == 0) sc->err = 2;
    return;
  }
  // Sort the top-k by (lower desc, id asc) and test adjacent pairs: needed when
  // no node outside the top-k survived, or as the output when the run stops
  // here for another reason.
  const bool walk_zero = b.fp32 ? (gs.xmax32[b.r] == 0u) : (gs.xmax64[b.r] == 0ull);
  const bool need_sort = s_kept == 0 || walk_zero || (b.fp32 && !s_prog) || b.r >= gs.max_iter;
  int P = 1;
  while (P < k) P <<= 1;
  if (!need_sort) P = 0;
  if (t == 0 && !need_sort) s_fail = 1;
  for (int i = t; i < P; i += kFinishThreads) {
    if (i < k) {
      const int v = act_out[i];
      double lo, up;
      bound_eval(b, v, lo, up);
      sm.srt.key[i] = key_of(lo);
      sm.srt.ext[i] = ext(v);
    } else {
      sm.srt.key[i] = 0ull;
      sm.srt.ext[i] = INT_MAX;
    }
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = t; q < P / 2; q += kFinishThreads) {
        const int i = 2 * q - (q & (stride - 1));
        const int j = i + stride;
        const bool up = ((i & size) == 0);
        const unsigned long long ki = sm.srt.key[i], kj = sm.srt.key[j];
        const int ei = sm.srt.ext[i], ej = sm.srt.ext[j];
        const bool j_before_i = kj > ki || (kj == ki && ej < ei);
        if (j_before_i == up) {
          sm.srt.key[i] = kj;
          sm.srt.key[j] = ki;
          sm.srt.ext[i] = ej;
          sm.srt.ext[j] = ei;
        }
      }
      __syncthreads();
    }
  }
  for (int i = t; i < (need_sort ? k : 0); i += kFinishThreads) {
    const int v = int_of ? int_of[sm.srt.ext[i]] : sm.srt.ext[i];
    double lo, up;
    bound_eval(b, v, lo, up);
    top_sorted[i] = v;
    top_lo[i] = lo;
    top_up[i] = up;
    if (i > 0 && up - b.eps >= __longlong_as_double((long long)sm.srt.key[i - 1])) s_fail = 1;
  }
  __syncthreads();
  if (t == 0) {
    const int kept = s_kept;
    const bool certified = kept == 0 && !s_fail;
    int status = -1;
    if (certified) status = KATZ_OK;
    else if (walk_zero) status = KATZ_W_EXACT_TIES;
    else if (b.fp32 && !s_prog) status = KATZ_W_PRECISION_LIMIT;
    else if (b.r >= gs.max_iter) status = KATZ_W_ITER_LIMIT;
    sc->iterations = b.r;
    sc->cur = cur ^ 1;
    sc->m = k + kept;
    if (status >= 0) {
      sc->status = status;
      sc->done = 1;
    }
  }
}

__global__ void __launch_bounds__(kFinishThreads) select_wg(const GraphSel* gsel, const int* r_dev) {
  select_graph(gsel[blockIdx.x], r_dev);
}

__global__ void __launch_bounds__(kFinishThreads) select_wg_one(GraphSel one) { select_graph(one, nullptr); }

}  // namespace

hipError_t launch_select_wg(const GraphSel* gsel, int count, const int* r_dev, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(select_wg, dim3(count), dim3(kFinishThreads), 0, s, gsel, r_dev);
  return hipGetLastError();
}

hipError_t launch_select_wg_one(const GraphSel& one, hipStream_t s) {
  hipLaunchKernelGGL(select_wg_one, dim3(1), dim3(kFinishThreads), 0, s, one);
  return hipGetLastError();
}

}  // namespace katz
