// Device kernels of the certified top-k Katz ranking (gfx950, wave64).
//
// One iteration r of Algorithm 1 (Section 3.2) is
//   walk_first (r = 1) / walk_step or walk_step_grouped (r >= 2)
//                                 walk step of Eq. (basic_recurrence) for every
//                                 row, fused with the update of c_r (and of the
//                                 FP32 margin accumulator); in a renumbered run,
//                                 step 2 also renames the column ids,
//   sel_hist / sel_scan / sel_compact (levels 0, 1), sel_finish
//                                 radix select of the k-th largest lower bound
//                                 over the active set M,
//   sel_apply                     deactivation u - eps < l(M[k]) and compaction
//                                 of M (converged() of Algorithm 1),
//   sel_check                     LDS sort of the top-k and the adjacent-pair
//                                 eps-separation test; sets the stop flag.
// Every kernel returns immediately once the run has stopped, so the host may
// enqueue iterations ahead of reading the flag.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "katz_device.h"

namespace katz {

int bin_of_host(int64_t len, const BinBounds& bb) { return bin_of_len(len, bb); }

namespace {

// ---------------------------------------------------------------------------
// Row sources for binning: a caller CSR, the slack CSR of a dynamic state, or
// a list of row ids of the slack CSR (the affected rows of one re-walk level).
// get(i) yields row id, offset and length of entry i; false marks a malformed
// CSR row.
// ---------------------------------------------------------------------------
template <class OffT>
struct CsrRows {
  const OffT* rp;
  long long nnz;
  static constexpr bool kCsr = true;
  __device__ __forceinline__ bool get(long long i, int& row, long long& off, long long& len) const {
    row = (int)i;
    off = (long long)rp[i];
    const long long end = (long long)rp[i + 1];
    len = end - off;
    return len >= 0 && len <= INT_MAX && off >= 0 && end <= nnz;
  }
};

struct SlackRows {
  const long long* off;
  const int* len;
  static constexpr bool kCsr = false;
  __device__ __forceinline__ bool get(long long i, int& row, long long& o, long long& l) const {
    row = (int)i;
    o = off[i];
    l = len[i];
    return true;
  }
};

struct ListRows {
  const int32_t* ids;
  const long long* off;
  const int* len;
  static constexpr bool kCsr = false;
  __device__ __forceinline__ bool get(long long i, int& row, long long& o, long long& l) const {
    row = ids[i];
    o = off[row];
    l = len[row];
    return true;
  }
};

// After the device-wide scans of the bin counts (bin-major) and of the segment
// counts: bin bases, bin sizes, segment total and the longest row.
__global__ void __launch_bounds__(kFinishThreads) prep_finalize(const long long* blk, int nblocks,
                                                                const long long* totals, RunScalars* sc) {
  if (sc->err) return;
  long long dm = 0;
  for (long long i = threadIdx.x; i < nblocks; i += kFinishThreads)
    dm = max(dm, blk[(long long)(NUM_BINS + 1) * nblocks + i]);
  for (int o = 32; o >= 1; o >>= 1) dm = max(dm, __shfl_xor(dm, o));
  __shared__ long long wm[kFinishThreads / kWave];
  if (lane_id() == 0) wm[threadIdx.x / kWave] = dm;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < kFinishThreads / kWave; ++i) dm = max(dm, wm[i]);
    sc->dmax = (int)dm;
    for (int b = 0; b < NUM_BINS; ++b) {
      const long long lo = blk[(long long)b * nblocks];
      const long long hi = b + 1 < NUM_BINS ? blk[(long long)(b + 1) * nblocks] : totals[0];
      sc->bin_base[b] = lo;
      sc->bin_count[b] = hi - lo;
    }
    sc->seg_total = totals[1];
  }
}

// Strict CSR checks: rows strictly increasing (no duplicates), no self-loops.
__global__ void __launch_bounds__(kWG) validate_strict(const RowDesc* desc, long long count,
                                                       const int32_t* col, long long n, RunScalars* sc) {
  const long long wv = ((long long)blockIdx.x * kWG + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (wv >= count) return;
  const RowDesc d = desc[wv];
  bool bad = false;
  for (int j = lane; j < d.len; j += kWave) {
    const int32_t u = col[d.off + j];
    if (u < 0 || u >= n || u == d.row) bad = true;
    if (j > 0 && col[d.off + j - 1] >= u) bad = true;
  }
  if (bad) atomicOr(&sc->err, 1);
}

// Symmetry: arc v->u must have u->v (a binary search of v in row u, whose
// entries are sorted by the strict check).  One wave per row of at most one
// segment's length, lanes striding over its arcs; longer rows go by segments
// (one wave per 4096-arc segment), so a hub row is checked by many waves.
__device__ __forceinline__ bool has_arc(const long long* row_off, const int* row_len, const int32_t* col, int u,
                                        int v) {
  long long lo = row_off[u], hi = row_off[u] + row_len[u];
  const long long end = hi;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo < end && col[lo] == v;
}

__device__ __forceinline__ bool check_arcs(const long long* row_off, const int* row_len, const int32_t* col,
                                           long long n, int v, long long off, int len) {
  bool bad = false;
  for (int j = lane_id(); j < len && !bad; j += kWave) {
    const int32_t u = col[off + j];
    bad = u < 0 || u >= n || !has_arc(row_off, row_len, col, u, v);
  }
  return bad;
}

__global__ void __launch_bounds__(kWG) validate_symmetry_rows(const RowDesc* desc, long long count,
                                                              const long long* row_off, const int* row_len,
                                                              const int32_t* col, long long n, RunScalars* sc) {
  const long long i = ((long long)blockIdx.x * kWG + threadIdx.x) / kWave;
  if (i >= count) return;
  const RowDesc d = desc[i];
  if (d.len > kBlockRowMax) return;   // checked by segments
  const bool bad = check_arcs(row_off, row_len, col, n, d.row, d.off, d.len);
  if (__ballot(bad) && lane_id() == 0) atomicOr(&sc->err, 1);
}

__global__ void __launch_bounds__(kWG) validate_symmetry_segs(const SegDesc* segs, long long nseg,
                                                              const HugeRow* huge, const long long* row_off,
                                                              const int* row_len, const int32_t* col, long long n,
                                                              RunScalars* sc) {
  const long long i = ((long long)blockIdx.x * kWG + threadIdx.x) / kWave;
  if (i >= nseg) return;
  const SegDesc sd = segs[i];
  const bool bad = check_arcs(row_off, row_len, col, n, huge[sd.hrow].row, sd.off, sd.len);
  if (__ballot(bad) && lane_id() == 0) atomicOr(&sc->err, 1);
}

__global__ void __launch_bounds__(kWG) desc_to_rows(const RowDesc* desc, long long count,
                                                    long long* row_off, int* row_len) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  const RowDesc d = desc[i];
  row_off[d.row] = d.off;
  row_len[d.row] = d.len;
}

// ---------------------------------------------------------------------------
// Walk step (Eq. (basic_recurrence)) with the fused bound epilogue.
// ---------------------------------------------------------------------------
// Largest walk entry an FP32 state's re-walk accepts under its stored scales.
constexpr float kRewalkLimit = 0x1p64f;

template <bool F32>
struct Epi {
  double sigma_r;
  int e_r;
};

// Per-iteration scale of the FP32 form: x~_r = T * 2^-e_r with 2^e_r above
// deg_max * max(x~_{r-1}), so max x~_r < 1; sigma_r = alpha sigma_{r-1} 2^e_r.
// At r = 1 the previous vector is all ones (max 1).
template <bool F32>
__device__ __forceinline__ Epi<F32> compute_epi_at(const IterArgs& a, int r) {
  Epi<F32> ep{1.0, 0};
  if constexpr (F32) {
    const float M = (r == 1) ? 1.0f : __uint_as_float(a.xmax32[r - 1]);
    int ex = 0;
    if (M > 0.0f) {
      (void)frexpf(M, &ex);
      ex += a.clog2_dmax;
    }
    ep.e_r = ex;
    ep.sigma_r = ldexp(a.alpha * a.sigma[r - 1], ex);
  }
  return ep;
}

template <bool F32>
__device__ __forceinline__ Epi<F32> compute_epi(const IterArgs& a) {
  return compute_epi_at<F32>(a, a.r);
}

// The stored walk entry of a row whose sum is t: s = alpha t (FP64 form) or
// x~ = t 2^-e_r (FP32 form).
template <bool F32>
__device__ __forceinline__ typename Prec<F32>::T x_entry(const IterArgs& a, const Epi<F32>& ep,
                                                         typename Prec<F32>::T t) {
  if constexpr (F32) return ldexpf(t, -ep.e_r);
  else return a.alpha * t;
}

// The row's previous c (and FP32 margin e), loaded as soon as the row id is
// known so the load overlaps the gathers instead of following them.
struct Prev {
  double c;
  float e;
  double hp;   // pass 2 of a two-pass step: the row's pass-1 sum (exact in FP64)
};

template <bool F32>
__device__ __forceinline__ Prev load_prev(const IterArgs& a, int row) {
  Prev p{0.0, 0.0f, 0.0};
  if (a.pass == 1) return p;   // pass 1 writes no epilogue
  if (a.r > 1 && !a.rewalk) {
    p.c = a.c[row];
    if constexpr (F32) p.e = a.e[row];
  }
  if (a.pass == 2) p.hp = (double)reinterpret_cast<const typename Prec<F32>::T*>(a.hot_part)[row];
  return p;
}

// The end of a row's sum t: pass 1 keeps it for pass 2; otherwise (pass 2 adds
// the pass-1 sum first) the bound epilogue.
template <bool F32>
__device__ __forceinline__ void finish_row(const IterArgs& a, const Epi<F32>& ep, int row,
                                           typename Prec<F32>::T t, double& vmax, const Prev& pv);

template <bool F32>
__device__ __forceinline__ void epilogue(const IterArgs& a, const Epi<F32>& ep, int row,
                                         typename Prec<F32>::T t, double& vmax, const Prev& pv) {
  if constexpr (!F32) {
    const double s = x_entry<F32>(a, ep, t);
    reinterpret_cast<double*>(a.x_out)[row] = s;
    if (a.rewalk) return;
    a.c[row] = (a.r == 1) ? s : pv.c + s;
    vmax = fmax(vmax, s);
  } else {
    const float xs = x_entry<F32>(a, ep, t);
    reinterpret_cast<float*>(a.x_out)[row] = xs;
    if (a.rewalk) {
      // A state's re-walk keeps the scales of its history, which were chosen
      // for max x~ < 1 on the graph of their time; an entry far above that
      // (or not a number) asks the host to re-run the state from level 1.
      if (!(xs <= kRewalkLimit)) a.sc->rescale = 1;
      return;
    }
    const double s = ep.sigma_r * (double)xs;
    const double e_prev = (a.r == 1) ? 0.0 : (double)pv.e;
    a.c[row] = (a.r == 1) ? s : pv.c + s;
    a.e[row] = __double2float_ru((e_prev + a.etap * s) * (1.0 + 0x1p-50));
    vmax = fmax(vmax, (double)xs);
  }
}

template <bool F32>
__device__ __forceinline__ void finish_row(const IterArgs& a, const Epi<F32>& ep, int row,
                                           typename Prec<F32>::T t, double& vmax, const Prev& pv) {
  using T = typename Prec<F32>::T;
  if (a.pass == 1) {
    reinterpret_cast<T*>(a.hot_part)[row] = t;
    return;
  }
  if (a.pass == 2) t = (T)pv.hp + t;
  epilogue<F32>(a, ep, row, t, vmax, pv);
}

// Where one stretch of a row reads its column ids and, in walk step 2 fused
// with the renumbering, where it writes the renamed ids.
struct Stretch {
  const int32_t* src;
  int32_t* dst;        // renumbering only
  int len;
};

// Strided row sum over G lanes: lane l adds elements l, l+G, l+2G, ... in
// order.  Loads are issued eight at a time (eight column ids, then eight
// gathers) so a lane keeps eight requests in flight; slots past the row end
// add an exact zero, which leaves the sum and its rounding unchanged.  Walk
// entries below a.hub_n are read from the workgroup's copy in LDS (after the
// internal renumbering these are the longest rows, i.e. the most-referenced
// nodes); the copy is exact, so the sum does not depend on where an entry
// was read.
//
// Renumber (walk step 2 of a renumbered static run): the column ids are the
// caller's; each is range-checked (an id outside 0..n-1 sets sc->col_err and
// adds zero, it is never used as an index), renamed through pmap and written
// out, and the neighbour's x_1 is formed from its length exactly as the first
// walk step stored it.  The values added, and their order, are those of the
// unfused step on the renamed columns, so the sum is bitwise the same.
constexpr int kBatch = 8;

template <bool F32, int G, bool Renumber>
__device__ __forceinline__ typename Prec<F32>::T strided_sum(const IterArgs& a, const typename Prec<F32>::T* hub,
                                                             const Stretch& st, int lane, const Epi<F32>& ep1) {
  using T = typename Prec<F32>::T;
  const T* x = reinterpret_cast<const T*>(a.x_in);
  const int H = a.hub_n;
  const int len = st.len;
  // Loads in flight per lane; the elements a lane adds, and their order, do
  // not depend on it (the FP64 renumbering step uses four to avoid spills).
  constexpr int NB = (Renumber && !F32) ? 4 : kBatch;
  T sum = 0;
  bool bad = false;
  for (int j0 = lane; j0 < len; j0 += NB * G) {
    int32_t c[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = j0 + u * G;
      int32_t cc = j < len ? st.src[j] : -1;
      if constexpr (Renumber) {
        if (j < len && (unsigned)cc >= (unsigned)a.n) {
          bad = true;
          cc = -1;
        }
      }
      c[u] = cc;
    }
    if constexpr (Renumber) {
      IdLen m[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) m[u] = c[u] < 0 ? IdLen{0, 0} : a.pmap[c[u]];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int j = j0 + u * G;
        if (j < len) st.dst[j] = m[u].id;
        sum += c[u] < 0 ? (T)0 : x_entry<F32>(a, ep1, (T)m[u].len);
      }
    } else {
      // A two-pass step takes only its class of entries (hot: column id below
      // hot_n); the others add an exact zero and issue no gather.
      T v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const bool take = c[u] >= 0 && (a.pass == 0 || ((c[u] < a.hot_n) == (a.pass == 1)));
        v[u] = take ? (c[u] < H ? hub[c[u]] : x[c[u]]) : (T)0;
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) sum += v[u];
    }
  }
  if (Renumber && bad) atomicOr(&a.sc->col_err, 1);
  return sum;
}

// The stretch of a whole row (desc.off indexes the walk's column array).
template <bool Renumber>
__device__ __forceinline__ Stretch row_stretch(const IterArgs& a, const RowDesc& d, bool valid) {
  if constexpr (Renumber) return Stretch{a.col_src + (valid ? a.coff[d.row] : 0), a.ncol + d.off, d.len};
  else return Stretch{a.col + d.off, nullptr, d.len};
}

// tid: the thread's index in its 256-thread group (the workgroup, or one of
// the groups of walk_step_grouped).
template <bool F32, int G, bool Renumber>
__device__ __forceinline__ void rows_group(const IterArgs& a, const typename Prec<F32>::T* hub, const Epi<F32>& ep,
                                           const Epi<F32>& ep1, long long lb, int bin, double& vmax, bool stop,
                                           int tid) {
  using T = typename Prec<F32>::T;
  constexpr int RPB = kWG / G;
  const int lane = tid & (G - 1);
  const long long i = lb * RPB + tid / G;
  const bool valid = i < a.bin_count[bin];
  RowDesc d{0, 0, 0};
  if (valid) d = a.desc[a.bin_base[bin] + i];
  Prev pv{0.0, 0.0f};
  if (valid && lane == 0) pv = load_prev<F32>(a, d.row);
  if (stop) return;
  T sum = strided_sum<F32, G, Renumber>(a, hub, row_stretch<Renumber>(a, d, valid), lane, ep1);
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, G);
  if (valid && lane == 0) finish_row<F32>(a, ep, d.row, sum, vmax, pv);
}

// Sum of one row or segment by a 256-thread group: 256 strided lanes, wave
// butterflies, then the four wave sums as (w0 + w1) + (w2 + w3) through part
// (the group's four LDS slots).  Contains workgroup barriers: every thread of
// the workgroup must call it the same number of times.
template <bool F32, bool Renumber>
__device__ __forceinline__ typename Prec<F32>::T group_sum(const IterArgs& a, const typename Prec<F32>::T* hub,
                                                           const Stretch& st, const Epi<F32>& ep1, int tid,
                                                           typename Prec<F32>::T* part) {
  using T = typename Prec<F32>::T;
  T sum = strided_sum<F32, kWG, Renumber>(a, hub, st, tid, ep1);
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
  if (lane_id() == 0) part[tid / kWave] = sum;
  __syncthreads();
  const T tot = (part[0] + part[1]) + (part[2] + part[3]);
  __syncthreads();
  return tot;
}

template <bool F32, bool Renumber>
__device__ __forceinline__ typename Prec<F32>::T block_sum(const IterArgs& a, const typename Prec<F32>::T* hub,
                                                           const Stretch& st, const Epi<F32>& ep1) {
  __shared__ typename Prec<F32>::T part[kWG / kWave];
  return group_sum<F32, Renumber>(a, hub, st, ep1, threadIdx.x, part);
}

// Per-workgroup maximum of the new walk entries, stored without atomics (a
// later kernel reduces the array).  All threads must call it.
template <bool F32>
__device__ __forceinline__ void store_block_max(const IterArgs& a, double vmax, long long slot) {
  if (a.pass == 1) return;   // uniform: pass 1 computes no walk entry
  __shared__ double wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = vmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    if constexpr (F32) reinterpret_cast<float*>(a.blkmax)[slot] = (float)m;
    else reinterpret_cast<double*>(a.blkmax)[slot] = m;
  }
}

// First walk step: x_0 = 1, so the sum over row v is its length, exactly.
template <bool F32>
__global__ void __launch_bounds__(kWG) walk_first(IterArgs a) {
  if (a.sc->err || a.sc->done) return;
  const Epi<F32> ep = compute_epi<F32>(a);
  if constexpr (F32) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sigma[1] = ep.sigma_r;
      a.sigma_sum[1] = ep.sigma_r;
    }
  }
  double vmax = 0.0;
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < a.count_first) {
    const RowDesc d = a.desc[i];
    epilogue<F32>(a, ep, d.row, (typename Prec<F32>::T)d.len, vmax, Prev{0.0, 0.0f});
  }
  store_block_max<F32>(a, vmax, blockIdx.x);
}

// 0 <= col < n for every arc (basic validation, before the first gather).
__global__ void __launch_bounds__(kWG) check_col_range(const int32_t* col, long long nnz, long long n,
                                                       RunScalars* sc) {
  bool bad = false;
  for (long long j = (long long)blockIdx.x * kWG + threadIdx.x; j < nnz; j += (long long)gridDim.x * kWG)
    if ((unsigned)col[j] >= (unsigned long long)n) bad = true;
  if (__ballot(bad) && lane_id() == 0) atomicOr(&sc->err, 1);
}

// Walk step r >= 2: every bin in one launch, heavy bins first.  The grid may
// be smaller than the work: workgroup b takes work items b, b + gridDim.x, ...
// (a persistent grid, which is what makes the LDS copy of the first a.hub_n
// walk entries worth its fill).  Renumber: step 2 of a renumbered static run,
// which also writes the renamed column ids (see strided_sum).
template <bool F32, bool Renumber>
__global__ void __launch_bounds__(kWG) walk_step(IterArgs a) {
  using T = typename Prec<F32>::T;
  // The stop flag (a launch enqueued ahead of the host's flag read skips its
  // work once the run has stopped) and the FP32 scale are read first and used
  // late, so their loads overlap the first descriptor loads.
  const bool stop = a.sc->err || a.sc->done;
  const long long total = a.first_block[NUM_BINS];
  // A persistent grid visits many work items per workgroup: stop at once.
  if (stop && (long long)gridDim.x < total) return;
  const Epi<F32> ep = compute_epi<F32>(a);
  const Epi<F32> ep1 = Renumber ? compute_epi_at<F32>(a, 1) : ep;
  extern __shared__ __align__(16) unsigned char walk_lds[];
  T* hub = reinterpret_cast<T*>(walk_lds);
  if (!Renumber && a.hub_n > 0) {
    const T* x = reinterpret_cast<const T*>(a.x_in);
    if (!stop)
      for (int i = threadIdx.x; i < a.hub_n; i += kWG) hub[i] = x[i];
    __syncthreads();
  }
  if constexpr (F32) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && !stop) {
      a.sigma[a.r] = ep.sigma_r;
      a.sigma_sum[a.r] = a.sigma_sum[a.r - 1] + ep.sigma_r;
    }
  }
  double vmax = 0.0;
  for (long long b = blockIdx.x; b < total; b += gridDim.x) {
    int bin = 0;
    while (bin < NUM_BINS && b >= a.first_block[bin + 1]) ++bin;
    const long long lb = b - a.first_block[bin];
    switch (bin) {
      case BIN_HUGE: {
        // One 4096-arc segment of a long row: its partial sum only; huge_combine
        // adds the partials of each row in segment order after this launch.
        const SegDesc sd = a.segs[lb];
        Stretch st{a.col + sd.off, nullptr, sd.len};
        if constexpr (Renumber) {
          const HugeRow h = a.huge[sd.hrow];
          st.src = a.col_src + a.coff[h.row] + (long long)(sd.part - h.part0) * kSeg;
          st.dst = a.ncol + sd.off;
        }
        if (stop) break;
        const T tot = block_sum<F32, Renumber>(a, hub, st, ep1);
        if (threadIdx.x == 0) {
          T* part = reinterpret_cast<T*>(a.partial);
          part[sd.part] = a.pass == 2 ? part[sd.part] + tot : tot;
        }
        break;
      }
      case BIN_B256: {
        const RowDesc d = a.desc[a.bin_base[BIN_B256] + lb];
        Prev pv{0.0, 0.0f, 0.0};
        if (threadIdx.x == 0) pv = load_prev<F32>(a, d.row);
        const Stretch st = row_stretch<Renumber>(a, d, true);
        if (stop) break;
        const T tot = block_sum<F32, Renumber>(a, hub, st, ep1);
        if (threadIdx.x == 0) finish_row<F32>(a, ep, d.row, tot, vmax, pv);
        break;
      }
      case BIN_W64: rows_group<F32, kBinLanes[BIN_W64], Renumber>(a, hub, ep, ep1, lb, BIN_W64, vmax, stop, threadIdx.x); break;
      case BIN_W16: rows_group<F32, kBinLanes[BIN_W16], Renumber>(a, hub, ep, ep1, lb, BIN_W16, vmax, stop, threadIdx.x); break;
      case BIN_G32: rows_group<F32, kBinLanes[BIN_G32], Renumber>(a, hub, ep, ep1, lb, BIN_G32, vmax, stop, threadIdx.x); break;
      case BIN_G16: rows_group<F32, kBinLanes[BIN_G16], Renumber>(a, hub, ep, ep1, lb, BIN_G16, vmax, stop, threadIdx.x); break;
      case BIN_G8: rows_group<F32, kBinLanes[BIN_G8], Renumber>(a, hub, ep, ep1, lb, BIN_G8, vmax, stop, threadIdx.x); break;
      case BIN_G4: rows_group<F32, kBinLanes[BIN_G4], Renumber>(a, hub, ep, ep1, lb, BIN_G4, vmax, stop, threadIdx.x); break;
      case BIN_EMPTY: {
        // Only at r = 2: the buffer of x_2 was never written for empty rows.
        const long long i = lb * kWG + threadIdx.x;
        if (!stop && a.pass != 1 && i < a.bin_count[BIN_EMPTY]) {
          const int row = a.desc[a.bin_base[BIN_EMPTY] + i].row;
          reinterpret_cast<T*>(a.x_out)[row] = (T)0;
        }
        break;
      }
      default: break;
    }
  }
  store_block_max<F32>(a, vmax, blockIdx.x);
}

// Walk step r >= 2 by workgroups of kWalkGroups 256-thread groups that share
// one LDS copy of the hub entries (a larger copy than a 256-thread workgroup
// can hold at the same number of waves per CU).  Each group works as one
// workgroup of walk_step does, with the same lane schedule per row, so every
// sum is bitwise the same.  Group g of workgroup w is virtual workgroup
// w * kWalkGroups + g.  The workgroup-sum items (long-row segments, rows of
// 1025..4096 arcs) come first and go in rounds that every group takes part in,
// an empty share when it has no item, since those sums meet at workgroup-wide
// barriers; the row-group items after them have no barriers.
template <bool F32>
__global__ void __launch_bounds__(kWG * kWalkGroups) walk_step_grouped(IterArgs a) {
  using T = typename Prec<F32>::T;
  constexpr int S = kWalkGroups;
  // The flags cannot change while a walk kernel runs, so every wave of the
  // workgroup takes the same branch here.
  if (a.sc->err || a.sc->done) return;
  const long long total = a.first_block[NUM_BINS];
  const Epi<F32> ep = compute_epi<F32>(a);
  extern __shared__ __align__(16) unsigned char walk_lds[];
  T* hub = reinterpret_cast<T*>(walk_lds);
  {
    const T* x = reinterpret_cast<const T*>(a.x_in);
    for (int i = threadIdx.x; i < a.hub_n; i += kWG * S) hub[i] = x[i];
    __syncthreads();
  }
  if constexpr (F32) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sigma[a.r] = ep.sigma_r;
      a.sigma_sum[a.r] = a.sigma_sum[a.r - 1] + ep.sigma_r;
    }
  }
  __shared__ T part[S][kWG / kWave];
  __shared__ double wm[S][kWG / kWave];
  const int grp = threadIdx.x / kWG;
  const int tid = threadIdx.x % kWG;
  const long long vb = (long long)blockIdx.x * S + grp;
  const long long nvb = (long long)gridDim.x * S;
  double vmax = 0.0;
  const long long n_seg = a.first_block[BIN_B256];
  const long long n_sum = a.first_block[BIN_W64];
  const long long rounds = (n_sum + nvb - 1) / nvb;
  for (long long q = 0; q < rounds; ++q) {
    const long long b = q * nvb + vb;
    Stretch st{a.col, nullptr, 0};
    SegDesc sd{0, 0, 0, 0, 0};
    RowDesc d{0, 0, 0};
    Prev pv{0.0, 0.0f, 0.0};
    if (b < n_seg) {
      sd = a.segs[b];
      st = Stretch{a.col + sd.off, nullptr, sd.len};
    } else if (b < n_sum) {
      d = a.desc[a.bin_base[BIN_B256] + (b - n_seg)];
      st = Stretch{a.col + d.off, nullptr, d.len};
      if (tid == 0) pv = load_prev<F32>(a, d.row);
    }
    const T tot = group_sum<F32, false>(a, hub, st, ep, tid, part[grp]);
    if (tid == 0) {
      if (b < n_seg) {
        T* pt = reinterpret_cast<T*>(a.partial);
        pt[sd.part] = a.pass == 2 ? pt[sd.part] + tot : tot;
      } else if (b < n_sum) {
        finish_row<F32>(a, ep, d.row, tot, vmax, pv);
      }
    }
  }
  for (long long b = n_sum + vb; b < total; b += nvb) {
    int bin = BIN_W64;
    while (bin < NUM_BINS && b >= a.first_block[bin + 1]) ++bin;
    const long long lb = b - a.first_block[bin];
    switch (bin) {
      case BIN_W64: rows_group<F32, kBinLanes[BIN_W64], false>(a, hub, ep, ep, lb, BIN_W64, vmax, false, tid); break;
      case BIN_W16: rows_group<F32, kBinLanes[BIN_W16], false>(a, hub, ep, ep, lb, BIN_W16, vmax, false, tid); break;
      case BIN_G32: rows_group<F32, kBinLanes[BIN_G32], false>(a, hub, ep, ep, lb, BIN_G32, vmax, false, tid); break;
      case BIN_G16: rows_group<F32, kBinLanes[BIN_G16], false>(a, hub, ep, ep, lb, BIN_G16, vmax, false, tid); break;
      case BIN_G8: rows_group<F32, kBinLanes[BIN_G8], false>(a, hub, ep, ep, lb, BIN_G8, vmax, false, tid); break;
      case BIN_G4: rows_group<F32, kBinLanes[BIN_G4], false>(a, hub, ep, ep, lb, BIN_G4, vmax, false, tid); break;
      case BIN_EMPTY: {
        const long long i = lb * kWG + tid;
        if (a.pass != 1 && i < a.bin_count[BIN_EMPTY]) {
          const int row = a.desc[a.bin_base[BIN_EMPTY] + i].row;
          reinterpret_cast<T*>(a.x_out)[row] = (T)0;
        }
        break;
      }
      default: break;
    }
  }
  // Per-group maxima, one slot per virtual workgroup (pass 1 computes none).
  if (a.pass == 1) return;
  for (int o = 32; o >= 1; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  if (lane_id() == 0) wm[grp][tid / kWave] = vmax;
  __syncthreads();
  if (tid == 0) {
    const double m = fmax(fmax(wm[grp][0], wm[grp][1]), fmax(wm[grp][2], wm[grp][3]));
    if constexpr (F32) reinterpret_cast<float*>(a.blkmax)[vb] = (float)m;
    else reinterpret_cast<double*>(a.blkmax)[vb] = m;
  }
}

// Rows longer than one segment: one wave per row adds the row's segment
// partials in segment order (lane l takes l, l+64, ...; then a butterfly) and
// runs the epilogue.  Launched after walk_step, so the kernel boundary makes the
// partials visible to every workgroup without fences.
template <bool F32>
__global__ void __launch_bounds__(kWG) huge_combine(IterArgs a) {
  if (a.sc->err || a.sc->done) return;
  using T = typename Prec<F32>::T;
  const Epi<F32> ep = compute_epi<F32>(a);
  double vmax = 0.0;
  const long long i = (long long)blockIdx.x * (kWG / kWave) + threadIdx.x / kWave;
  if (i < a.bin_count[BIN_HUGE]) {
    const HugeRow h = a.huge[i];
    const int lane = lane_id();
    Prev pv{0.0, 0.0f};
    if (lane == 0) pv = load_prev<F32>(a, h.row);
    const T* part = reinterpret_cast<const T*>(a.partial);
    T sum = 0;
    for (int s2 = lane; s2 < h.nseg; s2 += kWave) sum += part[h.part0 + s2];
    for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
    if (lane == 0) epilogue<F32>(a, ep, h.row, sum, vmax, pv);
  }
  store_block_max<F32>(a, vmax, a.blk_base + blockIdx.x);
}

__global__ void __launch_bounds__(kWG) reduce_blkmax(const void* blkmax, long long nb, int fp32,
                                                     unsigned* xmax32, unsigned long long* xmax64, int r,
                                                     const RunScalars* sc) {
  if (sc->err || sc->done) return;
  __shared__ double wm[kWG / kWave];
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < nb; i += (long long)gridDim.x * kWG)
    m = fmax(m, fp32 ? (double)reinterpret_cast<const float*>(blkmax)[i] : reinterpret_cast<const double*>(blkmax)[i]);
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    // Non-negative values: the IEEE bit patterns order like the values.
    if (fp32) atomicMax(&xmax32[r], __float_as_uint((float)m));
    else atomicMax(&xmax64[r], (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
// Top-k selection and converged() (Algorithm 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool stopped(const RunScalars* sc) { return sc->err || sc->done; }

__device__ __forceinline__ int ext_id(const SelArgs& a, int v) { return a.ext_of ? a.ext_of[v] : v; }
__device__ __forceinline__ int int_id(const SelArgs& a, int e) { return a.int_of ? a.int_of[e] : e; }

// Level-0 keys and histogram of bits [62:51] over the active list.
__global__ void __launch_bounds__(kWG) sel_hist0(SelArgs a) {
  if (stopped(a.sc)) return;
  __shared__ unsigned h[kDigits];
  for (int d = threadIdx.x; d < kDigits; d += kWG) h[d] = 0;
  __syncthreads();
  const int m = a.sc->m;
  const long long stride = (long long)gridDim.x * kWG;
  for (long long i0 = (long long)blockIdx.x * kWG; i0 < m; i0 += stride) {   // uniform trip count per wave
    const long long i = i0 + threadIdx.x;
    unsigned long long key = 0;
    if (i < m) {
      const int v = a.identity_in ? (int)i : a.act_in[i];
      double lo, up;
      bound_eval(a.b, v, lo, up);
      key = key_of(lo);
      a.keys[i] = key;
    }
    wave_hist_add(h, (unsigned)((key >> 51) & (kDigits - 1)), i < m);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kDigits; d += kWG)
    if (h[d]) atomicAdd(&a.hist[d], h[d]);
}

// Level-1 histogram of bits [50:39] over the level-0 candidates.
__global__ void __launch_bounds__(kWG) sel_hist1(SelArgs a) {
  if (stopped(a.sc)) return;
  const int cnt = a.sc->cand_count[0];
  if (cnt <= kSmallCand) return;
  __shared__ unsigned h[kDigits];
  for (int d = threadIdx.x; d < kDigits; d += kWG) h[d] = 0;
  __syncthreads();
  for (long long i0 = (long long)blockIdx.x * kWG; i0 < cnt; i0 += (long long)gridDim.x * kWG) {
    const long long i = i0 + threadIdx.x;
    const unsigned d = i < cnt ? (unsigned)((a.cand_key[0][i] >> 39) & (kDigits - 1)) : 0u;
    wave_hist_add(h, d, i < cnt);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kDigits; d += kWG)
    if (h[d]) atomicAdd(&a.hist[kDigits + d], h[d]);
}

__global__ void __launch_bounds__(kFinishThreads) sel_scan(SelArgs a, int level) {
  if (stopped(a.sc)) return;
  if (level == 1 && a.sc->cand_count[0] <= kSmallCand) return;
  unsigned* hist = a.hist + level * kDigits;
  const int need = (level == 0) ? a.k : a.sc->need;
  const Bucket bk = find_bucket(hist, kDigits, need, true);
  for (int d = threadIdx.x; d < kDigits; d += kFinishThreads) hist[d] = 0u;
  if (threadIdx.x == 0) {
    a.sc->need = bk.need;
    a.sc->prefix = (level == 0) ? (unsigned long long)bk.b : ((a.sc->prefix << kDigitBits) | (unsigned)bk.b);
    a.sc->level = level + 1;
  }
}

constexpr int kIPT = 8;                         // items per thread per append group
constexpr long long kGroup = (long long)kWG * kIPT;

__global__ void __launch_bounds__(kWG) sel_compact(SelArgs a, int level) {
  if (stopped(a.sc)) return;
  const int c0 = a.sc->cand_count[0];
  if (level == 1 && c0 <= kSmallCand) return;
  const unsigned long long pre = a.sc->prefix;
  const int shift = level == 0 ? 51 : 39;
  const int cnt = level == 0 ? a.sc->m : c0;
  for (long long g0 = (long long)blockIdx.x * kGroup; g0 < cnt; g0 += (long long)gridDim.x * kGroup) {
    unsigned long long key[kIPT];
    int v[kIPT];
    unsigned mask = 0;
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
      const long long i = g0 + (long long)j * kWG + threadIdx.x;
      key[j] = 0;
      v[j] = 0;
      if (i < cnt) {
        if (level == 0) {
          key[j] = a.keys[i];
          v[j] = a.identity_in ? (int)i : a.act_in[i];
        } else {
          key[j] = a.cand_key[0][i];
          v[j] = a.cand_v[0][i];
        }
        if ((key[j] >> shift) == pre) mask |= 1u << j;
      }
    }
    int pos = block_reserve(&a.sc->cand_count[level], mask);
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
      if (mask >> j & 1u) {
        a.cand_key[level][pos] = key[j];
        a.cand_v[level][pos] = v[j];
        ++pos;
      }
    }
  }
}

constexpr int kFinishIlp = 4;   // candidates per thread and pass of sel_finish

// Resolves the remaining digits of the k-th key and the id cut inside its ties.
__global__ void __launch_bounds__(kFinishThreads) sel_finish(SelArgs a) {
  if (stopped(a.sc)) return;
  __shared__ unsigned h[kDigits];
  __shared__ unsigned long long s_prefix, s_kmin, s_kmax;
  __shared__ int s_need, s_count;
  const bool from1 = a.sc->cand_count[0] > kSmallCand;
  const unsigned long long* ck = a.cand_key[from1 ? 1 : 0];
  const int32_t* cv = a.cand_v[from1 ? 1 : 0];
  const int cnt = a.sc->cand_count[from1 ? 1 : 0];
  if (threadIdx.x == 0) {
    s_prefix = a.sc->prefix;
    s_need = a.sc->need;
    s_count = cnt;
    s_kmin = ~0ull;
    s_kmax = 0ull;
  }
  __syncthreads();
  const int first = from1 ? 2 : 1;
  const bool track = cnt > kSmallCand;   // only a large candidate set repays the min/max
  for (int level = first; level < kSelectLevels; ++level) {
    const int shift = level < 5 ? 51 - kDigitBits * level : 0;
    const int width = level < 5 ? kDigitBits : 3;
    const int hishift = shift + width;
    // Every candidate carries the prefix resolved before the first level, and
    // the first pass finds their smallest and largest key.  A later digit on
    // which these two agree (with all bits above it) is that digit of every
    // candidate: its bucket holds all cnt of them and the rank inside it does
    // not change, so the pass is not needed.
    if (track && level > first && ((s_kmin ^ s_kmax) >> shift) == 0) {
      if (threadIdx.x == 0) s_prefix = (s_prefix << width) | ((s_kmin >> shift) & ((1ull << width) - 1ull));
      __syncthreads();
      continue;
    }
    for (int d = threadIdx.x; d < kDigits; d += kFinishThreads) h[d] = 0u;
    __syncthreads();
    const unsigned long long pre = s_prefix;
    // Candidates share their leading digits (all of them when many nodes tie
    // at the k-th key), so the counts go through the wave-aggregated add, with
    // kFinishIlp loads in flight per thread and the same trip count for every
    // thread.
    unsigned long long kmin = ~0ull, kmax = 0ull;
    for (int i0 = 0; i0 < cnt; i0 += kFinishIlp * kFinishThreads) {
      unsigned long long key[kFinishIlp];
#pragma unroll
      for (int u = 0; u < kFinishIlp; ++u) {
        const int i = i0 + u * kFinishThreads + (int)threadIdx.x;
        key[u] = i < cnt ? ck[i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kFinishIlp; ++u) {
        const int i = i0 + u * kFinishThreads + (int)threadIdx.x;
        wave_hist_add(h, (unsigned)((key[u] >> shift) & ((1u << width) - 1u)), i < cnt && (key[u] >> hishift) == pre);
        if (track && i < cnt) {
          kmin = key[u] < kmin ? key[u] : kmin;
          kmax = key[u] > kmax ? key[u] : kmax;
        }
      }
    }
    if (track && level == first) {
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long x = __shfl_xor(kmin, o), y = __shfl_xor(kmax, o);
        kmin = x < kmin ? x : kmin;
        kmax = y > kmax ? y : kmax;
      }
      if (lane_id() == 0) {
        atomicMin(&s_kmin, kmin);
        atomicMax(&s_kmax, kmax);
      }
    }
    __syncthreads();
    const Bucket bk = find_bucket(h, 1 << width, s_need, true);
    if (threadIdx.x == 0) {
      s_prefix = (pre << width) | (unsigned)bk.b;
      s_need = bk.need;
      s_count = bk.count;
    }
    __syncthreads();
  }
  const unsigned long long theta_key = s_prefix;
  const int need = s_need;        // how many of the tied keys belong to the top-k
  const int ties = s_count;       // how many active nodes carry exactly theta_key
  int cut = INT_MAX;
  if (need < ties) {
    // The need-th smallest external id among the ties: 31-bit ids, digits
    // [30:20], [19:9], [8:0], ascending.
    __shared__ int s_idpre, s_idneed;
    if (threadIdx.x == 0) {
      s_idpre = 0;
      s_idneed = need;
    }
    __syncthreads();
    const int widths[3] = {11, 11, 9};
    int shift = 31;
    for (int L = 0; L < 3; ++L) {
      const int width = widths[L];
      const int hishift = shift;
      shift -= width;
      for (int d = threadIdx.x; d < kDigits; d += kFinishThreads) h[d] = 0u;
      __syncthreads();
      const int pre = s_idpre;
      for (int i0 = 0; i0 < cnt; i0 += kFinishIlp * kFinishThreads) {
        bool tie[kFinishIlp];
        int v[kFinishIlp];
#pragma unroll
        for (int u = 0; u < kFinishIlp; ++u) {
          const int i = i0 + u * kFinishThreads + (int)threadIdx.x;
          tie[u] = i < cnt && ck[i] == theta_key;
          v[u] = i < cnt ? cv[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kFinishIlp; ++u) {
          const int e = tie[u] ? ext_id(a, v[u]) : 0;
          const bool in = tie[u] && (hishift >= 31 ? 0 : (e >> hishift)) == pre;
          wave_hist_add(h, (unsigned)((e >> shift) & ((1 << width) - 1)), in);
        }
      }
      __syncthreads();
      const Bucket bk = find_bucket(h, 1 << width, s_idneed, false);
      if (threadIdx.x == 0) {
        s_idpre = (pre << width) | bk.b;
        s_idneed = bk.need;
      }
      __syncthreads();
    }
    cut = s_idpre;
  }
  if (threadIdx.x == 0) {
    a.sc->theta_key = theta_key;
    a.sc->theta = __longlong_as_double((long long)theta_key);
    a.sc->cut_ext = cut;
  }
}

// converged(), first half: nodes past position k leave M when u - eps < l(M[k]).
__global__ void __launch_bounds__(kWG) sel_apply(SelArgs a) {
  if (stopped(a.sc)) return;
  __shared__ int s_prog;
  if (threadIdx.x == 0) s_prog = 0;
  const int m = a.sc->m;
  const unsigned long long tk = a.sc->theta_key;
  const double theta = a.sc->theta;
  const int cut = a.sc->cut_ext;
  const double eps = a.b.eps;
  bool prog = false;
  for (long long g0 = (long long)blockIdx.x * kGroup; g0 < m; g0 += (long long)gridDim.x * kGroup) {
    int v[kIPT];
    unsigned mt = 0, mk = 0;
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
      const long long i = g0 + (long long)j * kWG + threadIdx.x;
      v[j] = 0;
      if (i < m) {
        v[j] = a.identity_in ? (int)i : a.act_in[i];
        const unsigned long long key = a.keys[i];
        const bool top = key > tk || (key == tk && ext_id(a, v[j]) <= cut);
        bool keep = false;
        if (!top) {
          double lo, up;
          bound_eval(a.b, v[j], lo, up);
          keep = !(up - eps < theta);
        }
        if (top) mt |= 1u << j;
        if (keep) mk |= 1u << j;
        if ((top || keep) && !prog && can_progress(a.b, v[j])) prog = true;
      }
    }
    int pt = block_reserve(&a.sc->top_count, mt);
    int pk = block_reserve(&a.sc->kept_count, mk);
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
      if (mt >> j & 1u) {
        if (pt < a.k) a.act_out[pt] = v[j];
        ++pt;
      }
      if (mk >> j & 1u) {
        if ((long long)a.k + pk < a.n) a.act_out[a.k + pk] = v[j];
        ++pk;
      }
    }
  }
  if (prog) s_prog = 1;
  __syncthreads();
  if (threadIdx.x == 0 && s_prog) atomicOr(&a.sc->progress, 1);
}

// converged(), second half: sort the top-k by (l desc, id asc) in LDS and test
// every adjacent pair for eps-separation; decide whether the run stops.
__global__ void __launch_bounds__(kFinishThreads) sel_check(SelArgs a) {
  if (stopped(a.sc)) return;
  if (a.sc->top_count != a.k) {
    // The selection must produce exactly k top nodes; anything else is an
    // internal inconsistency and stops the run before ids are dereferenced.
    if (threadIdx.x == 0) a.sc->err = 2;
    return;
  }
  __shared__ unsigned long long skey[kMaxK];
  __shared__ int sext[kMaxK];
  __shared__ int s_fail;
  const int k = a.k;
  // The sorted top-k is needed for the pair test (only when no node outside
  // the top-k survived) and as the output when the run stops here for another
  // reason; otherwise the iteration goes on and the sort is skipped.
  const bool walk_zero = a.b.fp32 ? (a.xmax32[a.b.r] == 0u) : (a.xmax64[a.b.r] == 0ull);
  const bool need_sort = a.sc->kept_count == 0 || walk_zero || (a.b.fp32 && !a.sc->progress) ||
                         a.b.r >= a.max_iter;
  int P = 1;
  while (P < k) P <<= 1;
  if (!need_sort) P = 0;
  if (threadIdx.x == 0) s_fail = need_sort ? 0 : 1;
  for (int i = threadIdx.x; i < P; i += kFinishThreads) {
    if (i < k) {
      const int v = a.act_out[i];
      double lo, up;
      bound_eval(a.b, v, lo, up);
      skey[i] = key_of(lo);
      sext[i] = ext_id(a, v);
    } else {
      skey[i] = 0ull;
      sext[i] = INT_MAX;
    }
  }
  __syncthreads();
  // Bitonic sort, "before" = larger key, then smaller id.
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += kFinishThreads) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const bool up = ((i & size) == 0);
        const unsigned long long ki = skey[i], kj = skey[j];
        const int ei = sext[i], ej = sext[j];
        const bool j_before_i = kj > ki || (kj == ki && ej < ei);
        if (j_before_i == up) {
          skey[i] = kj;
          skey[j] = ki;
          sext[i] = ej;
          sext[j] = ei;
        }
      }
      __syncthreads();
    }
  }
  const double eps = a.b.eps;
  for (int i = threadIdx.x; i < (need_sort ? k : 0); i += kFinishThreads) {
    const int v = int_id(a, sext[i]);
    double lo, up;
    bound_eval(a.b, v, lo, up);
    a.top_sorted[i] = v;
    a.top_lo[i] = lo;
    a.top_up[i] = up;
    if (i > 0 && up - eps >= __longlong_as_double((long long)skey[i - 1])) s_fail = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    RunScalars* sc = a.sc;
    const int kept = sc->kept_count;
    const bool certified = kept == 0 && !s_fail;
    int status = -1;
    if (certified) status = KATZ_OK;
    else if (walk_zero) status = KATZ_W_EXACT_TIES;
    else if (a.b.fp32 && !sc->progress) status = KATZ_W_PRECISION_LIMIT;
    else if (a.b.r >= a.max_iter) status = KATZ_W_ITER_LIMIT;
    sc->iterations = a.b.r;
    sc->cur = a.act_out_idx;
    sc->m = k + kept;
    sc->top_count = 0;
    sc->kept_count = 0;
    sc->cand_count[0] = 0;
    sc->cand_count[1] = 0;
    sc->progress = 0;
    if (status >= 0) {
      sc->status = status;
      sc->done = 1;
    }
  }
}

// Final outputs: external ids and bounds of the ranked nodes, and the largest
// upper bound outside the top-k.
__global__ void __launch_bounds__(kWG) write_top(SelArgs a, uint8_t* mark, int32_t* ids, double* lo,
                                                 double* up) {
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i >= a.k) return;
  const int v = a.top_sorted[i];
  mark[v] = 1;
  ids[i] = ext_id(a, v);
  lo[i] = a.top_lo[i];
  up[i] = a.top_up[i];
}

__global__ void __launch_bounds__(kWG) rest_max(SelArgs a, const uint8_t* mark, unsigned long long* out) {
  double best = 0.0;
  bool any = false;
  for (long long v = (long long)blockIdx.x * kWG + threadIdx.x; v < a.n; v += (long long)gridDim.x * kWG) {
    if (mark[v]) continue;
    double lo, up;
    bound_eval(a.b, (int)v, lo, up);
    best = any ? fmax(best, up) : up;
    any = true;
  }
  __shared__ double wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) {
    const double y = __shfl_xor(best, o);
    best = fmax(best, y);
  }
  if (lane_id() == 0) wm[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void __launch_bounds__(kWG) all_bounds(BoundArgs b, long long n, const int32_t* ext_of,
                                                  double* lower, double* upper) {
  const long long v = (long long)blockIdx.x * kWG + threadIdx.x;
  if (v >= n) return;
  double lo, up;
  bound_eval(b, (int)v, lo, up);
  const int e = ext_of ? ext_of[v] : (int)v;
  lower[e] = lo;
  upper[e] = up;
}

__global__ void init_run(RunScalars* sc, long long n, double* sigma, double* sigma_sum, unsigned* xmax32,
                         unsigned long long* xmax64, int max_iter, unsigned* hist) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (t == 0) {
    RunScalars z{};
    z.m = (int)n;
    z.status = KATZ_OK;
    *sc = z;
    sigma[0] = 1.0;
    sigma_sum[0] = 0.0;
  }
  for (long long i = t; i <= max_iter; i += stride) {
    xmax32[i] = 0u;
    xmax64[i] = 0ull;
    if (i > 0) {
      sigma[i] = 0.0;
      sigma_sum[i] = 0.0;
    }
  }
  for (long long i = t; i < 2 * kDigits; i += stride) hist[i] = 0u;
}

// Internal renumbering: new id i = position of the row in the binned order
// (degree classes, longest first).  ext_of[i] is the caller's id of new node i.
__global__ void __launch_bounds__(kWG) relabel_ids(const RowDesc* desc, long long n, int32_t* ext_of,
                                                   int32_t* int_of, long long* coff, IdLen* pmap, long long* len_ll,
                                                   int* len32) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const RowDesc d = desc[i];
  ext_of[i] = d.row;
  int_of[d.row] = (int32_t)i;
  coff[i] = d.off;
  pmap[d.row] = IdLen{(int32_t)i, d.len};
  len_ll[i] = d.len;
  len32[i] = d.len;
}

// After walk step 2 of a renumbered run: a bad column id fails the run.
__global__ void fold_col_err(RunScalars* sc) {
  if (sc->col_err) sc->err = 1;
}

__global__ void reset_flags(RunScalars* sc) {
  sc->err = 0;
  sc->done = 0;
  sc->status = KATZ_OK;
  sc->top_count = 0;
  sc->kept_count = 0;
  sc->progress = 0;
  sc->cand_count[0] = 0;
  sc->cand_count[1] = 0;
  sc->dmax = 0;
  sc->col_err = 0;
  sc->rescale = 0;
}

}  // namespace

// Renumbering: new id i = position of row i in the binned order, the tables
// of both directions, and the offsets of the renumbered rows (noff, an
// exclusive scan of the lengths).  The renamed column ids are written by walk
// step 2 (walk_step<F32, true>), which reads every column id anyway.
hipError_t launch_relabel(const RowDesc* desc, long long n, int32_t* ext_of, int32_t* int_of, long long* coff,
                          IdLen* pmap, long long* len_ll, int* len32, long long* noff, long long* sums,
                          long long* total, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<long long>(1, (n + kWG - 1) / kWG);
  hipLaunchKernelGGL(relabel_ids, dim3(nb), dim3(kWG), 0, s, desc, n, ext_of, int_of, coff, pmap, len_ll, len32);
  return launch_scan_ll(len_ll, n, noff, sums, total, s);
}

hipError_t launch_reset_flags(RunScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(reset_flags, dim3(1), dim3(1), 0, s, sc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_prep_count(const void* row_ptr, int row_ptr_64, int64_t n, int64_t nnz, long long* blk,
                             int nblocks, RunScalars* sc, const BinBounds& bb, hipStream_t s) {
  if (row_ptr_64)
    hipLaunchKernelGGL(prep_count<CsrRows<int64_t>>, dim3(nblocks), dim3(kWG), 0, s,
                       CsrRows<int64_t>{(const int64_t*)row_ptr, (long long)nnz}, (long long)n, blk, nblocks, sc, bb);
  else
    hipLaunchKernelGGL(prep_count<CsrRows<int32_t>>, dim3(nblocks), dim3(kWG), 0, s,
                       CsrRows<int32_t>{(const int32_t*)row_ptr, (long long)nnz}, (long long)n, blk, nblocks, sc, bb);
  return hipGetLastError();
}

hipError_t launch_prep_scan(long long* blk, int nblocks, long long* sums, long long* totals, RunScalars* sc,
                            hipStream_t s) {
  hipError_t e = launch_scan_ll(blk, (long long)NUM_BINS * nblocks, blk, sums, totals, s);
  if (e != hipSuccess) return e;
  e = launch_scan_ll(blk + (long long)NUM_BINS * nblocks, nblocks, blk + (long long)NUM_BINS * nblocks, sums,
                     totals + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_finalize, dim3(1), dim3(kFinishThreads), 0, s, (const long long*)blk, nblocks,
                     (const long long*)totals, sc);
  return hipGetLastError();
}

hipError_t launch_prep_scatter(const void* row_ptr, int row_ptr_64, int64_t n, const long long* blk,
                               int nblocks, RowDesc* desc, SegDesc* segs, HugeRow* huge, RunScalars* sc,
                               const BinBounds& bb, hipStream_t s) {
  if (row_ptr_64)
    hipLaunchKernelGGL(prep_scatter<CsrRows<int64_t>>, dim3(nblocks), dim3(kWG), 0, s,
                       CsrRows<int64_t>{(const int64_t*)row_ptr, 0}, (long long)n, blk, nblocks, desc, segs, huge,
                       sc, bb);
  else
    hipLaunchKernelGGL(prep_scatter<CsrRows<int32_t>>, dim3(nblocks), dim3(kWG), 0, s,
                       CsrRows<int32_t>{(const int32_t*)row_ptr, 0}, (long long)n, blk, nblocks, desc, segs, huge,
                       sc, bb);
  return hipGetLastError();
}

hipError_t launch_prep_rows(const int32_t* ids, long long count, const long long* off, const int* len,
                            long long* blk, int nblocks, long long* sums, long long* totals, RowDesc* desc,
                            SegDesc* segs, HugeRow* huge, RunScalars* sc, const BinBounds& bb, hipStream_t s) {
  if (ids) {
    const ListRows rows{ids, off, len};
    hipLaunchKernelGGL(prep_count<ListRows>, dim3(nblocks), dim3(kWG), 0, s, rows, count, blk, nblocks, sc, bb);
    const hipError_t e = launch_prep_scan(blk, nblocks, sums, totals, sc, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_scatter<ListRows>, dim3(nblocks), dim3(kWG), 0, s, rows, count, (const long long*)blk,
                       nblocks, desc, segs, huge, sc, bb);
  } else {
    const SlackRows rows{off, len};
    hipLaunchKernelGGL(prep_count<SlackRows>, dim3(nblocks), dim3(kWG), 0, s, rows, count, blk, nblocks, sc, bb);
    const hipError_t e = launch_prep_scan(blk, nblocks, sums, totals, sc, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_scatter<SlackRows>, dim3(nblocks), dim3(kWG), 0, s, rows, count, (const long long*)blk,
                       nblocks, desc, segs, huge, sc, bb);
  }
  return hipGetLastError();
}

hipError_t launch_validate_strict(const RowDesc* desc, long long n, const SegDesc* segs, long long nseg,
                                  const HugeRow* huge, const int32_t* col, int undirected, long long* row_off,
                                  int* row_len, RunScalars* sc, hipStream_t s) {
  const long long blocks = (n * kWave + kWG - 1) / kWG;
  hipLaunchKernelGGL(validate_strict, dim3((unsigned)blocks), dim3(kWG), 0, s, desc, n, col, n, sc);
  if (undirected) {
    const long long nb = (n + kWG - 1) / kWG;
    hipLaunchKernelGGL(desc_to_rows, dim3((unsigned)nb), dim3(kWG), 0, s, desc, n, row_off, row_len);
    hipLaunchKernelGGL(validate_symmetry_rows, dim3((unsigned)blocks), dim3(kWG), 0, s, desc, n,
                       (const long long*)row_off, (const int*)row_len, col, n, sc);
    if (nseg > 0) {
      const long long sb = (nseg * kWave + kWG - 1) / kWG;
      hipLaunchKernelGGL(validate_symmetry_segs, dim3((unsigned)sb), dim3(kWG), 0, s, segs, nseg, huge,
                         (const long long*)row_off, (const int*)row_len, col, n, sc);
    }
  }
  return hipGetLastError();
}

hipError_t launch_walk_first(const IterArgs& a, int fp32, long long n, long long nnz, int validate,
                             hipStream_t s) {
  if (validate && nnz > 0) {
    const long long nb = std::min<long long>((nnz + kWG - 1) / kWG, 4096);
    hipLaunchKernelGGL(check_col_range, dim3((unsigned)nb), dim3(kWG), 0, s, a.col, nnz, n, a.sc);
  }
  const unsigned grid = (unsigned)std::max<long long>(1, (a.count_first + kWG - 1) / kWG);
  if (fp32) hipLaunchKernelGGL(walk_first<true>, dim3(grid), dim3(kWG), 0, s, a);
  else hipLaunchKernelGGL(walk_first<false>, dim3(grid), dim3(kWG), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_check_col_range(const int32_t* col, long long nnz, long long n, RunScalars* sc, hipStream_t s) {
  if (nnz > 0) {
    const long long nb = std::min<long long>((nnz + kWG - 1) / kWG, 4096);
    hipLaunchKernelGGL(check_col_range, dim3((unsigned)nb), dim3(kWG), 0, s, col, nnz, n, sc);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_blkmax(const void* blkmax, long long nb, int fp32, unsigned* xmax32,
                                unsigned long long* xmax64, int r, const RunScalars* sc, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<long long>(64, std::max<long long>(1, (nb + kWG - 1) / kWG));
  hipLaunchKernelGGL(reduce_blkmax, dim3(grid), dim3(kWG), 0, s, blkmax, nb, fp32, xmax32, xmax64, r, sc);
  return hipGetLastError();
}

// walk_step, then huge_combine when there are rows longer than one segment.
// *blocks_used: workgroup maxima written to a.blkmax (both launches).
// Workgroups of a kernel that the device holds at once: a persistent grid
// larger than this would run its last workgroups after all the others.
long long resident_blocks(const void* kernel, size_t lds, int block) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t, int>, long long> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return LLONG_MAX;
  }
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_tuple(dev, kernel, lds, block);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  long long v = LLONG_MAX;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0 && cus > 0)
    v = (long long)per_cu * cus;
  else
    (void)hipGetLastError();
  cache[key] = v;
  return v;
}

// One launch of the walk kernel over every work item (the grouped kernel
// when groups = kWalkGroups); returns the workgroup-maximum slots it writes.
hipError_t launch_walk_kernel(const IterArgs& a, int fp32, long long total_blocks, long long max_grid,
                              long long* used_out, hipStream_t s, bool renumber, int groups) {
  long long g = total_blocks > 0 ? total_blocks : 1;
  const size_t lds = (size_t)a.hub_n * (fp32 ? sizeof(float) : sizeof(double));
  if (!renumber && groups == kWalkGroups) {
    // Workgroups of kWalkGroups groups; slots = virtual workgroups.
    g = (g + kWalkGroups - 1) / kWalkGroups;
    const void* k = fp32 ? (const void*)walk_step_grouped<true> : (const void*)walk_step_grouped<false>;
    if (max_grid > 0) g = std::min(g, max_grid);
    g = std::max<long long>(1, std::min(g, resident_blocks(k, lds, kWG * kWalkGroups)));
    if (fp32) hipLaunchKernelGGL(walk_step_grouped<true>, dim3((unsigned)g), dim3(kWG * kWalkGroups), lds, s, a);
    else hipLaunchKernelGGL(walk_step_grouped<false>, dim3((unsigned)g), dim3(kWG * kWalkGroups), lds, s, a);
    *used_out = g * kWalkGroups;
  } else {
    if (max_grid > 0) {
      const void* k = renumber ? (fp32 ? (const void*)walk_step<true, true> : (const void*)walk_step<false, true>)
                               : (fp32 ? (const void*)walk_step<true, false> : (const void*)walk_step<false, false>);
      g = std::min(g, std::min(max_grid, resident_blocks(k, renumber ? 0 : lds, kWG)));
    }
    if (renumber) {
      if (fp32) hipLaunchKernelGGL((walk_step<true, true>), dim3((unsigned)g), dim3(kWG), 0, s, a);
      else hipLaunchKernelGGL((walk_step<false, true>), dim3((unsigned)g), dim3(kWG), 0, s, a);
    } else {
      if (fp32) hipLaunchKernelGGL((walk_step<true, false>), dim3((unsigned)g), dim3(kWG), lds, s, a);
      else hipLaunchKernelGGL((walk_step<false, false>), dim3((unsigned)g), dim3(kWG), lds, s, a);
    }
    *used_out = g;
  }
  return hipGetLastError();
}

hipError_t launch_walk_step(const IterArgs& a, int fp32, long long total_blocks, long long max_grid,
                            long long* blocks_used, hipStream_t s, bool renumber, int groups) {
  if (a.hub_n > 0 && max_grid <= 0) return hipErrorInvalidValue;   // the copy pays only on a persistent grid
  // col_src may be null for a graph without arcs.
  if (renumber && (a.hub_n > 0 || !a.coff || !a.pmap || !a.ncol || a.r != 2)) return hipErrorInvalidValue;
  if (groups != 1 && groups != kWalkGroups) return hipErrorInvalidValue;
  const bool split = a.hot_n > 0 && !renumber && !a.rewalk;
  if (split && !a.hot_part) return hipErrorInvalidValue;
  long long used = 0;
  hipError_t e;
  if (split) {
    // Pass 1: the hot entries (with the LDS copy); pass 2: the others, without
    // a copy (its gathers miss it), then the epilogue.
    IterArgs p1 = a;
    p1.pass = 1;
    long long unused = 0;
    e = launch_walk_kernel(p1, fp32, total_blocks, max_grid, &unused, s, false, groups);
    if (e != hipSuccess) return e;
    IterArgs p2 = a;
    p2.pass = 2;
    p2.hub_n = 0;
    e = launch_walk_kernel(p2, fp32, total_blocks, max_grid, &used, s, false, groups);
  } else {
    IterArgs p0 = a;
    p0.pass = 0;
    e = launch_walk_kernel(p0, fp32, total_blocks, max_grid, &used, s, renumber, groups);
  }
  if (e != hipSuccess) return e;
  const long long nh = a.bin_count[BIN_HUGE];
  if (nh > 0) {
    IterArgs c = a;
    c.pass = 0;   // the segment partials already hold both passes
    c.blk_base = used;
    const long long cg = (nh + kWG / kWave - 1) / (kWG / kWave);
    if (fp32) hipLaunchKernelGGL(huge_combine<true>, dim3((unsigned)cg), dim3(kWG), 0, s, c);
    else hipLaunchKernelGGL(huge_combine<false>, dim3((unsigned)cg), dim3(kWG), 0, s, c);
    used += cg;
  }
  if (renumber) hipLaunchKernelGGL(fold_col_err, dim3(1), dim3(1), 0, s, a.sc);
  *blocks_used = used;
  return hipGetLastError();
}

hipError_t launch_select_iteration(const SelArgs& a, int grid, hipStream_t s, unsigned long long* sort_key,
                                   int32_t* sort_ext) {
  hipLaunchKernelGGL(sel_hist0, dim3(grid), dim3(kWG), 0, s, a);
  hipLaunchKernelGGL(sel_scan, dim3(1), dim3(kFinishThreads), 0, s, a, 0);
  hipLaunchKernelGGL(sel_compact, dim3(grid), dim3(kWG), 0, s, a, 0);
  hipLaunchKernelGGL(sel_hist1, dim3(grid), dim3(kWG), 0, s, a);
  hipLaunchKernelGGL(sel_scan, dim3(1), dim3(kFinishThreads), 0, s, a, 1);
  hipLaunchKernelGGL(sel_compact, dim3(grid), dim3(kWG), 0, s, a, 1);
  hipLaunchKernelGGL(sel_finish, dim3(1), dim3(kFinishThreads), 0, s, a);
  hipLaunchKernelGGL(sel_apply, dim3(grid), dim3(kWG), 0, s, a);
  if (sort_key) return launch_large_check(a, sort_key, sort_ext, s);
  hipLaunchKernelGGL(sel_check, dim3(1), dim3(kFinishThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_write_result(const SelArgs& a, uint8_t* mark, int32_t* out_ids, double* out_lo,
                               double* out_up, unsigned long long* rest_bits, int grid, hipStream_t s) {
  hipLaunchKernelGGL(write_top, dim3((a.k + kWG - 1) / kWG), dim3(kWG), 0, s, a, mark, out_ids, out_lo, out_up);
  hipLaunchKernelGGL(rest_max, dim3(std::min(grid, 512)), dim3(kWG), 0, s, a, (const uint8_t*)mark, rest_bits);
  return hipGetLastError();
}

hipError_t launch_all_bounds(const BoundArgs& b, int64_t n, const int32_t* ext_of, double* lower,
                             double* upper, hipStream_t s) {
  const unsigned nb = (unsigned)((n + kWG - 1) / kWG);
  hipLaunchKernelGGL(all_bounds, dim3(nb), dim3(kWG), 0, s, b, (long long)n, ext_of, lower, upper);
  return hipGetLastError();
}

hipError_t launch_init_run(RunScalars* sc, int64_t n, double* sigma, double* sigma_sum, unsigned* xmax32,
                           unsigned long long* xmax64, int max_iter, unsigned* hist, hipStream_t s) {
  hipLaunchKernelGGL(init_run, dim3(16), dim3(kWG), 0, s, sc, (long long)n, sigma, sigma_sum, xmax32, xmax64,
                     max_iter, hist);
  return hipGetLastError();
}

}  // namespace katz
