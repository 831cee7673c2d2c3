// Batched form: Algorithm 1 over many independent graphs at once, each with its
// own alpha, k and eps.
//
// The graphs are not copied: their rows are binned together under global row
// ids (graph g owns ids gbase[g] .. gbase[g+1] - 1), and every row carries the
// graph id that locates its column array, its node base and its alpha.  One
// iteration is three launches whose arguments never change, so a block of
// iterations can be captured into a hipGraph and replayed:
//   walk_batch     walk step of every row whose graph is still iterating,
//   select_wg      one workgroup per graph (converged() of Algorithm 1),
//   batch_advance  FP32 scales of the next iteration; r += 1.
// The iteration number r lives in device memory.  The walk vector's r = 0
// buffer holds ones, so the first iteration is an ordinary walk step.
#include <algorithm>

#include "katz_device.h"

namespace katz {
namespace {

struct BatchRows {
  const int* gid_of;
  const long long* gbase;
  const void* const* grp;
  const int* grp64;
  const long long* gnnz;
  static constexpr bool kCsr = false;
  __device__ __forceinline__ bool get(long long i, int& row, long long& off, long long& len) const {
    const int g = gid_of[i];
    const long long v = i - gbase[g];
    row = (int)i;
    long long o0, o1;
    if (grp64[g]) {
      o0 = reinterpret_cast<const long long*>(grp[g])[v];
      o1 = reinterpret_cast<const long long*>(grp[g])[v + 1];
    } else {
      o0 = reinterpret_cast<const int*>(grp[g])[v];
      o1 = reinterpret_cast<const int*>(grp[g])[v + 1];
    }
    off = o0;
    len = o1 - o0;
    return len >= 0 && len <= INT_MAX && o0 >= 0 && o1 <= gnnz[g];
  }
};

__global__ void __launch_bounds__(kWG) fill_gid(const long long* gbase, int count, long long total, int* gid_of) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= total) return;
  int lo = 0, hi = count;   // largest g with gbase[g] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (gbase[mid] <= i) lo = mid; else hi = mid;
  }
  gid_of[i] = lo;
}

// Per graph: row_ptr[0] = 0 and row_ptr[n] = nnz.
__global__ void batch_csr_ends(const void* const* grp, const int* grp64, const long long* gbase,
                               const long long* gnnz, int count, RunScalars* sc) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const long long n = gbase[g + 1] - gbase[g];
  long long a, b;
  if (grp64[g]) {
    a = reinterpret_cast<const long long*>(grp[g])[0];
    b = reinterpret_cast<const long long*>(grp[g])[n];
  } else {
    a = reinterpret_cast<const int*>(grp[g])[0];
    b = reinterpret_cast<const int*>(grp[g])[n];
  }
  if (a != 0 || b != gnnz[g]) atomicOr(&sc->err, 1);
}

// The graphs' arcs, and rows, are numbered one after another (graph g's arcs
// are gabase[g] .. gabase[g+1]-1 of the whole batch), and each workgroup takes
// one fixed-size chunk of them, so big and small graphs cost alike per arc.
// Largest g with base[g] <= i: the graph owning index i (empty graphs own none).
__device__ __forceinline__ int owner_of(const long long* base, int count, long long i) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

constexpr int kColChunk = 16384;   // arcs per workgroup
constexpr int kRowChunk = 4096;    // rows per workgroup

// 0 <= col < n_g for every arc.
__global__ void __launch_bounds__(kWG) batch_col_range(const int32_t* const* gcol, const long long* gabase,
                                                       const long long* gbase, int count, RunScalars* sc) {
  const long long a0 = (long long)blockIdx.x * kColChunk;
  const long long a1 = min(a0 + kColChunk, gabase[count]);
  bool bad = false;
  for (int g = owner_of(gabase, count, a0); g < count && gabase[g] < a1; ++g) {
    const unsigned long long n = (unsigned long long)(gbase[g + 1] - gbase[g]);
    const int32_t* col = gcol[g];
    const long long s = max(a0, gabase[g]) - gabase[g];
    const long long e = min(a1, gabase[g + 1]) - gabase[g];
    for (long long j0 = s + threadIdx.x; j0 < e; j0 += 8 * kWG) {
      int32_t c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const long long j = j0 + (long long)u * kWG;
        c[u] = j < e ? col[j] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if ((unsigned long long)(unsigned)c[u] >= n) bad = true;
    }
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(&sc->err, 1);
}

// Longest row of every graph: one atomic max per workgroup and graph met.
__global__ void __launch_bounds__(kWG) batch_dmax(const void* const* grp, const int* grp64, const long long* gbase,
                                                  int count, int* gdmax) {
  __shared__ int wm[kWG / kWave];
  const long long r0 = (long long)blockIdx.x * kRowChunk;
  const long long r1 = min(r0 + kRowChunk, gbase[count]);
  for (int g = owner_of(gbase, count, r0); g < count && gbase[g] < r1; ++g) {
    const long long s = max(r0, gbase[g]) - gbase[g];
    const long long e = min(r1, gbase[g + 1]) - gbase[g];
    int m = 0;
    if (grp64[g]) {
      const long long* rp = reinterpret_cast<const long long*>(grp[g]);
      for (long long v = s + threadIdx.x; v < e; v += kWG) m = max(m, (int)min(rp[v + 1] - rp[v], (long long)INT_MAX));
    } else {
      const int* rp = reinterpret_cast<const int*>(grp[g]);
      for (long long v = s + threadIdx.x; v < e; v += kWG) m = max(m, rp[v + 1] - rp[v]);
    }
    for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o));
    if (lane_id() == 0) wm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int bm = max(max(wm[0], wm[1]), max(wm[2], wm[3]));
      if (bm > 0) atomicMax(&gdmax[g], bm);
    }
    __syncthreads();
  }
}

template <bool F32>
__device__ __forceinline__ bool graph_live(const BatchWalk& a, int g) {
  const RunScalars& s = a.gsc[g];
  return !s.done && !s.err;
}

template <bool F32>
__device__ __forceinline__ typename Prec<F32>::T batch_strided_sum(const typename Prec<F32>::T* x,
                                                                   const int32_t* cp, int len, int lane, int G) {
  using T = typename Prec<F32>::T;
  T sum = 0;
  constexpr int B = 8;
  for (int j0 = lane; j0 < len; j0 += B * G) {
    int32_t c[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int j = j0 + u * G;
      c[u] = j < len ? cp[j] : -1;
    }
    T v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = c[u] >= 0 ? x[c[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < B; ++u) sum += v[u];
  }
  return sum;
}

// Per-row inputs of the epilogue, loaded as soon as the row and its graph are
// known so that the loads overlap the gathers: the previous c (and FP32 margin
// e) of the row, and the graph's alpha (FP64) or FP32 scale of iteration r.
struct BatchIn {
  double c;
  double scale;
  double etap;
  float e;
  int ex;
};

template <bool F32>
__device__ __forceinline__ BatchIn batch_prefetch(const BatchWalk& a, int r, int g, int row) {
  BatchIn p{0.0, 0.0, 0.0, 0.0f, 0};
  if (r > 1) p.c = a.c[row];
  if constexpr (F32) {
    const long long at = (long long)g * a.stride + r;
    if (r > 1) p.e = a.e[row];
    p.ex = a.gexp[at];
    p.scale = a.gsigma[at];
    p.etap = a.etap[at];
  } else {
    p.scale = a.galpha[g];
  }
  return p;
}

// Row epilogue of the batched walk (same arithmetic as the single-graph one,
// with the graph's alpha and FP32 scale).
template <bool F32>
__device__ __forceinline__ void batch_epilogue(const BatchWalk& a, int r, int row, typename Prec<F32>::T t,
                                               double& vmax, const BatchIn& p) {
  const int out = r & 1;
  if constexpr (!F32) {
    const double s = p.scale * t;
    reinterpret_cast<double*>(a.xbuf[out])[row] = s;
    a.c[row] = (r == 1) ? s : p.c + s;
    vmax = fmax(vmax, s);
  } else {
    const float xs = ldexpf(t, -p.ex);
    reinterpret_cast<float*>(a.xbuf[out])[row] = xs;
    const double s = p.scale * (double)xs;
    const double e_prev = (r == 1) ? 0.0 : (double)p.e;
    a.c[row] = (r == 1) ? s : p.c + s;
    a.e[row] = __double2float_ru((e_prev + p.etap * s) * (1.0 + 0x1p-50));
    vmax = fmax(vmax, (double)xs);
  }
}

__device__ __forceinline__ void graph_max_atomic(const BatchWalk& a, int r, int g, double m, bool f32) {
  if (f32) atomicMax(&a.gxmax32[(long long)g * a.stride + r], __float_as_uint((float)m));
  else atomicMax(&a.gxmax64[(long long)g * a.stride + r], (unsigned long long)__double_as_longlong(m));
}

// Per-workgroup maximum of the new walk entries.  A workgroup whose rows belong
// to one graph stores (graph, maximum) in its slot, and batch_reduce_max folds
// the slots into the per-graph maxima (no same-address atomics in the walk);
// rows of several graphs in one workgroup (only where a bin crosses a graph
// boundary) update the per-graph maxima with atomics.  All threads call it.
template <bool F32>
__device__ __forceinline__ void batch_store_max(const BatchWalk& a, int r, int g, double vmax, long long slot) {
  __shared__ int s_g[kWG / kWave];
  __shared__ double s_m[kWG / kWave];
  const unsigned long long present = __ballot(g >= 0);
  const int src = present ? __ffsll((long long)present) - 1 : 0;
  const int g0 = __shfl(g, src);
  const bool uniform = __all(g < 0 || g == g0);
  double m = vmax;
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (a.direct_max) {
    if (uniform) {
      if (lane_id() == 0 && present && m > 0.0) graph_max_atomic(a, r, g0, m, F32);
    } else if (g >= 0 && vmax > 0.0) {
      graph_max_atomic(a, r, g, vmax, F32);
    }
    return;
  }
  if (!uniform && g >= 0 && vmax > 0.0) graph_max_atomic(a, r, g, vmax, F32);
  if (lane_id() == 0) {
    s_g[threadIdx.x / kWave] = present == 0 ? -1 : (uniform ? g0 : -2);
    s_m[threadIdx.x / kWave] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int bg = -1;
    bool mixed = false;
    double bm = 0.0;
    for (int w = 0; w < kWG / kWave; ++w) {
      if (s_g[w] < 0) {
        mixed = mixed || s_g[w] == -2;
        continue;
      }
      if (bg < 0) bg = s_g[w];
      if (s_g[w] != bg) mixed = true;
      bm = fmax(bm, s_m[w]);
    }
    if (mixed) {
      for (int w = 0; w < kWG / kWave; ++w)
        if (s_g[w] >= 0 && s_m[w] > 0.0) graph_max_atomic(a, r, s_g[w], s_m[w], F32);
      bg = -1;
    }
    a.blk_g[a.blk_base + slot] = bm > 0.0 ? bg : -1;
    a.blk_m[a.blk_base + slot] = bm;
  }
}

// Folds the workgroup slots of one iteration into the per-graph maxima: each
// workgroup reduces a contiguous run of slots in LDS (one entry per graph) and
// issues one atomic per graph it saw.
template <bool F32>
__global__ void __launch_bounds__(kWG) batch_reduce_max(BatchWalk a, long long nb) {
  const int r = *a.r_dev;
  if (r >= a.stride) return;
  extern __shared__ unsigned long long gmax_lds[];
  for (int i = threadIdx.x; i < a.count; i += kWG) gmax_lds[i] = 0ull;
  __syncthreads();
  const long long per = (nb + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = min(nb, lo + per);
  for (long long e = lo + threadIdx.x; e < hi; e += kWG) {
    const int g = a.blk_g[e];
    if (g < 0) continue;
    const double m = a.blk_m[e];
    const unsigned long long bits =
        F32 ? (unsigned long long)__float_as_uint((float)m) : (unsigned long long)__double_as_longlong(m);
    atomicMax(&gmax_lds[g], bits);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.count; i += kWG) {
    const unsigned long long v = gmax_lds[i];
    if (!v) continue;
    if constexpr (F32) atomicMax(&a.gxmax32[(long long)i * a.stride + r], (unsigned)v);
    else atomicMax(&a.gxmax64[(long long)i * a.stride + r], v);
  }
}

// gi: the graph of every row of this work item (its liveness already known),
// or -1 when the item holds rows of several graphs (looked up per row).
template <bool F32, int G>
__device__ __forceinline__ void batch_rows_group(const BatchWalk& a, int r, long long lb, int bin, int gi, int& g_out,
                                                 double& vmax) {
  using T = typename Prec<F32>::T;
  constexpr int RPB = kWG / G;
  const int lane = threadIdx.x & (G - 1);
  const long long i = lb * RPB + threadIdx.x / G;
  bool valid = i < a.bin_count[bin];
  RowDesc d{0, 0, 0};
  int g = gi;
  if (valid) {
    d = a.desc[a.bin_base[bin] + i];
    if (gi < 0) {
      g = a.gid_of[d.row];
      valid = graph_live<F32>(a, g);
    }
  }
  BatchIn p{0.0, 0.0, 0.0, 0.0f, 0};
  if (valid && lane == 0) p = batch_prefetch<F32>(a, r, g, d.row);
  T sum = 0;
  if (valid) {
    const T* x = reinterpret_cast<const T*>(a.xbuf[(r + 1) & 1]) + a.gbase[g];
    sum = batch_strided_sum<F32>(x, a.gcol[g] + d.off, d.len, lane, G);
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, G);
  if (valid && lane == 0) {
    if (gi >= 0) {
      batch_epilogue<F32>(a, r, d.row, sum, vmax, p);
      g_out = g;
    } else {
      // Rows of several graphs in one item: fold this row's entry into its
      // graph's maximum at once (such items are rare).
      double m = 0.0;
      batch_epilogue<F32>(a, r, d.row, sum, m, p);
      if (m > 0.0) graph_max_atomic(a, r, g, m, F32);
    }
  }
}

template <bool F32>
__device__ __forceinline__ typename Prec<F32>::T batch_block_sum(const typename Prec<F32>::T* x, const int32_t* cp,
                                                                 int len) {
  using T = typename Prec<F32>::T;
  __shared__ T part[kWG / kWave];
  T sum = batch_strided_sum<F32>(x, cp, len, threadIdx.x, kWG);
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
  if (lane_id() == 0) part[threadIdx.x / kWave] = sum;
  __syncthreads();
  const T tot = (part[0] + part[1]) + (part[2] + part[3]);
  __syncthreads();
  return tot;
}

// Work items are taken from this iteration's list of live items (built by
// batch_live_items); work item b writes workgroup slot b.  The grid may be
// smaller than the list (persistent workgroups take items with a grid stride).
template <bool F32>
__global__ void __launch_bounds__(kWG) walk_batch(BatchWalk a) {
  using T = typename Prec<F32>::T;
  const int r = *a.r_dev;
  if (r >= a.stride) return;
  // With XCD lists, the workgroups that the hardware places on XCD x (ids
  // x, x + 8, ...) take the items of list x only.
  const int x = blockIdx.x % a.xcd_groups;
  const long long n_items = a.n_items[x];
  const int* list = a.items + (long long)x * a.item_cap;
  const long long step = gridDim.x / a.xcd_groups;
  const T* xin = reinterpret_cast<const T*>(a.xbuf[(r + 1) & 1]);
  for (long long t = blockIdx.x / a.xcd_groups; t < n_items; t += step) {
    const long long b = list[t];
    const int gi = a.item_g[b];
    double vmax = 0.0;
    int g_mine = -1;
    int bin = 0;
    while (bin < NUM_BINS && b >= a.first_block[bin + 1]) ++bin;
    const long long lb = b - a.first_block[bin];
    switch (bin) {
      case BIN_HUGE: {
        // One segment of a long row (item graph gi): its partial sum only;
        // batch_huge_combine adds each row's partials in segment order.
        const SegDesc sd = a.segs[lb];
        const T tot = batch_block_sum<F32>(xin + a.gbase[gi], a.gcol[gi] + sd.off, sd.len);
        if (threadIdx.x == 0) reinterpret_cast<T*>(a.partial)[sd.part] = tot;
        break;
      }
      case BIN_B256: {
        const RowDesc d = a.desc[a.bin_base[BIN_B256] + lb];
        BatchIn p{0.0, 0.0, 0.0, 0.0f, 0};
        if (threadIdx.x == 0) p = batch_prefetch<F32>(a, r, gi, d.row);
        const T tot = batch_block_sum<F32>(xin + a.gbase[gi], a.gcol[gi] + d.off, d.len);
        if (threadIdx.x == 0) {
          batch_epilogue<F32>(a, r, d.row, tot, vmax, p);
          g_mine = gi;
        }
        break;
      }
      case BIN_W64:
        for (int k = 0; k < a.tile; ++k) batch_rows_group<F32, kBinLanes[BIN_W64]>(a, r, lb * a.tile + k, BIN_W64, gi, g_mine, vmax);
        break;
      case BIN_W16:
        for (int k = 0; k < a.tile; ++k) batch_rows_group<F32, kBinLanes[BIN_W16]>(a, r, lb * a.tile + k, BIN_W16, gi, g_mine, vmax);
        break;
      case BIN_G32:
        for (int k = 0; k < a.tile; ++k) batch_rows_group<F32, kBinLanes[BIN_G32]>(a, r, lb * a.tile + k, BIN_G32, gi, g_mine, vmax);
        break;
      case BIN_G16:
        for (int k = 0; k < a.tile; ++k) batch_rows_group<F32, kBinLanes[BIN_G16]>(a, r, lb * a.tile + k, BIN_G16, gi, g_mine, vmax);
        break;
      case BIN_G8:
        for (int k = 0; k < a.tile; ++k) batch_rows_group<F32, kBinLanes[BIN_G8]>(a, r, lb * a.tile + k, BIN_G8, gi, g_mine, vmax);
        break;
      case BIN_G4:
        for (int k = 0; k < a.tile; ++k) batch_rows_group<F32, kBinLanes[BIN_G4]>(a, r, lb * a.tile + k, BIN_G4, gi, g_mine, vmax);
        break;
      case BIN_EMPTY: {
        // Rows without arcs: x_r = 0 (and c_1 = 0, e = 0 at r = 1).
        for (int k = 0; k < a.tile; ++k) {
          const long long i = (lb * a.tile + k) * kWG + threadIdx.x;
          if (i < a.bin_count[BIN_EMPTY]) {
            const int row = a.desc[a.bin_base[BIN_EMPTY] + i].row;
            const int g = gi >= 0 ? gi : a.gid_of[row];
            if (gi >= 0 || graph_live<F32>(a, g)) {
              reinterpret_cast<T*>(a.xbuf[r & 1])[row] = (T)0;
              if (r == 1) {
                a.c[row] = 0.0;
                if constexpr (F32) a.e[row] = 0.0f;
              }
            }
          }
        }
        break;
      }
      default: break;
    }
    batch_store_max<F32>(a, r, g_mine, vmax, b);
  }
}

// Graph of each work item: the graph of all its rows, or -1 when its rows
// belong to several graphs (rows of a bin are in global-id order, so the
// first and last row decide).  Segments and single-row items have one graph.
__global__ void __launch_bounds__(kWG) batch_item_graphs(BatchWalk a, long long total, int* item_g) {
  const long long b = (long long)blockIdx.x * kWG + threadIdx.x;
  if (b >= total) return;
  int bin = 0;
  while (bin < NUM_BINS && b >= a.first_block[bin + 1]) ++bin;
  const long long lb = b - a.first_block[bin];
  int g = -1;
  if (bin == BIN_HUGE) {
    g = a.gid_of[a.huge[a.segs[lb].hrow].row];
  } else {
    const long long rpb = bin == BIN_B256 ? 1 : (long long)bin_rows_per_group(bin) * a.tile;
    const long long i0 = lb * rpb;
    const long long i1 = min(i0 + rpb, a.bin_count[bin]) - 1;
    const int g0 = a.gid_of[a.desc[a.bin_base[bin] + i0].row];
    const int g1 = a.gid_of[a.desc[a.bin_base[bin] + i1].row];
    g = g0 == g1 ? g0 : -1;
  }
  item_g[b] = g;
}

// This iteration's work items: those whose graph is still iterating, and every
// item with rows of several graphs.  One atomic per workgroup appends the
// workgroup's items (their order does not matter: each writes its own slot);
// with XCD lists, one atomic per wave and list.
__global__ void __launch_bounds__(kWG) batch_live_items(BatchWalk a, long long total, int* items, int* n_items) {
  const int r = *a.r_dev;
  if (r >= a.stride) return;
  const long long b = (long long)blockIdx.x * kWG + threadIdx.x;
  bool keep = false;
  int x = 0;
  if (b < total) {
    const int g = a.item_g[b];
    keep = g < 0 || graph_live<true>(a, g);
    if (a.xcd_groups > 1) x = g >= 0 ? a.xcd_of[g] : (int)(b % a.xcd_groups);
  }
  if (a.xcd_groups == 1) {
    const int pos = block_reserve(n_items, keep ? 1u : 0u);
    if (keep) items[pos] = (int)b;
    return;
  }
  unsigned long long pending = __ballot(keep);
  while (pending) {                                    // at most one round per list
    const int leader = __ffsll((long long)pending) - 1;
    const int xl = __shfl(x, leader);
    const unsigned long long same = __ballot(keep && x == xl) & pending;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(&n_items[xl], __popcll(same));
    base = __shfl(base, leader);
    if ((same >> lane_id()) & 1ull) items[(long long)xl * a.item_cap + base + __popcll(same & lanemask_lt())] = (int)b;
    pending &= ~same;
  }
}

// Rows longer than one segment: one wave per row of a live graph adds the
// row's partials in segment order and runs the epilogue.
template <bool F32>
__global__ void __launch_bounds__(kWG) batch_huge_combine(BatchWalk a, long long n_huge) {
  using T = typename Prec<F32>::T;
  const int r = *a.r_dev;
  if (r >= a.stride) return;
  double vmax = 0.0;
  int g_mine = -1;
  const long long i = (long long)blockIdx.x * (kWG / kWave) + threadIdx.x / kWave;
  if (i < n_huge) {
    const HugeRow h = a.huge[i];
    const int g = a.gid_of[h.row];
    if (graph_live<F32>(a, g)) {            // uniform over the wave
      const int lane = lane_id();
      BatchIn p{0.0, 0.0, 0.0, 0.0f, 0};
      if (lane == 0) p = batch_prefetch<F32>(a, r, g, h.row);
      const T* part = reinterpret_cast<const T*>(a.partial);
      T sum = 0;
      for (int s2 = lane; s2 < h.nseg; s2 += kWave) sum += part[h.part0 + s2];
      for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
      if (lane == 0) {
        batch_epilogue<F32>(a, r, h.row, sum, vmax, p);
        g_mine = g;
      }
    }
  }
  batch_store_max<F32>(a, r, g_mine, vmax, blockIdx.x);
}

// After the selection of iteration r: FP32 scales of iteration r + 1 for every
// graph still iterating, then r += 1.  Counts the stopped graphs.
__global__ void __launch_bounds__(kFinishThreads) batch_advance(int* r_dev, int count, RunScalars* gsc,
                                                                const unsigned* gxmax32, double* gsigma,
                                                                double* gsigsum, int* gexp, const double* galpha,
                                                                const int* gclog2, int stride, int fp32,
                                                                int* ndone, int* n_items) {
  const int r = *r_dev;
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = 0;
  __syncthreads();
  int done = 0;
  for (int g = threadIdx.x; g < count; g += kFinishThreads) {
    const RunScalars& s = gsc[g];
    if (s.done || s.err) {
      ++done;
      continue;
    }
    if (fp32 && r + 1 < stride) {
      const long long at = (long long)g * stride;
      const float M = __uint_as_float(gxmax32[at + r]);
      int ex = 0;
      if (M > 0.0f) {
        (void)frexpf(M, &ex);
        ex += gclog2[g];
      }
      const double sg = ldexp(galpha[g] * gsigma[at + r], ex);
      gexp[at + r + 1] = ex;
      gsigma[at + r + 1] = sg;
      gsigsum[at + r + 1] = gsigsum[at + r] + sg;
    }
  }
  atomicAdd(&s_done, done);
  __syncthreads();
  if (threadIdx.x == 0) {
    *r_dev = r + 1;
    *ndone = s_done;
    for (int x = 0; x < kXcds; ++x) n_items[x] = 0;   // the next iteration's lists are rebuilt from zero
  }
}

__global__ void __launch_bounds__(kWG) fill_ones(void* x, long long n, int fp32) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  if (fp32) reinterpret_cast<float*>(x)[i] = 1.0f;
  else reinterpret_cast<double*>(x)[i] = 1.0;
}

// The bound factors of the graph's final iteration.
__device__ BoundArgs final_bounds(const GraphSel& gs) {
  const int r = gs.sc->iterations;
  BoundArgs b = gs.b;
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
  return b;
}

// Per graph outputs: caller ids (local) and bounds of the ranked nodes, which
// are also marked (by internal id) for batch_rest.  Block g handles graph g.
__global__ void __launch_bounds__(kWG) batch_write(const GraphSel* gsel, int32_t* const* out_ids,
                                                   double* const* out_lo, double* const* out_up, uint8_t* mark) {
  const GraphSel& gs = gsel[blockIdx.x];
  for (int i = threadIdx.x; i < gs.k; i += kWG) {
    const int v = gs.top_sorted[i];
    mark[v] = 1;
    out_ids[blockIdx.x][i] = (gs.ext_of ? gs.ext_of[v] : v) - gs.base;
    out_lo[blockIdx.x][i] = gs.top_lo[i];
    out_up[blockIdx.x][i] = gs.top_up[i];
  }
}

// The largest upper bound outside each graph's top-k: blockIdx.y is the graph,
// blockIdx.x a slice of its nodes; rest_bits[g] collects the maxima (bit
// patterns of non-negative doubles order like the values).
__global__ void __launch_bounds__(kWG) batch_rest(const GraphSel* gsel, const uint8_t* mark,
                                                  unsigned long long* rest_bits) {
  const GraphSel& gs = gsel[blockIdx.y];
  const BoundArgs b = final_bounds(gs);
  double best = 0.0;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < gs.n; i += (long long)gridDim.x * kWG) {
    const int v = gs.base + (int)i;
    if (mark[v]) continue;
    double lo, up;
    bound_eval(b, v, lo, up);
    best = fmax(best, up);
  }
  __shared__ double wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) best = fmax(best, __shfl_xor(best, o));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    if (m > 0.0) atomicMax(&rest_bits[blockIdx.y], (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
// Internal renumbering of a batch: each graph's nodes are renamed by their
// position in the graph's own binned order (longest class first, ties by
// caller id), inside the graph's id range gbase[g] .. gbase[g+1]-1, as a
// single-graph call renames them; the walk then reads renamed column ids
// (graph-local) from one array.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bin_of_pos(const RunScalars* sc, long long p) {
  int b = 0;
  while (b + 1 < NUM_BINS && p >= sc->bin_base[b + 1]) ++b;
  return b;
}

// Binned positions are bin-major and, inside a bin, in global row order, so the
// rows of graph g in bin b are one run of positions: record its first and last.
__global__ void __launch_bounds__(kWG) batch_runs(const RowDesc* desc, long long total, const long long* gbase,
                                                  int count, const RunScalars* sc, long long* run_first,
                                                  long long* run_last) {
  const long long p = (long long)blockIdx.x * kWG + threadIdx.x;
  if (p >= total) return;
  const int b = bin_of_pos(sc, p);
  const long long lo = sc->bin_base[b], hi = lo + sc->bin_count[b];
  const int g = owner_of(gbase, count, desc[p].row);
  if (p == lo || owner_of(gbase, count, desc[p - 1].row) != g) run_first[(long long)g * NUM_BINS + b] = p;
  if (p == hi - 1 || owner_of(gbase, count, desc[p + 1].row) != g) run_last[(long long)g * NUM_BINS + b] = p;
}

// Per graph: where each bin's run starts among the graph's new ids.
__global__ void batch_run_starts(const long long* run_first, const long long* run_last, int count,
                                 long long* run_start) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  long long acc = 0;
  for (int b = 0; b < NUM_BINS; ++b) {
    const long long i = (long long)g * NUM_BINS + b;
    run_start[i] = acc;
    if (run_first[i] >= 0) acc += run_last[i] - run_first[i] + 1;
  }
}

// New id of every row, both directions of the renaming, the caller offset and
// length of each renamed row, and pmap[caller id] = {graph-local new id, length}.
__global__ void __launch_bounds__(kWG) batch_relabel(const RowDesc* desc, long long total, const long long* gbase,
                                                     int count, const RunScalars* sc, const long long* run_first,
                                                     const long long* run_start, int32_t* ext_of, int32_t* int_of,
                                                     long long* coff, IdLen* pmap, long long* len_ll, int* len32) {
  const long long p = (long long)blockIdx.x * kWG + threadIdx.x;
  if (p >= total) return;
  const int b = bin_of_pos(sc, p);
  const RowDesc d = desc[p];
  const int g = owner_of(gbase, count, d.row);
  const long long ri = (long long)g * NUM_BINS + b;
  const long long i = gbase[g] + run_start[ri] + (p - run_first[ri]);
  ext_of[i] = d.row;
  int_of[d.row] = (int32_t)i;
  coff[i] = d.off;
  pmap[d.row] = IdLen{(int32_t)(i - gbase[g]), d.len};
  len_ll[i] = d.len;
  len32[i] = d.len;
}

// Renamed column ids of one stretch of a row (arcs in their original order).
template <int G>
__device__ __forceinline__ void batch_rename(const int32_t* src, int32_t* dst, int len, int lane, const IdLen* pm) {
  for (int j0 = lane; j0 < len; j0 += 8 * G) {
    int32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * G;
      c[u] = j < len ? src[j] : -1;
    }
    int32_t m[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m[u] = c[u] < 0 ? 0 : pm[c[u]].id;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * G;
      if (j < len) dst[j] = m[u];
    }
  }
}

// G lanes per renamed row of one bin (rows first .. first+cnt-1 of desc).
template <int G>
__global__ void __launch_bounds__(kWG) batch_rename_rows(const RowDesc* desc, long long first, long long cnt,
                                                         const int* gid_of, const long long* gbase,
                                                         const int32_t* const* gcol, const long long* coff,
                                                         const IdLen* pmap, int32_t* ncol) {
  constexpr int RPB = kWG / G;
  const long long i = first + (long long)blockIdx.x * RPB + threadIdx.x / G;
  if (i >= first + cnt) return;
  const RowDesc d = desc[i];
  const int g = gid_of[d.row];
  batch_rename<G>(gcol[g] + coff[d.row], ncol + d.off, d.len, threadIdx.x & (G - 1), pmap + gbase[g]);
}

// One workgroup per 4096-arc segment of a long renamed row.
__global__ void __launch_bounds__(kWG) batch_rename_segments(const SegDesc* segs, const HugeRow* huge,
                                                             const long long* noff, const int* gid_of,
                                                             const long long* gbase, const int32_t* const* gcol,
                                                             const long long* coff, const IdLen* pmap,
                                                             int32_t* ncol) {
  const SegDesc sd = segs[blockIdx.x];
  const int row = huge[sd.hrow].row;
  const int g = gid_of[row];
  batch_rename<kWG>(gcol[g] + coff[row] + (sd.off - noff[row]), ncol + sd.off, sd.len, threadIdx.x,
                    pmap + gbase[g]);
}

template <int G>
void launch_rename_bin(const RowDesc* desc, long long first, long long cnt, const int* gid_of,
                       const long long* gbase, const int32_t* const* gcol, const long long* coff,
                       const IdLen* pmap, int32_t* ncol, hipStream_t s) {
  if (cnt <= 0) return;
  constexpr int RPB = kWG / G;
  const unsigned nb = (unsigned)((cnt + RPB - 1) / RPB);
  hipLaunchKernelGGL(batch_rename_rows<G>, dim3(nb), dim3(kWG), 0, s, desc, first, cnt, gid_of, gbase, gcol, coff,
                     pmap, ncol);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_batch_prep(const long long* gbase, const void* const* grp, const int* grp64, const long long* gnnz,
                             const long long* gabase, const int32_t* const* gcol, int count, long long total_n,
                             long long total_nnz, int* gid_of, long long* blk, int nblocks, long long* sums,
                             long long* totals, RowDesc* desc, SegDesc* segs, HugeRow* huge, RunScalars* sc,
                             int validate, const BinBounds& bb, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<long long>(1, (total_n + kWG - 1) / kWG);
  hipLaunchKernelGGL(fill_gid, dim3(nb), dim3(kWG), 0, s, gbase, count, total_n, gid_of);
  hipLaunchKernelGGL(batch_csr_ends, dim3((count + 255) / 256), dim3(256), 0, s, grp, grp64, gbase, gnnz, count, sc);
  if (validate && total_nnz > 0) {
    const unsigned gx = (unsigned)((total_nnz + kColChunk - 1) / kColChunk);
    hipLaunchKernelGGL(batch_col_range, dim3(gx), dim3(kWG), 0, s, gcol, gabase, gbase, count, sc);
  }
  const BatchRows rows{gid_of, gbase, grp, grp64, gnnz};
  hipLaunchKernelGGL(prep_count<BatchRows>, dim3(nblocks), dim3(kWG), 0, s, rows, total_n, blk, nblocks, sc, bb);
  hipError_t e = launch_prep_scan(blk, nblocks, sums, totals, sc, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_scatter<BatchRows>, dim3(nblocks), dim3(kWG), 0, s, rows, total_n, (const long long*)blk,
                     nblocks, desc, segs, huge, sc, bb);
  return hipGetLastError();
}

hipError_t launch_batch_dmax(const void* const* grp, const int* grp64, const long long* gbase, int count,
                             long long total_n, int* gdmax, hipStream_t s) {
  if (total_n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((total_n + kRowChunk - 1) / kRowChunk);
  hipLaunchKernelGGL(batch_dmax, dim3(nb), dim3(kWG), 0, s, grp, grp64, gbase, count, gdmax);
  return hipGetLastError();
}

hipError_t launch_fill_ones(void* x, long long n, int fp32, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<long long>(1, (n + kWG - 1) / kWG);
  hipLaunchKernelGGL(fill_ones, dim3(nb), dim3(kWG), 0, s, x, n, fp32);
  return hipGetLastError();
}

// One walk step of the batch: walk_batch (on at most max_grid workgroups when
// max_grid > 0), batch_huge_combine for rows longer than one segment, and
// batch_reduce_max for the per-graph maxima.
// Workgroups of the batched walk kernel the device holds at once (the cap of a
// persistent grid; queried before the iterations are captured).
long long batch_walk_resident(int fp32) {
  return resident_blocks(fp32 ? (const void*)walk_batch<true> : (const void*)walk_batch<false>, 0, kWG);
}

hipError_t launch_walk_batch(const BatchWalk& a, long long total_blocks, long long max_grid, long long n_huge,
                             hipStream_t s) {
  const long long items = std::max<long long>(1, total_blocks);
  long long g = max_grid > 0 ? std::min(items, max_grid) : items;   // max_grid: see batch_walk_resident
  // Every XCD gets the same number of workgroups (a persistent grid rounds
  // down, staying within the resident count; one per item rounds up).
  g = max_grid > 0 ? std::max<long long>(a.xcd_groups, g / a.xcd_groups * a.xcd_groups)
                   : (g + a.xcd_groups - 1) / a.xcd_groups * a.xcd_groups;
  const unsigned grid = (unsigned)g;
  BatchWalk w = a;
  w.blk_base = 0;
  if (a.fp32) hipLaunchKernelGGL(walk_batch<true>, dim3(grid), dim3(kWG), 0, s, w);
  else hipLaunchKernelGGL(walk_batch<false>, dim3(grid), dim3(kWG), 0, s, w);
  long long nb = items;
  if (n_huge > 0) {
    const unsigned cg = (unsigned)((n_huge + kWG / kWave - 1) / (kWG / kWave));
    BatchWalk c = a;
    c.blk_base = items;
    if (a.fp32) hipLaunchKernelGGL(batch_huge_combine<true>, dim3(cg), dim3(kWG), 0, s, c, n_huge);
    else hipLaunchKernelGGL(batch_huge_combine<false>, dim3(cg), dim3(kWG), 0, s, c, n_huge);
    nb += cg;
  }
  if (!a.direct_max) {
    const unsigned rg = (unsigned)std::min<long long>(64, (nb + 4095) / 4096);
    const size_t lds = sizeof(unsigned long long) * (size_t)a.count;
    if (a.fp32) hipLaunchKernelGGL(batch_reduce_max<true>, dim3(rg), dim3(kWG), lds, s, a, nb);
    else hipLaunchKernelGGL(batch_reduce_max<false>, dim3(rg), dim3(kWG), lds, s, a, nb);
  }
  return hipGetLastError();
}

hipError_t launch_batch_advance(int* r_dev, int count, RunScalars* gsc, const unsigned* gxmax32, double* gsigma,
                                double* gsigsum, int* gexp, const double* galpha, const int* gclog2, int stride,
                                int fp32, int* ndone, int* n_items, hipStream_t s) {
  hipLaunchKernelGGL(batch_advance, dim3(1), dim3(kFinishThreads), 0, s, r_dev, count, gsc, gxmax32, gsigma, gsigsum,
                     gexp, galpha, gclog2, stride, fp32, ndone, n_items);
  return hipGetLastError();
}

hipError_t launch_batch_item_graphs(const BatchWalk& a, long long total_blocks, int* item_g, hipStream_t s) {
  if (total_blocks <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((total_blocks + kWG - 1) / kWG);
  hipLaunchKernelGGL(batch_item_graphs, dim3(nb), dim3(kWG), 0, s, a, total_blocks, item_g);
  return hipGetLastError();
}

hipError_t launch_batch_live_items(const BatchWalk& a, long long total_blocks, int* items, int* n_items,
                                   hipStream_t s) {
  const unsigned nb = (unsigned)std::max<long long>(1, (total_blocks + kWG - 1) / kWG);
  hipLaunchKernelGGL(batch_live_items, dim3(nb), dim3(kWG), 0, s, a, total_blocks, items, n_items);
  return hipGetLastError();
}

hipError_t launch_batch_write(const GraphSel* gsel, int count, long long max_n, int32_t* const* out_ids,
                              double* const* out_lo, double* const* out_up, uint8_t* mark,
                              unsigned long long* rest_bits, hipStream_t s) {
  hipLaunchKernelGGL(batch_write, dim3(count), dim3(kWG), 0, s, gsel, out_ids, out_lo, out_up, mark);
  const unsigned bx = (unsigned)std::max<long long>(1, std::min<long long>(64, (max_n + 4095) / 4096));
  hipLaunchKernelGGL(batch_rest, dim3(bx, count), dim3(kWG), 0, s, gsel, (const uint8_t*)mark, rest_bits);
  return hipGetLastError();
}


// Renaming tables of a batch from its first binning (desc, bins in sc); then
// noff = exclusive scan of the renamed lengths.  run_* hold count * NUM_BINS
// entries; run_first and run_last must be all -1 on entry.
hipError_t launch_batch_relabel(const RowDesc* desc, long long total, const long long* gbase, int count,
                                const RunScalars* sc, long long* run_first, long long* run_last,
                                long long* run_start, int32_t* ext_of, int32_t* int_of, long long* coff, IdLen* pmap,
                                long long* len_ll, int* len32, long long* noff, long long* sums, long long* tot,
                                hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((total + kWG - 1) / kWG);
  hipLaunchKernelGGL(batch_runs, dim3(nb), dim3(kWG), 0, s, desc, total, gbase, count, sc, run_first, run_last);
  hipLaunchKernelGGL(batch_run_starts, dim3((count + 255) / 256), dim3(256), 0, s, (const long long*)run_first,
                     (const long long*)run_last, count, run_start);
  hipLaunchKernelGGL(batch_relabel, dim3(nb), dim3(kWG), 0, s, desc, total, gbase, count, sc,
                     (const long long*)run_first, (const long long*)run_start, ext_of, int_of, coff, pmap, len_ll,
                     len32);
  return launch_scan_ll(len_ll, total, noff, sums, tot, s);
}

// Renamed column ids of every renamed row (bins of the second binning).
hipError_t launch_batch_rename(const RowDesc* desc, const long long* bin_base, const long long* bin_count,
                               const SegDesc* segs, long long seg_total, const HugeRow* huge, const long long* noff,
                               const int* gid_of, const long long* gbase, const int32_t* const* gcol,
                               const long long* coff, const IdLen* pmap, int32_t* ncol, hipStream_t s) {
  if (seg_total > 0)
    hipLaunchKernelGGL(batch_rename_segments, dim3((unsigned)seg_total), dim3(kWG), 0, s, segs, huge, noff, gid_of,
                       gbase, gcol, coff, pmap, ncol);
  launch_rename_bin<kWG>(desc, bin_base[BIN_B256], bin_count[BIN_B256], gid_of, gbase, gcol, coff, pmap, ncol, s);
  launch_rename_bin<64>(desc, bin_base[BIN_W64], bin_count[BIN_W64], gid_of, gbase, gcol, coff, pmap, ncol, s);
  launch_rename_bin<16>(desc, bin_base[BIN_W16], bin_count[BIN_W16], gid_of, gbase, gcol, coff, pmap, ncol, s);
  launch_rename_bin<32>(desc, bin_base[BIN_G32], bin_count[BIN_G32], gid_of, gbase, gcol, coff, pmap, ncol, s);
  launch_rename_bin<16>(desc, bin_base[BIN_G16], bin_count[BIN_G16], gid_of, gbase, gcol, coff, pmap, ncol, s);
  launch_rename_bin<8>(desc, bin_base[BIN_G8], bin_count[BIN_G8], gid_of, gbase, gcol, coff, pmap, ncol, s);
  launch_rename_bin<4>(desc, bin_base[BIN_G4], bin_count[BIN_G4], gid_of, gbase, gcol, coff, pmap, ncol, s);
  return hipGetLastError();
}

}  // namespace katz
