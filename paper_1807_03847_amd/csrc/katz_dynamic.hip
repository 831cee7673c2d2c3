// Kernels of the dynamic update (Section 4, Algorithm 2).
//
// The state keeps the graph as a CSR with per-row slack: row v occupies
// pool[row_off[v] .. row_off[v] + row_cap[v]) with its row_len[v] arcs sorted
// at the front.  A batch of edge insertions I and deletions D is applied as a
// sorted merge per touched row (in place when the new length fits the row's
// capacity, otherwise into a fresh region at the pool's end).
//
// Walk counts are then recomputed level by level over the affected set
// C_1 = touched rows, C_{i+1} = C_i u {w : w -> x, x in C_i} (the breadth-first
// search over the reverse graph of Algorithm 2; undirected graphs are their own
// reverse), with the same row kernels as the static walk step, so every
// recomputed entry is bitwise the value a static run on the new graph computes.
#include <algorithm>

#include "katz_device.h"

namespace katz {
namespace {

__device__ __forceinline__ long long slack_cap(long long len) { return len + max(2ll, len >> 3); }

template <class OffT>
__global__ void __launch_bounds__(kWG) slack_caps(const OffT* rp, long long n, int* row_len, int* row_cap,
                                                  long long* cap_ll) {
  const long long v = (long long)blockIdx.x * kWG + threadIdx.x;
  if (v >= n) return;
  const long long len = (long long)rp[v + 1] - (long long)rp[v];
  const long long cap = slack_cap(len);
  row_len[v] = (int)len;
  row_cap[v] = (int)cap;
  cap_ll[v] = cap;
}

// Device-wide exclusive scan in three phases: per-chunk sums, a one-block scan
// of the sums, per-chunk scans that start from their chunk offset.
constexpr int kScanPer = 16;
constexpr long long kScanChunk = (long long)kWG * kScanPer;

__global__ void __launch_bounds__(kWG) scan_chunk_sums(const long long* in, long long count, long long* sums) {
  const long long base = (long long)blockIdx.x * kScanChunk;
  long long acc = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const long long i = base + (long long)j * kWG + threadIdx.x;
    if (i < count) acc += in[i];
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ long long ws[kWG / kWave];
  if (lane_id() == 0) ws[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ void __launch_bounds__(kFinishThreads) scan_sums(long long* sums, long long nb, long long* total) {
  block_exclusive_scan_ll(sums, nb, total);
}

__global__ void __launch_bounds__(kWG) scan_chunk_apply(const long long* in, long long count, const long long* sums,
                                                        long long* out) {
  const long long base = (long long)blockIdx.x * kScanChunk;
  // Thread t owns elements base + t*kScanPer .. + kScanPer - 1 (contiguous).
  long long loc[kScanPer];
  long long acc = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const long long i = base + (long long)threadIdx.x * kScanPer + j;
    loc[j] = i < count ? in[i] : 0;
    acc += loc[j];
  }
  long long inc = acc;
  const int lane = lane_id();
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  __shared__ long long ws[kWG / kWave];
  if (lane == kWave - 1) ws[threadIdx.x / kWave] = inc;
  __syncthreads();
  long long before = sums[blockIdx.x] + inc - acc;
  for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) before += ws[w];
  for (int j = 0; j < kScanPer; ++j) {
    const long long i = base + (long long)threadIdx.x * kScanPer + j;
    if (i < count) out[i] = before;
    before += loc[j];
  }
}

// One wave per row: copy the caller's CSR row into the slack pool.
// Flattened passes over the positions of a row-partitioned array (the arcs of
// a CSR, the slots of a slack pool): wave w takes kFlatPer * kWave consecutive
// positions, lane l the positions c0 + q kWave + l, so every load and store
// instruction of the wave covers kWave consecutive positions whatever the row
// lengths (a hub row is spread over many waves, short rows share one).  A
// lane finds the row of its first position by a binary search over the row
// offsets and follows the rows forward from there.
constexpr int kFlatPer = 16;

template <class OffT>
__device__ __forceinline__ long long row_at(const OffT* off, long long rows, long long p) {
  long long lo = 0, hi = rows - 1;   // the last row i with off[i] <= p
  while (lo < hi) {
    const long long mid = (lo + hi + 1) >> 1;
    if ((long long)off[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

unsigned flat_blocks(long long positions) {
  const long long waves = (positions + (long long)kWave * kFlatPer - 1) / ((long long)kWave * kFlatPer);
  return (unsigned)std::max<long long>(1, (waves * kWave + kWG - 1) / kWG);
}

// Row v of the CSR copied to pool[row_off[v] ..].
template <class OffT>
__global__ void __launch_bounds__(kWG) copy_rows_to_pool(const OffT* rp, const int32_t* col, long long n,
                                                         long long nnz, const long long* row_off, int32_t* pool) {
  const long long c0 = ((long long)blockIdx.x * kWG + threadIdx.x) / kWave * ((long long)kWave * kFlatPer);
  if (c0 >= nnz) return;
  const int lane = lane_id();
  long long v = -1, start = 0, end = 0;
  for (int q = 0; q < kFlatPer; ++q) {
    const long long j = c0 + (long long)q * kWave + lane;
    if (j >= nnz) break;
    if (v < 0) {
      v = row_at(rp, n, j);
      start = (long long)rp[v];
      end = (long long)rp[v + 1];
    }
    while (j >= end && v + 1 < n) {
      ++v;
      start = end;
      end = (long long)rp[v + 1];
    }
    pool[row_off[v] + (j - start)] = col[j];
  }
}

// The checks a state needs of its CSR, one pass over the arcs: every column
// id in range, no self-loop, each row strictly ascending (sorted, no
// neighbour twice).  A 256-thread workgroup takes 4096 consecutive arcs,
// thread t the arcs c0 + q 256 + t; the starts of the rows they fall in are
// staged in the LDS (up to kStrictRows of them; a chunk that crosses more,
// through runs of empty rows, follows the rows forward per thread instead),
// and each arc finds its row there by a fixed-step binary search.  Offsets
// are checked by the binning pass; inconsistent ones cannot make this pass
// read out of bounds (rows stay in 0..n-1, arcs in 0..nnz-1) and flag the
// graph.
constexpr int kStrictThreads = 256;
constexpr int kStrictPer = 16;
constexpr int kStrictChunk = kStrictThreads * kStrictPer;
constexpr int kStrictRows = 2048;

template <class OffT>
__global__ void __launch_bounds__(kStrictThreads) check_rows_strict(const OffT* rp, const int32_t* col, long long n,
                                                                    long long nnz, RunScalars* sc) {
  __shared__ long long rel[kStrictRows];   // row starts of the chunk (absolute arc positions)
  __shared__ long long s_r0;
  __shared__ int s_rows;
  const long long c0 = (long long)blockIdx.x * kStrictChunk;
  if (c0 >= nnz) return;                   // uniform over the workgroup
  const int t = threadIdx.x;
  const long long c1 = (c0 + kStrictChunk < nnz ? c0 + kStrictChunk : nnz) - 1;
  if (t == 0) {
    const long long r0 = row_at(rp, n, c0);
    const long long r1 = row_at(rp, n, c1);
    s_r0 = r0;
    s_rows = r1 >= r0 ? (int)(r1 - r0 + 1 < kStrictRows + 1 ? r1 - r0 + 1 : kStrictRows + 1) : 1;
  }
  __syncthreads();
  const long long r0 = s_r0;
  const bool staged = s_rows <= kStrictRows;
  const int rows = staged ? s_rows : 0;
  for (int k = t; k < rows; k += kStrictThreads) rel[k] = (long long)rp[r0 + k];
  __syncthreads();
  bool bad = false;
  long long v = -1, start = 0, end = 0;   // the forward walk of an unstaged chunk
#pragma unroll 4
  for (int q = 0; q < kStrictPer; ++q) {
    const long long j = c0 + (long long)q * kStrictThreads + t;
    if (j > c1) break;
    long long row, rs, re;
    if (staged) {
      int lo = 0;   // the last staged row k with rel[k] <= j
#pragma unroll
      for (int step = kStrictRows / 2; step > 0; step >>= 1) {
        const int m = lo + step;
        if (m < rows && rel[m] <= j) lo = m;
      }
      row = r0 + lo;
      rs = rel[lo];
      re = lo + 1 < rows ? rel[lo + 1] : (long long)rp[row + 1];
    } else {
      if (v < 0) {
        v = row_at(rp, n, j);
        start = (long long)rp[v];
        end = (long long)rp[v + 1];
      }
      while (j >= end && v + 1 < n) {
        ++v;
        start = end;
        end = (long long)rp[v + 1];
      }
      row = v;
      rs = start;
      re = end;
    }
    const int32_t u = col[j];
    bad = bad || j < rs || j >= re || u < 0 || (long long)u >= n || (long long)u == row ||
          (j > rs && j > 0 && col[j - 1] >= u);
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(&sc->err, 1);
}
__device__ __forceinline__ long long lower_bound_i32(const int32_t* a, long long len, int32_t x) {
  long long lo = 0, hi = len;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// A renumbered state stores internal ids, each row sorted by the caller ids
// of its entries (the static order of that row's sum).  ext_of / int_of map
// internal <-> caller ids; null maps are the identity (a state in caller order).
__device__ __forceinline__ int32_t ext_or_id(const int32_t* ext_of, int32_t x) { return ext_of ? ext_of[x] : x; }

// First position in a row whose entry's caller id is not below e.
__device__ __forceinline__ long long lower_bound_ext(const int32_t* row, long long len, int32_t e,
                                                     const int32_t* ext_of) {
  long long lo = 0, hi = len;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (ext_or_id(ext_of, row[mid]) < e) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Inserted arcs must be absent and deleted arcs present (Section 4: I n E = {},
// D c E).  Pairs [0, n_ins) are insertions, [n_ins, n_ins + n_del) deletions,
// in caller ids.
__global__ void __launch_bounds__(kWG) batch_exist(const int32_t* a, const int32_t* b, long long n_ins,
                                                   long long total, const long long* row_off, const int* row_len,
                                                   const int32_t* pool, const int32_t* ext_of, const int32_t* int_of,
                                                   int* err) {
  const long long j = (long long)blockIdx.x * kWG + threadIdx.x;
  if (j >= total) return;
  const int32_t u = int_of ? int_of[a[j]] : a[j], v = b[j];
  const int32_t* row = pool + row_off[u];
  const long long len = row_len[u];
  const long long p = lower_bound_ext(row, len, v, ext_of);
  const bool found = p < len && ext_or_id(ext_of, row[p]) == v;
  if ((j < n_ins) == found) atomicOr(err, 1);
}

// Caller ids -> internal ids, in place.
__global__ void __launch_bounds__(kWG) map_ids(int32_t* ids, long long count, const int32_t* int_of) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < count) ids[i] = int_of[ids[i]];
}

// Renumbering of a new state: internal id i = position of the caller's row in
// the binned order (as in a static call); the slack capacities in internal order.
__global__ void __launch_bounds__(kWG) state_relabel(const RowDesc* desc, long long n, const int* row_cap,
                                                     int32_t* ext_of, int32_t* int_of, long long* cap_ll) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const int v = desc[i].row;
  ext_of[i] = v;
  int_of[v] = (int32_t)i;
  cap_ll[i] = row_cap[v];
}

// One wave per internal row i: the caller's row ext_of[i], entries renamed and
// kept in their order, copied to the internal pool.
// The renumbered slack CSR.  Pass 1, one thread per internal row i: its
// length and capacity, and where its old row starts (old row ext_of[i]).
template <class OffT>
__global__ void __launch_bounds__(kWG) rename_meta(const int32_t* ext_of, long long n, const OffT* off_old,
                                                   const int* len_old, const int* cap_old, int* len_new,
                                                   int* cap_new, long long* src_of) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const int v = ext_of[i];
  len_new[i] = len_old[v];
  cap_new[i] = cap_old[v];
  src_of[i] = (long long)off_old[v];
}

// Pass 2: a 256-thread workgroup takes 4096 consecutive slots of the new
// pool, thread t the slots c0 + q 256 + t (q = 0 .. 15), so each load and
// store instruction covers consecutive words.  Slot p lies in internal row i
// (off_new ascending; every capacity is at least 2, so a chunk touches at most
// 2050 rows); the first len_new[i] slots of a row take the old row's entries
// renamed through int_of, the rest stay free.  The chunk's row starts are
// staged in the LDS, each slot finds its row there by a fixed-step binary
// search, and the loads of the sixteen slots of a thread are issued phase by
// phase (row data, old entries, renaming gathers), none waiting on another
// slot's.
constexpr int kRenameThreads = 256;
constexpr int kRenamePer = 16;
constexpr int kRenameChunk = kRenameThreads * kRenamePer;
constexpr int kRenameRows = kRenameChunk / 2 + 2;

__global__ void __launch_bounds__(kRenameThreads) rename_slots(const long long* off_new, long long n,
                                                               long long used_new, const int* len_new,
                                                               const long long* src_of, const int32_t* pool_old,
                                                               const int32_t* int_of, int32_t* pool_new) {
  __shared__ int rel[kRenameRows];   // row starts of the chunk, relative to c0
  __shared__ long long s_r0;
  __shared__ int s_rows;
  const long long c0 = (long long)blockIdx.x * kRenameChunk;
  if (c0 >= used_new) return;        // uniform over the workgroup
  const int t = threadIdx.x;
  const long long c1 = (c0 + kRenameChunk < used_new ? c0 + kRenameChunk : used_new) - 1;
  if (t == 0) {
    const long long r0 = row_at(off_new, n, c0);
    const long long r1 = row_at(off_new, n, c1);
    s_r0 = r0;
    s_rows = (int)(r1 - r0 + 1);
  }
  __syncthreads();
  const long long r0 = s_r0;
  const int rows = s_rows < kRenameRows ? s_rows : kRenameRows;
  for (int k = t; k < rows; k += kRenameThreads) rel[k] = (int)(off_new[r0 + k] - c0);
  __syncthreads();
  int kk[kRenamePer], jj[kRenamePer];
#pragma unroll
  for (int q = 0; q < kRenamePer; ++q) {
    const int x = q * kRenameThreads + t;
    int lo = 0;   // the last row k with rel[k] <= x (rel[0] <= 0 <= x)
#pragma unroll
    for (int step = 2048; step > 0; step >>= 1) {
      const int m = lo + step;
      if (m < rows && rel[m] <= x) lo = m;
    }
    kk[q] = lo;
    jj[q] = x - rel[lo];
  }
  long long addr[kRenamePer];
#pragma unroll
  for (int q = 0; q < kRenamePer; ++q) {
    const bool in = c0 + q * kRenameThreads + t <= c1;
    const long long i = r0 + kk[q];
    const int len = in ? len_new[i] : 0;
    addr[q] = jj[q] < len ? src_of[i] + jj[q] : -1;
  }
  int32_t c[kRenamePer];
#pragma unroll
  for (int q = 0; q < kRenamePer; ++q) c[q] = addr[q] >= 0 ? pool_old[addr[q]] : -1;
#pragma unroll
  for (int q = 0; q < kRenamePer; ++q)
    if (c[q] >= 0) pool_new[c0 + q * kRenameThreads + t] = int_of[c[q]];
}
// Candidate lengths of the touched rows; marks them.
__global__ void __launch_bounds__(kWG) touched_lengths(const int32_t* rows, long long t, const int* delta,
                                                       const int* row_len, long long* new_len, uint8_t* mark) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= t) return;
  const int w = rows[i];
  new_len[i] = (long long)row_len[w] + delta[i];
  mark[w] = 1;
}

// Maximum row length after the batch: untouched rows as they are, touched rows
// at their candidate length.
__global__ void __launch_bounds__(kWG) max_len_after(const int* row_len, const uint8_t* mark, long long n,
                                                     const long long* new_len, long long t, int* out) {
  int m = 0;
  for (long long v = (long long)blockIdx.x * kWG + threadIdx.x; v < n; v += (long long)gridDim.x * kWG)
    if (!mark[v]) m = max(m, row_len[v]);
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < t; i += (long long)gridDim.x * kWG)
    m = max(m, (int)new_len[i]);
  __shared__ int wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, max(max(wm[0], wm[1]), max(wm[2], wm[3])));
}

__global__ void __launch_bounds__(kWG) unmark_rows(const int32_t* rows, long long t, uint8_t* mark) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < t) mark[rows[i]] = 0;
}

// One workgroup per touched row w: new row = (old row \ del) u ins, in caller-id
// order, written to scratch[sbase[i] ..].  ins and del hold caller ids, sorted
// per row; the row's entries are stored ids (internal in a renumbered state).
__global__ void __launch_bounds__(kWG) merge_rows(const int32_t* rows, const long long* ins_off, const int* ins_cnt,
                                                  const int32_t* ins_dst, const long long* del_off,
                                                  const int* del_cnt, const int32_t* del_dst,
                                                  const long long* sbase, const long long* row_off,
                                                  const int* row_len, const int32_t* pool, const int32_t* ext_of,
                                                  const int32_t* int_of, int32_t* scratch) {
  const long long i = blockIdx.x;
  const int w = rows[i];
  const int32_t* old = pool + row_off[w];
  const long long len = row_len[w];
  const int32_t* ins = ins_dst + ins_off[i];
  const int32_t* del = del_dst + del_off[i];
  const int ni = ins_cnt[i], nd = del_cnt[i];
  int32_t* out = scratch + sbase[i];
  for (long long j = threadIdx.x; j < len; j += kWG) {
    const int32_t x = old[j];
    const int32_t e = ext_or_id(ext_of, x);
    const long long pd = lower_bound_i32(del, nd, e);
    if (pd < nd && del[pd] == e) continue;
    const long long pi = lower_bound_i32(ins, ni, e);
    out[j - pd + pi] = x;
  }
  for (int j = threadIdx.x; j < ni; j += kWG) {
    const int32_t e = ins[j];
    const long long po = lower_bound_ext(old, len, e, ext_of);
    const long long pd = lower_bound_i32(del, nd, e);
    out[j + po - pd] = int_of ? int_of[e] : e;
  }
}

__global__ void __launch_bounds__(kWG) copy_back_rows(const int32_t* rows, const long long* sbase,
                                                      const long long* new_len, const long long* dest_off,
                                                      const int* dest_cap, const int32_t* scratch,
                                                      long long* row_off, int* row_len, int* row_cap,
                                                      int32_t* pool) {
  const long long i = blockIdx.x;
  const int w = rows[i];
  const long long len = new_len[i];
  const long long dst = dest_off[i];
  for (long long j = threadIdx.x; j < len; j += kWG) pool[dst + j] = scratch[sbase[i] + j];
  if (threadIdx.x == 0) {
    row_off[w] = dst;
    row_len[w] = (int)len;
    row_cap[w] = dest_cap[i];
  }
}

// Breadth-first expansion over the frontier's arcs, flattened: flen holds the
// frontier rows' lengths, turned into their exclusive scan foff (total: their
// sum) before the expansion.  Thread t of a chunk takes kExpandPer consecutive
// arcs (one binary search for the row of its first arc, then a walk forward);
// every neighbour not yet in C joins C at `level` and the next frontier.  The
// appends and the arc count of the new frontier (the arcs its own expansion
// will scan) are aggregated per workgroup: one atomic each per chunk.  The
// earlier design gave every frontier row sixteen waves and every wave its own
// atomics; on serving batches of R-MAT 24 that cost 2.6 ms per expansion.
constexpr int kExpandPer = 8;
constexpr long long kExpandChunk = (long long)kWG * kExpandPer;

__global__ void __launch_bounds__(kWG) frontier_lengths(const int32_t* frontier, long long f, const int* row_len,
                                                        long long* flen) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < f) flen[i] = row_len[frontier[i]];
}

__global__ void __launch_bounds__(kWG) frontier_expand(const int32_t* frontier, long long f, const long long* foff,
                                                       const long long* total, const long long* row_off,
                                                       const int* row_len, const int32_t* pool, int* level_of,
                                                       int level, int32_t* next, int* next_count,
                                                       unsigned long long* next_arcs) {
  __shared__ int s_cnt[kWG / kWave];
  __shared__ unsigned long long s_arcs[kWG / kWave];
  __shared__ int s_base;
  const long long T = *total;
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  // The trip count is uniform per workgroup (it depends on blockIdx only).
  for (long long c0 = (long long)blockIdx.x * kExpandChunk; c0 < T; c0 += (long long)gridDim.x * kExpandChunk) {
    const long long a0 = c0 + (long long)threadIdx.x * kExpandPer;
    int32_t uu[kExpandPer];
    unsigned mask = 0;
    unsigned long long arcs = 0;
    if (a0 < T) {
      long long lo = 0, hi = f - 1;   // the last frontier row starting at or before a0
      while (lo < hi) {
        const long long mid = (lo + hi + 1) >> 1;
        if (foff[mid] <= a0) lo = mid;
        else hi = mid - 1;
      }
      long long i = lo;
      long long start = foff[i];
      long long end = i + 1 < f ? foff[i + 1] : T;
      const int32_t* row = pool + row_off[frontier[i]];
#pragma unroll
      for (int k = 0; k < kExpandPer; ++k) {
        const long long a = a0 + k;
        uu[k] = 0;
        if (a < T) {
          while (a >= end) {   // rows of length 0 are skipped
            ++i;
            start = end;
            end = i + 1 < f ? foff[i + 1] : T;
            row = pool + row_off[frontier[i]];
          }
          const int32_t u = row[a - start];
          uu[k] = u;
          // Most neighbours of a large frontier are in C already: a plain read
          // skips the atomic for them (a stale 0 only costs the atomic).
          if (level_of[u] == 0 && atomicCAS(&level_of[u], 0, level) == 0) {
            mask |= 1u << k;
            arcs += (unsigned long long)row_len[u];
          }
        }
      }
    }
    const int nf = __popc(mask);
    int inc = nf;
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    for (int o = 32; o >= 1; o >>= 1) arcs += __shfl_xor(arcs, o);
    if (lane == kWave - 1) s_cnt[wid] = inc;
    if (lane == 0) s_arcs[wid] = arcs;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
      s_base = tot ? atomicAdd(next_count, tot) : 0;
      const unsigned long long at = s_arcs[0] + s_arcs[1] + s_arcs[2] + s_arcs[3];
      if (at) atomicAdd(next_arcs, at);
    }
    __syncthreads();
    int pos = s_base + inc - nf;
    for (int w = 0; w < wid; ++w) pos += s_cnt[w];
#pragma unroll
    for (int k = 0; k < kExpandPer; ++k)
      if (mask >> k & 1u) next[pos++] = uu[k];
    __syncthreads();   // s_cnt / s_base are rewritten by the next chunk
  }
}

__global__ void __launch_bounds__(kWG) set_levels(const int32_t* rows, long long t, int* level_of, int level) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < t) level_of[rows[i]] = level;
}

__global__ void __launch_bounds__(kWG) clear_levels(const int32_t* rows, long long t, int* level_of) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < t) level_of[rows[i]] = 0;
}

// c(w) = x_1(w) + x_2(w) + ... + x_r(w), accumulated in the static order.
__global__ void __launch_bounds__(kWG) c_from_history(const int32_t* rows, long long count, double* const* X,
                                                      int r, double* c) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  const int w = rows ? rows[i] : (int)i;
  double acc = X[1][w];
  for (int l = 2; l <= r; ++l) acc = acc + X[l][w];
  c[w] = acc;
}

__global__ void __launch_bounds__(kWG) max_of_vector(const double* x, long long n, unsigned long long* out) {
  double m = 0.0;
  for (long long v = (long long)blockIdx.x * kWG + threadIdx.x; v < n; v += (long long)gridDim.x * kWG)
    m = fmax(m, x[v]);
  __shared__ double wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(out, (unsigned long long)__double_as_longlong(fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]))));
}

// FP32 form (Section 3.3): the walk epilogue of level i adds s_i = sigma_i x~_i
// to c and raises the margin e by eta'_i s_i (rounded upward); recomputed here
// for the re-walked rows with the same operations in the same order, so a row
// ends with the bits a walk over the whole history would give it.
__global__ void __launch_bounds__(kWG) c_from_history_f32(const int32_t* rows, long long count, float* const* X,
                                                          const double* sigma, const double* etap, int r,
                                                          double* c, float* e) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  const int w = rows ? rows[i] : (int)i;
  double acc = 0.0;
  float m = 0.0f;
  for (int l = 1; l <= r; ++l) {
    const double s = sigma[l] * (double)X[l][w];
    const double e_prev = (l == 1) ? 0.0 : (double)m;
    acc = (l == 1) ? s : acc + s;
    m = __double2float_ru((e_prev + etap[l] * s) * (1.0 + 0x1p-50));
  }
  c[w] = acc;
  e[w] = m;
}

__global__ void __launch_bounds__(kWG) max_of_vector_f32(const float* x, long long n, unsigned* out) {
  float m = 0.0f;
  for (long long v = (long long)blockIdx.x * kWG + threadIdx.x; v < n; v += (long long)gridDim.x * kWG)
    m = fmaxf(m, x[v]);
  __shared__ float wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

// min over the active list of the lower bound (as non-negative IEEE bits).
__global__ void __launch_bounds__(kWG) min_lower_active(BoundArgs b, const int32_t* act, const int* m_ptr,
                                                        unsigned long long* out, uint8_t* mark) {
  const int m = *m_ptr;
  unsigned long long best = ~0ull;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < m; i += (long long)gridDim.x * kWG) {
    const int v = act[i];
    double lo, up;
    bound_eval(b, v, lo, up);
    best = min(best, key_of(lo));
    mark[v] = 1;
  }
  __shared__ unsigned long long wm[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long y = __shfl_xor(best, o);
    best = min(best, y);
  }
  if (lane_id() == 0) wm[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) atomicMin(out, min(min(wm[0], wm[1]), min(wm[2], wm[3])));
}

// Reactivation (Algorithm 2): M <- M u {w : u(w) >= min_{x in M} l(x) - eps}.
__global__ void __launch_bounds__(kWG) reactivate(BoundArgs b, long long n, const unsigned long long* min_bits,
                                                  uint8_t* mark, int32_t* out, int* count) {
  const double thr = __longlong_as_double((long long)*min_bits) - b.eps;
  constexpr int IPT = 8;
  const long long group = (long long)kWG * IPT;
  for (long long g0 = (long long)blockIdx.x * group; g0 < n; g0 += (long long)gridDim.x * group) {
    unsigned mask = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const long long v = g0 + (long long)j * kWG + threadIdx.x;
      if (v >= n) continue;
      bool keep;
      if (mark[v]) {
        keep = true;
        mark[v] = 0;
      } else {
        double lo, up;
        bound_eval(b, (int)v, lo, up);
        keep = up >= thr;
      }
      if (keep) mask |= 1u << j;
    }
    int pos = block_reserve(count, mask);
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      if (mask >> j & 1u) out[pos++] = (int)(g0 + (long long)j * kWG + threadIdx.x);
  }
}

__global__ void __launch_bounds__(kWG) gather_int(const int32_t* rows, long long t, const int* src, int* out) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < t) out[i] = src[rows[i]];
}

__global__ void __launch_bounds__(kWG) gather_ll(const int32_t* rows, long long t, const long long* src,
                                                 long long* out) {
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  if (i < t) out[i] = src[rows[i]];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static unsigned blocks_for(long long count, int per_block = kWG) {
  return (unsigned)std::max<long long>(1, (count + per_block - 1) / per_block);
}

hipError_t launch_scan_ll(const long long* in, long long count, long long* out, long long* sums,
                          long long* total, hipStream_t s) {
  const long long nb = std::max<long long>(1, (count + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(scan_chunk_sums, dim3((unsigned)nb), dim3(kWG), 0, s, in, count, sums);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kFinishThreads), 0, s, sums, nb, total);
  hipLaunchKernelGGL(scan_chunk_apply, dim3((unsigned)nb), dim3(kWG), 0, s, in, count, (const long long*)sums, out);
  return hipGetLastError();
}

long long scan_sums_capacity(long long count) { return std::max<long long>(1, (count + kScanChunk - 1) / kScanChunk); }

hipError_t launch_slack_caps(const void* rp, int rp64, long long n, int* row_len, int* row_cap, long long* cap_ll,
                             hipStream_t s) {
  if (rp64)
    hipLaunchKernelGGL(slack_caps<int64_t>, dim3(blocks_for(n)), dim3(kWG), 0, s, (const int64_t*)rp, n, row_len,
                       row_cap, cap_ll);
  else
    hipLaunchKernelGGL(slack_caps<int32_t>, dim3(blocks_for(n)), dim3(kWG), 0, s, (const int32_t*)rp, n, row_len,
                       row_cap, cap_ll);
  return hipGetLastError();
}

hipError_t launch_copy_rows_to_pool(const void* rp, int rp64, const int32_t* col, long long n, long long nnz,
                                    const long long* row_off, int32_t* pool, hipStream_t s) {
  if (n <= 0 || nnz <= 0) return hipSuccess;
  const unsigned nb = flat_blocks(nnz);
  if (rp64)
    hipLaunchKernelGGL(copy_rows_to_pool<int64_t>, dim3(nb), dim3(kWG), 0, s, (const int64_t*)rp, col, n, nnz,
                       row_off, pool);
  else
    hipLaunchKernelGGL(copy_rows_to_pool<int32_t>, dim3(nb), dim3(kWG), 0, s, (const int32_t*)rp, col, n, nnz,
                       row_off, pool);
  return hipGetLastError();
}

hipError_t launch_check_rows_strict(const void* rp, int rp64, const int32_t* col, long long n, long long nnz,
                                    RunScalars* sc, hipStream_t s) {
  if (n <= 0 || nnz <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((nnz + kStrictChunk - 1) / kStrictChunk);
  if (rp64)
    hipLaunchKernelGGL(check_rows_strict<int64_t>, dim3(nb), dim3(kStrictThreads), 0, s, (const int64_t*)rp, col, n,
                       nnz, sc);
  else
    hipLaunchKernelGGL(check_rows_strict<int32_t>, dim3(nb), dim3(kStrictThreads), 0, s, (const int32_t*)rp, col, n,
                       nnz, sc);
  return hipGetLastError();
}

hipError_t launch_map_ids(int32_t* ids, long long count, const int32_t* int_of, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(map_ids, dim3(blocks_for(count)), dim3(kWG), 0, s, ids, count, int_of);
  return hipGetLastError();
}

hipError_t launch_state_relabel(const RowDesc* desc, long long n, const int* row_cap, int32_t* ext_of,
                               int32_t* int_of, long long* cap_ll, hipStream_t s) {
  hipLaunchKernelGGL(state_relabel, dim3(blocks_for(n)), dim3(kWG), 0, s, desc, n, row_cap, ext_of, int_of, cap_ll);
  return hipGetLastError();
}

hipError_t launch_state_rename_rows(const int32_t* ext_of, const int32_t* int_of, long long n,
                                   const void* off_old, int off64, const int* len_old, const int* cap_old,
                                   const int32_t* pool_old, const long long* off_new, long long used_new,
                                   int* len_new, int* cap_new, int32_t* pool_new, long long* src_of, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (off64)
    hipLaunchKernelGGL(rename_meta<long long>, dim3(blocks_for(n)), dim3(kWG), 0, s, ext_of, n,
                       (const long long*)off_old, len_old, cap_old, len_new, cap_new, src_of);
  else
    hipLaunchKernelGGL(rename_meta<int>, dim3(blocks_for(n)), dim3(kWG), 0, s, ext_of, n, (const int*)off_old,
                       len_old, cap_old, len_new, cap_new, src_of);
  if (used_new > 0)
    hipLaunchKernelGGL(rename_slots, dim3((unsigned)((used_new + kRenameChunk - 1) / kRenameChunk)),
                       dim3(kRenameThreads), 0, s, off_new, n, used_new, len_new, src_of, pool_old, int_of, pool_new);
  return hipGetLastError();
}

hipError_t launch_batch_exist(const int32_t* a, const int32_t* b, long long n_ins, long long total,
                              const long long* row_off, const int* row_len, const int32_t* pool,
                              const int32_t* ext_of, const int32_t* int_of, int* err, hipStream_t s) {
  if (total > 0)
    hipLaunchKernelGGL(batch_exist, dim3(blocks_for(total)), dim3(kWG), 0, s, a, b, n_ins, total, row_off, row_len,
                       pool, ext_of, int_of, err);
  return hipGetLastError();
}

hipError_t launch_touched_lengths(const int32_t* rows, long long t, const int* delta, const int* row_len,
                                  long long* new_len, uint8_t* mark, hipStream_t s) {
  hipLaunchKernelGGL(touched_lengths, dim3(blocks_for(t)), dim3(kWG), 0, s, rows, t, delta, row_len, new_len, mark);
  return hipGetLastError();
}

hipError_t launch_max_len_after(const int* row_len, const uint8_t* mark, long long n, const long long* new_len,
                                long long t, int* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(n), 512);
  hipLaunchKernelGGL(max_len_after, dim3(nb), dim3(kWG), 0, s, row_len, mark, n, new_len, t, out);
  return hipGetLastError();
}

hipError_t launch_unmark_rows(const int32_t* rows, long long t, uint8_t* mark, hipStream_t s) {
  hipLaunchKernelGGL(unmark_rows, dim3(blocks_for(t)), dim3(kWG), 0, s, rows, t, mark);
  return hipGetLastError();
}

hipError_t launch_merge_rows(const int32_t* rows, long long t, const long long* ins_off, const int* ins_cnt,
                             const int32_t* ins_dst, const long long* del_off, const int* del_cnt,
                             const int32_t* del_dst, const long long* sbase, const long long* row_off,
                             const int* row_len, const int32_t* pool, const int32_t* ext_of, const int32_t* int_of,
                             int32_t* scratch, hipStream_t s) {
  if (t > 0)
    hipLaunchKernelGGL(merge_rows, dim3((unsigned)t), dim3(kWG), 0, s, rows, ins_off, ins_cnt, ins_dst, del_off,
                       del_cnt, del_dst, sbase, row_off, row_len, pool, ext_of, int_of, scratch);
  return hipGetLastError();
}

hipError_t launch_copy_back_rows(const int32_t* rows, long long t, const long long* sbase, const long long* new_len,
                                 const long long* dest_off, const int* dest_cap, const int32_t* scratch,
                                 long long* row_off, int* row_len, int* row_cap, int32_t* pool, hipStream_t s) {
  if (t > 0)
    hipLaunchKernelGGL(copy_back_rows, dim3((unsigned)t), dim3(kWG), 0, s, rows, sbase, new_len, dest_off, dest_cap,
                       scratch, row_off, row_len, row_cap, pool);
  return hipGetLastError();
}

hipError_t launch_frontier_expand(const int32_t* frontier, long long f, const long long* row_off, const int* row_len,
                                  const int32_t* pool, int* level_of, int level, int32_t* next, int* next_count,
                                  unsigned long long* next_arcs, long long* foff, long long* sums, long long* total,
                                  unsigned long long arcs_hint, hipStream_t s) {
  if (f <= 0) return hipSuccess;
  hipLaunchKernelGGL(frontier_lengths, dim3(blocks_for(f)), dim3(kWG), 0, s, frontier, f, row_len, foff);
  const hipError_t e = launch_scan_ll(foff, f, foff, sums, total, s);
  if (e != hipSuccess) return e;
  // Grid-stride chunks: sized from the host's estimate of the arcs (0: not
  // known), at most 2048 workgroups; the kernel reads the exact total.
  const long long est = arcs_hint ? (long long)arcs_hint : 2048 * kExpandChunk;
  const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(2048, (est + kExpandChunk - 1) / kExpandChunk));
  hipLaunchKernelGGL(frontier_expand, dim3(grid), dim3(kWG), 0, s, frontier, f, (const long long*)foff,
                     (const long long*)total, row_off, row_len, pool, level_of, level, next, next_count, next_arcs);
  return hipGetLastError();
}

hipError_t launch_set_levels(const int32_t* rows, long long t, int* level_of, int level, hipStream_t s) {
  if (t > 0) hipLaunchKernelGGL(set_levels, dim3(blocks_for(t)), dim3(kWG), 0, s, rows, t, level_of, level);
  return hipGetLastError();
}

hipError_t launch_clear_levels(const int32_t* rows, long long t, int* level_of, hipStream_t s) {
  if (t > 0) hipLaunchKernelGGL(clear_levels, dim3(blocks_for(t)), dim3(kWG), 0, s, rows, t, level_of);
  return hipGetLastError();
}

hipError_t launch_c_from_history(const int32_t* rows, long long count, double* const* X, int r, double* c,
                                 hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(c_from_history, dim3(blocks_for(count)), dim3(kWG), 0, s, rows, count, X, r, c);
  return hipGetLastError();
}

hipError_t launch_max_of_vector(const double* x, long long n, unsigned long long* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(n), 512);
  hipLaunchKernelGGL(max_of_vector, dim3(nb), dim3(kWG), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_c_from_history_f32(const int32_t* rows, long long count, float* const* X, const double* sigma,
                                     const double* etap, int r, double* c, float* e, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(c_from_history_f32, dim3(blocks_for(count)), dim3(kWG), 0, s, rows, count, X, sigma, etap, r,
                       c, e);
  return hipGetLastError();
}

hipError_t launch_max_of_vector_f32(const float* x, long long n, unsigned* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(n), 512);
  hipLaunchKernelGGL(max_of_vector_f32, dim3(nb), dim3(kWG), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_min_lower_active(const BoundArgs& b, const int32_t* act, const int* m_ptr,
                                   unsigned long long* min_bits, uint8_t* mark, long long n, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(n), 512);
  hipLaunchKernelGGL(min_lower_active, dim3(nb), dim3(kWG), 0, s, b, act, m_ptr, min_bits, mark);
  return hipGetLastError();
}

hipError_t launch_reactivate_all(const BoundArgs& b, long long n, const unsigned long long* min_bits,
                                 uint8_t* mark, int32_t* out, int* count, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>(blocks_for(n), 2048);
  hipLaunchKernelGGL(reactivate, dim3(nb), dim3(kWG), 0, s, b, n, min_bits, mark, out, count);
  return hipGetLastError();
}

hipError_t launch_gather_int(const int32_t* rows, long long t, const int* src, int* out, hipStream_t s) {
  if (t > 0) hipLaunchKernelGGL(gather_int, dim3(blocks_for(t)), dim3(kWG), 0, s, rows, t, src, out);
  return hipGetLastError();
}

hipError_t launch_gather_ll(const int32_t* rows, long long t, const long long* src, long long* out, hipStream_t s) {
  if (t > 0) hipLaunchKernelGGL(gather_ll, dim3(blocks_for(t)), dim3(kWG), 0, s, rows, t, src, out);
  return hipGetLastError();
}

}  // namespace katz
