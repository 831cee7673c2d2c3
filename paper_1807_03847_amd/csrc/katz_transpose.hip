// The reverse graph on the device.  Inbound Katz centrality counts the walks
// that end at a node, which are the outbound walks of the reverse graph
// (Section 2.1), and Algorithm 2's breadth-first search runs over reverse arcs
// (Section 4): both need the transpose of a CSR.
//
// The transpose is a stable least-significant-digit radix sort of the arcs by
// target, with the source as payload.  The arcs enter in source order (CSR
// order), so every reversed row lists its sources in ascending order
// (repeated arcs kept, in input order) and the result does not depend on
// scheduling: a run on the reverse graph sums each row in a fixed order.
//
// One pass over digit d of the target ids:
//   radix_count    tile t of kTile arcs: how many carry each digit value;
//                  stored digit-major, count[v * tiles + t];
//   (scan)         an exclusive scan of count gives every (value, tile) its
//                  first output slot;
//   radix_scatter  each tile orders its arcs by digit in LDS, input order
//                  kept: round j takes arcs j*kRadixWG .. of the tile, waves
//                  find their lanes' ranks among equal digits with ballots,
//                  and per-value running counts carry the order across waves
//                  and rounds; the tile then leaves in that order, each
//                  value's arcs as one contiguous run.
// Afterwards row_starts turns the sorted targets into the row offsets.
#include <algorithm>

#include "katz_device.h"

namespace katz {
namespace {

constexpr int kRadixMaxBits = 8;
constexpr int kRadixBins = 1 << kRadixMaxBits;
constexpr int kRadixWG = 1024;                               // threads of the radix kernels
constexpr int kRadixWaves = kRadixWG / kWave;
constexpr int kTileRounds = 6;                               // 6144-arc tiles: two workgroups per CU fit the LDS
constexpr long long kTile = (long long)kRadixWG * kTileRounds;   // arcs per tile
constexpr int kExpandPer = 16;                              // arcs per thread of expand_sources

// src[j] = the row of arc j.  A 256-thread workgroup takes 4096 consecutive
// arcs, thread t the arcs c0 + q 256 + t (each store instruction covers
// consecutive arcs).  The starts of the rows the chunk crosses are staged in
// the LDS (up to kExpandRows of them) and each arc finds its row there by a
// fixed-step binary search; a chunk that crosses more rows (runs of empty
// rows) follows the rows forward per thread from a binary search over the
// offsets.
constexpr int kExpandThreads = 256;
constexpr int kExpandChunk = kExpandThreads * kExpandPer;
constexpr int kExpandRows = 2048;

template <class OffT>
__device__ __forceinline__ long long last_row_at_or_before(const OffT* rp, long long n, long long j) {
  long long lo = 0, hi = n - 1;   // the last row v with rp[v] <= j
  while (lo < hi) {
    const long long mid = (lo + hi + 1) >> 1;
    if ((long long)rp[mid] <= j) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class OffT>
__global__ void __launch_bounds__(kExpandThreads) expand_sources(const OffT* rp, long long n, long long nnz,
                                                                 int32_t* src) {
  __shared__ long long rel[kExpandRows];
  __shared__ long long s_r0;
  __shared__ int s_rows;
  const long long c0 = (long long)blockIdx.x * kExpandChunk;
  if (c0 >= nnz) return;   // uniform over the workgroup
  const int t = threadIdx.x;
  const long long c1 = (c0 + kExpandChunk < nnz ? c0 + kExpandChunk : nnz) - 1;
  if (t == 0) {
    const long long r0 = last_row_at_or_before(rp, n, c0);
    const long long r1 = last_row_at_or_before(rp, n, c1);
    s_r0 = r0;
    s_rows = (int)(r1 - r0 + 1 < kExpandRows + 1 ? r1 - r0 + 1 : kExpandRows + 1);
  }
  __syncthreads();
  const long long r0 = s_r0;
  const bool staged = s_rows <= kExpandRows;
  const int rows = staged ? s_rows : 0;
  for (int k = t; k < rows; k += kExpandThreads) rel[k] = (long long)rp[r0 + k];
  __syncthreads();
  if (staged) {
#pragma unroll 4
    for (int q = 0; q < kExpandPer; ++q) {
      const long long j = c0 + (long long)q * kExpandThreads + t;
      if (j > c1) break;
      int lo = 0;   // the last staged row k with rel[k] <= j
#pragma unroll
      for (int step = kExpandRows / 2; step > 0; step >>= 1) {
        const int m = lo + step;
        if (m < rows && rel[m] <= j) lo = m;
      }
      src[j] = (int32_t)(r0 + lo);
    }
  } else {
    long long v = -1, end = 0;
    for (int q = 0; q < kExpandPer; ++q) {
      const long long j = c0 + (long long)q * kExpandThreads + t;
      if (j > c1) break;
      if (v < 0) {
        v = last_row_at_or_before(rp, n, j);
        end = (long long)rp[v + 1];
      }
      while (j >= end) {   // empty rows are skipped
        ++v;
        end = (long long)rp[v + 1];
      }
      src[j] = (int32_t)v;
    }
  }
}

__device__ __forceinline__ unsigned digit_of(int32_t key, int shift, unsigned mask) {
  return ((unsigned)key >> shift) & mask;
}

__global__ void __launch_bounds__(kRadixWG) radix_count(const int32_t* key, long long nnz, int shift, int bits,
                                                        long long tiles, long long* count) {
  __shared__ unsigned h[kRadixBins];
  const unsigned mask = (1u << bits) - 1u;
  for (int d = threadIdx.x; d < kRadixBins; d += kRadixWG) h[d] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kTile;
  // Every key of the thread is loaded before the first count, so the tile's
  // loads are in flight together.
  int32_t kr[kTileRounds];
#pragma unroll
  for (int j = 0; j < kTileRounds; ++j) {
    const long long i = base + (long long)j * kRadixWG + threadIdx.x;
    kr[j] = i < nnz ? key[i] : -1;
  }
#pragma unroll
  for (int j = 0; j < kTileRounds; ++j)
    if (kr[j] >= 0) atomicAdd(&h[digit_of(kr[j], shift, mask)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d <= (int)mask; d += kRadixWG) count[(long long)d * tiles + blockIdx.x] = h[d];
}

// Places the tile's arcs at their sorted positions, stable.  first: the
// exclusive scan of count (first output slot of each (value, tile)).  The
// tile is first ordered by digit in LDS (input order kept inside a digit),
// then written out in that order, so each digit's arcs of the tile leave as
// one contiguous run instead of lane-by-lane scattered words.
__global__ void __launch_bounds__(kRadixWG) radix_scatter(const int32_t* key_in, const int32_t* val_in, long long nnz,
                                                          int shift, int bits, long long tiles,
                                                          const long long* first, int32_t* key_out,
                                                          int32_t* val_out) {
  extern __shared__ __align__(16) int32_t stage[];      // kTile keys, then kTile values
  int32_t* sk = stage;
  int32_t* sv = stage + kTile;
  __shared__ long long gbase[kRadixBins];                // global first slot of each value for this tile
  __shared__ int lbase[kRadixBins];                      // tile-local first slot of each value
  __shared__ int run[kRadixBins];                        // arcs of each value placed so far
  __shared__ int wcnt[kRadixWaves][kRadixBins];          // this round's count of each value per wave
  const unsigned mask = (1u << bits) - 1u;
  const int nvals = (int)mask + 1;
  const long long scanned = (long long)nvals * tiles;
  const int t = threadIdx.x;
  // This tile's count of value d is the step of the scan to the next entry.
  if (t < nvals) {
    const long long idx = (long long)t * tiles + blockIdx.x;
    const long long nxt = idx + 1 < scanned ? first[idx + 1] : nnz;
    gbase[t] = first[idx];
    lbase[t] = (int)(nxt - first[idx]);
    run[t] = 0;
  }
  __syncthreads();
  const int w = t / kWave;
  const int lane = lane_id();
  const long long tile0 = (long long)blockIdx.x * kTile;
  const int tile_len = (int)(nnz - tile0 < kTile ? nnz - tile0 : kTile);
  // The thread's keys and payloads of every round, loaded at once (their
  // latency is paid once per tile instead of once per round).
  int32_t kr[kTileRounds], vr[kTileRounds];
#pragma unroll
  for (int j = 0; j < kTileRounds; ++j) {
    const int li = j * kRadixWG + t;
    kr[j] = li < tile_len ? key_in[tile0 + li] : 0;
    vr[j] = li < tile_len ? val_in[tile0 + li] : 0;
  }
  if (w == 0) {   // exclusive scan of the tile's counts: four values per lane, then the wave
    int c[kRadixBins / kWave];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < kRadixBins / kWave; ++q) {
      const int d = lane * (kRadixBins / kWave) + q;
      c[q] = d < nvals ? lbase[d] : 0;
      sum += c[q];
    }
    int incl = sum;
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    int acc = incl - sum;
#pragma unroll
    for (int q = 0; q < kRadixBins / kWave; ++q) {
      const int d = lane * (kRadixBins / kWave) + q;
      if (d < nvals) lbase[d] = acc;
      acc += c[q];
    }
  }
  __syncthreads();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
  for (int j = 0; j < kTileRounds; ++j) {
    const int li = j * kRadixWG + t;
    const bool valid = li < tile_len;
    const int32_t k = kr[j], v = vr[j];
    const unsigned d = digit_of(k, shift, mask);
    // Lanes of this wave with the same digit: intersect the ballots of every
    // digit bit.
    unsigned long long same = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const unsigned long long on = __ballot((d >> b) & 1u);
      same &= ((d >> b) & 1u) ? on : ~on;
    }
    const int rank = __popcll(same & below);
    for (int x = t; x < kRadixWaves * kRadixBins; x += kRadixWG) (&wcnt[0][0])[x] = 0;
    __syncthreads();
    if (valid && rank == 0) wcnt[w][d] = __popcll(same);
    __syncthreads();
    if (valid) {
      int pos = lbase[d] + run[d] + rank;
      for (int u = 0; u < w; ++u) pos += wcnt[u][d];
      sk[pos] = k;
      sv[pos] = v;
    }
    __syncthreads();   // every lane has read run[] before it moves on
    if (t < nvals) {
      int add = 0;
      for (int u = 0; u < kRadixWaves; ++u) add += wcnt[u][t];
      run[t] += add;
    }
    __syncthreads();   // run[] updated before the next round reads it
  }
  // The tile in digit order: consecutive slots of one value go to
  // consecutive global positions.
  for (int li = t; li < tile_len; li += kRadixWG) {
    const int32_t k = sk[li];
    const unsigned d = digit_of(k, shift, mask);
    const long long pos = gbase[d] + (li - lbase[d]);
    key_out[pos] = k;
    val_out[pos] = sv[li];
  }
}

// Row offsets of the reverse graph from its sorted targets: rt_ptr[v] = the
// first position whose target is at least v.
__global__ void __launch_bounds__(kWG) row_starts(const int32_t* key, long long nnz, long long n, long long* rt_ptr) {
  const long long p = (long long)blockIdx.x * kWG + threadIdx.x;
  if (p > nnz) return;
  const long long lo = p == 0 ? 0 : (long long)key[p - 1] + 1;   // targets lo .. hi start at p
  const long long hi = p == nnz ? n : (long long)key[p];
  for (long long v = lo; v <= hi; ++v) rt_ptr[v] = p;
}

// Sets sc->err when a CSR differs from another (offsets or column ids).
template <class OffT>
__global__ void __launch_bounds__(kWG) csr_equal(const OffT* rp, const int32_t* col, const long long* rt_ptr,
                                                 const int32_t* rt_col, long long n, long long nnz, RunScalars* sc) {
  const long long stride = (long long)gridDim.x * kWG;
  bool bad = false;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i <= n; i += stride)
    bad = bad || (long long)rp[i] != rt_ptr[i];
  for (long long j = (long long)blockIdx.x * kWG + threadIdx.x; j < nnz; j += stride) bad = bad || col[j] != rt_col[j];
  if (bad) atomicOr(&sc->err, 1);
}

int bits_for(long long n) {
  int b = 1;
  while (b < 31 && (1ll << b) < n) ++b;
  return b;
}

}  // namespace

size_t transpose_scratch_bytes(long long n, long long nnz) {
  const long long tiles = std::max<long long>(1, (nnz + kTile - 1) / kTile);
  const long long table = (long long)kRadixBins * tiles;
  auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
  (void)n;
  return 3 * r((size_t)std::max<long long>(nnz, 1) * 4) + r((size_t)table * 8) +
         r((size_t)scan_sums_capacity(table) * 8) + r(8);
}

hipError_t launch_transpose(const void* rp, int rp64, const int32_t* col, long long n, long long nnz, void* scratch,
                            long long* rt_ptr, int32_t* rt_col, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nnz == 0) {
    return hipMemsetAsync(rt_ptr, 0, sizeof(long long) * (size_t)(n + 1), s);
  }
  const long long tiles = (nnz + kTile - 1) / kTile;
  const long long table = (long long)kRadixBins * tiles;
  auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* p = static_cast<char*>(scratch);
  int32_t* src = reinterpret_cast<int32_t*>(p);
  p += r((size_t)nnz * 4);
  int32_t* ka = reinterpret_cast<int32_t*>(p);
  p += r((size_t)nnz * 4);
  int32_t* kb = reinterpret_cast<int32_t*>(p);
  p += r((size_t)nnz * 4);
  long long* cnt = reinterpret_cast<long long*>(p);
  p += r((size_t)table * 8);
  long long* sums = reinterpret_cast<long long*>(p);
  p += r((size_t)scan_sums_capacity(table) * 8);
  long long* total = reinterpret_cast<long long*>(p);

  // Digit widths: the fewest passes of at most kRadixMaxBits bits, split evenly.
  const int total_bits = bits_for(n);
  const int passes = (total_bits + kRadixMaxBits - 1) / kRadixMaxBits;
  const int width = (total_bits + passes - 1) / passes;
  // Ping-pong buffers: pass q reads set (passes - q) & 1 and writes set
  // (passes - 1 - q) & 1, so the last pass leaves the payload in rt_col.  The
  // first pass reads its keys from col and its payload from the sources,
  // which are expanded into the set it reads.
  int32_t* vbuf[2] = {rt_col, src};
  int32_t* kbuf[2] = {ka, kb};
  const unsigned eg = (unsigned)((nnz + kExpandChunk - 1) / kExpandChunk);
  int32_t* src0 = vbuf[passes & 1];
  if (rp64)
    hipLaunchKernelGGL(expand_sources<long long>, dim3(eg), dim3(kExpandThreads), 0, s, (const long long*)rp, n, nnz,
                       src0);
  else hipLaunchKernelGGL(expand_sources<int>, dim3(eg), dim3(kExpandThreads), 0, s, (const int*)rp, n, nnz, src0);
  const int32_t* kin = col;
  const int32_t* vin = src0;
  int shift = 0;
  for (int q = 0; q < passes; ++q) {
    const int bits = std::min(width, total_bits - shift);
    const int set = (passes - 1 - q) & 1;
    int32_t* kout = kbuf[set];
    int32_t* vout = vbuf[set];
    hipLaunchKernelGGL(radix_count, dim3((unsigned)tiles), dim3(kRadixWG), 0, s, kin, nnz, shift, bits, tiles, cnt);
    const hipError_t e = launch_scan_ll(cnt, (long long)(1 << bits) * tiles, cnt, sums, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter, dim3((unsigned)tiles), dim3(kRadixWG), sizeof(int32_t) * 2 * kTile, s, kin,
                       vin, nnz, shift, bits, tiles, (const long long*)cnt, kout, vout);
    kin = kout;
    vin = vout;
    shift += bits;
  }
  const unsigned rg = (unsigned)((nnz + 1 + kWG - 1) / kWG);
  hipLaunchKernelGGL(row_starts, dim3(rg), dim3(kWG), 0, s, kin, nnz, n, rt_ptr);
  return hipGetLastError();
}

hipError_t launch_csr_equal(const void* rp, int rp64, const int32_t* col, const long long* rt_ptr,
                            const int32_t* rt_col, long long n, long long nnz, RunScalars* sc, hipStream_t s) {
  const long long work = std::max(n + 1, nnz);
  const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(4096, (work + kWG - 1) / kWG));
  if (rp64)
    hipLaunchKernelGGL(csr_equal<long long>, dim3(grid), dim3(kWG), 0, s, (const long long*)rp, col, rt_ptr, rt_col, n,
                       nnz, sc);
  else
    hipLaunchKernelGGL(csr_equal<int>, dim3(grid), dim3(kWG), 0, s, (const int*)rp, col, rt_ptr, rt_col, n, nnz, sc);
  return hipGetLastError();
}

}  // namespace katz
