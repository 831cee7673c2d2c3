// Device helpers shared by the kernel sources (inline, header-only).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "katz_internal.h"

namespace katz {

__host__ __device__ inline int bin_of_len(long long len, const BinBounds& bb) {
  return len <= 0 ? BIN_EMPTY
       : len <= bb.g4 ? BIN_G4
       : len <= bb.g8 ? BIN_G8
       : len <= bb.g16 ? BIN_G16
       : len <= bb.g32 ? BIN_G32
       : len <= bb.w16 ? BIN_W16
       : len <= bb.w64 ? BIN_W64
       : len <= kBlockRowMax ? BIN_B256
       : BIN_HUGE;
}


__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

// Wave-aggregated append: one atomic per wave.  Every lane of the wave must call it.
__device__ __forceinline__ int wave_append(int* counter, bool pred) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return -1;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return base + __popcll(mask & lanemask_lt());
}

// Histogram increment of a wave: h[d] += 1 for every lane with pred.  The
// lanes that share the first active lane's digit add with one LDS atomic (when
// keys share their leading digits, per-lane atomics would queue on one
// address); the others add one by one (spread digits do not collide).  Every
// lane of the wave must call it.
__device__ __forceinline__ void wave_hist_add(unsigned* h, unsigned d, bool pred) {
  const unsigned long long active = __ballot(pred);
  if (!active) return;
  const int leader = __ffsll((long long)active) - 1;
  const unsigned dl = __shfl(d, leader);
  const unsigned long long same = __ballot(pred && d == dl);
  if (lane_id() == leader) atomicAdd(&h[dl], (unsigned)__popcll(same));
  else if (pred && d != dl) atomicAdd(&h[d], 1u);
}

template <bool F32> struct Prec;
template <> struct Prec<false> { using T = double; };
template <> struct Prec<true> { using T = float; };

template <bool F32>
__device__ __forceinline__ typename Prec<F32>::T ldx(const void* x, int32_t j) {
  return reinterpret_cast<const typename Prec<F32>::T*>(x)[j];
}

// ---------------------------------------------------------------------------
// Bound evaluation (Section 3.1, Theorem 1).
//   FP64 form:  l = c + alpha s (undirected) or c;  u = c + beta s.
//   FP32 form:  s = sigma_r x~, with every rounding of the walk vector bounded
//               by the per-node accumulator e and the global factors; the
//               interval [lo, up] contains the exact l_r and u_r.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bound_eval(const BoundArgs& b, int v, double& lo, double& up) {
  const double cv = b.c[v];
  if (!b.fp32) {
    const double s = reinterpret_cast<const double*>(b.x)[v];
    lo = b.undirected ? cv + b.alpha * s : cv;
    up = cv + b.beta * s;
  } else {
    const double s = b.sigma[b.r] * (double)reinterpret_cast<const float*>(b.x)[v];
    const double down = (double)b.e[v] * b.f_e + b.tau_coef * b.sigma_sum[b.r];
    const double l = cv * b.f_lo_c + s * b.f_lo_s - down;
    lo = l > 0.0 ? l : 0.0;
    up = cv * b.f_hi_c + down + s * b.f_hi_s;
  }
}

// FP32 form: true while the part of the interval that further iterations
// shrink still exceeds 1/16 of the part they cannot shrink (rounding margin).
__device__ __forceinline__ bool can_progress(const BoundArgs& b, int v) {
  if (!b.fp32) return true;
  const double cv = b.c[v];
  const double s = b.sigma[b.r] * (double)reinterpret_cast<const float*>(b.x)[v];
  const double down = (double)b.e[v] * b.f_e + b.tau_coef * b.sigma_sum[b.r];
  const double intrinsic = s * (b.f_hi_s - b.f_lo_s);
  const double margin = 2.0 * down + 2.0 * b.kappa * cv;
  return intrinsic * 16.0 > margin;
}

__device__ __forceinline__ unsigned long long key_of(double lo) {
  return (unsigned long long)__double_as_longlong(lo);
}


// Exclusive scan of a long long array of length len with one 1024-thread block.
__device__ inline void block_exclusive_scan_ll(long long* a, long long len, long long* total_out) {
  __shared__ long long wsum[kFinishThreads / kWave];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int t = threadIdx.x;
  const int lane = lane_id();
  const int w = t / kWave;
  for (long long base = 0; base < len; base += kFinishThreads) {
    const long long i = base + t;
    long long x = i < len ? a[i] : 0;
    long long inc = x;
    for (int o = 1; o < kWave; o <<= 1) {
      long long y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
      long long ws = lane < kFinishThreads / kWave ? wsum[lane] : 0;
      long long wi = ws;
      for (int o = 1; o < kWave; o <<= 1) {
        long long y = __shfl_up(wi, o);
        if (lane >= o) wi += y;
      }
      if (lane < kFinishThreads / kWave) wsum[lane] = wi - ws;   // exclusive wave offsets
    }
    __syncthreads();
    const long long c0 = carry;
    if (i < len) a[i] = c0 + wsum[w] + inc - x;
    __syncthreads();
    if (t == kFinishThreads - 1) carry = c0 + wsum[w] + inc;
    __syncthreads();
  }
  if (t == 0 && total_out) *total_out = carry;
}


// Inside one 1024-thread block: the bucket of hist[0..nb) (nb <= 4096) that holds
// rank `need` (1-based), counting from the largest bucket (desc) or the
// smallest.  Thread t owns positions 4t..4t+3 of that order.
struct Bucket {
  int b;
  int need;   // rank inside the bucket
  int count;  // items in the bucket
};

__device__ inline Bucket find_bucket(const unsigned* h, int nb, int need, bool desc) {
  __shared__ long long wsum[kFinishThreads / kWave];
  __shared__ Bucket res;
  const int t = threadIdx.x;
  const int lane = lane_id();
  const int w = t / kWave;
  unsigned loc[4];
  long long tot = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pos = 4 * t + j;
    const int bin = desc ? nb - 1 - pos : pos;
    loc[j] = (pos < nb) ? h[bin] : 0u;
    tot += loc[j];
  }
  long long inc = tot;
  for (int o = 1; o < kWave; o <<= 1) {
    long long y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    long long ws = lane < kFinishThreads / kWave ? wsum[lane] : 0;
    long long wi = ws;
    for (int o = 1; o < kWave; o <<= 1) {
      long long y = __shfl_up(wi, o);
      if (lane >= o) wi += y;
    }
    if (lane < kFinishThreads / kWave) wsum[lane] = wi - ws;
  }
  __syncthreads();
  long long cum = wsum[w] + inc - tot;   // items before this thread's positions
  if (cum < need && need <= cum + tot) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (need <= cum + (long long)loc[j]) {
        const int pos = 4 * t + j;
        res.b = desc ? nb - 1 - pos : pos;
        res.need = (int)(need - cum);
        res.count = (int)loc[j];
        break;
      }
      cum += loc[j];
    }
  }
  __syncthreads();
  const Bucket r = res;
  __syncthreads();
  return r;
}

// Exclusive scan of one int per thread over a 256-thread workgroup; returns the
// thread's prefix and writes the total to *total (all threads).
__device__ inline int block_scan_256(int x, int* total) {
  __shared__ int ws[kWG / kWave];
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  int inc = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) ws[w] = inc;
  __syncthreads();
  int before = 0, all = 0;
  for (int i = 0; i < kWG / kWave; ++i) {
    if (i < w) before += ws[i];
    all += ws[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// Appends for a group of 256 x IPT items (IPT per thread): bit j of `mask` flags
// the thread's j-th item.  One atomic per workgroup reserves the group's slots;
// returns the thread's first slot (its flagged items take consecutive slots).
// Every thread of the workgroup must call it.
__device__ inline int block_reserve(int* counter, unsigned mask) {
  __shared__ int s_base;
  int total = 0;
  const int ex = block_scan_256(__popc(mask), &total);
  if (threadIdx.x == 0) s_base = total > 0 ? atomicAdd(counter, total) : 0;
  __syncthreads();
  const int base = s_base;
  __syncthreads();
  return base + ex;
}

// Binning kernels, shared by every row source (header-only templates; each
// kernel source instantiates its own copies).
namespace {
// ---------------------------------------------------------------------------
// Prep: per-block bin counts, maximum degree, CSR checks.
// blk layout: [NUM_BINS + 1][nblocks]; column NUM_BINS counts huge segments.
// ---------------------------------------------------------------------------
template <class Rows>
__global__ void __launch_bounds__(kWG) prep_count(Rows rows, long long count, long long* blk, int nblocks,
                                                  RunScalars* sc, BinBounds bb) {
  __shared__ int cnt[NUM_BINS + 1];
  if (threadIdx.x <= NUM_BINS) cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  int dmax = 0;
  bool bad = false;
  if (i < count) {
    int row;
    long long off, len;
    if (!rows.get(i, row, off, len)) {
      bad = true;
    } else {
      const int b = bin_of_len(len, bb);
      atomicAdd(&cnt[b], 1);
      if (b == BIN_HUGE) atomicAdd(&cnt[NUM_BINS], (int)((len + kSeg - 1) / kSeg));
      dmax = (int)len;
    }
  }
  if constexpr (Rows::kCsr) {
    if (i == 0 && ((long long)rows.rp[0] != 0 || (long long)rows.rp[count] != rows.nnz)) bad = true;
  }
  __shared__ int wmax[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o));
  if (lane_id() == 0) wmax[threadIdx.x / kWave] = dmax;
  if (bad) atomicOr(&sc->err, 1);
  __syncthreads();
  if (threadIdx.x <= NUM_BINS) blk[(long long)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
  // Column NUM_BINS + 1: the block's longest row (reduced by prep_finalize).
  if (threadIdx.x == 0)
    blk[(long long)(NUM_BINS + 1) * nblocks + blockIdx.x] = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
}

template <class Rows>
__global__ void __launch_bounds__(kWG) prep_scatter(Rows rows, long long count, const long long* blk,
                                                    int nblocks, RowDesc* desc, SegDesc* segs,
                                                    HugeRow* huge, RunScalars* sc, BinBounds bb) {
  if (sc->err) return;
  __shared__ int wcnt[NUM_BINS][kWG / kWave];
  __shared__ int wseg[kWG / kWave];
  const long long i = (long long)blockIdx.x * kWG + threadIdx.x;
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  long long off = 0, len = 0;
  int row = 0;
  int bin = -1;
  int nseg = 0;
  if (i < count) {
    rows.get(i, row, off, len);
    bin = bin_of_len(len, bb);
    if (bin == BIN_HUGE) nseg = (int)((len + kSeg - 1) / kSeg);
  }
  int rank_in_wave = 0;
  for (int b = 0; b < NUM_BINS; ++b) {
    const unsigned long long mask = __ballot(bin == b);
    if (bin == b) rank_in_wave = __popcll(mask & lanemask_lt());
    if (lane == 0) wcnt[b][w] = __popcll(mask);
  }
  // Segment offsets of huge rows inside the wave (inclusive scan of nseg).
  int sinc = nseg;
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(sinc, o);
    if (lane >= o) sinc += y;
  }
  if (lane == kWave - 1) wseg[w] = sinc;
  __syncthreads();
  if (i < count) {
    int before = 0;
    for (int ww = 0; ww < w; ++ww) before += wcnt[bin][ww];
    const long long pos = blk[(long long)bin * nblocks + blockIdx.x] + before + rank_in_wave;
    desc[pos] = RowDesc{off, (int32_t)row, (int32_t)len};
    if (bin == BIN_HUGE) {
      int sbefore = 0;
      for (int ww = 0; ww < w; ++ww) sbefore += wseg[ww];
      const long long part0 = blk[(long long)NUM_BINS * nblocks + blockIdx.x] + sbefore + sinc - nseg;
      const long long hidx = pos - sc->bin_base[BIN_HUGE];
      huge[hidx] = HugeRow{(int32_t)row, (int32_t)len, nseg, (int32_t)part0};
      for (int sg = 0; sg < nseg; ++sg) {
        const int slen = (int)min((long long)kSeg, len - (long long)sg * kSeg);
        segs[part0 + sg] = SegDesc{off + (long long)sg * kSeg, slen, (int32_t)(part0 + sg), (int32_t)hidx, 0};
      }
    }
  }
}

}  // namespace

}  // namespace katz
