// R-MAT input graphs built on the GPU (input data only; no Katz arithmetic).
//
// The same graph as sg_rmat in gen.cpp, bit for bit: the same counter-based
// draws (SplitMix64's finaliser over a Weyl sequence keyed by seed and stream,
// Steele, Lea, Flood, OOPSLA 2014), the same quadrant recursion (Chakrabarti,
// Zhan, Faloutsos, SDM 2004) and the same relabelling permutation (computed
// on the host by gen.cpp and passed in), then both arcs of every non-loop
// draw, sorted and deduplicated into canonical CSR.  The host build of scale
// 27 (2^31 draws, 4.3e9 arcs) takes minutes; here the arcs are packed into
// 64-bit keys (source << scale | target), sorted with a device radix sort and
// compacted, which takes seconds.
//
// Device memory: two key arrays of 8 bytes per arc before deduplication
// (34 GB each at scale 27) plus the sort's temporary storage, all freed when
// sg_gpu_rmat_finish has written the caller's arrays.
#include <hip/hip_runtime.h>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <cstdint>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr long long kChunk = (long long)kThreads * kPerThread;   // keys per compaction block

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t mix64_host(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Both arcs of draw i as keys (u << scale | v); a self-loop gives two copies
// of the sentinel n << scale, which sorts after every arc.
__global__ void __launch_bounds__(kThreads) rmat_keys(int scale, long long draws, uint64_t key, double a,
                                                      double ab, double abc, const int32_t* perm,
                                                      unsigned long long* keys) {
  const long long stride = (long long)gridDim.x * kThreads;
  const unsigned long long sentinel = (1ull << scale) << scale;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < draws; i += stride) {
    long long src = 0, dst = 0;
    const uint64_t c0 = (uint64_t)i * (uint64_t)scale;
    for (int l = 0; l < scale; ++l) {
      const double p = (double)(mix64(key + (c0 + (uint64_t)l + 1) * kGolden) >> 11) * (1.0 / 9007199254740992.0);
      const long long ge_a = p >= a, ge_ab = p >= ab, ge_abc = p >= abc;
      src = (src << 1) | ge_ab;
      dst = (dst << 1) | ((ge_a & (ge_ab ^ 1)) | ge_abc);
    }
    unsigned long long k0 = sentinel, k1 = sentinel;
    if (src != dst) {
      const unsigned long long u = perm ? (unsigned long long)perm[src] : (unsigned long long)src;
      const unsigned long long v = perm ? (unsigned long long)perm[dst] : (unsigned long long)dst;
      k0 = (u << scale) | v;
      k1 = (v << scale) | u;
    }
    keys[2 * i] = k0;
    keys[2 * i + 1] = k1;
  }
}

// Keys kept by the compaction: the first of each run of equal keys, never
// the sentinel.  counts[b] = kept keys of chunk b.
__global__ void __launch_bounds__(kThreads) count_kept(const unsigned long long* keys, long long total,
                                                       unsigned long long sentinel, unsigned long long* counts) {
  const long long base = (long long)blockIdx.x * kChunk;
  unsigned c = 0;
  for (int t = 0; t < kPerThread; ++t) {
    const long long j = base + (long long)t * kThreads + threadIdx.x;
    if (j < total) {
      const unsigned long long k = keys[j];
      c += (k != sentinel && (j == 0 || keys[j - 1] != k)) ? 1u : 0u;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
  __shared__ unsigned ws[kThreads / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (unsigned long long)ws[0] + ws[1] + ws[2] + ws[3];
}

// Writes the kept keys of chunk b, in order, from offset offs[b]: the column
// id of each, and the row offsets of the rows from the previous kept key's
// row (exclusive) to its own (inclusive).
__global__ void __launch_bounds__(kThreads) write_kept(const unsigned long long* keys, long long total,
                                                       unsigned long long sentinel, int scale,
                                                       const unsigned long long* offs, int64_t* row_ptr,
                                                       int32_t* col) {
  const long long base = (long long)blockIdx.x * kChunk;
  __shared__ unsigned ws[kThreads / 64];
  __shared__ unsigned long long running;
  if (threadIdx.x == 0) running = offs[blockIdx.x];
  __syncthreads();
  const unsigned long long mask = (1ull << scale) - 1ull;
  const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
  for (int t = 0; t < kPerThread; ++t) {
    const long long j = base + (long long)t * kThreads + threadIdx.x;
    unsigned long long k = 0, prev = 0;
    bool keep = false;
    if (j < total) {
      k = keys[j];
      prev = j > 0 ? keys[j - 1] : 0ull;
      keep = k != sentinel && (j == 0 || prev != k);
    }
    const unsigned long long ballot = __ballot(keep);
    const unsigned before = (unsigned)__popcll(ballot & ((1ull << lane) - 1ull));
    if (lane == 0) ws[w] = (unsigned)__popcll(ballot);
    __syncthreads();
    unsigned wbase = 0;
    for (int q = 0; q < w; ++q) wbase += ws[q];
    const unsigned long long pos = running + wbase + before;
    if (keep) {
      col[pos] = (int32_t)(k & mask);
      const long long u = (long long)(k >> scale);
      const long long pu = j > 0 ? (long long)(prev >> scale) : -1;
      for (long long r = pu + 1; r <= u; ++r) row_ptr[r] = (int64_t)pos;
    }
    __syncthreads();
    if (threadIdx.x == 0) running += (unsigned long long)ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
  }
}

// Rows after the last kept key's row end at nnz.
__global__ void __launch_bounds__(kThreads) tail_rows(int64_t* row_ptr, long long first, long long n, long long nnz) {
  for (long long r = first + (long long)blockIdx.x * kThreads + threadIdx.x; r <= n; r += (long long)gridDim.x * kThreads)
    row_ptr[r] = (int64_t)nnz;
}

struct Build {
  int scale = 0;
  long long n = 0, total = 0, nnz = 0, nchunks = 0;
  unsigned long long* keys[2] = {nullptr, nullptr};
  int cur = 0;
  unsigned long long* counts = nullptr;
  unsigned long long* offs = nullptr;
  void* temp = nullptr;
  hipStream_t s = nullptr;
  ~Build() {
    for (auto* p : keys)
      if (p) (void)hipFree(p);
    if (counts) (void)hipFree(counts);
    if (offs) (void)hipFree(offs);
    if (temp) (void)hipFree(temp);
  }
};

}  // namespace

extern "C" {

// Generates R-MAT(scale, edge_factor, a, b, c) with the permutation `perm_host`
// (n entries, or null for no relabelling) on the current device and stream.
// Returns 0 and a handle with the arc count after deduplication, -1 for
// invalid arguments, -2 for a HIP failure (out of memory included).
int sg_gpu_rmat_begin(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed,
                      const int32_t* perm_host, void* stream, void** handle, int64_t* nnz) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || !handle || !nnz) return -1;
  Build* B = new Build;
  B->scale = scale;
  B->n = 1ll << scale;
  B->total = 2ll * edge_factor * B->n;
  B->s = (hipStream_t)stream;
  const long long draws = (long long)edge_factor * B->n;
  const uint64_t key = mix64_host(seed * kGolden + mix64_host(1 + 0x632BE59BD9B4E019ull));
  int32_t* perm = nullptr;
  auto fail = [&](int rc) {
    if (perm) (void)hipFree(perm);
    delete B;
    return rc;
  };
  if (hipMalloc((void**)&B->keys[0], sizeof(unsigned long long) * B->total) != hipSuccess ||
      hipMalloc((void**)&B->keys[1], sizeof(unsigned long long) * B->total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(-2);
  }
  if (perm_host) {
    if (hipMalloc((void**)&perm, sizeof(int32_t) * B->n) != hipSuccess ||
        hipMemcpyAsync(perm, perm_host, sizeof(int32_t) * B->n, hipMemcpyHostToDevice, B->s) != hipSuccess) {
      (void)hipGetLastError();
      return fail(-2);
    }
  }
  hipLaunchKernelGGL(rmat_keys, dim3(8192), dim3(kThreads), 0, B->s, scale, draws, key, a, a + b, a + b + c, perm,
                     B->keys[0]);
  if (hipGetLastError() != hipSuccess) return fail(-2);
  rocprim::double_buffer<unsigned long long> db(B->keys[0], B->keys[1]);
  size_t temp_bytes = 0;
  const unsigned end_bit = 2 * scale + 1;
  if (rocprim::radix_sort_keys(nullptr, temp_bytes, db, (size_t)B->total, 0, end_bit, B->s) != hipSuccess)
    return fail(-2);
  if (hipMalloc(&B->temp, temp_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(-2);
  }
  if (rocprim::radix_sort_keys(B->temp, temp_bytes, db, (size_t)B->total, 0, end_bit, B->s) != hipSuccess)
    return fail(-2);
  B->cur = db.current() == B->keys[0] ? 0 : 1;
  (void)hipFree(B->temp);
  B->temp = nullptr;
  // Kept keys per chunk and their offsets.
  B->nchunks = (B->total + kChunk - 1) / kChunk;
  if (hipMalloc((void**)&B->counts, sizeof(unsigned long long) * B->nchunks) != hipSuccess ||
      hipMalloc((void**)&B->offs, sizeof(unsigned long long) * (B->nchunks + 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(-2);
  }
  const unsigned long long sentinel = (unsigned long long)B->n << scale;
  hipLaunchKernelGGL(count_kept, dim3((unsigned)B->nchunks), dim3(kThreads), 0, B->s, B->keys[B->cur], B->total,
                     sentinel, B->counts);
  if (hipGetLastError() != hipSuccess) return fail(-2);
  temp_bytes = 0;
  if (rocprim::exclusive_scan(nullptr, temp_bytes, B->counts, B->offs, 0ull, (size_t)B->nchunks + 0,
                              rocprim::plus<unsigned long long>(), B->s) != hipSuccess)
    return fail(-2);
  if (hipMalloc(&B->temp, temp_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(-2);
  }
  if (rocprim::exclusive_scan(B->temp, temp_bytes, B->counts, B->offs, 0ull, (size_t)B->nchunks,
                              rocprim::plus<unsigned long long>(), B->s) != hipSuccess)
    return fail(-2);
  unsigned long long last_off = 0, last_cnt = 0;
  if (hipMemcpyAsync(&last_off, B->offs + (B->nchunks - 1), sizeof(last_off), hipMemcpyDeviceToHost, B->s) !=
          hipSuccess ||
      hipMemcpyAsync(&last_cnt, B->counts + (B->nchunks - 1), sizeof(last_cnt), hipMemcpyDeviceToHost, B->s) !=
          hipSuccess ||
      hipStreamSynchronize(B->s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(-2);
  }
  if (perm) (void)hipFree(perm);
  perm = nullptr;
  B->nnz = (long long)(last_off + last_cnt);
  *nnz = B->nnz;
  *handle = B;
  return 0;
}

// Writes row_ptr (n + 1 int64) and col (nnz int32, device arrays of the
// caller) and frees the handle.  Returns 0 or -2.
int sg_gpu_rmat_finish(void* handle, int64_t* row_ptr, int32_t* col) {
  Build* B = static_cast<Build*>(handle);
  const unsigned long long sentinel = (unsigned long long)B->n << B->scale;
  int rc = 0;
  hipLaunchKernelGGL(write_kept, dim3((unsigned)B->nchunks), dim3(kThreads), 0, B->s, B->keys[B->cur], B->total,
                     sentinel, B->scale, B->offs, row_ptr, col);
  // Rows after the last arc's row: the last kept key is the last key below the sentinel.
  long long last_row = -1;
  if (B->nnz > 0) {
    unsigned long long kl = 0;
    // The kept keys are the distinct keys, and the largest is at col[nnz-1]'s
    // row; find it from the sorted keys: the last key that is not the sentinel.
    long long lo = 0, hi = B->total;   // first index holding the sentinel
    while (lo < hi) {
      const long long mid = (lo + hi) / 2;
      unsigned long long km = 0;
      if (hipMemcpyAsync(&km, B->keys[B->cur] + mid, sizeof(km), hipMemcpyDeviceToHost, B->s) != hipSuccess ||
          hipStreamSynchronize(B->s) != hipSuccess) {
        (void)hipGetLastError();
        rc = -2;
        break;
      }
      if (km < sentinel) lo = mid + 1; else hi = mid;
    }
    if (rc == 0) {
      if (hipMemcpyAsync(&kl, B->keys[B->cur] + (lo - 1), sizeof(kl), hipMemcpyDeviceToHost, B->s) != hipSuccess ||
          hipStreamSynchronize(B->s) != hipSuccess) {
        (void)hipGetLastError();
        rc = -2;
      }
      last_row = (long long)(kl >> B->scale);
    }
  }
  if (rc == 0) {
    hipLaunchKernelGGL(tail_rows, dim3(1024), dim3(kThreads), 0, B->s, row_ptr, last_row + 1, B->n, B->nnz);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(B->s) != hipSuccess) {
      (void)hipGetLastError();
      rc = -2;
    }
  }
  delete B;
  return rc;
}

// Frees a handle without writing outputs.
void sg_gpu_rmat_abort(void* handle) { delete static_cast<Build*>(handle); }

}  // extern "C"
