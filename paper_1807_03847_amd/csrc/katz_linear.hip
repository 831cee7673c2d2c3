// Vector kernels of the paper's two comparison methods (katz_solve), which
// use the walk kernels for their sparse matrix-vector products y = alpha A v:
//   * Foster's heuristic (Section 2.2): f_{i+1} = alpha A f_i + 1, stopped
//     when the largest change of an entry falls below the tolerance;
//   * conjugate gradients on Eq. (la), (I - alpha A) z = 1, then the Katz
//     vector alpha A z (Section 1).
// Reductions (maxima, dot products) are deterministic: each workgroup writes
// its partial result to its own slot, and one workgroup combines the slots in
// slot order, so a run's iterates do not depend on scheduling.
#include <algorithm>
#include <cstdint>

#include "katz_device.h"

namespace katz {
namespace {

constexpr int kRedBlocks = 1024;   // workgroups of a reduction pass (slots)

__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double w[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (lane_id() == 0) w[threadIdx.x / kWave] = v;
  __syncthreads();
  const double t = (w[0] + w[1]) + (w[2] + w[3]);
  __syncthreads();
  return t;
}

__device__ __forceinline__ double block_max_d(double v) {
  __shared__ double w[kWG / kWave];
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (lane_id() == 0) w[threadIdx.x / kWave] = v;
  __syncthreads();
  const double t = fmax(fmax(w[0], w[1]), fmax(w[2], w[3]));
  __syncthreads();
  return t;
}

__global__ void __launch_bounds__(kWG) fill_value(double* x, long long n, double v) {
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long long)gridDim.x * kWG) x[i] = v;
}

// Foster step: f_new = y + 1 (y = alpha A f); slot = max |f_new - f| of the
// workgroup's entries.
__global__ void __launch_bounds__(kWG) foster_step(const double* y, const double* f, double* f_new, long long n,
                                                   double* slots) {
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long long)gridDim.x * kWG) {
    const double v = y[i] + 1.0;
    f_new[i] = v;
    m = fmax(m, fabs(v - f[i]));
  }
  m = block_max_d(m);
  if (threadIdx.x == 0) slots[blockIdx.x] = m;
}

// q = p - y (y = alpha A p: q = (I - alpha A) p); slot = sum of p q.
__global__ void __launch_bounds__(kWG) cg_apply(const double* p, const double* y, double* q, long long n,
                                                double* slots) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long long)gridDim.x * kWG) {
    const double v = p[i] - y[i];
    q[i] = v;
    s += p[i] * v;
  }
  s = block_sum_d(s);
  if (threadIdx.x == 0) slots[blockIdx.x] = s;
}

// z += a p; r -= a q; slot = sum of r r (the new residual).
__global__ void __launch_bounds__(kWG) cg_update(double* z, double* r, const double* p, const double* q,
                                                 const double* a_ptr, long long n, double* slots) {
  const double a = *a_ptr;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long long)gridDim.x * kWG) {
    z[i] = z[i] + a * p[i];
    const double v = r[i] - a * q[i];
    r[i] = v;
    s += v * v;
  }
  s = block_sum_d(s);
  if (threadIdx.x == 0) slots[blockIdx.x] = s;
}

// p = r + b p.
__global__ void __launch_bounds__(kWG) cg_direction(double* p, const double* r, const double* b_ptr, long long n) {
  const double b = *b_ptr;
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long long)gridDim.x * kWG)
    p[i] = r[i] + b * p[i];
}

// Combines the slots of a reduction in slot order: op 0 = sum, 1 = max.
// out[0] = the result; with the CG scalars also the step sizes:
//   mode 1 (after cg_apply):  s[1] = s[0] / out  (a = r.r / p.q)
//   mode 2 (after cg_update): s[2] = out / s[0]  (b = r'.r' / r.r), s[0] = out
__global__ void __launch_bounds__(kWG) combine_slots(const double* slots, int nslots, int op, double* out,
                                                     double* scal, int mode) {
  double v = 0.0;
  // Each thread combines a fixed stride of slots in order, then the block
  // combines the threads in a fixed tree: deterministic.
  for (int i = threadIdx.x; i < nslots; i += kWG) v = op ? fmax(v, slots[i]) : v + slots[i];
  v = op ? block_max_d(v) : block_sum_d(v);
  if (threadIdx.x == 0) {
    out[0] = v;
    if (mode == 1) scal[1] = scal[0] / v;
    if (mode == 2) {
      scal[2] = v / scal[0];
      scal[0] = v;
    }
  }
}

// scores = x + add (Foster: f - 1), written through ext_of (internal -> caller id).
__global__ void __launch_bounds__(kWG) write_scores(const double* x, double add, long long n, const int32_t* ext_of,
                                                    double* out) {
  for (long long i = (long long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long long)gridDim.x * kWG)
    out[ext_of ? ext_of[i] : i] = x[i] + add;
}

unsigned grid_of(long long n) {
  return (unsigned)std::max<long long>(1, std::min<long long>((n + kWG - 1) / kWG, kRedBlocks));
}

}  // namespace

int linear_reduce_slots() { return kRedBlocks; }

hipError_t launch_fill_value(double* x, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_value, dim3(grid_of(n)), dim3(kWG), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_foster_step(const double* y, const double* f, double* f_new, long long n, double* slots,
                              double* out, hipStream_t s) {
  const unsigned g = grid_of(n);
  hipLaunchKernelGGL(foster_step, dim3(g), dim3(kWG), 0, s, y, f, f_new, n, slots);
  hipLaunchKernelGGL(combine_slots, dim3(1), dim3(kWG), 0, s, (const double*)slots, (int)g, 1, out,
                     (double*)nullptr, 0);
  return hipGetLastError();
}

// scal: [0] r.r, [1] a, [2] b (device).  out: [0] p.q, then [1] the new r.r.
hipError_t launch_cg_apply(const double* p, const double* y, double* q, long long n, double* slots, double* out,
                           double* scal, hipStream_t s) {
  const unsigned g = grid_of(n);
  hipLaunchKernelGGL(cg_apply, dim3(g), dim3(kWG), 0, s, p, y, q, n, slots);
  hipLaunchKernelGGL(combine_slots, dim3(1), dim3(kWG), 0, s, (const double*)slots, (int)g, 0, out, scal, 1);
  return hipGetLastError();
}

hipError_t launch_cg_update(double* z, double* r, const double* p, const double* q, long long n, double* slots,
                            double* out, double* scal, hipStream_t s) {
  const unsigned g = grid_of(n);
  hipLaunchKernelGGL(cg_update, dim3(g), dim3(kWG), 0, s, z, r, p, q, (const double*)(scal + 1), n, slots);
  hipLaunchKernelGGL(combine_slots, dim3(1), dim3(kWG), 0, s, (const double*)slots, (int)g, 0, out, scal, 2);
  return hipGetLastError();
}

hipError_t launch_cg_direction(double* p, const double* r, const double* scal, long long n, hipStream_t s) {
  hipLaunchKernelGGL(cg_direction, dim3(grid_of(n)), dim3(kWG), 0, s, p, r, scal + 2, n);
  return hipGetLastError();
}

hipError_t launch_write_scores(const double* x, double add, long long n, const int32_t* ext_of, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(write_scores, dim3(grid_of(n)), dim3(kWG), 0, s, x, add, n, ext_of, out);
  return hipGetLastError();
}

}  // namespace katz
