// Plain FP64 bound iteration for Katz ranking, in C++ with OpenMP.
//
// TEST INFRASTRUCTURE ONLY: this is the oracle, built into its own library
// (oracle/libkatz_ref.so) and loaded by oracle/cpp.py.  Only the tests, the
// smoke check and the benchmark's CPU-baseline leg may load it; the product
// never links or loads it, and it includes nothing from the product.
//
// Paper: van der Grinten, Bergamini, Green, Bader, Meyerhenke, "Scalable Katz
// Ranking Computation in Large Static and Dynamic Graphs", ESA 2018.
//
// It computes exactly what oracle/katz.py computes (Algorithm 1 of Section 3.2
// with the top-k criterion of Section 3.1), with the same arithmetic in the
// same order, so the two agree bit for bit:
//   * the scaled walk vector x_r = alpha * (A x_{r-1}), x_0 = 1 (Eq.
//     (basic_recurrence) with alpha^r folded in), each row summed left to
//     right in CSR order starting from 0.0, alpha applied after the sum;
//   * c_r = c_{r-1} + x_r;
//   * l_r = c_r + alpha x_r on undirected graphs, else c_r; u_r = c_r + beta x_r
//     with gamma = d_max / (1 - alpha d_max) and beta = fl(alpha gamma)
//     (Theorem 1);
//   * converged(): order M by (lower bound descending, id ascending); theta is
//     the k-th lower bound; a node after position k whose u - eps < theta
//     leaves M; more than k nodes left means not certified; otherwise every
//     adjacent pair of the top-k must satisfy u(M[i]) - eps < l(M[i-1]).
//   * the loop is a do-while (the first test follows iteration 1); it also
//     stops at max_iter (status 1) and when the walk vector is all zero
//     (status 3: the bounds are exact and an unseparated pair is a true tie).
// Built with -ffp-contract=off so no multiply-add is fused.
//
// Only the top-k positions of the order must be exact, so the partial sort is
// a selection of the k-th element followed by a sort of the k first (library
// primitives; the comparison is a strict total order, so the selected set and
// its order do not depend on the thread count).  The row loop of the walk runs
// in parallel over rows; every row is still summed sequentially, so the
// result does not depend on the thread count either.
#include <omp.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

struct Entry {          // one active node and its lower bound
  double lo;
  int32_t v;
};

// Before = larger lower bound, then smaller id.
inline bool before(const Entry& a, const Entry& b) { return a.lo > b.lo || (a.lo == b.lo && a.v < b.v); }

int64_t max_degree(int64_t n, const int64_t* rp) {
  int64_t d = 0;
#pragma omp parallel for reduction(max : d) schedule(static)
  for (int64_t v = 0; v < n; ++v) d = std::max<int64_t>(d, rp[v + 1] - rp[v]);
  return d;
}

// Rows lo..hi-1 of x_new = alpha * (A x) (xn indexed by row), and c += x_new
// when c is given; returns whether some new entry is nonzero.
bool walk(int64_t lo, int64_t hi, const int64_t* rp, const int32_t* col, double alpha, const double* x, double* xn,
          double* c) {
  bool any = false;
#pragma omp parallel for schedule(dynamic, 2048) reduction(|| : any)
  for (int64_t v = lo; v < hi; ++v) {
    double t = 0.0;
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) t += x[col[j]];
    const double s = alpha * t;
    xn[v - lo] = s;
    if (c) c[v] = c[v] + s;
    any = any || s != 0.0;
  }
  return any;
}

void node_bounds(int64_t n, const double* c, const double* x, double alpha, double beta, int undirected,
                 double* lo, double* up) {
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    lo[v] = undirected ? c[v] + alpha * x[v] : c[v];
    up[v] = c[v] + beta * x[v];
  }
}

// converged() of Algorithm 1 over the active set M (ids).  On return M holds
// the top-k in ranking order followed by the nodes kept after position k.
bool converged(std::vector<int32_t>& M, const double* lo, const double* up, int64_t k, double eps,
               std::vector<Entry>& buf) {
  const int64_t m = (int64_t)M.size();
  buf.resize(m);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) buf[i] = Entry{lo[M[i]], M[i]};
  std::nth_element(buf.begin(), buf.begin() + (k - 1), buf.end(), before);
  std::sort(buf.begin(), buf.begin() + k, before);
  const double theta = buf[k - 1].lo;
  int64_t kept = k;
  for (int64_t i = k; i < m; ++i) {
    const int32_t v = buf[i].v;
    if (!(up[v] - eps < theta)) buf[kept++] = buf[i];
  }
  M.resize(kept);
  for (int64_t i = 0; i < kept; ++i) M[i] = buf[i].v;
  if (kept > k) return false;
  for (int64_t i = 1; i < k; ++i)
    if (up[M[i]] - eps >= lo[M[i - 1]]) return false;
  return true;
}

// The thread count of one call: set for the call, restored on return, so a
// call with threads > 0 leaves later calls with threads <= 0 on OpenMP's
// default.
struct ThreadScope {
  int saved;
  explicit ThreadScope(int threads) : saved(omp_get_max_threads()) {
    if (threads > 0) omp_set_num_threads(threads);
  }
  ~ThreadScope() { omp_set_num_threads(saved); }
};

}  // namespace

extern "C" {

struct ko_result {
  double alpha, gamma, beta;
  double rest_upper_max;   // max u_r over V minus the top-k; -inf when k = n
  int64_t active_final;    // |M| at the end
  int32_t iterations;      // r
  int32_t status;          // 0 ok, 1 iteration limit, 3 exact ties
};

// Runs Algorithm 1 on (n, row_ptr, col).  alpha <= 0 selects 1/(1 + d_max).
// topk / lower / upper: [k] outputs in ranking order.  c_out, x_out,
// lower_all, upper_all: optional [n] outputs (c_r, x_r, l_r, u_r of every
// node).  threads <= 0 keeps OpenMP's default.  Returns 0, or -1 for invalid
// arguments (alpha outside (0, 1/d_max), k outside [1, n], eps < 0,
// max_iter < 1), -2 when memory runs out.
int ko_rank_static(int64_t n, const int64_t* row_ptr, const int32_t* col, double alpha, int64_t k, double eps,
                   int32_t undirected, int32_t max_iter, int32_t threads, int32_t* topk, double* lower,
                   double* upper, double* c_out, double* x_out, double* lower_all, double* upper_all,
                   ko_result* res) {
  const ThreadScope scope(threads);
  if (n < 1 || k < 1 || k > n || !(eps >= 0.0) || max_iter < 1) return -1;
  const int64_t dmax = max_degree(n, row_ptr);
  if (alpha <= 0.0) alpha = 1.0 / (1.0 + (double)dmax);
  if (!(alpha > 0.0) || !(alpha * (double)dmax < 1.0)) return -1;
  const double gamma = (double)dmax / (1.0 - alpha * (double)dmax);
  const double beta = alpha * gamma;
  try {
    std::vector<double> x(n, 1.0), xn(n), c(n, 0.0), lo(n), up(n);
    std::vector<int32_t> M(n);
    std::vector<Entry> buf;
    for (int64_t v = 0; v < n; ++v) M[v] = (int32_t)v;
    int r = 0, status = 0;
    for (;;) {
      ++r;
      const bool any = walk(0, n, row_ptr, col, alpha, x.data(), xn.data(), c.data());
      x.swap(xn);
      node_bounds(n, c.data(), x.data(), alpha, beta, undirected, lo.data(), up.data());
      if (converged(M, lo.data(), up.data(), k, eps, buf)) {
        status = 0;
        break;
      }
      if (!any) {
        status = 3;
        break;
      }
      if (r >= max_iter) {
        status = 1;
        break;
      }
    }
    // Outputs: the top-k in ranking order and the largest upper bound outside it.
    std::vector<uint8_t> top(n, 0);
    for (int64_t i = 0; i < k; ++i) {
      const int32_t v = M[i];
      top[v] = 1;
      topk[i] = v;
      lower[i] = lo[v];
      upper[i] = up[v];
    }
    double rest = -std::numeric_limits<double>::infinity();
#pragma omp parallel for reduction(max : rest) schedule(static)
    for (int64_t v = 0; v < n; ++v)
      if (!top[v]) rest = std::max(rest, up[v]);
    if (c_out) std::memcpy(c_out, c.data(), sizeof(double) * n);
    if (x_out) std::memcpy(x_out, x.data(), sizeof(double) * n);
    if (lower_all) std::memcpy(lower_all, lo.data(), sizeof(double) * n);
    if (upper_all) std::memcpy(upper_all, up.data(), sizeof(double) * n);
    res->alpha = alpha;
    res->gamma = gamma;
    res->beta = beta;
    res->rest_upper_max = rest;
    res->active_final = (int64_t)M.size();
    res->iterations = r;
    res->status = status;
  } catch (const std::bad_alloc&) {
    return -2;
  }
  return 0;
}

// l_r and u_r of every node after exactly r iterations (no convergence test).
int ko_bounds(int64_t n, const int64_t* row_ptr, const int32_t* col, double alpha, int32_t r, int32_t undirected,
              int32_t threads, double* lower, double* upper) {
  const ThreadScope scope(threads);
  if (n < 1 || r < 1) return -1;
  const int64_t dmax = max_degree(n, row_ptr);
  if (alpha <= 0.0) alpha = 1.0 / (1.0 + (double)dmax);
  if (!(alpha > 0.0) || !(alpha * (double)dmax < 1.0)) return -1;
  const double gamma = (double)dmax / (1.0 - alpha * (double)dmax);
  const double beta = alpha * gamma;
  try {
    std::vector<double> x(n, 1.0), xn(n), c(n, 0.0);
    for (int i = 0; i < r; ++i) {
      walk(0, n, row_ptr, col, alpha, x.data(), xn.data(), c.data());
      x.swap(xn);
    }
    node_bounds(n, c.data(), x.data(), alpha, beta, undirected, lower, upper);
  } catch (const std::bad_alloc&) {
    return -2;
  }
  return 0;
}

// One walk step over rows lo..hi-1 only (x_out[v - lo] for those rows), the
// loop the iteration runs; x_in holds all n entries.  Used to time a bounded
// sample of a graph too large for a full single-thread run.
int ko_walk_rows(int64_t n, const int64_t* row_ptr, const int32_t* col, double alpha, int64_t lo, int64_t hi,
                 int32_t threads, const double* x_in, double* x_out) {
  const ThreadScope scope(threads);
  if (lo < 0 || hi > n || lo > hi) return -1;
  walk(lo, hi, row_ptr, col, alpha, x_in, x_out, nullptr);
  return 0;
}

int ko_max_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
