// Host driver for the sanitizer build of the C++ oracle and the graph
// generators: small graphs of every generator through every oracle entry
// point.  Exit status 0 when every call succeeded and every result is sane;
// the sanitizers abort on the first error they find.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
struct ko_result {
  double alpha, gamma, beta;
  double rest_upper_max;
  int64_t active_final;
  int32_t iterations;
  int32_t status;
};
int ko_rank_static(int64_t n, const int64_t* row_ptr, const int32_t* col, double alpha, int64_t k, double eps,
                   int32_t undirected, int32_t max_iter, int32_t threads, int32_t* topk, double* lower,
                   double* upper, double* c_out, double* x_out, double* lower_all, double* upper_all,
                   ko_result* res);
int ko_bounds(int64_t n, const int64_t* row_ptr, const int32_t* col, double alpha, int32_t r, int32_t undirected,
              int32_t threads, double* lower, double* upper);
int ko_walk_rows(int64_t n, const int64_t* row_ptr, const int32_t* col, double alpha, int64_t lo, int64_t hi,
                 int32_t threads, double* x_in, double* x_out);
void* sg_er(int64_t n, int64_t m_edges, uint64_t seed);
void* sg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed, int32_t relabel);
void* sg_ba(int64_t n, int32_t m, uint64_t seed);
int64_t sg_n(void* h);
int64_t sg_nnz(void* h);
void sg_export(void* h, int64_t* row_ptr, int32_t* col);
void sg_free(void* h);
void sg_permutation(int64_t n, uint64_t seed, int32_t* out);
void sg_rmat_pairs(int32_t scale, double a, double b, double c, uint64_t seed, int32_t relabel, uint64_t stream,
                   uint64_t first, int64_t count, int32_t* u, int32_t* v);
void sg_draw(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, uint64_t* out);
}

static int check_graph(void* h, const char* name) {
  if (!h) {
    std::printf("%s: generator failed\n", name);
    return 1;
  }
  const int64_t n = sg_n(h), nnz = sg_nnz(h);
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> col(nnz > 0 ? nnz : 1);
  sg_export(h, rp.data(), col.data());
  sg_free(h);
  for (int threads : {1, 3}) {
    const int64_t k = n < 20 ? n : 20;
    std::vector<int32_t> topk(k);
    std::vector<double> lo(k), up(k), c(n), x(n), la(n), ua(n);
    ko_result res{};
    const int rc = ko_rank_static(n, rp.data(), col.data(), 0.0, k, 1e-9, 1, 200, threads, topk.data(), lo.data(),
                                  up.data(), c.data(), x.data(), la.data(), ua.data(), &res);
    if (rc < 0) {
      std::printf("%s: rank rc=%d\n", name, rc);
      return 1;
    }
    for (int64_t i = 0; i < k; ++i)
      if (!(lo[i] <= up[i])) {
        std::printf("%s: bounds out of order\n", name);
        return 1;
      }
    std::vector<double> bl(n), bu(n);
    if (ko_bounds(n, rp.data(), col.data(), 0.0, 4, 1, threads, bl.data(), bu.data()) < 0) return 1;
    std::vector<double> xi(n, 1.0), xo(n);
    if (ko_walk_rows(n, rp.data(), col.data(), 0.5 / (1 + n), 0, n, threads, xi.data(), xo.data()) < 0) return 1;
  }
  std::printf("%s: n=%lld nnz=%lld ok\n", name, (long long)n, (long long)nnz);
  return 0;
}

int main() {
  int bad = 0;
  bad |= check_graph(sg_er(800, 3200, 5), "er");
  bad |= check_graph(sg_rmat(10, 8, 0.57, 0.19, 0.19, 3, 1), "rmat10");
  bad |= check_graph(sg_ba(1500, 5, 7), "ba");
  bad |= check_graph(sg_er(50, 0, 1), "empty");
  std::vector<int32_t> perm(1000), u(500), v(500);
  sg_permutation(1000, 9, perm.data());
  sg_rmat_pairs(10, 0.57, 0.19, 0.19, 3, 1, 7, 0, 500, u.data(), v.data());
  std::vector<uint64_t> d(100);
  sg_draw(1, 2, 3, 100, d.data());
  std::printf(bad ? "FAILED\n" : "all ok\n");
  return bad;
}
