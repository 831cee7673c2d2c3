// Seeded synthetic graph generators (input data only; no Katz arithmetic here).
//
// Every random draw comes from a counter-based generator: the value for
// (seed, stream, counter) is a pure function of those three integers, so a
// graph depends only on its seed, never on the thread count.  The mixing
// function is the SplitMix64 finaliser (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), applied to a Weyl sequence.
//
// Output format: canonical CSR with int64 row offsets and int32 columns.
// Undirected graphs hold both arcs of every edge; rows are sorted, without
// duplicates and without self-loops.
//
// Generators:
//   * Erdos-Renyi G(n, M): M distinct undirected edges drawn uniformly
//     without replacement.
//   * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): edge_factor * 2^scale
//     edge draws, quadrant probabilities (a, b, c, d), no noise; seeded random
//     relabelling of the vertices (as in Graph500), then symmetrise, drop
//     self-loops, deduplicate.  Two passes (count, then fill) regenerate the
//     edges from the counter so no edge list is ever stored.
//   * Barabasi-Albert preferential attachment (Batagelj-Brandes linear-time
//     scheme, "Efficient generation of large random networks", Phys Rev E
//     2005): an (m+1)-clique seed, then each new vertex picks m distinct
//     targets by uniform draws from the endpoint list.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <unordered_set>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter-based draw: a 64-bit value for (seed, stream, counter).
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t counter) {
  uint64_t key = mix64(seed * kGolden + mix64(stream + 0x632BE59BD9B4E019ull));
  return mix64(key + (counter + 1) * kGolden);
}

// Uniform double in [0, 1) with 53 random bits.
inline double draw_unit(uint64_t seed, uint64_t stream, uint64_t counter) {
  return (double)(draw(seed, stream, counter) >> 11) * (1.0 / 9007199254740992.0);
}

// Uniform integer in [0, bound) by Lemire's multiply-shift (bias < 2^-64 * bound).
inline uint64_t draw_below(uint64_t seed, uint64_t stream, uint64_t counter, uint64_t bound) {
  unsigned __int128 p = (unsigned __int128)draw(seed, stream, counter) * bound;
  return (uint64_t)(p >> 64);
}

struct Graph {
  int64_t n = 0;
  int64_t nnz = 0;
  int64_t* row_ptr = nullptr;  // n + 1
  int32_t* col = nullptr;      // nnz
};

void free_graph(Graph* g) {
  if (!g) return;
  std::free(g->row_ptr);
  std::free(g->col);
  delete g;
}

// Sort each row, drop duplicates, and compact into a fresh array.
// `deg` holds the filled length of each row, `start` the row starts of `raw`.
Graph* finish_csr(int64_t n, const int64_t* start, int64_t* deg, int32_t* raw) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* b = raw + start[v];
    int32_t* e = b + deg[v];
    std::sort(b, e);
    deg[v] = std::unique(b, e) - b;
  }
  Graph* g = new Graph;
  g->n = n;
  g->row_ptr = (int64_t*)std::malloc(sizeof(int64_t) * (n + 1));
  if (!g->row_ptr) { free_graph(g); return nullptr; }
  g->row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) g->row_ptr[v + 1] = g->row_ptr[v] + deg[v];
  g->nnz = g->row_ptr[n];
  g->col = (int32_t*)std::malloc(sizeof(int32_t) * (g->nnz > 0 ? g->nnz : 1));
  if (!g->col) { free_graph(g); return nullptr; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v)
    std::memcpy(g->col + g->row_ptr[v], raw + start[v], sizeof(int32_t) * deg[v]);
  return g;
}

// Build a symmetric CSR from a generator of undirected pairs.  `pair(i, &u, &v)`
// returns false for a discarded draw.  Called twice per edge index (count pass
// and fill pass), so it must be a pure function of i.
template <class PairFn>
Graph* symmetric_csr(int64_t n, int64_t draws, PairFn pair) {
  int64_t* cnt = (int64_t*)std::calloc(n + 1, sizeof(int64_t));
  if (!cnt) return nullptr;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < draws; ++i) {
    int64_t u, v;
    if (!pair(i, &u, &v)) continue;
    __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
  }
  int64_t* start = (int64_t*)std::malloc(sizeof(int64_t) * (n + 1));
  if (!start) { std::free(cnt); return nullptr; }
  start[0] = 0;
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + cnt[v];
  int64_t total = start[n];
  int32_t* raw = (int32_t*)std::malloc(sizeof(int32_t) * (total > 0 ? total : 1));
  if (!raw) { std::free(cnt); std::free(start); return nullptr; }
  std::memset(cnt, 0, sizeof(int64_t) * (n + 1));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < draws; ++i) {
    int64_t u, v;
    if (!pair(i, &u, &v)) continue;
    int64_t pu = __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
    int64_t pv = __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    raw[start[u] + pu] = (int32_t)v;
    raw[start[v] + pv] = (int32_t)u;
  }
  Graph* g = finish_csr(n, start, cnt, raw);
  std::free(raw);
  std::free(start);
  std::free(cnt);
  return g;
}

// Seeded uniform random permutation (Fisher-Yates, counter-based draws).
int32_t* random_permutation(int64_t n, uint64_t seed) {
  int32_t* p = (int32_t*)std::malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  if (!p) return nullptr;
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)draw_below(seed, 2, (uint64_t)i, (uint64_t)(i + 1));
    std::swap(p[i], p[j]);
  }
  return p;
}

}  // namespace

extern "C" {

void sg_free(void* h) { free_graph((Graph*)h); }
int64_t sg_n(void* h) { return ((Graph*)h)->n; }
int64_t sg_nnz(void* h) { return ((Graph*)h)->nnz; }
void sg_export(void* h, int64_t* row_ptr, int32_t* col) {
  Graph* g = (Graph*)h;
  std::memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * (g->n + 1));
  if (g->nnz) std::memcpy(col, g->col, sizeof(int32_t) * g->nnz);
}

// Erdos-Renyi G(n, M): the first M distinct non-loop pairs of the draw sequence.
void* sg_er(int64_t n, int64_t m_edges, uint64_t seed) {
  if (n < 2 || m_edges < 0 || m_edges > n * (n - 1) / 2) return nullptr;
  std::vector<uint64_t> keys;
  keys.reserve(m_edges);
  std::unordered_set<uint64_t> seen;
  seen.reserve(m_edges * 2);
  for (uint64_t i = 0; (int64_t)keys.size() < m_edges; ++i) {
    uint64_t u = draw_below(seed, 1, 2 * i, (uint64_t)n);
    uint64_t v = draw_below(seed, 1, 2 * i + 1, (uint64_t)n);
    if (u == v) continue;
    if (u > v) std::swap(u, v);
    uint64_t key = (u << 32) | v;
    if (seen.insert(key).second) keys.push_back(key);
  }
  return symmetric_csr(n, m_edges, [&](int64_t i, int64_t* u, int64_t* v) {
    *u = (int64_t)(keys[i] >> 32);
    *v = (int64_t)(keys[i] & 0xffffffffull);
    return true;
  });
}

// R-MAT with seeded relabelling; symmetrised, deduplicated, no self-loops.
void* sg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
              uint64_t seed, int32_t relabel) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return nullptr;
  const int64_t n = (int64_t)1 << scale;
  const int64_t draws = (int64_t)edge_factor * n;
  int32_t* perm = nullptr;
  if (relabel) {
    perm = random_permutation(n, seed);
    if (!perm) return nullptr;
  }
  const double ab = a + b, abc = a + b + c;
  auto pair = [&](int64_t i, int64_t* u, int64_t* v) {
    int64_t src = 0, dst = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double p = draw_unit(seed, 1, (uint64_t)i * (uint64_t)scale + (uint64_t)l);
      int64_t bit = (int64_t)1 << (scale - 1 - l);
      if (p < a) {
      } else if (p < ab) {
        dst |= bit;
      } else if (p < abc) {
        src |= bit;
      } else {
        src |= bit;
        dst |= bit;
      }
    }
    if (src == dst) return false;
    *u = perm ? perm[src] : src;
    *v = perm ? perm[dst] : dst;
    return true;
  };
  Graph* g = symmetric_csr(n, draws, pair);
  std::free(perm);
  return g;
}

// Barabasi-Albert by the Batagelj-Brandes endpoint-list scheme with m distinct
// targets per new vertex (a repeated target is redrawn).
void* sg_ba(int64_t n, int32_t m, uint64_t seed) {
  if (m < 1 || n < m + 2) return nullptr;
  const int64_t edges = (int64_t)m * (m + 1) / 2 + (n - m - 1) * (int64_t)m;
  std::vector<int32_t> ends;
  ends.reserve(2 * edges);
  for (int32_t i = 0; i <= m; ++i)
    for (int32_t j = i + 1; j <= m; ++j) {
      ends.push_back(i);
      ends.push_back(j);
    }
  uint64_t counter = 0;
  std::vector<int32_t> picked;
  for (int64_t v = m + 1; v < n; ++v) {
    picked.clear();
    const uint64_t pool = ends.size();
    while ((int32_t)picked.size() < m) {
      int32_t t = ends[draw_below(seed, 3, counter++, pool)];
      if (std::find(picked.begin(), picked.end(), t) == picked.end()) picked.push_back(t);
    }
    for (int32_t t : picked) {
      ends.push_back((int32_t)v);
      ends.push_back(t);
    }
  }
  return symmetric_csr(n, (int64_t)ends.size() / 2, [&](int64_t i, int64_t* u, int64_t* v) {
    *u = ends[2 * i];
    *v = ends[2 * i + 1];
    return true;
  });
}

// Raw counter-based draws, exposed so tests can pin the generator itself.
void sg_draw(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, uint64_t* out) {
  for (int64_t i = 0; i < count; ++i) out[i] = draw(seed, stream, first + (uint64_t)i);
}

}  // extern "C"
