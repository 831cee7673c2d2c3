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

// Counter-based draw: a 64-bit value for (seed, stream, counter).  The key
// depends only on (seed, stream); Draws caches it for loops over counters.
inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed * kGolden + mix64(stream + 0x632BE59BD9B4E019ull));
}

inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t counter) {
  return mix64(stream_key(seed, stream) + (counter + 1) * kGolden);
}

struct Draws {
  uint64_t key;
  Draws(uint64_t seed, uint64_t stream) : key(stream_key(seed, stream)) {}
  uint64_t at(uint64_t counter) const { return mix64(key + (counter + 1) * kGolden); }
  double unit(uint64_t counter) const { return (double)(at(counter) >> 11) * (1.0 / 9007199254740992.0); }
};

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

// Sort each row of `raw` (row v at start[v], deg[v] entries), drop
// duplicates, and compact the rows in place into canonical CSR.  Row v moves
// to row_ptr[v] <= start[v], and row_ptr[v + 1] <= start[v + 1]; rows are moved
// in increasing order, so a move never overwrites a row not yet moved.  `raw`
// is shrunk to the final size and becomes the graph's column array; `start` is
// overwritten by the row offsets (it must hold n + 1 entries).
Graph* finish_csr(int64_t n, int64_t* start, int64_t* deg, int32_t* raw) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* b = raw + start[v];
    int32_t* e = b + deg[v];
    std::sort(b, e);
    deg[v] = std::unique(b, e) - b;
  }
  int64_t pos = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t from = start[v];
    start[v] = pos;
    if (deg[v] > 0 && from != pos) std::memmove(raw + pos, raw + from, sizeof(int32_t) * deg[v]);
    pos += deg[v];
  }
  start[n] = pos;
  Graph* g = new Graph;
  g->n = n;
  g->nnz = pos;
  g->row_ptr = start;
  int32_t* shrunk = (int32_t*)std::realloc(raw, sizeof(int32_t) * (pos > 0 ? pos : 1));
  g->col = shrunk ? shrunk : raw;
  return g;
}

// Build a symmetric CSR from a generator of undirected pairs.  `pair(i, &u, &v)`
// returns false for a discarded draw.  Called twice per edge index (count pass
// and fill pass), so it must be a pure function of i.  `perm` (nullable)
// relabels both endpoints.  Peak memory: the arc array (4 bytes per arc before
// deduplication) and two n-sized offset arrays.
//
// The passes take the draws in blocks: a block's pairs are generated first,
// then the relabel and counter addresses of the whole block are prefetched
// before they are used, so the random accesses of a block overlap (one draw
// costs a few hundred instructions, too many for the core to run ahead to the
// next draw's memory accesses by itself).  The arc order inside a row depends
// on the thread schedule, but rows are sorted afterwards.
constexpr int kBlock = 512;

template <class PairFn>
int block_pairs(int64_t b0, int64_t draws, PairFn& pair, const int32_t* perm, int64_t* us, int64_t* vs) {
  int m = 0;
  const int64_t b1 = std::min<int64_t>(b0 + kBlock, draws);
  for (int64_t i = b0; i < b1; ++i) {
    int64_t u, v;
    if (!pair(i, &u, &v)) continue;
    us[m] = u;
    vs[m] = v;
    ++m;
  }
  if (perm) {
    for (int j = 0; j < m; ++j) {
      __builtin_prefetch(perm + us[j]);
      __builtin_prefetch(perm + vs[j]);
    }
    for (int j = 0; j < m; ++j) {
      us[j] = perm[us[j]];
      vs[j] = perm[vs[j]];
    }
  }
  return m;
}

template <class PairFn>
Graph* symmetric_csr(int64_t n, int64_t draws, PairFn pair, const int32_t* perm = nullptr) {
  int64_t* cnt = (int64_t*)std::calloc(n + 1, sizeof(int64_t));
  if (!cnt) return nullptr;
#pragma omp parallel
  {
    int64_t us[kBlock], vs[kBlock];
#pragma omp for schedule(static)
    for (int64_t b0 = 0; b0 < draws; b0 += kBlock) {
      const int m = block_pairs(b0, draws, pair, perm, us, vs);
      for (int j = 0; j < m; ++j) {
        __builtin_prefetch(cnt + us[j], 1);
        __builtin_prefetch(cnt + vs[j], 1);
      }
      for (int j = 0; j < m; ++j) {
        __atomic_fetch_add(&cnt[us[j]], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&cnt[vs[j]], 1, __ATOMIC_RELAXED);
      }
    }
  }
  int64_t* start = (int64_t*)std::malloc(sizeof(int64_t) * (n + 1));
  if (!start) { std::free(cnt); return nullptr; }
  start[0] = 0;
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + cnt[v];
  int64_t total = start[n];
  int32_t* raw = (int32_t*)std::malloc(sizeof(int32_t) * (total > 0 ? total : 1));
  if (!raw) { std::free(cnt); std::free(start); return nullptr; }
  std::memset(cnt, 0, sizeof(int64_t) * (n + 1));
#pragma omp parallel
  {
    int64_t us[kBlock], vs[kBlock], pu[kBlock], pv[kBlock];
#pragma omp for schedule(static)
    for (int64_t b0 = 0; b0 < draws; b0 += kBlock) {
      const int m = block_pairs(b0, draws, pair, perm, us, vs);
      for (int j = 0; j < m; ++j) {
        __builtin_prefetch(cnt + us[j], 1);
        __builtin_prefetch(cnt + vs[j], 1);
        __builtin_prefetch(start + us[j]);
        __builtin_prefetch(start + vs[j]);
      }
      for (int j = 0; j < m; ++j) {
        pu[j] = start[us[j]] + __atomic_fetch_add(&cnt[us[j]], 1, __ATOMIC_RELAXED);
        pv[j] = start[vs[j]] + __atomic_fetch_add(&cnt[vs[j]], 1, __ATOMIC_RELAXED);
      }
      for (int j = 0; j < m; ++j) {
        __builtin_prefetch(raw + pu[j], 1);
        __builtin_prefetch(raw + pv[j], 1);
      }
      for (int j = 0; j < m; ++j) {
        raw[pu[j]] = (int32_t)vs[j];
        raw[pv[j]] = (int32_t)us[j];
      }
    }
  }
  Graph* g = finish_csr(n, start, cnt, raw);
  std::free(cnt);
  return g;
}

// Seeded uniform random permutation (Fisher-Yates, counter-based draws) into p[n].
void fill_permutation(int64_t n, uint64_t seed, int32_t* p) {
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  const Draws d(seed, 2);
  for (int64_t i = n - 1; i > 0; --i) {
    const unsigned __int128 m = (unsigned __int128)d.at((uint64_t)i) * (uint64_t)(i + 1);
    std::swap(p[i], p[(int64_t)(m >> 64)]);
  }
}

int32_t* random_permutation(int64_t n, uint64_t seed) {
  int32_t* p = (int32_t*)std::malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  if (p) fill_permutation(n, seed, p);
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
// Hands the graph's two arrays to the caller (who frees each with
// sg_free_array) and frees the rest of the handle.
void sg_detach(void* h, int64_t** row_ptr, int32_t** col) {
  Graph* g = (Graph*)h;
  *row_ptr = g->row_ptr;
  *col = g->col;
  delete g;
}
void sg_free_array(void* p) { std::free(p); }

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
  const Draws d(seed, 1);
  auto pair = [&](int64_t i, int64_t* u, int64_t* v) {
    int64_t src = 0, dst = 0;
    // Quadrant of each level from one uniform p: [0, a) top-left, [a, a+b)
    // top-right (dst bit), [a+b, a+b+c) bottom-left (src bit), the rest
    // bottom-right (both bits); most significant bit first.  Written without
    // branches (the outcome is random, so branches would mispredict).
    const uint64_t c0 = (uint64_t)i * (uint64_t)scale;
    for (int32_t l = 0; l < scale; ++l) {
      const double p = d.unit(c0 + (uint64_t)l);
      const int64_t ge_a = p >= a, ge_ab = p >= ab, ge_abc = p >= abc;
      src = (src << 1) | ge_ab;
      dst = (dst << 1) | ((ge_a & (ge_ab ^ 1)) | ge_abc);
    }
    if (src == dst) return false;
    *u = src;
    *v = dst;
    return true;
  };
  Graph* g = symmetric_csr(n, draws, pair, perm);
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

// The relabelling permutation of sg_rmat(scale, ..., seed) for n = 2^scale
// (used by the GPU build of the same graph).
void sg_permutation(int64_t n, uint64_t seed, int32_t* out) { fill_permutation(n, seed, out); }

// Endpoint pairs drawn from the R-MAT distribution of sg_rmat(scale, ...,
// seed) -- the same quadrant recursion and the same relabelling -- from the
// counter stream `stream` (the graph itself uses stream 1), pairs first ..
// first + count - 1.  Self-loops are kept; callers filter what they need.
// Used for edge insertions that follow the graph's own degree distribution.
void sg_rmat_pairs(int32_t scale, double a, double b, double c, uint64_t seed, int32_t relabel,
                   uint64_t stream, uint64_t first, int64_t count, int32_t* out_u, int32_t* out_v) {
  const int64_t n = (int64_t)1 << scale;
  int32_t* perm = relabel ? random_permutation(n, seed) : nullptr;
  const double ab = a + b, abc = a + b + c;
  const Draws d(seed, stream);
  for (int64_t i = 0; i < count; ++i) {
    int64_t src = 0, dst = 0;
    const uint64_t c0 = (first + (uint64_t)i) * (uint64_t)scale;
    for (int32_t l = 0; l < scale; ++l) {
      const double p = d.unit(c0 + (uint64_t)l);
      const int64_t ge_a = p >= a, ge_ab = p >= ab, ge_abc = p >= abc;
      src = (src << 1) | ge_ab;
      dst = (dst << 1) | ((ge_a & (ge_ab ^ 1)) | ge_abc);
    }
    out_u[i] = perm ? perm[src] : (int32_t)src;
    out_v[i] = perm ? perm[dst] : (int32_t)dst;
  }
  std::free(perm);
}

// Raw counter-based draws, exposed so tests can pin the generator itself.
void sg_draw(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, uint64_t* out) {
  for (int64_t i = 0; i < count; ++i) out[i] = draw(seed, stream, first + (uint64_t)i);
}

}  // extern "C"
