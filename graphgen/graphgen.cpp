// Seeded synthetic graph generators.
//
// This module produces INPUTS only: symmetric CSR graphs of the shapes used to
// exercise label propagation (planted partition, R-MAT power law, 2-D k-nearest
// -neighbour "road" graphs, batches of planted graphs).  It contains none of the
// community-detection arithmetic; both the CPU oracle and the GPU library read
// the graphs it writes.
//
// Randomness: splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014) seeds xoshiro256** (Blackman & Vigna,
// "Scrambled linear pseudorandom number generators", 2018).  Every parallel
// chunk owns its own stream, so output is independent of the thread count.
// The file is built without -march / fast-math so results are bit-identical on
// any x86-64 host running the same binary.
//
// CSR conventions: offsets int64[n+1], cols int32[nnz] sorted ascending within
// each row, no self-loops, no duplicates, symmetric (j in row i <=> i in row j);
// weights uint32[nnz] with w_ij == w_ji, or NULL for unit weights.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t splitmix64_next(uint64_t &x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

struct Xoshiro256ss {
  uint64_t s[4];
  // One independent stream per (seed, stream) pair.
  Xoshiro256ss(uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ (stream * 0xd1b54a32d192ed03ULL);
    for (int k = 0; k < 4; ++k) s[k] = splitmix64_next(x);
  }
  uint64_t next() {
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0,1)
  // Unbiased integer in [0, bound) by rejection.
  uint64_t below(uint64_t bound) {
    if (bound <= 1) return 0;
    const uint64_t lim = UINT64_MAX - (UINT64_MAX % bound);
    for (;;) {
      uint64_t r = next();
      if (r < lim) return r % bound;
    }
  }
};

// Symmetric per-pair hash used for weights: depends only on {u, v}.
inline uint32_t pair_weight(uint64_t seed, int64_t u, int64_t v, uint32_t wmin, uint32_t wmax) {
  if (u > v) std::swap(u, v);
  uint64_t x = seed ^ 0x5851f42d4c957f2dULL;
  x ^= (uint64_t)u * 0x9e3779b97f4a7c15ULL;
  uint64_t h = splitmix64_next(x);
  h ^= (uint64_t)v * 0xc2b2ae3d27d4eb4fULL;
  uint64_t y = h;
  h = splitmix64_next(y);
  const uint64_t span = (uint64_t)wmax - (uint64_t)wmin + 1;
  return (uint32_t)((uint64_t)wmin + h % span);
}

// Progress lines on stderr (GRAPHGEN_VERBOSE=1): long generations print each
// phase as it ends so a supervising process sees activity.
inline bool verbose() {
  static const bool v = getenv("GRAPHGEN_VERBOSE") && getenv("GRAPHGEN_VERBOSE")[0] == '1';
  return v;
}
inline double now_s() { return omp_get_wtime(); }
inline void progress(const char *what, double t0) {
  if (verbose()) {
    fprintf(stderr, "graphgen: %s done at %.1f s\n", what, now_s() - t0);
    fflush(stderr);
  }
}

inline void atomic_inc(int64_t *p) { __atomic_fetch_add(p, (int64_t)1, __ATOMIC_RELAXED); }
inline int64_t atomic_fetch_inc(int64_t *p) { return __atomic_fetch_add(p, (int64_t)1, __ATOMIC_RELAXED); }

}  // namespace

extern "C" {

typedef struct gg_graph {
  int64_t n;         // vertices (sum over graphs for a batch)
  int64_t nnz;       // directed CSR entries (each undirected edge twice)
  int64_t *offsets;  // int64[n+1]; for a batch: offsets into the concatenated cols
  int32_t *cols;     // int32[nnz]; for a batch: LOCAL ids within the graph
  uint32_t *weights; // uint32[nnz] or NULL (unit weights)
  int64_t num_graphs;   // 1 for a single graph
  int64_t *vtx_base;    // int64[num_graphs+1] (batch only, else NULL)
  int64_t *edge_base;   // int64[num_graphs+1] (batch only, else NULL)
} gg_graph;

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->offsets);
  free(g->cols);
  free(g->weights);
  free(g->vtx_base);
  free(g->edge_base);
  memset(g, 0, sizeof(*g));
}

}  // extern "C"

namespace {

// Builds a symmetric, deduplicated, self-loop-free CSR from an edge source that
// can be replayed: src(chunk, emit) calls emit(u, v) for each generated
// undirected edge of that chunk, identically on every call.  Two passes (count,
// scatter) keep peak memory at one pre-deduplication column array.
template <class Src>
int build_sym_csr(int64_t n, int64_t nchunks, Src src, uint64_t wseed, uint32_t wmin,
                  uint32_t wmax, int unit_weights, gg_graph *out) {
  memset(out, 0, sizeof(*out));
  out->n = n;
  out->num_graphs = 1;
  const double t0 = now_s();
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nchunks; ++c) {
    src(c, [&](int64_t u, int64_t v) {
      if (u == v) return;
      atomic_inc(&cnt[u]);
      atomic_inc(&cnt[v]);
    });
  }
  progress("degree count", t0);
  // Exclusive prefix sum -> row starts (pre-dedup).
  int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!start) { free(cnt); return -2; }
  int64_t acc = 0;
  for (int64_t i = 0; i < n; ++i) { start[i] = acc; acc += cnt[i]; }
  start[n] = acc;
  const int64_t raw = acc;
  int32_t *tmp = (int32_t *)malloc((size_t)std::max<int64_t>(raw, 1) * sizeof(int32_t));
  if (!tmp) { free(cnt); free(start); return -2; }
  // cnt becomes the per-row cursor.
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) cnt[i] = start[i];
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nchunks; ++c) {
    src(c, [&](int64_t u, int64_t v) {
      if (u == v) return;
      tmp[atomic_fetch_inc(&cnt[u])] = (int32_t)v;
      tmp[atomic_fetch_inc(&cnt[v])] = (int32_t)u;
    });
  }
  progress("scatter", t0);
  // Sort and deduplicate each row; cnt[i] := new degree.
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int32_t *b = tmp + start[i], *e = tmp + start[i + 1];
    std::sort(b, e);
    cnt[i] = std::unique(b, e) - b;
  }
  progress("row sort", t0);
  int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!off) { free(cnt); free(start); free(tmp); return -2; }
  acc = 0;
  for (int64_t i = 0; i < n; ++i) { off[i] = acc; acc += cnt[i]; }
  off[n] = acc;
  const int64_t nnz = acc;
  int32_t *cols = (int32_t *)malloc((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));
  uint32_t *w = nullptr;
  if (!unit_weights) w = (uint32_t *)malloc((size_t)std::max<int64_t>(nnz, 1) * sizeof(uint32_t));
  if (!cols || (!unit_weights && !w)) {
    free(cnt); free(start); free(tmp); free(off); free(cols); free(w);
    return -2;
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = cnt[i];
    memcpy(cols + off[i], tmp + start[i], (size_t)d * sizeof(int32_t));
    if (w)
      for (int64_t k = 0; k < d; ++k) w[off[i] + k] = pair_weight(wseed, i, cols[off[i] + k], wmin, wmax);
  }
  free(cnt);
  free(start);
  free(tmp);
  progress("compaction", t0);
  out->nnz = nnz;
  out->offsets = off;
  out->cols = cols;
  out->weights = w;
  return 0;
}

// Fisher-Yates permutation of [0, n).
std::vector<int32_t> random_permutation(int64_t n, uint64_t seed) {
  std::vector<int32_t> p((size_t)n);
  for (int64_t i = 0; i < n; ++i) p[(size_t)i] = (int32_t)i;
  Xoshiro256ss rng(seed, 0x7065726dULL);
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)rng.below((uint64_t)i + 1);
    std::swap(p[(size_t)i], p[(size_t)j]);
  }
  return p;
}

// Geometric skipping over the pairs (v, w), w < v < s, each kept with
// probability p (Batagelj & Brandes, "Efficient generation of large random
// networks", Phys. Rev. E 71, 2005).
template <class Emit>
void gnp_pairs(int64_t s, double p, Xoshiro256ss &rng, Emit emit) {
  if (s < 2 || p <= 0.0) return;
  if (p >= 1.0) {
    for (int64_t v = 1; v < s; ++v)
      for (int64_t w = 0; w < v; ++w) emit(v, w);
    return;
  }
  const double lp = std::log(1.0 - p);
  int64_t v = 1, w = -1;
  while (v < s) {
    const double r = rng.uniform();
    w = w + 1 + (int64_t)std::floor(std::log(1.0 - r) / lp);
    while (w >= v && v < s) { w -= v; ++v; }
    if (v < s) emit(v, w);
  }
}

// One planted-partition graph into a sorted, deduplicated symmetric edge list.
// Blocks are consecutive id ranges [floor(b n / k), floor((b+1) n / k)).
struct PlantedParams { int64_t n, k; double p_in; int64_t inter_pairs; };

void planted_edges(const PlantedParams &P, uint64_t seed, uint64_t stream_base,
                   std::vector<std::pair<int32_t, int32_t>> &edges) {
  edges.clear();
  for (int64_t b = 0; b < P.k; ++b) {
    const int64_t lo = b * P.n / P.k, hi = (b + 1) * P.n / P.k;
    Xoshiro256ss rng(seed, stream_base + (uint64_t)b);
    gnp_pairs(hi - lo, P.p_in, rng, [&](int64_t v, int64_t w) {
      edges.emplace_back((int32_t)(lo + w), (int32_t)(lo + v));
    });
  }
  if (P.k > 1) {
    Xoshiro256ss rng(seed, stream_base + (uint64_t)P.k);
    for (int64_t t = 0; t < P.inter_pairs; ++t) {
      const int64_t u = (int64_t)rng.below((uint64_t)P.n);
      // Block of u: the b with floor(b n / k) <= u < floor((b+1) n / k).
      int64_t b = (u * P.k) / P.n;
      while (b + 1 < P.k && (b + 1) * P.n / P.k <= u) ++b;
      while (b > 0 && b * P.n / P.k > u) --b;
      int64_t v;
      for (;;) {
        v = (int64_t)rng.below((uint64_t)P.n);
        const int64_t lo = b * P.n / P.k, hi = (b + 1) * P.n / P.k;
        if (v < lo || v >= hi) break;
      }
      edges.emplace_back((int32_t)std::min(u, v), (int32_t)std::max(u, v));
    }
  }
}

}  // namespace

extern "C" {

// Planted partition: n vertices in k consecutive blocks; each intra-block pair
// kept with probability p_in; inter_pairs uniform pairs in different blocks.
// Unit weights when wmax == 0, else uniform per undirected edge in [wmin, wmax].
int gg_planted(int64_t n, int64_t k, double p_in, int64_t inter_pairs, uint32_t wmin,
               uint32_t wmax, uint64_t seed, gg_graph *out) {
  if (!out || n < 0 || n >= ((int64_t)1 << 31) || k < 1 || k > std::max<int64_t>(n, 1)) return -1;
  PlantedParams P{n, k, p_in, inter_pairs};
  std::vector<std::pair<int32_t, int32_t>> edges;
  planted_edges(P, seed, 0, edges);
  const int64_t m = (int64_t)edges.size();
  const int64_t chunk = 1 << 16;
  const int64_t nchunks = (m + chunk - 1) / chunk;
  auto src = [&](int64_t c, auto emit) {
    const int64_t lo = c * chunk, hi = std::min(m, lo + chunk);
    for (int64_t t = lo; t < hi; ++t) emit(edges[(size_t)t].first, edges[(size_t)t].second);
  };
  return build_sym_csr(n, nchunks, src, seed, wmin, wmax, wmax == 0, out);
}

// R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004): edge_factor * 2^scale
// edges, each placed by `scale` independent quadrant choices with
// probabilities a, b, c, d = 1-a-b-c (no noise).  With permute != 0 vertex ids
// are relabelled by a seeded random permutation (as Graph500 does).  Self
// loops and duplicates are removed, the result symmetrised.  Unit weights when
// wmax == 0, else uniform per undirected edge in [wmin, wmax].
int gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, int permute,
            uint32_t wmin, uint32_t wmax, uint64_t seed, gg_graph *out) {
  if (!out || scale < 1 || scale > 30 || edge_factor < 1) return -1;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edge_factor << scale;
  const uint64_t ta = (uint64_t)std::llround(a * 4294967296.0);
  const uint64_t tab = (uint64_t)std::llround((a + b) * 4294967296.0);
  const uint64_t tabc = (uint64_t)std::llround((a + b + c) * 4294967296.0);
  std::vector<int32_t> perm;
  if (permute) perm = random_permutation(n, seed);
  const int64_t chunk = 1 << 20;
  const int64_t nchunks = (m + chunk - 1) / chunk;
  auto src = [&](int64_t ch, auto emit) {
    Xoshiro256ss rng(seed, 0x524d4154ULL + (uint64_t)ch * 2 + 1);
    const int64_t lo = ch * chunk, hi = std::min(m, lo + chunk);
    for (int64_t t = lo; t < hi; ++t) {
      int64_t u = 0, v = 0;
      uint64_t bits = 0;
      int have = 0;
      for (int lvl = 0; lvl < scale; ++lvl) {
        if (have == 0) { bits = rng.next(); have = 2; }
        const uint64_t r = bits & 0xffffffffULL;
        bits >>= 32;
        --have;
        const int q = r < ta ? 0 : r < tab ? 1 : r < tabc ? 2 : 3;
        u = (u << 1) | (q >> 1);
        v = (v << 1) | (q & 1);
      }
      if (permute) { u = perm[(size_t)u]; v = perm[(size_t)v]; }
      emit(u, v);
    }
  };
  return build_sym_csr(n, nchunks, src, seed, wmin, wmax, wmax == 0, out);
}

// Random geometric "road-like" graph: n points uniform in the unit square, each
// joined to its k nearest neighbours (Euclidean, ties by index), union
// symmetrised.  Unit weights.
int gg_road_knn(int64_t n, int k, uint64_t seed, gg_graph *out) {
  if (!out || n < 0 || n >= ((int64_t)1 << 31) || k < 1 || k > 16) return -1;
  if (n == 0) {
    memset(out, 0, sizeof(*out));
    out->num_graphs = 1;
    out->offsets = (int64_t *)calloc(1, sizeof(int64_t));
    out->cols = (int32_t *)malloc(sizeof(int32_t));
    return out->offsets && out->cols ? 0 : -2;
  }
  std::vector<double> x((size_t)n), y((size_t)n);
  {
    Xoshiro256ss rng(seed, 0x726f6164ULL);
    for (int64_t i = 0; i < n; ++i) { x[(size_t)i] = rng.uniform(); y[(size_t)i] = rng.uniform(); }
  }
  const int64_t g = std::max<int64_t>(1, (int64_t)std::floor(std::sqrt((double)n / 2.0)));
  const double cell = 1.0 / (double)g;
  auto cell_of = [&](double t) { int64_t c = (int64_t)(t * (double)g); return c >= g ? g - 1 : c; };
  std::vector<int64_t> cstart((size_t)(g * g + 1), 0);
  std::vector<int32_t> bucket((size_t)n);
  for (int64_t i = 0; i < n; ++i) cstart[(size_t)(cell_of(y[(size_t)i]) * g + cell_of(x[(size_t)i]) + 1)]++;
  for (int64_t c = 0; c < g * g; ++c) cstart[(size_t)c + 1] += cstart[(size_t)c];
  {
    std::vector<int64_t> cur(cstart.begin(), cstart.end() - 1);
    for (int64_t i = 0; i < n; ++i) bucket[(size_t)cur[(size_t)(cell_of(y[(size_t)i]) * g + cell_of(x[(size_t)i]))]++] = (int32_t)i;
  }
  const int kk = (int)std::min<int64_t>(k, n - 1);
  std::vector<int32_t> nbr((size_t)n * (size_t)std::max(kk, 1), -1);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    if (kk <= 0) continue;
    double bd[16];
    int32_t bi[16];
    int have = 0;
    const double xi = x[(size_t)i], yi = y[(size_t)i];
    const int64_t cx = cell_of(xi), cy = cell_of(yi);
    auto consider = [&](int32_t j) {
      if (j == (int32_t)i) return;
      const double dx = x[(size_t)j] - xi, dy = y[(size_t)j] - yi;
      const double d = dx * dx + dy * dy;
      if (have == kk && (d > bd[kk - 1] || (d == bd[kk - 1] && j > bi[kk - 1]))) return;
      int p = have < kk ? have++ : kk - 1;
      while (p > 0 && (bd[p - 1] > d || (bd[p - 1] == d && bi[p - 1] > j))) {
        bd[p] = bd[p - 1];
        bi[p] = bi[p - 1];
        --p;
      }
      bd[p] = d;
      bi[p] = j;
    };
    for (int64_t r = 0;; ++r) {
      for (int64_t yy = cy - r; yy <= cy + r; ++yy) {
        if (yy < 0 || yy >= g) continue;
        const bool edge_row = (yy == cy - r || yy == cy + r);
        for (int64_t xx = cx - r; xx <= cx + r; ++xx) {
          if (xx < 0 || xx >= g) continue;
          if (!edge_row && xx != cx - r && xx != cx + r) continue;
          const int64_t c = yy * g + xx;
          for (int64_t t = cstart[(size_t)c]; t < cstart[(size_t)c + 1]; ++t) consider(bucket[(size_t)t]);
        }
      }
      const double reach = (double)r * cell;
      if (have == kk && bd[kk - 1] < reach * reach) break;
      if (r > 2 * g + 2) break;  // whole square covered
    }
    for (int t = 0; t < have; ++t) nbr[(size_t)i * kk + t] = bi[t];
  }
  const int64_t chunk = 1 << 16;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  auto src = [&](int64_t ch, auto emit) {
    const int64_t lo = ch * chunk, hi = std::min(n, lo + chunk);
    for (int64_t i = lo; i < hi; ++i)
      for (int t = 0; t < kk; ++t) {
        const int32_t j = nbr[(size_t)i * kk + t];
        if (j >= 0) emit(i, j);
      }
  };
  return build_sym_csr(n, nchunks, src, seed, 1, 1, 1, out);
}

// A batch of independent planted-partition graphs, concatenated.  Graph g has
//   N_g = round(exp(U[ln nmin, ln nmax])) vertices,
//   k_g = round(exp(U[ln kmin, ln kmax])) blocks, clamped to [1, max(1, N_g/10)],
//   target mean degree d_g ~ U[dmin, dmax] of which `inter_deg` is inter-block:
//   p_in = (d_g - inter_deg) / (N_g/k_g - 1) clamped to [0, 1], and
//   round(N_g * inter_deg / 2) uniform inter-block pairs.
// cols hold LOCAL ids (0..N_g-1); offsets index the concatenated cols array
// (offsets[vtx_base[g]] == edge_base[g]).  Unit weights.
int gg_batched_planted(int64_t num_graphs, int64_t nmin, int64_t nmax, int64_t kmin, int64_t kmax,
                       double dmin, double dmax, double inter_deg, uint64_t seed, gg_graph *out) {
  if (!out || num_graphs < 0 || nmin < 1 || nmax < nmin || kmin < 1 || kmax < kmin) return -1;
  memset(out, 0, sizeof(*out));
  std::vector<PlantedParams> P((size_t)num_graphs);
  {
    Xoshiro256ss rng(seed, 0x62617463ULL);
    for (int64_t g = 0; g < num_graphs; ++g) {
      const double un = rng.uniform(), uk = rng.uniform(), ud = rng.uniform();
      const int64_t n = (int64_t)std::llround(std::exp(std::log((double)nmin) + un * (std::log((double)nmax) - std::log((double)nmin))));
      int64_t k = (int64_t)std::llround(std::exp(std::log((double)kmin) + uk * (std::log((double)kmax) - std::log((double)kmin))));
      k = std::max<int64_t>(1, std::min<int64_t>(k, std::max<int64_t>(1, n / 10)));
      const double d = dmin + ud * (dmax - dmin);
      const double s = (double)n / (double)k;
      double p = s > 1.0 ? (d - inter_deg) / (s - 1.0) : 0.0;
      p = std::min(1.0, std::max(0.0, p));
      const int64_t inter = (int64_t)std::llround((double)n * inter_deg / 2.0);
      P[(size_t)g] = PlantedParams{n, k, p, inter};
    }
  }
  out->num_graphs = num_graphs;
  out->vtx_base = (int64_t *)calloc((size_t)num_graphs + 1, sizeof(int64_t));
  out->edge_base = (int64_t *)calloc((size_t)num_graphs + 1, sizeof(int64_t));
  if (!out->vtx_base || !out->edge_base) { gg_free(out); return -2; }
  for (int64_t g = 0; g < num_graphs; ++g) out->vtx_base[g + 1] = out->vtx_base[g] + P[(size_t)g].n;
  const int64_t ntot = out->vtx_base[num_graphs];
  if (ntot >= ((int64_t)1 << 40)) { gg_free(out); return -1; }
  // Per-graph degrees first (sorted unique symmetric lists), then concatenate.
  std::vector<std::vector<int32_t>> rows_cols((size_t)num_graphs);
  std::vector<std::vector<int64_t>> rows_off((size_t)num_graphs);
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < num_graphs; ++g) {
    std::vector<std::pair<int32_t, int32_t>> e;
    planted_edges(P[(size_t)g], seed, ((uint64_t)g + 1) << 24, e);
    const int64_t n = P[(size_t)g].n;
    std::vector<std::pair<int32_t, int32_t>> d;
    d.reserve(e.size() * 2);
    for (auto &pr : e) {
      if (pr.first == pr.second) continue;
      d.emplace_back(pr.first, pr.second);
      d.emplace_back(pr.second, pr.first);
    }
    std::vector<std::pair<int32_t, int32_t>>().swap(e);
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    std::vector<int64_t> off((size_t)n + 1, 0);
    std::vector<int32_t> cols(d.size());
    for (size_t t = 0; t < d.size(); ++t) { off[(size_t)d[t].first + 1]++; cols[t] = d[t].second; }
    for (int64_t i = 0; i < n; ++i) off[(size_t)i + 1] += off[(size_t)i];
    rows_cols[(size_t)g].swap(cols);
    rows_off[(size_t)g].swap(off);
  }
  if (err) { gg_free(out); return err; }
  for (int64_t g = 0; g < num_graphs; ++g)
    out->edge_base[g + 1] = out->edge_base[g] + (int64_t)rows_cols[(size_t)g].size();
  const int64_t nnz = out->edge_base[num_graphs];
  out->n = ntot;
  out->nnz = nnz;
  out->offsets = (int64_t *)malloc(((size_t)ntot + 1) * sizeof(int64_t));
  out->cols = (int32_t *)malloc((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));
  if (!out->offsets || !out->cols) { gg_free(out); return -2; }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < num_graphs; ++g) {
    const int64_t vb = out->vtx_base[g], eb = out->edge_base[g], n = P[(size_t)g].n;
    for (int64_t i = 0; i < n; ++i) out->offsets[vb + i] = eb + rows_off[(size_t)g][(size_t)i];
    if (!rows_cols[(size_t)g].empty())
      memcpy(out->cols + eb, rows_cols[(size_t)g].data(), rows_cols[(size_t)g].size() * sizeof(int32_t));
  }
  out->offsets[ntot] = nnz;
  return 0;
}

}  // extern "C"
