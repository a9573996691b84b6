// GSL-LPA oracle: a plain, slow, single-threaded CPU implementation.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or
// load this file; only the test suite, the smoke check and the CPU baseline leg
// of the benchmark use it.  It shares no code, header or table with the GPU
// path.
//
// What it computes (Sahu, "GSL-LPA: Fast Label Propagation Algorithm (LPA) for
// Community Detection with no Internally-Disconnected Communities",
// arXiv:2403.01261):
//   * oracle_lpa          -- Alg. 3 (lpa / lpaMove / scanCommunities) with the
//                            label rule of Eq. 2, then the split of Alg. 2.
//   * oracle_lpa_f32      -- the same with fp32 weights summed in fp64.
//   * oracle_split_bfs    -- Alg. 2 (split disconnected communities by BFS).
//   * oracle_split_lp     -- Alg. 1 (min-label LP, with or without pruning).
//   * oracle_modularity   -- Eq. 1, second form.
//   * oracle_disconnected -- Alg. 4 (find internally-disconnected communities).
//
// Readings where the paper leaves a choice (all are listed with the design
// notes of the repository):
//   - Sweeps are synchronous: every vertex of sweep t reads the labels that
//     sweep t-1 left; changes become visible only when the sweep ends.  (The
//     paper's lpaMove writes C[i] in place inside a parallel loop, Alg. 3,
//     which is schedule-dependent.)
//   - Among labels of maximum summed weight the smallest label wins; the
//     vertex's own label gets no preference.
//   - A vertex whose row holds no entry other than self loops keeps its label.
//   - Every row entry with j != i contributes its weight (duplicates add, a
//     zero weight still makes its label a candidate).
//   - Weights are unsigned 32-bit integers summed exactly in 64 bits; NULL
//     weights mean unit weights.
//   - Convergence is the literal test dN / N <= tau in double precision, and
//     N counts every vertex.
//   - Alg. 2's garbled lines are read as: c = C[i]; BFS follows j when
//     C[j] == C[i]; seeds are taken in ascending vertex order.  Hence
//     C'[v] = smallest vertex id of v's connected piece of its community.
//   - Pruning (Alg. 3 "mark processed / mark neighbours unprocessed") under
//     synchronous sweeps: a vertex is processed in sweep t+1 iff one of its
//     neighbours changed label in sweep t; every vertex is unprocessed in
//     sweep 0.
//   - Modularity with zero total edge weight is defined as 0.
//
// Error behaviour: functions return 0 on success, -1 on invalid arguments
// (negative sizes, offsets not starting at 0 / decreasing, column or label
// out of range), -2 on allocation failure.
#include <cstdint>
#include <cstring>
#include <deque>
#include <vector>

namespace {

bool valid_csr(int64_t n, const int64_t *off, const int32_t *cols) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return false;
  if (n == 0) return true;
  if (!off || off[0] != 0) return false;
  for (int64_t i = 0; i < n; ++i)
    if (off[i + 1] < off[i]) return false;
  if (off[n] > 0 && !cols) return false;
  for (int64_t e = 0; e < off[n]; ++e)
    if (cols[e] < 0 || (int64_t)cols[e] >= n) return false;
  return true;
}

bool valid_labels(int64_t n, const int32_t *lab) {
  if (n > 0 && !lab) return false;
  for (int64_t i = 0; i < n; ++i)
    if (lab[i] < 0 || (int64_t)lab[i] >= n) return false;
  return true;
}

// Weight of entry e: uint32 weights summed in 64-bit integers, or fp32
// weights summed in fp64 (the paper's precision, Sec. 5.1.2); NULL weights
// are 1.
inline uint64_t weight_of(const uint32_t *w, int64_t e) { return w ? (uint64_t)w[e] : 1u; }
inline double weight_of(const float *w, int64_t e) { return w ? (double)w[e] : 1.0; }

// scanCommunities (Alg. 3): the per-vertex label -> summed weight table,
// skipping self loops, as a sparse accumulator (sums in CSR entry order).
// Returns the most weighted label (smallest on ties) or -1 if the table is
// empty.
template <class W, class Acc>
struct Scanner {
  std::vector<Acc> sum;
  std::vector<int64_t> stamp;
  std::vector<int32_t> touched;
  int64_t epoch = 0;
  explicit Scanner(int64_t n) : sum((size_t)n, 0), stamp((size_t)n, -1) {}

  int32_t best_label(int64_t i, const int64_t *off, const int32_t *cols, const W *w, const int32_t *C) {
    ++epoch;
    touched.clear();
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      const int64_t j = cols[e];
      if (j == i) continue;
      const int32_t c = C[j];
      if (stamp[(size_t)c] != epoch) {
        stamp[(size_t)c] = epoch;
        sum[(size_t)c] = 0;
        touched.push_back(c);
      }
      sum[(size_t)c] += weight_of(w, e);
    }
    int32_t best = -1;
    Acc best_w = 0;
    for (int32_t c : touched) {
      const Acc s = sum[(size_t)c];
      if (best < 0 || s > best_w || (s == best_w && c < best)) {
        best = c;
        best_w = s;
      }
    }
    return best;
  }
};

// bfsVisitForEach (Alg. 2 / Alg. 4): BFS from s over entries (u, v) with
// f_if(v); every visited vertex is marked in vis and passed to f_do.
template <class FIf, class FDo>
void bfs_visit_for_each(std::vector<uint8_t> &vis, const int64_t *off, const int32_t *cols,
                        int64_t s, FIf f_if, FDo f_do) {
  std::deque<int64_t> q;
  vis[(size_t)s] = 1;
  q.push_back(s);
  while (!q.empty()) {
    const int64_t u = q.front();
    q.pop_front();
    f_do(u);
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int64_t v = cols[e];
      if (vis[(size_t)v] || !f_if(v)) continue;
      vis[(size_t)v] = 1;
      q.push_back(v);
    }
  }
}

void split_bfs(int64_t n, const int64_t *off, const int32_t *cols, const int32_t *C, int32_t *Cp) {
  // Alg. 2: C'[i] = i, then for each unvisited vertex in ascending order,
  // label everything reachable inside its community with the seed's label.
  std::vector<uint8_t> vis((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) Cp[i] = (int32_t)i;
  for (int64_t i = 0; i < n; ++i) {
    if (vis[(size_t)i]) continue;
    const int32_t c = C[i];
    const int32_t cp = Cp[i];
    bfs_visit_for_each(vis, off, cols, i, [&](int64_t j) { return C[j] == c; },
                       [&](int64_t j) { Cp[j] = cp; });
  }
}

}  // namespace

extern "C" {

// Alg. 3 (lpa) with synchronous sweeps, optional pruning, optional split.
//   n, off, cols, w : CSR (w may be NULL: unit weights)
//   max_iters, tol  : MAX_ITERATIONS and tau
//   prune           : nonzero -> process only vertices whose neighbour changed
//   split           : nonzero -> apply Alg. 2 after the sweeps
//   labels_out      : int32[n] final labels
//   iters_out       : sweeps performed (may be NULL)
//   dn_hist         : int64[max_iters], dN of each performed sweep (may be NULL)
//   history         : int32[max_iters * n], labels after each sweep (may be NULL)
//   processed_hist  : int64[max_iters], vertices processed per sweep (may be NULL)
}  // extern "C"

namespace {

template <class W, class Acc>
int lpa_impl(int64_t n, const int64_t *off, const int32_t *cols, const W *w, int32_t max_iters, double tol,
             int prune, int split, int32_t *labels_out, int32_t *iters_out, int64_t *dn_hist,
             int32_t *history, int64_t *processed_hist) {
  if (!valid_csr(n, off, cols) || max_iters < 0 || !(tol >= 0.0 && tol <= 1.0)) return -1;
  if (n > 0 && !labels_out) return -1;
  if (iters_out) *iters_out = 0;
  if (n == 0) return 0;
  // Vertex membership C = [0 .. |V|); all vertices unprocessed.
  std::vector<int32_t> C((size_t)n), Cn((size_t)n);
  for (int64_t i = 0; i < n; ++i) C[(size_t)i] = (int32_t)i;
  std::vector<uint8_t> unprocessed((size_t)n, 1), next_unprocessed((size_t)n, 0);
  Scanner<W, Acc> scan(n);
  int32_t l = 0;
  for (; l < max_iters;) {
    // lpaMove: every unprocessed vertex reads C (the previous sweep's labels);
    // changes go to Cn and take effect when the sweep ends.
    Cn = C;
    std::fill(next_unprocessed.begin(), next_unprocessed.end(), 0);
    int64_t dN = 0, processed = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (prune && !unprocessed[(size_t)i]) continue;
      ++processed;  // mark i as processed
      const int32_t cstar = scan.best_label(i, off, cols, w, C.data());
      if (cstar < 0 || cstar == C[(size_t)i]) continue;
      Cn[(size_t)i] = cstar;
      ++dN;
      for (int64_t e = off[i]; e < off[i + 1]; ++e) next_unprocessed[(size_t)cols[e]] = 1;
    }
    C.swap(Cn);
    if (prune) unprocessed.swap(next_unprocessed);
    if (dn_hist) dn_hist[l] = dN;
    if (processed_hist) processed_hist[l] = processed;
    if (history) memcpy(history + (size_t)l * (size_t)n, C.data(), (size_t)n * sizeof(int32_t));
    ++l;
    if ((double)dN / (double)n <= tol) break;  // converged?
  }
  if (iters_out) *iters_out = l;
  if (split)
    split_bfs(n, off, cols, C.data(), labels_out);
  else
    memcpy(labels_out, C.data(), (size_t)n * sizeof(int32_t));
  return 0;
}

}  // namespace

extern "C" {

int oracle_lpa(int64_t n, const int64_t *off, const int32_t *cols, const uint32_t *w, int32_t max_iters,
               double tol, int prune, int split, int32_t *labels_out, int32_t *iters_out, int64_t *dn_hist,
               int32_t *history, int64_t *processed_hist) {
  return lpa_impl<uint32_t, uint64_t>(n, off, cols, w, max_iters, tol, prune, split, labels_out, iters_out,
                                      dn_hist, history, processed_hist);
}

// The same with fp32 weights summed in fp64 in CSR entry order (the paper's
// precision).  Weights must be finite and >= 0.
int oracle_lpa_f32(int64_t n, const int64_t *off, const int32_t *cols, const float *w, int32_t max_iters,
                   double tol, int prune, int split, int32_t *labels_out, int32_t *iters_out, int64_t *dn_hist,
                   int32_t *history, int64_t *processed_hist) {
  if (w && n > 0 && off)
    for (int64_t e = 0; e < off[n]; ++e)
      if (!(w[e] >= 0.0f) || w[e] > 3.4e38f) return -1;
  return lpa_impl<float, double>(n, off, cols, w, max_iters, tol, prune, split, labels_out, iters_out, dn_hist,
                                 history, processed_hist);
}

// Alg. 2 (splitDisconnectedBfs).
int oracle_split_bfs(int64_t n, const int64_t *off, const int32_t *cols, const int32_t *labels_in,
                     int32_t *labels_out) {
  if (!valid_csr(n, off, cols) || !valid_labels(n, labels_in)) return -1;
  if (n > 0 && !labels_out) return -1;
  split_bfs(n, off, cols, labels_in, labels_out);
  return 0;
}

// Alg. 1 (splitDisconnectedLp): min-label propagation restricted to same-
// community neighbours, in place, until no label changes.  prune != 0 is the
// LPP variant.  rounds_out (may be NULL) receives the number of passes.
int oracle_split_lp(int64_t n, const int64_t *off, const int32_t *cols, const int32_t *labels_in,
                    int prune, int32_t *labels_out, int64_t *rounds_out) {
  if (!valid_csr(n, off, cols) || !valid_labels(n, labels_in)) return -1;
  if (n > 0 && !labels_out) return -1;
  const int32_t *C = labels_in;
  int32_t *Cp = labels_out;
  std::vector<uint8_t> unprocessed((size_t)n, 1);
  for (int64_t i = 0; i < n; ++i) Cp[i] = (int32_t)i;
  int64_t rounds = 0;
  for (;;) {
    int64_t dN = 0;
    ++rounds;
    for (int64_t i = 0; i < n; ++i) {
      if (!unprocessed[(size_t)i]) continue;
      if (prune) unprocessed[(size_t)i] = 0;
      int32_t cmin = Cp[i];
      for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        const int64_t j = cols[e];
        if (C[j] == C[i] && Cp[j] < cmin) cmin = Cp[j];
      }
      if (cmin == Cp[i]) continue;
      Cp[i] = cmin;
      ++dN;
      if (prune)
        for (int64_t e = off[i]; e < off[i + 1]; ++e)
          if (C[cols[e]] == C[i]) unprocessed[(size_t)cols[e]] = 1;
    }
    if (dN == 0) break;
  }
  if (rounds_out) *rounds_out = rounds;
  return 0;
}

// Eq. 1, second form: Q = sum_c [sigma_c / 2m - (Sigma_c / 2m)^2], where
// sigma_c sums w over CSR entries (i, j) with C_i = C_j = c, Sigma_c sums w
// over entries with C_i = c, and 2m sums w over all entries.  The sums are
// exact integers; Q = I / 2m - S2 / (2m)^2 with I = sum_c sigma_c and
// S2 = sum_c Sigma_c^2, evaluated once in double precision.
// Also reports the integer parts (may be NULL): parts[0] = 2m, parts[1] = I,
// parts[2] = low 64 bits of S2, parts[3] = high 64 bits of S2.
int oracle_modularity(int64_t n, const int64_t *off, const int32_t *cols, const uint32_t *w,
                      const int32_t *labels, double *q_out, uint64_t *parts) {
  if (!valid_csr(n, off, cols) || !valid_labels(n, labels) || !q_out) return -1;
  std::vector<uint64_t> sigma((size_t)n, 0), Sigma((size_t)n, 0);
  uint64_t two_m = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      const uint64_t we = weight_of(w, e);
      const int32_t c = labels[i];
      two_m += we;
      Sigma[(size_t)c] += we;
      if (labels[cols[e]] == c) sigma[(size_t)c] += we;
    }
  uint64_t I = 0;
  unsigned __int128 S2 = 0;
  for (int64_t c = 0; c < n; ++c) {
    I += sigma[(size_t)c];
    S2 += (unsigned __int128)Sigma[(size_t)c] * Sigma[(size_t)c];
  }
  if (parts) {
    parts[0] = two_m;
    parts[1] = I;
    parts[2] = (uint64_t)S2;
    parts[3] = (uint64_t)(S2 >> 64);
  }
  if (two_m == 0) {
    *q_out = 0.0;
    return 0;
  }
  const double M = (double)two_m;
  *q_out = (double)I / M - (double)S2 / (M * M);
  return 0;
}

// Alg. 4 (disconnectedCommunities): D[c] = 1 iff community c's vertices are
// not all reachable from its first vertex through same-community entries.
//   D_out     : uint8[n] indexed by label (may be NULL)
//   count_out : number of disconnected communities (may be NULL)
int oracle_disconnected(int64_t n, const int64_t *off, const int32_t *cols, const int32_t *labels,
                        uint8_t *D_out, int64_t *count_out) {
  if (!valid_csr(n, off, cols) || !valid_labels(n, labels)) return -1;
  std::vector<int64_t> S((size_t)n, 0);  // communitySizes
  for (int64_t i = 0; i < n; ++i) S[(size_t)labels[i]]++;
  std::vector<uint8_t> D((size_t)n, 0), vis((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = labels[i];
    if (S[(size_t)c] == 0) continue;
    int64_t reached = 0;
    bfs_visit_for_each(vis, off, cols, i, [&](int64_t j) { return labels[j] == c; },
                       [&](int64_t) { ++reached; });
    if (reached < S[(size_t)c]) D[(size_t)c] = 1;
    S[(size_t)c] = 0;
  }
  int64_t cnt = 0;
  for (int64_t c = 0; c < n; ++c) cnt += D[(size_t)c];
  if (D_out) memcpy(D_out, D.data(), (size_t)n);
  if (count_out) *count_out = cnt;
  return 0;
}

}  // extern "C"
