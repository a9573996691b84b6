// Split pass (Alg. 2 / Alg. 1): every vertex receives the smallest vertex id
// of its connected piece inside its own community.
//
// The paper's BFS (Alg. 2) and min-label propagation (Alg. 1) both reach that
// labelling; here it is computed as connected components of the subgraph of
// entries (u, v) with C[u] == C[v], by a lock-free union-find whose unions
// always hang the larger root below the smaller one.  Ids therefore decrease
// along every parent chain and the final root of each component is its
// smallest vertex, whatever order the unions happen in.
//
// The edges are taken in the order of Afforest (Sutton, Ben-Nun & Barak,
// IPDPS 2018): first the first two intra-community entries of every row,
// flattened, then a representative component per
// community -- the root some vertex of the community points at after the
// flattening, nearly always the community's big piece -- and then every entry
// of every row whose vertex is not in its community's representative.  A
// skipped vertex u loses nothing: an entry (u, v) with v in another community
// needs no union; with v skipped too, u and v are already in the same
// component (a community has one representative); otherwise the mirrored
// entry (v, u) is processed from v's side in the second pass (the graph is
// symmetric).
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

// Parent pointers are read with cache-friendly relaxed loads that may return
// an older value.  That is safe because a pointer only ever moves to an
// ancestor: a stale read still names an ancestor (or the vertex itself while
// it was a root), ids decrease along every chain, and a vertex that is not a
// root never becomes one again.  Every hook is a device-scope compare-and-swap
// on a root; when it fails, the value it returns is the current parent, and
// the search resumes from there, so each retry moves to a strictly smaller id.
__device__ __forceinline__ int32_t ld_parent(const int32_t *p, int32_t x) {
  return __hip_atomic_load(const_cast<int32_t *>(p) + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x (as far as this thread can see) with path halving: writing an
// ancestor into a non-root's pointer is harmless whatever races with it.
__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t x) {
  for (;;) {
    const int32_t p = ld_parent(parent, x);
    if (p == x) return x;
    const int32_t gp = ld_parent(parent, p);
    if (gp != p)
      __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = gp;
  }
}

__device__ __forceinline__ void unite(int32_t *parent, int32_t a, int32_t b) {
  a = find_root(parent, a);
  b = find_root(parent, b);
  for (;;) {
    if (a == b) return;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    // A fresh read first: when many threads hold the same stale pair of
    // roots (hubs of a power-law graph), only the first needs the atomic.
    int32_t expected = __hip_atomic_load(parent + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (expected == a &&  // hang root a (larger) below b (smaller)
        __hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
    a = find_root(parent, expected);  // a was hooked meanwhile: continue above it
    b = find_root(parent, b);
  }
}

__global__ void split_init(int32_t *parent, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    parent[i] = (int32_t)i;
}

constexpr int kLinkFirst = 2;  // intra-community entries per row linked before the hooks

// First pass: the first kLinkFirst intra-community entries of every row
// (scanning at most kLinkScan entries), then a flattening.  Taking
// intra-community entries (not simply the first entries, which may all lead
// to other communities) leaves nearly every community in one piece.
constexpr int kLinkScan = 16;
constexpr int kLinkChunk = 8;
__global__ __launch_bounds__(256) void split_link_first(const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ cols,
                                                        const int32_t *__restrict__ C,
                                                        int32_t *parent, int64_t n,
                                                        const int32_t *__restrict__ gid,
                                                        const uint8_t *__restrict__ sel) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    // rows of graphs outside the selection stay singletons (their labels are
    // their own ids, so no entry could link them anyway)
    if (gid && !sel[gid[u]]) continue;
    const int64_t b = off[u];
    const int64_t e = off[u + 1] < b + kLinkScan ? off[u + 1] : b + kLinkScan;
    const int32_t cu = C[u];
    int seen = 0;
    // kLinkChunk entries and their labels are loaded at once (one round trip
    // instead of one per entry), then linked in row order.
    for (int64_t p0 = b; p0 < e && seen < kLinkFirst; p0 += kLinkChunk) {
      int32_t v[kLinkChunk];
      bool hit[kLinkChunk];
#pragma unroll
      for (int k = 0; k < kLinkChunk; ++k) v[k] = p0 + k < e ? cols[p0 + k] : (int32_t)u;
#pragma unroll
      for (int k = 0; k < kLinkChunk; ++k) hit[k] = v[k] != (int32_t)u && C[v[k]] == cu;
#pragma unroll
      for (int k = 0; k < kLinkChunk; ++k)
        if (hit[k] && seen < kLinkFirst) {
          unite(parent, (int32_t)u, v[k]);
          ++seen;
        }
    }
  }
}

__global__ void split_flatten(int32_t *parent, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    parent[i] = find_root(parent, (int32_t)i);
}

// Representative component of every community: the root of some vertex of
// the community (racing plain stores: any of them is a valid choice).
__global__ void split_rep(const int32_t *__restrict__ C, const int32_t *__restrict__ parent, int64_t n,
                          int32_t *__restrict__ rep) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) rep[C[i]] = parent[i];
}

// After the flattening every vertex points at its root.  The second pass
// reads, per row entry, one packed word cp[v] = (C[v] << 32) | root(v) taken
// then (a single gather instead of two): an entry joins nothing new when v is
// in another community or was already in u's component at that time
// (components only grow, so a stale snapshot never skips a needed union).
__global__ void split_pack(const int32_t *__restrict__ C, const int32_t *__restrict__ parent, int64_t n,
                           unsigned long long *__restrict__ cp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    cp[i] = ((unsigned long long)(uint32_t)C[i] << 32) | (uint32_t)parent[i];
}

__device__ __forceinline__ void hook_entry(int32_t *parent, const unsigned long long *__restrict__ cp,
                                           int32_t u, uint32_t cu, uint32_t ru, int32_t v) {
  if (v == u) return;
  const unsigned long long x = cp[v];
  if ((uint32_t)(x >> 32) != cu || (uint32_t)x == ru) return;
  unite(parent, u, v);
}

// Second pass, one thread per vertex (short rows): every entry of the rows of
// vertices outside their community's representative (entries already linked
// cost one snapshot compare).
__global__ __launch_bounds__(256) void split_hook_thread(const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ cols,
                                                         const unsigned long long *__restrict__ cp,
                                                         int32_t *parent,
                                                         const int32_t *__restrict__ list,
                                                         int64_t first, int64_t count,
                                                         const int32_t *__restrict__ rep) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += stride) {
    const int32_t u = list ? list[first + idx] : (int32_t)(first + idx);
    const unsigned long long xu = cp[u];
    if (rep[xu >> 32] == (int32_t)(uint32_t)xu) continue;
    const int64_t e = off[u + 1];
    int64_t p = off[u];
    // the link rounds joined the first kLinkFirst intra-community entries
    // found within kLinkScan entries: skip them
    for (int linked = 0; p < e && p < off[u] + kLinkScan && linked < kLinkFirst; ++p) {
      const int32_t v = cols[p];
      if (v != u && (uint32_t)(cp[v] >> 32) == (uint32_t)(xu >> 32))
        ++linked;
    }
    for (; p < e; ++p) hook_entry(parent, cp, u, (uint32_t)(xu >> 32), (uint32_t)xu, cols[p]);
  }
}

// Same with a group of G lanes per vertex (G <= 64, or the 256-thread block).
template <int G>
__global__ __launch_bounds__(256) void split_hook_group(const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ cols,
                                                        const unsigned long long *__restrict__ cp,
                                                        int32_t *parent,
                                                        const int32_t *__restrict__ list,
                                                        int64_t first, int64_t count,
                                                        const int32_t *__restrict__ rep) {
  constexpr int GPB = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  for (int64_t idx = (int64_t)blockIdx.x * GPB + g; idx < count; idx += (int64_t)gridDim.x * GPB) {
    const int32_t u = list ? list[first + idx] : (int32_t)(first + idx);
    const unsigned long long xu = cp[u];
    if (rep[xu >> 32] == (int32_t)(uint32_t)xu) continue;  // uniform over the group
    const int64_t e = off[u + 1];
    for (int64_t p = off[u] + lane; p < e; p += G)
      hook_entry(parent, cp, u, (uint32_t)(xu >> 32), (uint32_t)xu, cols[p]);
  }
}

__global__ void split_compress(int32_t *parent, int32_t *out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = find_root(parent, (int32_t)i);
}

// Renumbered graph: root of every vertex, and per root the smallest
// original id of its component.  Most vertices of a block usually share one
// root (the giant piece), so the block first folds the candidates for the
// root of its first vertex in LDS and sends one atomic for them.
__global__ __launch_bounds__(256) void split_root_min(int32_t *parent, const int32_t *__restrict__ orig,
                                                      int64_t np, int32_t *minorig) {
  __shared__ int32_t lead, lead_min;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < np; base += stride) {
    const int64_t p = base + threadIdx.x;
    int32_t r = -1, o = 0;
    if (p < np) {
      r = find_root(parent, (int32_t)p);
      parent[p] = r;
      o = orig[p];
    }
    if (threadIdx.x == 0) {
      lead = r;
      lead_min = 0x7fffffff;
    }
    __syncthreads();
    if (r >= 0 && r == lead) atomicMin(&lead_min, o);  // LDS
    else if (r >= 0) atomicMin(&minorig[r], o);
    __syncthreads();
    if (threadIdx.x == 0 && lead >= 0) atomicMin(&minorig[lead], lead_min);
    __syncthreads();
  }
}

// The root is looked up again here: split_root_min's store of the root into
// parent[p] can be overwritten by another thread's path halving with an
// intermediate ancestor, so parent[p] alone need not be the root.
__global__ void split_out(const int32_t *__restrict__ parent, const int32_t *__restrict__ orig,
                          const int32_t *__restrict__ minorig, int64_t np, int64_t n, int32_t *out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int32_t v = orig[p];
    if (p < np) {
      int32_t r = (int32_t)p, q = parent[p];
      while (q != r) {  // read-only walk: no unions or writes happen any more
        r = q;
        q = parent[q];
      }
      out[v] = minorig[r];
    } else {
      out[v] = v;
    }
  }
}

__global__ void fill_i32(int32_t *p, int32_t v, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void check_labels(const int32_t *labels, int64_t n, unsigned long long *bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int found = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t c = labels[i];
    found |= (c < 0 || (int64_t)c >= n);
  }
  if (__ballot(found) && threadIdx.x % kWave == 0) atomicAdd(bad, 1ull);
}

int grid_cap(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// The paper's other split technique (Alg. 1): min-label propagation restricted
// to intra-community entries, repeated until no label changes.  Labels start
// as the vertex ids and only decrease, so the fixed point -- every vertex
// holds the smallest id of its piece -- is the union-find result; the rounds
// update labels in place (a stale read only delays convergence).  With
// pruning (LPP) a vertex is processed only if a neighbour of its community
// changed in the previous round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t ld_lab(const int32_t *p, int64_t i) {
  return __hip_atomic_load(const_cast<int32_t *>(p) + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_lab(int32_t *p, int64_t i, int32_t v) {
  __hip_atomic_store(p + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int G>
__global__ __launch_bounds__(256) void split_lp_round(const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ cols,
                                                      const int32_t *__restrict__ C, int32_t *lab,
                                                      const int32_t *__restrict__ list, int64_t first,
                                                      int64_t count, const uint8_t *__restrict__ fin,
                                                      uint8_t *fout, unsigned long long *changed) {
  constexpr int GPB = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  unsigned long long nchg = 0;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
    const int64_t idx = base + g;
    int32_t u = -1;
    if (idx < count) {
      u = list ? list[first + idx] : (int32_t)(first + idx);
      if (fin && !fin[u]) u = -1;
    }
    int32_t m = 0x7fffffff, cu = 0;
    int64_t b = 0, e = 0;
    if (u >= 0) {
      cu = C[u];
      b = off[u];
      e = off[u + 1];
      m = ld_lab(lab, u);
    }
    const int32_t own = m;
    for (int64_t p = b + lane; p < e; p += G) {
      const int32_t v = cols[p];
      if (C[v] == cu) {
        const int32_t lv = ld_lab(lab, v);
        m = lv < m ? lv : m;
      }
    }
    constexpr int W = G < kWave ? G : kWave;
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
      const int32_t y = __shfl_xor(m, o, W);
      m = y < m ? y : m;
    }
    if constexpr (G > kWave) {  // the whole block is one group: combine its waves
      __shared__ int32_t wmin[256 / kWave];
      if (threadIdx.x % kWave == 0) wmin[threadIdx.x / kWave] = m;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < 256 / kWave; ++w) m = wmin[w] < m ? wmin[w] : m;
      __syncthreads();
    }
    if (u >= 0 && m < own) {
      if (lane == 0) {
        st_lab(lab, u, m);
        nchg += 1;
      }
      if (fout)
        for (int64_t p = b + lane; p < e; p += G) {
          const int32_t v = cols[p];
          if (C[v] == cu && !fout[v]) fout[v] = 1;
        }
    }
  }
  if (nchg) atomicAdd(changed, nchg);
}

__global__ void split_lp_init(int32_t *lab, uint8_t *f0, uint8_t *f1, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    lab[i] = (int32_t)i;
    if (f0) f0[i] = 1;
    if (f1) f1[i] = 0;
  }
}

__global__ void clear_u8(uint8_t *p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

}  // namespace

hipError_t launch_split_lp_init(int32_t *lab, uint8_t *f0, uint8_t *f1, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  split_lp_init<<<grid_cap(n, 256, 256 * 16), 256, 0, s>>>(lab, f0, f1, n);
  return hipGetLastError();
}

// One round over every tier; fin / fout NULL for LP, the flag arrays of this
// and the next round for LPP (fin is cleared afterwards for reuse).
hipError_t launch_split_lp_round(const int64_t *off, const int32_t *cols, int64_t n, const int32_t *C,
                                 int32_t *lab, const int32_t *list, const int64_t *tier_count_host,
                                 const int64_t *tier_start_host, const TierConfig &cfg, uint8_t *fin,
                                 uint8_t *fout, unsigned long long *changed, hipStream_t s) {
  constexpr int kCap = 256 * 16;
  for (int t = 1; t < kNumTiers; ++t) {
    const int64_t cnt = tier_count_host[t], first = tier_start_host[t];
    if (cnt <= 0) continue;
    const int64_t d = cfg.bound[t];
    if (d <= 8)
      split_lp_round<1><<<grid_cap(cnt, 256, kCap), 256, 0, s>>>(off, cols, C, lab, list, first, cnt, fin, fout,
                                                                  changed);
    else if (d <= 32)
      split_lp_round<8><<<grid_cap(cnt, 32, kCap), 256, 0, s>>>(off, cols, C, lab, list, first, cnt, fin, fout,
                                                                 changed);
    else if (d <= 512)
      split_lp_round<64><<<grid_cap(cnt, 4, kCap), 256, 0, s>>>(off, cols, C, lab, list, first, cnt, fin, fout,
                                                                 changed);
    else
      split_lp_round<256><<<grid_cap(cnt, 1, kCap), 256, 0, s>>>(off, cols, C, lab, list, first, cnt, fin,
                                                                  fout, changed);
  }
  if (fin && n > 0) clear_u8<<<grid_cap(n, 256, kCap), 256, 0, s>>>(fin, n);
  return hipGetLastError();
}

namespace {

// Alg. 4 on top of the split: a community is disconnected iff it has more
// than one connected piece, and every piece has exactly one root (the vertex
// whose piece label is its own id).  One count per root, summed per community
// with one atomic per run of lanes holding the same label.
__global__ __launch_bounds__(256) void dc_pieces(const int32_t *__restrict__ labels,
                                                 const int32_t *__restrict__ comp, int64_t n,
                                                 int32_t *__restrict__ pieces) {
  const int wl = threadIdx.x % kWave;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    const int32_t c = (v < n && comp[v] == (int32_t)v) ? labels[v] : -1;
    unsigned long long pending = __ballot(c >= 0);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int32_t lc = __shfl(c, leader);
      const unsigned long long same = __ballot(c == lc);
      if (wl == leader) atomicAdd(&pieces[lc], (int32_t)__popcll(same));
      pending &= ~same;
    }
  }
}

__global__ __launch_bounds__(256) void dc_flags(const int32_t *__restrict__ pieces, int64_t n,
                                                uint8_t *__restrict__ D, unsigned long long *count) {
  __shared__ unsigned long long red[256 / kWave];
  unsigned long long cnt = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    const bool d = pieces[c] > 1;
    if (D) D[c] = d ? 1 : 0;
    cnt += d ? 1 : 0;
  }
  cnt = block_sum(cnt, red);
  if (threadIdx.x == 0 && cnt) atomicAdd(count, cnt);
}

}  // namespace

hipError_t launch_disconnected(const int32_t *labels, const int32_t *comp, int64_t n, int32_t *pieces,
                               uint8_t *D, unsigned long long *count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_i32<<<grid_cap(n, 256, 256 * 16), 256, 0, s>>>(pieces, 0, n);
  dc_pieces<<<grid_cap(n, 256, 256 * 16), 256, 0, s>>>(labels, comp, n, pieces);
  dc_flags<<<grid_cap(n, 256, 256 * 16), 256, 0, s>>>(pieces, n, D, count);
  return hipGetLastError();
}

// Split on a graph whose vertices are grouped by tier (tier t occupies
// [tier_start[t], tier_start[t] + tier_count[t]) of `list`, or of the ids
// themselves when list is NULL).
//  orig == NULL : the graph is in caller ids; out[i] = smallest id of i's piece.
//  orig != NULL : the graph is the renumbered copy of its n non-isolated
//                 vertices, orig[p] the caller id of vertex p (orig holds
//                 n_total entries, isolated vertices last); out is written in
//                 caller ids with the smallest caller id of each piece.
hipError_t launch_split(const int64_t *off, const int32_t *cols, int64_t n, const int32_t *C,
                        int32_t *parent, int32_t *out, const int32_t *list,
                        const int64_t *tier_count_host, const int64_t *tier_start_host,
                        const int32_t *orig, int32_t *minorig, int64_t n_total, int32_t *rep,
                        unsigned long long *cp, const TierConfig &cfg, hipStream_t s, const int32_t *gid,
                        const uint8_t *sel) {
  constexpr int kCap = 256 * 16;
  if (n > 0) {
    split_init<<<grid_cap(n, 256, kCap), 256, 0, s>>>(parent, n);
    split_link_first<<<grid_cap(n, 256, kCap), 256, 0, s>>>(off, cols, C, parent, n, gid, sel);
    split_flatten<<<grid_cap(n, 256, kCap), 256, 0, s>>>(parent, n);
    split_rep<<<grid_cap(n, 256, kCap), 256, 0, s>>>(C, parent, n, rep);
    split_pack<<<grid_cap(n, 256, kCap), 256, 0, s>>>(C, parent, n, cp);
  }
  for (int t = 1; t < kNumTiers; ++t) {
    const int64_t cnt = tier_count_host[t], first = tier_start_host[t];
    if (cnt <= 0) continue;
    // lanes per row follow the tier's degree bound (any kernel is correct
    // for any degree; this only balances the work)
    const int64_t d = cfg.bound[t];
    if (d <= 8)
      split_hook_thread<<<grid_cap(cnt, 256, kCap), 256, 0, s>>>(off, cols, cp, parent, list, first, cnt,
                                                                  rep);
    else if (d <= 32)
      split_hook_group<8><<<grid_cap(cnt, 32, kCap), 256, 0, s>>>(off, cols, cp, parent, list, first, cnt,
                                                                   rep);
    else if (d <= 512)
      split_hook_group<64><<<grid_cap(cnt, 4, kCap), 256, 0, s>>>(off, cols, cp, parent, list, first, cnt,
                                                                   rep);
    else
      split_hook_group<256><<<grid_cap(cnt, 1, kCap), 256, 0, s>>>(off, cols, cp, parent, list, first, cnt,
                                                                    rep);
  }
  if (!orig) {
    if (n > 0) split_compress<<<grid_cap(n, 256, kCap), 256, 0, s>>>(parent, out, n);
  } else {
    if (n > 0) {
      fill_i32<<<grid_cap(n, 256, kCap), 256, 0, s>>>(minorig, 0x7fffffff, n);
      split_root_min<<<grid_cap(n, 256, kCap), 256, 0, s>>>(parent, orig, n, minorig);
    }
    if (n_total > 0) split_out<<<grid_cap(n_total, 256, kCap), 256, 0, s>>>(parent, orig, minorig, n, n_total, out);
  }
  return hipGetLastError();
}

hipError_t launch_check_labels(const int32_t *labels, int64_t n, unsigned long long *bad,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  check_labels<<<grid_cap(n, 256, 256 * 16), 256, 0, s>>>(labels, n, bad);
  return hipGetLastError();
}

}  // namespace gsl
