// Split pass (Alg. 2 / Alg. 1): every vertex receives the smallest vertex id
// of its connected piece inside its own community.
//
// The paper's BFS (Alg. 2) and min-label propagation (Alg. 1) both reach that
// labelling; here it is computed as connected components of the subgraph of
// entries (u, v) with C[u] == C[v], by a lock-free union-find whose unions
// always hang the larger root below the smaller one.  Ids therefore decrease
// along every parent chain and the final root of each component is its
// smallest vertex, whatever order the unions happen in.  Each undirected edge
// is united once (from the row of its larger endpoint, v < u).
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

__device__ __forceinline__ int32_t ld_parent(const int32_t *p, int32_t x) {
  return __hip_atomic_load(const_cast<int32_t *>(p) + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving (a vertex's parent only ever moves to another,
// smaller ancestor, so racing halvings are harmless).
__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t x) {
  for (;;) {
    const int32_t p = ld_parent(parent, x);
    if (p == x) return x;
    const int32_t gp = ld_parent(parent, p);
    if (gp != p)
      __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}

__device__ __forceinline__ void unite(int32_t *parent, int32_t a, int32_t b) {
  for (;;) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    if (a == b) return;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    int32_t expected = a;  // hang root a (larger) below b (smaller)
    if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

__global__ void split_init(int32_t *parent, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    parent[i] = (int32_t)i;
}

// One thread per vertex (short rows).
__global__ __launch_bounds__(256) void split_hook_thread(const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ cols,
                                                         const int32_t *__restrict__ C,
                                                         int32_t *parent,
                                                         const int32_t *__restrict__ list,
                                                         int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += stride) {
    const int32_t u = list[idx];
    const int32_t cu = C[u];
    for (int64_t p = off[u]; p < off[u + 1]; ++p) {
      const int32_t v = cols[p];
      if (v < u && C[v] == cu) unite(parent, u, v);
    }
  }
}

// A group of G lanes per vertex (G <= 64) or, with G == blockDim.x, a block.
template <int G>
__global__ __launch_bounds__(256) void split_hook_group(const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ cols,
                                                        const int32_t *__restrict__ C,
                                                        int32_t *parent,
                                                        const int32_t *__restrict__ list,
                                                        int64_t count) {
  constexpr int GPB = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  for (int64_t idx = (int64_t)blockIdx.x * GPB + g; idx < count; idx += (int64_t)gridDim.x * GPB) {
    const int32_t u = list[idx];
    const int32_t cu = C[u];
    const int64_t e = off[u + 1];
    for (int64_t p = off[u] + lane; p < e; p += G) {
      const int32_t v = cols[p];
      if (v < u && C[v] == cu) unite(parent, u, v);
    }
  }
}

__global__ void split_compress(int32_t *parent, int32_t *out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = find_root(parent, (int32_t)i);
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

// tier_count_host / tier_start_host: the plan of the graph (tier t occupies
// list[tier_start[t] - tier_start[1] ...]).
hipError_t launch_split(const int64_t *off, const int32_t *cols, int64_t n, const int32_t *C,
                        int32_t *parent, int32_t *out, const int32_t *list,
                        const int64_t *tier_count_host, const int64_t *tier_start_host,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  constexpr int kCap = 256 * 16;
  split_init<<<grid_cap(n, 256, kCap), 256, 0, s>>>(parent, n);
  for (int t = 1; t < kNumTiers; ++t) {
    const int64_t cnt = tier_count_host[t];
    if (cnt <= 0) continue;
    const int32_t *l = list + (tier_start_host[t] - tier_start_host[1]);
    if (t == 1)
      split_hook_thread<<<grid_cap(cnt, 256, kCap), 256, 0, s>>>(off, cols, C, parent, l, cnt);
    else if (t <= 3)
      split_hook_group<8><<<grid_cap(cnt, 32, kCap), 256, 0, s>>>(off, cols, C, parent, l, cnt);
    else if (t <= 6)
      split_hook_group<64><<<grid_cap(cnt, 4, kCap), 256, 0, s>>>(off, cols, C, parent, l, cnt);
    else
      split_hook_group<256><<<grid_cap(cnt, 1, kCap), 256, 0, s>>>(off, cols, C, parent, l, cnt);
  }
  split_compress<<<grid_cap(n, 256, kCap), 256, 0, s>>>(parent, out, n);
  return hipGetLastError();
}

hipError_t launch_check_labels(const int32_t *labels, int64_t n, unsigned long long *bad,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  check_labels<<<grid_cap(n, 256, 256 * 16), 256, 0, s>>>(labels, n, bad);
  return hipGetLastError();
}

}  // namespace gsl
