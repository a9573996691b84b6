// Batches of independent graphs run as one graph.
//
// A batch is laid out as one CSR over the concatenated vertex ranges, with
// global vertex ids: graph g owns vertices [vtx_base[g], vtx_base[g+1]) and
// entries [edge_base[g], edge_base[g+1]).  The graphs share no edge, so every
// sweep, the split and the per-graph convergence tests see exactly what each
// graph would see alone; only the vertex ids carry the graph's base.  The
// kernels here build that layout from the caller's local-id input and turn the
// result back into local labels.
//
// Work is spread over fixed tiles of consecutive entries (or vertices); a
// tile finds its first graph by binary search over the base array and each
// thread steps forward from there, so graph sizes that differ by 1000x do not
// unbalance the launch.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {
namespace {

constexpr int kBlock = 256;
constexpr int kPerThread = 16;
constexpr int64_t kTile = (int64_t)kBlock * kPerThread;

// Last g in [0, G) with base[g] <= x (base non-decreasing, base[0] <= x).
__device__ int64_t graph_of(const int64_t *__restrict__ base, int64_t G, int64_t x) {
  int64_t lo = 0, hi = G - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (base[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// First graph of each tile, found once per block.
__device__ int64_t tile_graph(const int64_t *__restrict__ base, int64_t G, int64_t x0) {
  __shared__ int64_t g0;
  __syncthreads();
  if (threadIdx.x == 0) g0 = graph_of(base, G, x0);
  __syncthreads();
  return g0;
}

// Concatenated input: cols hold local ids; out = cols + vtx_base[graph].
__global__ __launch_bounds__(kBlock) void globalize_cols(const int32_t *__restrict__ cols,
                                                         const int64_t *__restrict__ edge_base,
                                                         const int64_t *__restrict__ vtx_base, int64_t G,
                                                         int64_t nnz, int32_t *__restrict__ out) {
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < nnz; t0 += (int64_t)gridDim.x * kTile) {
    int64_t g = tile_graph(edge_base, G, t0);
    const int64_t tend = t0 + kTile < nnz ? t0 + kTile : nnz;
    if (edge_base[g + 1] >= tend) {
      // the whole tile lies in graph g (most tiles): one base, all loads at once
      const int32_t vb = (int32_t)vtx_base[g];
#pragma unroll
      for (int j = 0; j < kPerThread; ++j) {
        const int64_t e = t0 + (int64_t)j * kBlock + threadIdx.x;
        if (e < tend) out[e] = cols[e] + vb;
      }
      continue;
    }
#pragma unroll 4
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t e = t0 + (int64_t)j * kBlock + threadIdx.x;
      if (e >= nnz) break;
      while (edge_base[g + 1] <= e) ++g;
      out[e] = cols[e] + (int32_t)vtx_base[g];
    }
  }
}

// Separate graphs: entry counts offsets[n] - offsets[0], or -1 when the
// offsets decrease somewhere (block per graph).
__global__ __launch_bounds__(kBlock) void graph_entries(const GraphDesc *__restrict__ d, int64_t G,
                                                        int64_t *__restrict__ cnt) {
  for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
    const GraphDesc x = d[g];
    int bad = 0;
    for (int64_t i = threadIdx.x; i < x.n; i += kBlock) bad |= x.offsets[i] > x.offsets[i + 1] ? 1 : 0;
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) cnt[g] = bad ? -1 : (x.n > 0 ? x.offsets[x.n] - x.offsets[0] : 0);
  }
}

// Separate graphs -> one global CSR: offsets shifted to the graph's entry
// base, cols shifted to its vertex base, weights copied (1 where a graph
// passes none).
__global__ __launch_bounds__(kBlock) void gather_offsets(const GraphDesc *__restrict__ d,
                                                         const int64_t *__restrict__ vtx_base,
                                                         const int64_t *__restrict__ edge_base, int64_t G,
                                                         int64_t N, int64_t eshift, int64_t *__restrict__ off) {
  if (blockIdx.x == 0 && threadIdx.x == 0) off[N] = eshift + edge_base[G];
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < N; t0 += (int64_t)gridDim.x * kTile) {
    int64_t g = tile_graph(vtx_base, G, t0);
#pragma unroll 4
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t v = t0 + (int64_t)j * kBlock + threadIdx.x;
      if (v >= N) break;
      while (vtx_base[g + 1] <= v) ++g;
      const int64_t *o = d[g].offsets;
      off[v] = eshift + edge_base[g] + (o[v - vtx_base[g]] - o[0]);
    }
  }
}

// Base arrays must start at 0, end at the totals and never decrease.
__global__ void check_bases(const int64_t *__restrict__ vtx_base, const int64_t *__restrict__ edge_base,
                            int64_t G, int64_t N, int64_t nnz, unsigned long long *bad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g > G) return;
  bool ok = true;
  if (g == 0) ok = vtx_base[0] == 0 && edge_base[0] == 0;
  else ok = vtx_base[g] >= vtx_base[g - 1] && edge_base[g] >= edge_base[g - 1];
  if (g == G) ok = ok && vtx_base[G] == N && edge_base[G] == nnz;
  if (!ok) atomicOr(bad, 1ull);
}

__global__ __launch_bounds__(kBlock) void gather_entries(const GraphDesc *__restrict__ d,
                                                         const int64_t *__restrict__ vtx_base,
                                                         const int64_t *__restrict__ edge_base, int64_t G,
                                                         int64_t nnz, int64_t vshift, int32_t *__restrict__ cols,
                                                         uint32_t *__restrict__ w, uint32_t *__restrict__ bad) {
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < nnz; t0 += (int64_t)gridDim.x * kTile) {
    int64_t g = tile_graph(edge_base, G, t0);
#pragma unroll 4
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t e = t0 + (int64_t)j * kBlock + threadIdx.x;
      if (e >= nnz) break;
      while (edge_base[g + 1] <= e) ++g;
      const GraphDesc x = d[g];
      const int64_t src = x.offsets[0] + (e - edge_base[g]);
      int32_t c = x.cols[src];
      if ((uint64_t)(uint32_t)c >= (uint64_t)(vtx_base[g + 1] - vtx_base[g])) {
        // out of range: flag the graph and keep the batch safe to run
        atomicOr(&bad[g], 1u);
        c = 0;
      }
      cols[e] = c + (int32_t)(vshift + vtx_base[g]);
      if (w) w[e] = x.weights ? x.weights[src] : 1u;
    }
  }
}

// Global labels -> local labels (in place).
__global__ __launch_bounds__(kBlock) void localize(int32_t *__restrict__ lab, const int64_t *__restrict__ vtx_base,
                                                   int64_t G, int64_t N) {
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < N; t0 += (int64_t)gridDim.x * kTile) {
    int64_t g = tile_graph(vtx_base, G, t0);
#pragma unroll 4
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t v = t0 + (int64_t)j * kBlock + threadIdx.x;
      if (v >= N) break;
      while (vtx_base[g + 1] <= v) ++g;
      lab[v] -= (int32_t)vtx_base[g];
    }
  }
}

// Local labels of the batch -> each graph's own output array (graphs flagged
// bad keep their output untouched).
__global__ __launch_bounds__(kBlock) void scatter_labels(const GraphDesc *__restrict__ d,
                                                         const int32_t *__restrict__ lab,
                                                         const int64_t *__restrict__ vtx_base,
                                                         const uint32_t *__restrict__ bad, int64_t G, int64_t N) {
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < N; t0 += (int64_t)gridDim.x * kTile) {
    int64_t g = tile_graph(vtx_base, G, t0);
#pragma unroll 4
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t v = t0 + (int64_t)j * kBlock + threadIdx.x;
      if (v >= N) break;
      while (vtx_base[g + 1] <= v) ++g;
      if (!bad[g]) d[g].labels_out[v - vtx_base[g]] = lab[v];
    }
  }
}

// One graph: offsets[0] == 0, non-decreasing, cols in [0, n).
__global__ __launch_bounds__(kBlock) void check_graph(const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ cols, int64_t n, int64_t nnz,
                                                      unsigned long long *bad) {
  int b = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t == 0 && off[0] != 0) b = 1;
  for (int64_t i = t; i < n; i += stride) b |= off[i] > off[i + 1] ? 1 : 0;
  for (int64_t e = t; e < nnz; e += stride) b |= (uint64_t)(uint32_t)cols[e] >= (uint64_t)n ? 2 : 0;
  if (b) atomicOr(bad, (unsigned long long)b);
}

// ---- sessions (continuous batching) ----
// Block per range (grid-stride): the vertices of a newly admitted graph get
// its slot, their own global id as label and the active flag of both sweeps
// parities (its first sweep processes every vertex, whatever the pruning
// state of the others).
__global__ __launch_bounds__(kBlock) void session_admit(const SessionRange *__restrict__ r, int64_t count,
                                                        int32_t *__restrict__ gid, int32_t *__restrict__ lab,
                                                        uint8_t *__restrict__ act0, uint8_t *__restrict__ act1) {
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const SessionRange x = r[i];
    for (int64_t v = x.vb + threadIdx.x; v < x.vb + x.n; v += kBlock) {
      gid[v] = x.slot;
      lab[v] = (int32_t)v;
      act0[v] = 1;
      act1[v] = 1;
    }
  }
}

// Per-slot loop state of admitted graphs: convergence limit, no sweep yet,
// running unless max_iters is 0.
__global__ void session_slots(const SessionRange *__restrict__ r, int64_t count, int32_t max_iters, double tol,
                              int64_t *__restrict__ glimit, int32_t *__restrict__ giters,
                              uint8_t *__restrict__ gdone, int64_t *__restrict__ gdn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const SessionRange x = r[i];
  glimit[x.slot] = x.limit;
  giters[x.slot] = 0;
  gdn[x.slot] = 0;
  gdone[x.slot] = max_iters <= 0 ? 1 : 0;
}

// Labels for the split of the finishing graphs: theirs as they are, every
// other vertex its own id (a vertex whose label no neighbour shares joins
// nothing, so the split passes over the other graphs at little cost).
__global__ __launch_bounds__(kBlock) void session_split_labels(const int32_t *__restrict__ lab,
                                                               const int32_t *__restrict__ gid,
                                                               const uint8_t *__restrict__ sel, int64_t n,
                                                               int32_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
    out[v] = sel[gid[v]] ? lab[v] : (int32_t)v;
}

// Block per finishing graph: its split labels as local ids into its output,
// its vertices handed to the dead slot.
__global__ __launch_bounds__(kBlock) void session_finish(const SessionRange *__restrict__ r, int64_t count,
                                                         const int32_t *__restrict__ split,
                                                         int32_t *__restrict__ gid, int32_t dead) {
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const SessionRange x = r[i];
    for (int64_t k = threadIdx.x; k < x.n; k += kBlock) {
      x.labels_out[k] = split[x.vb + k] - (int32_t)x.vb;
      gid[x.vb + k] = dead;
    }
  }
}

// Block per live graph: its CSR rows, entries, weights and labels copied from
// one arena buffer to the other at its new position (ids shifted by the
// vertex move, offsets by the entry move), its vertices given its slot and
// both active flags.
__global__ __launch_bounds__(kBlock) void session_move(const SessionRange *__restrict__ r, int64_t count,
                                                       const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
                                                       const uint32_t *__restrict__ w, const int32_t *__restrict__ lab,
                                                       int64_t *__restrict__ off2, int32_t *__restrict__ cols2,
                                                       uint32_t *__restrict__ w2, int32_t *__restrict__ lab2,
                                                       int32_t *__restrict__ gid, uint8_t *__restrict__ act0,
                                                       uint8_t *__restrict__ act1) {
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const SessionRange x = r[i];
    const int32_t dv = (int32_t)(x.new_vb - x.vb);
    const int64_t de = x.new_eb - x.eb;
    for (int64_t k = threadIdx.x; k < x.n; k += kBlock) {
      off2[x.new_vb + k] = off[x.vb + k] + de;
      lab2[x.new_vb + k] = lab[x.vb + k] + dv;
      gid[x.new_vb + k] = x.slot;
      act0[x.new_vb + k] = 1;
      act1[x.new_vb + k] = 1;
    }
    for (int64_t e = threadIdx.x; e < x.nnz; e += kBlock) {
      cols2[x.new_eb + e] = cols[x.eb + e] + dv;
      if (w) w2[x.new_eb + e] = w[x.eb + e];
    }
  }
}

unsigned tiles(int64_t count) {
  const int64_t t = (count + kTile - 1) / kTile;
  const int64_t cap = 256 * 64;
  return (unsigned)(t < 1 ? 1 : (t > cap ? cap : t));
}

}  // namespace

hipError_t launch_check_graph(const int64_t *off, const int32_t *cols, int64_t n, int64_t nnz,
                              unsigned long long *bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t work = n > nnz ? n : nnz;
  const int64_t b = (work + 4 * kBlock - 1) / (4 * kBlock);
  check_graph<<<(unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b)), kBlock, 0, s>>>(off, cols, n, nnz, bad);
  return hipGetLastError();
}

hipError_t launch_globalize_cols(const int32_t *cols, const int64_t *edge_base, const int64_t *vtx_base,
                                 int64_t G, int64_t nnz, int32_t *out, hipStream_t s) {
  if (nnz <= 0 || G <= 0) return hipSuccess;
  globalize_cols<<<tiles(nnz), kBlock, 0, s>>>(cols, edge_base, vtx_base, G, nnz, out);
  return hipGetLastError();
}

hipError_t launch_check_bases(const int64_t *vtx_base, const int64_t *edge_base, int64_t G, int64_t N,
                              int64_t nnz, unsigned long long *bad, hipStream_t s) {
  check_bases<<<(unsigned)((G + 1 + 255) / 256), 256, 0, s>>>(vtx_base, edge_base, G, N, nnz, bad);
  return hipGetLastError();
}

hipError_t launch_graph_entries(const GraphDesc *d, int64_t G, int64_t *cnt, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  graph_entries<<<(unsigned)(G < 4096 ? G : 4096), kBlock, 0, s>>>(d, G, cnt);
  return hipGetLastError();
}

hipError_t launch_gather(const GraphDesc *d, const int64_t *vtx_base, const int64_t *edge_base, int64_t G,
                         int64_t N, int64_t nnz, int64_t vshift, int64_t eshift, int64_t *off, int32_t *cols,
                         uint32_t *w, uint32_t *bad, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  gather_offsets<<<tiles(N + 1), kBlock, 0, s>>>(d, vtx_base, edge_base, G, N, eshift, off);
  if (nnz > 0)
    gather_entries<<<tiles(nnz), kBlock, 0, s>>>(d, vtx_base, edge_base, G, nnz, vshift, cols, w, bad);
  return hipGetLastError();
}

hipError_t launch_session_admit(const SessionRange *r, int64_t count, int32_t *gid, int32_t *lab, uint8_t *act0,
                                uint8_t *act1, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  session_admit<<<(unsigned)(count < 4096 ? count : 4096), kBlock, 0, s>>>(r, count, gid, lab, act0, act1);
  return hipGetLastError();
}

hipError_t launch_session_slots(const SessionRange *r, int64_t count, int32_t max_iters, double tol, int64_t *glimit,
                                int32_t *giters, uint8_t *gdone, int64_t *gdn, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  session_slots<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(r, count, max_iters, tol, glimit, giters, gdone, gdn);
  return hipGetLastError();
}

hipError_t launch_session_split_labels(const int32_t *lab, const int32_t *gid, const uint8_t *sel, int64_t n,
                                       int32_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  session_split_labels<<<tiles(n), kBlock, 0, s>>>(lab, gid, sel, n, out);
  return hipGetLastError();
}

hipError_t launch_session_finish(const SessionRange *r, int64_t count, const int32_t *split, int32_t *gid,
                                 int32_t dead, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  session_finish<<<(unsigned)(count < 4096 ? count : 4096), kBlock, 0, s>>>(r, count, split, gid, dead);
  return hipGetLastError();
}

hipError_t launch_session_move(const SessionRange *r, int64_t count, const int64_t *off, const int32_t *cols,
                               const uint32_t *w, const int32_t *lab, int64_t *off2, int32_t *cols2, uint32_t *w2,
                               int32_t *lab2, int32_t *gid, uint8_t *act0, uint8_t *act1, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  session_move<<<(unsigned)(count < 4096 ? count : 4096), kBlock, 0, s>>>(r, count, off, cols, w, lab, off2, cols2,
                                                                         w2, lab2, gid, act0, act1);
  return hipGetLastError();
}

hipError_t launch_localize(int32_t *lab, const int64_t *vtx_base, int64_t G, int64_t N, hipStream_t s) {
  if (N <= 0 || G <= 0) return hipSuccess;
  localize<<<tiles(N), kBlock, 0, s>>>(lab, vtx_base, G, N);
  return hipGetLastError();
}

hipError_t launch_scatter_labels(const GraphDesc *d, const int32_t *lab, const int64_t *vtx_base,
                                 const uint32_t *bad, int64_t G, int64_t N, hipStream_t s) {
  if (N <= 0 || G <= 0) return hipSuccess;
  scatter_labels<<<tiles(N), kBlock, 0, s>>>(d, lab, vtx_base, bad, G, N);
  return hipGetLastError();
}

}  // namespace gsl
