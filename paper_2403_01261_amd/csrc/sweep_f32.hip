// Sweeps with fp32 weights summed in fp64 -- the paper's precision
// (Sec. 5.1.2: float weights, double accumulators).  The label rule is Eq. 2
// as in sweep.hip: per processed vertex the label of largest summed weight
// among its row entries (j != i), smallest label on ties; a row without such
// entries keeps its label.
//
// Same tiers, loop state, pruning and change records as the integer path;
// only the accumulation differs.  Tables keep labels and fp64 sums in two
// LDS arrays (12 bytes per slot).  The thread tier sums in CSR entry order,
// like the oracle; LDS and hub tables add with atomics, so a sum may differ
// from the entry-order sum in its last bits when weights span more than 2^29
// in magnitude -- only exact ties can then resolve differently.  Hubs (rows
// longer than the last tier) sum chunk by chunk in LDS and fold the distinct
// labels into a global table per hub (the global-memory fallback), which one
// workgroup per hub scans for the winner.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

// (sum, label) pairs: larger sum first, then smaller label; label kNoLabel
// (with sum -1) is "no candidate".
__device__ __forceinline__ bool better(double w, uint32_t l, double bw, uint32_t bl) {
  if (l == kNoLabel) return false;
  return bl == kNoLabel || w > bw || (w == bw && l < bl);
}

template <int W>
__device__ __forceinline__ void shfl_best(double &w, uint32_t &l) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    const double ow = __shfl_xor(w, o, W);
    const uint32_t ol = (uint32_t)__shfl_xor((int)l, o, W);
    if (better(ow, ol, w, l)) {
      w = ow;
      l = ol;
    }
  }
}

__device__ __forceinline__ float wf(const SweepArgs &a, int64_t p) {
  return a.w ? reinterpret_cast<const float *>(a.w)[p] : 1.0f;
}

__device__ __forceinline__ void change(const SweepArgs &a, int32_t v, uint32_t cstar, LocalCounts &lc) {
  if (a.inplace)
    __hip_atomic_store(const_cast<int32_t *>(a.C) + v, (int32_t)cstar, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  else
    a.Cn[v] = (int32_t)cstar;
  a.chg[v] = 1;
  lc.dn += 1;
}

__device__ __forceinline__ void flush(const SweepArgs &a, const LocalCounts &lc, unsigned long long *red) {
  const unsigned long long dn = block_sum(lc.dn, red);
  const unsigned long long pr = block_sum(lc.processed, red);
  const unsigned long long ed = block_sum(lc.edges, red);
  const unsigned long long mk = block_sum(lc.marked, red);
  if (threadIdx.x == 0) {
    unsigned long long *r = a.part + (size_t)blockIdx.x * kCountFields;
    r[0] = dn;
    r[1] = pr;
    r[2] = ed;
    r[3] = mk;
    r[4] = 0;  // fp64 sums do not overflow
  }
}

// Adds w to `label` in an LDS table (keys / sums, 2^log2s slots).  Returns the
// slot if this call claimed it, else -1.
__device__ __forceinline__ int lds_insert_f64(uint32_t *keys, double *sums, int log2s, uint32_t label,
                                              double w) {
  const uint32_t mask = (1u << log2s) - 1u;
  uint32_t h = slot_hash(label, log2s);
  for (;;) {
    const uint32_t prev = atomicCAS(&keys[h], kEmptyKey, label);
    if (prev == kEmptyKey || prev == label) {
      atomicAdd(&sums[h], w);
      return prev == kEmptyKey ? (int)h : -1;
    }
    h = (h + 1u) & mask;
  }
}

// Tier 1: a thread per vertex, row in registers, sums in entry order.
template <int D>
__global__ __launch_bounds__(256) void sweepf_thread(SweepArgs a, const int32_t *__restrict__ list, int64_t first,
                                                     int64_t count) {
  __shared__ unsigned long long red[256 / kWave];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  LocalCounts lc;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += stride) {
    const int32_t v = list ? list[first + idx] : (int32_t)(first + idx);
    if (!sweep_takes(a, sv, v)) continue;
    const int64_t b = a.off[v];
    const int d = (int)(a.off[v + 1] - b);
    int32_t col[D];
    uint32_t lab[D];
    double w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) col[k] = k < d ? a.cols[b + k] : v;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      lab[k] = col[k] != v ? (uint32_t)a.C[col[k]] : kNoLabel;
      w[k] = k < d ? (double)wf(a, b + k) : 0.0;
    }
    double bw = -1.0;
    uint32_t bl = kNoLabel;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (lab[k] == kNoLabel) continue;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < D; ++m) s += lab[m] == lab[k] ? w[m] : 0.0;
      if (better(s, lab[k], bw, bl)) {
        bw = s;
        bl = lab[k];
      }
    }
    lc.processed += 1;
    lc.edges += (unsigned long long)d;
    if (bl != kNoLabel && bl != (uint32_t)a.C[v]) {
      change(a, v, bl, lc);
      if (sv.mark)
#pragma unroll
        for (int k = 0; k < D; ++k)
          if (k < d) {
            if (!sv.nact[col[k]]) sv.nact[col[k]] = 1;
            lc.marked += 1;
          }
    }
  }
  flush(a, lc, red);
}

// Tiers 2-7: a group of G lanes per vertex (a wave slice, or the block), K
// entries per lane, LDS keys / sums of 2^LOG2S slots per group.
template <int G, int LOG2S, int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void sweepf_lds(SweepArgs a, const int32_t *__restrict__ list, int64_t first,
                                                    int64_t count) {
  static_assert(G <= 64 || G == BLOCK, "group is a wave slice or the block");
  constexpr int GPB = BLOCK / G;
  constexpr int S = 1 << LOG2S;
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t keys[GPB * S];
  __shared__ double sums[GPB * S];
  __shared__ double rw[NW];
  __shared__ uint32_t rl[NW];
  __shared__ unsigned long long red[NW];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  for (int s = threadIdx.x; s < GPB * S; s += BLOCK) {
    keys[s] = kEmptyKey;
    sums[s] = 0.0;
  }
  __syncthreads();
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t *Tk = keys + g * S;
  double *Ts = sums + g * S;
  LocalCounts lc;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
    const int64_t idx = base + g;
    int32_t v = -1;
    if (idx < count) {
      v = list ? list[first + idx] : (int32_t)(first + idx);
      if (!sweep_takes(a, sv, v)) v = -1;
    }
    int64_t b = 0, e = 0;
    int log2s = 1;
    if (v >= 0) {
      b = a.off[v];
      e = a.off[v + 1];
      log2s = table_log2(e - b, 1, LOG2S);
    }
    int32_t j[K];
    uint32_t lab[K];
    double wt[K];
    int slot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t p = b + lane + (int64_t)k * G;
      const bool in = p < e;
      j[k] = in ? a.cols[p] : -1;
      wt[k] = in ? (double)wf(a, p) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) lab[k] = (j[k] >= 0 && j[k] != v) ? (uint32_t)a.C[j[k]] : kNoLabel;
#pragma unroll
    for (int k = 0; k < K; ++k) slot[k] = lab[k] != kNoLabel ? lds_insert_f64(Tk, Ts, log2s, lab[k], wt[k]) : -1;
    __syncthreads();
    double bw = -1.0;
    uint32_t bl = kNoLabel;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (slot[k] < 0) continue;
      const double s = Ts[slot[k]];
      if (better(s, Tk[slot[k]], bw, bl)) {
        bw = s;
        bl = Tk[slot[k]];
      }
      Tk[slot[k]] = kEmptyKey;
      Ts[slot[k]] = 0.0;
    }
    if constexpr (G <= 64) {
      shfl_best<G>(bw, bl);
    } else {
      shfl_best<kWave>(bw, bl);
      if (threadIdx.x % kWave == 0) {
        rw[threadIdx.x / kWave] = bw;
        rl[threadIdx.x / kWave] = bl;
      }
      __syncthreads();
      bw = -1.0;
      bl = kNoLabel;
#pragma unroll
      for (int w = 0; w < NW; ++w)
        if (better(rw[w], rl[w], bw, bl)) {
          bw = rw[w];
          bl = rl[w];
        }
    }
    if (v >= 0) {
      if (lane == 0) {
        lc.processed += 1;
        lc.edges += (unsigned long long)(e - b);
      }
      if (bl != kNoLabel && bl != (uint32_t)a.C[v]) {
        if (lane == 0) change(a, v, bl, lc);
        if (sv.mark)
#pragma unroll
          for (int k = 0; k < K; ++k)
            if (j[k] >= 0) {
              if (!sv.nact[j[k]]) sv.nact[j[k]] = 1;
              lc.marked += 1;
            }
      }
    }
    __syncthreads();
  }
  flush(a, lc, red);
}

// Hubs.  Chunk c of hub k holds entries [c * kHubChunk, ...) of the row; the
// hub's global table has kHubSlotsPerChunk slots per chunk (at least twice
// the row length), starting at kHubSlotsPerChunk * chunk_start[k].
constexpr int kHubBlockF = 256;
constexpr int kHubKF = kHubChunk / kHubBlockF;
constexpr int kHubSlotsPerChunk = 2 * kHubChunk;
constexpr int kHubLdsLog2 = 12;
static_assert((1 << kHubLdsLog2) >= 2 * kHubChunk, "chunk table must hold every chunk entry");

__device__ __forceinline__ int64_t owner_of(const int64_t *start, int64_t lo, int64_t hi, int64_t x) {
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (start[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kHubBlockF) void hubf_insert(SweepArgs a, const int32_t *__restrict__ hubs,
                                                          const int64_t *__restrict__ chunk_start, int64_t H,
                                                          uint32_t *gkeys, double *gsums) {
  __shared__ uint32_t keys[1 << kHubLdsLog2];
  __shared__ double sums[1 << kHubLdsLog2];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  const int64_t c = blockIdx.x;
  const int64_t k = owner_of(chunk_start, 0, H, c);
  const int32_t v = hubs ? hubs[k] : (int32_t)k;
  if (!sweep_takes(a, sv, v)) return;  // uniform over the block
  const int64_t rb = a.off[v], re = a.off[v + 1];
  const int64_t b = rb + (c - chunk_start[k]) * kHubChunk;
  const int64_t e = b + kHubChunk < re ? b + kHubChunk : re;
  for (int s = threadIdx.x; s < (1 << kHubLdsLog2); s += kHubBlockF) {
    keys[s] = kEmptyKey;
    sums[s] = 0.0;
  }
  __syncthreads();
  int slot[kHubKF];
#pragma unroll
  for (int q = 0; q < kHubKF; ++q) {
    const int64_t p = b + threadIdx.x + (int64_t)q * kHubBlockF;
    slot[q] = -1;
    if (p < e) {
      const int32_t jj = a.cols[p];
      if (jj != v) slot[q] = lds_insert_f64(keys, sums, kHubLdsLog2, (uint32_t)a.C[jj], (double)wf(a, p));
    }
  }
  __syncthreads();
  // fold the chunk's distinct labels into the hub's global table
  const int64_t tbase = (int64_t)kHubSlotsPerChunk * chunk_start[k];
  const uint64_t tsize = (uint64_t)kHubSlotsPerChunk * (uint64_t)(chunk_start[k + 1] - chunk_start[k]);
#pragma unroll
  for (int q = 0; q < kHubKF; ++q) {
    if (slot[q] < 0) continue;
    const uint32_t label = keys[slot[q]];
    const double s = sums[slot[q]];
    uint64_t h = ((uint64_t)(label * 2654435761u) * tsize) >> 32;
    for (;;) {
      uint32_t expected = kEmptyKey;
      const bool won = __hip_atomic_compare_exchange_strong(gkeys + tbase + h, &expected, label, __ATOMIC_RELAXED,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (won || expected == label) {
        __hip_atomic_fetch_add(gsums + tbase + h, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      h = h + 1 == tsize ? 0 : h + 1;
    }
  }
}

// One workgroup per hub: winner of the hub's table (which it clears),
// decision and, when marking, the flags of the whole row.
__global__ __launch_bounds__(kHubBlockF) void hubf_decide(SweepArgs a, const int32_t *__restrict__ hubs,
                                                          const int64_t *__restrict__ chunk_start, uint32_t *gkeys,
                                                          double *gsums) {
  __shared__ double rw[kHubBlockF / kWave];
  __shared__ uint32_t rl[kHubBlockF / kWave];
  __shared__ int changed;
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  const int64_t k = blockIdx.x;
  const int32_t v = hubs ? hubs[k] : (int32_t)k;
  if (!sweep_takes(a, sv, v)) return;  // uniform; its table is empty
  const int64_t tbase = (int64_t)kHubSlotsPerChunk * chunk_start[k];
  const int64_t tsize = (int64_t)kHubSlotsPerChunk * (chunk_start[k + 1] - chunk_start[k]);
  double bw = -1.0;
  uint32_t bl = kNoLabel;
  for (int64_t s = threadIdx.x; s < tsize; s += kHubBlockF) {
    const uint32_t l = gkeys[tbase + s];
    if (l == kEmptyKey) continue;
    const double w = gsums[tbase + s];
    if (better(w, l, bw, bl)) {
      bw = w;
      bl = l;
    }
    gkeys[tbase + s] = kEmptyKey;
    gsums[tbase + s] = 0.0;
  }
  shfl_best<kWave>(bw, bl);
  if (threadIdx.x % kWave == 0) {
    rw[threadIdx.x / kWave] = bw;
    rl[threadIdx.x / kWave] = bl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bw = -1.0;
    bl = kNoLabel;
    for (int w = 0; w < kHubBlockF / kWave; ++w)
      if (better(rw[w], rl[w], bw, bl)) {
        bw = rw[w];
        bl = rl[w];
      }
    const int64_t d = a.off[v + 1] - a.off[v];
    const int sweep = sv.it;
    const bool ch = bl != kNoLabel && bl != (uint32_t)a.C[v];
    changed = ch ? 1 : 0;
    LocalCounts lc;
    if (ch) change(a, v, bl, lc);
    atomicAdd(a.processed + sweep, 1ull);
    atomicAdd(a.tier + 0, 1ull);
    atomicAdd(a.edges + sweep, (unsigned long long)d);
    atomicAdd(a.tier + 1, (unsigned long long)d);
    if (ch) {
      atomicAdd(a.dn + sweep, 1ull);
      atomicAdd(a.tier + 2, 1ull);
      if (sv.mark) atomicAdd(a.tier + 3, (unsigned long long)d);
    }
  }
  __syncthreads();
  if (changed && sv.mark)
    for (int64_t p = a.off[v] + threadIdx.x; p < a.off[v + 1]; p += kHubBlockF) {
      const int32_t jj = a.cols[p];
      if (!sv.nact[jj]) sv.nact[jj] = 1;
    }
}

__global__ void check_f32(const float *__restrict__ w, int64_t nnz, unsigned long long *bad) {
  int b = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
    b |= (w[e] >= 0.0f && w[e] <= 3.4e38f) ? 0 : 1;
  if (__ballot(b) && threadIdx.x % kWave == 0) atomicOr(bad, 1ull);
}

__global__ void fill_keys(uint32_t *keys, double *sums, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    keys[i] = kEmptyKey;
    sums[i] = 0.0;
  }
}

int grid_f(int64_t items, int per_block) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > kMaxTierGrid ? kMaxTierGrid : g);
}

}  // namespace

// Tiers 1-7 with the default bounds (8/16/32/64/128/512/2048).
hipError_t launch_sweep_tier_f32(int tier, const SweepArgs &a, const int32_t *list, int64_t first, int64_t count,
                                 int *grid_out, hipStream_t s) {
  *grid_out = 0;
  if (count <= 0) return hipSuccess;
  int grid = 0;
  switch (tier) {
    case 1:
      grid = grid_f(count, 256);
      sweepf_thread<8><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 2:
      grid = grid_f(count, 256 / 8);
      sweepf_lds<8, 5, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 3:
      grid = grid_f(count, 256 / 16);
      sweepf_lds<16, 6, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 4:
      grid = grid_f(count, 256 / 32);
      sweepf_lds<32, 7, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 5:
      grid = grid_f(count, 256 / 64);
      sweepf_lds<64, 8, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 6:
      grid = grid_f(count, 256 / 64);
      sweepf_lds<64, 10, 256, 8><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 7:
      grid = grid_f(count, 1);
      sweepf_lds<256, 12, 256, 8><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    default:
      return hipErrorInvalidValue;
  }
  *grid_out = grid;
  return hipGetLastError();
}

hipError_t launch_hub_f32(const SweepArgs &a, const int32_t *hubs, const int64_t *chunk_start, int64_t H,
                          int64_t chunks, uint32_t *gkeys, double *gsums, hipStream_t s) {
  if (H <= 0) return hipSuccess;
  hubf_insert<<<(unsigned)chunks, kHubBlockF, 0, s>>>(a, hubs, chunk_start, H, gkeys, gsums);
  hubf_decide<<<(unsigned)H, kHubBlockF, 0, s>>>(a, hubs, chunk_start, gkeys, gsums);
  return hipGetLastError();
}

int64_t hub_f32_slots(int64_t chunks) { return (int64_t)kHubSlotsPerChunk * chunks; }

hipError_t launch_hub_f32_clear(uint32_t *gkeys, double *gsums, int64_t slots, hipStream_t s) {
  if (slots <= 0) return hipSuccess;
  fill_keys<<<grid_f(slots, 256), 256, 0, s>>>(gkeys, gsums, slots);
  return hipGetLastError();
}

hipError_t launch_check_f32(const float *w, int64_t nnz, unsigned long long *bad, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  check_f32<<<grid_f(nnz, 256 * 4), 256, 0, s>>>(w, nnz, bad);
  return hipGetLastError();
}

}  // namespace gsl
