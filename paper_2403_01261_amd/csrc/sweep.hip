// Label-propagation sweep kernels (lpaMove + scanCommunities of Alg. 3, the
// label rule of Eq. 2), synchronous form.
//
// Every kernel processes the vertices of one degree tier.  For a vertex i it
// sums w over the row entries (i, j), j != i, per label C[j], takes the label
// of largest sum (smallest label on ties; a row without such entries keeps its
// label) and, if that label differs from C[i], writes it to Cn[i], sets
// chg[i] and counts the change.  C is only read during a sweep; a separate
// apply kernel copies Cn into C for the changed vertices afterwards, so every
// vertex reads the labels of the previous sweep.
//
// Pruning: with `dense` clear, only vertices flagged in `act` are processed;
// with `mark` set, every neighbour of a changed vertex is flagged in `nact`
// for the next sweep.  Processing more vertices than flagged never changes a
// result (an unflagged vertex already holds the argmax of its unchanged
// neighbourhood), so the host may run a sweep dense instead of marking.
//
// Weights are summed exactly in 32-bit integers; every sweep checks that no
// row's total weight reaches 2^32 and raises `overflow` otherwise.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

__device__ __forceinline__ void record_change(const SweepArgs &a, int32_t v, uint32_t cstar,
                                              LocalCounts &lc) {
  a.Cn[v] = (int32_t)cstar;
  a.chg[v] = 1;
  lc.dn += 1;
}

// Block totals of the per-thread counts, stored as this block's record.
__device__ __forceinline__ void flush_counts(const SweepArgs &a, const LocalCounts &lc,
                                             unsigned long long *red) {
  const unsigned long long dn = block_sum(lc.dn, red);
  const unsigned long long pr = block_sum(lc.processed, red);
  const unsigned long long ed = block_sum(lc.edges, red);
  const unsigned long long mk = block_sum(lc.marked, red);
  const unsigned long long ov = block_sum(lc.overflow, red);
  if (threadIdx.x == 0) {
    unsigned long long *r = a.part + (size_t)blockIdx.x * kCountFields;
    r[0] = dn;
    r[1] = pr;
    r[2] = ed;
    r[3] = mk;
    r[4] = ov;
  }
}

// ---------------------------------------------------------------------------
// Tier 1: one thread per vertex, degree <= D.  The row's labels and weights
// stay in registers; the weight of a label is the sum over equal entries.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void sweep_thread(SweepArgs a, const int32_t *__restrict__ list,
                                                    int64_t first, int64_t count) {
  __shared__ unsigned long long red[256 / kWave];
  LocalCounts lc;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += stride) {
    const int32_t v = list ? list[first + idx] : (int32_t)(first + idx);
    if (!a.dense && !a.act[v]) continue;
    const int64_t b = a.off[v];
    const int d = (int)(a.off[v + 1] - b);
    int32_t col[D];
    uint32_t lab[D], w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) col[k] = k < d ? a.cols[b + k] : v;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      lab[k] = col[k] != v ? (uint32_t)a.C[col[k]] : kNoLabel;
      w[k] = k < d ? (a.w ? a.w[b + k] : 1u) : 0u;
    }
    unsigned long long rowsum = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) rowsum += w[k];
    unsigned long long best = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (lab[k] == kNoLabel) continue;
      uint32_t s = 0;
#pragma unroll
      for (int m = 0; m < D; ++m) s += lab[m] == lab[k] ? w[m] : 0u;
      const unsigned long long key = argmax_key(lab[k], s);
      best = key > best ? key : best;
    }
    lc.processed += 1;
    lc.edges += (unsigned long long)d;
    lc.overflow += rowsum >> 32 ? 1 : 0;
    if (best) {
      const uint32_t cstar = key_label(best);
      if (cstar != (uint32_t)a.C[v]) {
        record_change(a, v, cstar, lc);
        if (a.mark)
#pragma unroll
          for (int k = 0; k < D; ++k)
            if (k < d) {
              if (!a.nact[col[k]]) a.nact[col[k]] = 1;
              lc.marked += 1;
            }
      }
    }
  }
  flush_counts(a, lc, red);
}

// ---------------------------------------------------------------------------
// Tiers 2-8: a group of G lanes per vertex -- a slice of a wavefront (G <= 64)
// or the whole workgroup (G == BLOCK) -- with a private LDS table of up to
// 2^LOG2S slots.  Every lane owns at most K row entries (the tier bound is
// G * K), loads them all before inserting, and remembers the slots it
// claimed: after the barrier the claimers read the final sums of their own
// slots (the argmax candidates) and clear them, so no lane scans empty slots.
// All groups of a block move through the insert / read phases together.
// ---------------------------------------------------------------------------
template <int G, int LOG2S, int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void sweep_lds(SweepArgs a, const int32_t *__restrict__ list,
                                                   int64_t first, int64_t count) {
  static_assert(G <= 64 || G == BLOCK, "group is a wave slice or the block");
  constexpr int GPB = BLOCK / G;
  constexpr int S = 1 << LOG2S;
  constexpr int NW = BLOCK / kWave;
  __shared__ unsigned long long tab[GPB * S];
  __shared__ unsigned long long red[NW];
  __shared__ unsigned long long red2[NW];
  for (int s = threadIdx.x; s < GPB * S; s += BLOCK) tab[s] = kEmptySlot;
  __syncthreads();
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  unsigned long long *T = tab + g * S;
  LocalCounts lc;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
    const int64_t idx = base + g;
    int32_t v = -1;
    if (idx < count) {
      v = list ? list[first + idx] : (int32_t)(first + idx);
      if (!a.dense && !a.act[v]) v = -1;
    }
    int64_t b = 0, e = 0;
    int log2s = 1;
    if (v >= 0) {
      b = a.off[v];
      e = a.off[v + 1];
      log2s = table_log2(e - b, 1, LOG2S);
    }
    int32_t j[K];
    uint32_t wt[K], lab[K];
    int slot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t p = b + lane + (int64_t)k * G;
      const bool in = p < e;
      j[k] = in ? a.cols[p] : -1;
      wt[k] = in ? (a.w ? a.w[p] : 1u) : 0u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) lab[k] = (j[k] >= 0 && j[k] != v) ? (uint32_t)a.C[j[k]] : kNoLabel;
    unsigned long long rowsum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) rowsum += wt[k];
#pragma unroll
    for (int k = 0; k < K; ++k) slot[k] = lab[k] != kNoLabel ? lds_insert(T, log2s, lab[k], wt[k]) : -1;
    __syncthreads();
    unsigned long long best = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (slot[k] >= 0) {
        const unsigned long long x = T[slot[k]];
        const unsigned long long key = argmax_key((uint32_t)(x >> 32), (uint32_t)x);
        best = key > best ? key : best;
        T[slot[k]] = kEmptySlot;
      }
    }
    if constexpr (G <= 64) {
      best = group_max<G>(best);
      rowsum = group_sum<G>(rowsum);
    } else {
      best = group_max<kWave>(best);
      rowsum = wave_sum(rowsum);
      if (threadIdx.x % kWave == 0) {
        red[threadIdx.x / kWave] = best;
        red2[threadIdx.x / kWave] = rowsum;
      }
      __syncthreads();
      best = 0;
      rowsum = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        best = red[w] > best ? red[w] : best;
        rowsum += red2[w];
      }
    }
    if (v >= 0) {
      if (lane == 0) {
        lc.processed += 1;
        lc.edges += (unsigned long long)(e - b);
        lc.overflow += rowsum >> 32 ? 1 : 0;
      }
      if (best) {
        const uint32_t cstar = key_label(best);
        if (cstar != (uint32_t)a.C[v]) {
          if (lane == 0) record_change(a, v, cstar, lc);
          if (a.mark) {
#pragma unroll
            for (int k = 0; k < K; ++k)
              if (j[k] >= 0) {
                if (!a.nact[j[k]]) a.nact[j[k]] = 1;
                lc.marked += 1;
              }
          }
        }
      }
    }
    __syncthreads();
  }
  flush_counts(a, lc, red);
}

// Copies the new label of every changed vertex into C, clears chg and, when
// requested, clears the active flags consumed by the sweep.  Four vertices per
// thread; the flag arrays are padded to a multiple of 4 bytes.
__global__ __launch_bounds__(256) void apply_changes(int32_t *__restrict__ C,
                                                     const int32_t *__restrict__ Cn,
                                                     uint8_t *__restrict__ chg,
                                                     uint8_t *__restrict__ act_clear, int64_t n) {
  const int64_t quads = (n + 3) / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < quads; q += stride) {
    uint32_t word = reinterpret_cast<uint32_t *>(chg)[q];
    if (act_clear) reinterpret_cast<uint32_t *>(act_clear)[q] = 0u;
    if (!word) continue;
    reinterpret_cast<uint32_t *>(chg)[q] = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if ((word >> (8 * k)) & 0xffu) {
        const int64_t v = 4 * q + k;
        C[v] = Cn[v];
      }
  }
}

__global__ void init_labels(int32_t *C, int32_t *Cn, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    C[i] = (int32_t)i;
    Cn[i] = (int32_t)i;
  }
}

__global__ void fill_u64(uint64_t *p, uint64_t v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void fill_u8(uint8_t *p, uint8_t v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint32_t v4 = 0x01010101u * v;
  const int64_t words = count / 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    reinterpret_cast<uint32_t *>(p)[i] = v4;
  for (int64_t i = words * 4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = v;
}

int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

hipError_t launch_sweep_tier(int tier, const SweepArgs &a, const int32_t *list, int64_t first,
                             int64_t count, int *grid_out, hipStream_t s) {
  *grid_out = 0;
  if (count <= 0) return hipSuccess;
  constexpr int kCap = kMaxTierGrid;
  int grid = 0;
  switch (tier) {
    case 1:
      grid = grid_for(count, 256, kCap);
      sweep_thread<8><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 2:
      grid = grid_for(count, 256 / 8, kCap);
      sweep_lds<8, 5, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 3:
      grid = grid_for(count, 256 / 16, kCap);
      sweep_lds<16, 6, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 4:
      grid = grid_for(count, 256 / 32, kCap);
      sweep_lds<32, 7, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 5:
      grid = grid_for(count, 256 / 64, kCap);
      sweep_lds<64, 8, 256, 2><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 6:
      grid = grid_for(count, 256 / 64, kCap);
      sweep_lds<64, 10, 256, 8><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    case 7:
      grid = grid_for(count, 1, kCap);
      sweep_lds<256, 12, 256, 8><<<grid, 256, 0, s>>>(a, list, first, count);
      break;
    default:
      return hipErrorInvalidValue;
  }
  *grid_out = grid;
  return hipGetLastError();
}

namespace {
__global__ void reduce_counts(const unsigned long long *__restrict__ part, TierGrids g,
                              unsigned long long (*tier_stats)[4], unsigned long long *dn,
                              unsigned long long *processed, unsigned long long *edges,
                              unsigned long long *overflow) {
  __shared__ unsigned long long red[256 / kWave];
  const int t = blockIdx.x;
  const int nb = g.g[t];
  if (nb <= 0) return;
  const unsigned long long *r = part + (size_t)t * kMaxTierGrid * kCountFields;
  unsigned long long v[kCountFields] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int f = 0; f < kCountFields; ++f) v[f] += r[(size_t)b * kCountFields + f];
#pragma unroll
  for (int f = 0; f < kCountFields; ++f) v[f] = block_sum(v[f], red);
  if (threadIdx.x == 0) {
    atomicAdd(&tier_stats[t][2], v[0]);
    atomicAdd(&tier_stats[t][0], v[1]);
    atomicAdd(&tier_stats[t][1], v[2]);
    atomicAdd(&tier_stats[t][3], v[3]);
    atomicAdd(dn, v[0]);
    atomicAdd(processed, v[1]);
    atomicAdd(edges, v[2]);
    if (v[4]) atomicAdd(overflow, v[4]);
  }
}
}  // namespace

hipError_t launch_reduce_counts(const unsigned long long *part, TierGrids g,
                                unsigned long long (*tier_stats)[4], unsigned long long *dn,
                                unsigned long long *processed, unsigned long long *edges,
                                unsigned long long *overflow, hipStream_t s) {
  reduce_counts<<<kNumTiers, 256, 0, s>>>(part, g, tier_stats, dn, processed, edges, overflow);
  return hipGetLastError();
}

hipError_t launch_apply(int32_t *C, const int32_t *Cn, uint8_t *chg, uint8_t *act_clear, int64_t n,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  apply_changes<<<grid_for((n + 3) / 4, 256, 256 * 32), 256, 0, s>>>(C, Cn, chg, act_clear, n);
  return hipGetLastError();
}

hipError_t launch_init_labels(int32_t *C, int32_t *Cn, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  init_labels<<<grid_for(n, 256, 256 * 32), 256, 0, s>>>(C, Cn, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_u64<<<grid_for(count, 256, 256 * 32), 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_u8<<<grid_for((count + 3) / 4, 256, 256 * 32), 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

}  // namespace gsl
