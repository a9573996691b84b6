// Degree-ordered renumbering of the graph.
//
// The plan's list orders the vertices hubs first and isolated vertices last;
// new id p stands for old vertex list[p].  A renumbered copy of the CSR lets
// every tier kernel walk a contiguous id range (coalesced offsets, rows and
// flags) and packs the labels of the highest-degree vertices -- the targets of
// most label gathers -- into a few megabytes that stay in L2.  Labels keep
// their original-id values, so the smallest-label tie-break and the output are
// unchanged; only storage positions move.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

constexpr int kScanBlock = 1024;

__global__ void reorder_invert(const int32_t *__restrict__ list, int64_t n, int32_t *__restrict__ old2new) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    old2new[list[p]] = (int32_t)p;
}

// off2[p + 1] = degree of list[p] for the np non-isolated rows; off2[0] = 0.
// Also the initial labels of all n vertices (an isolated vertex keeps its
// own, even where an entry of a graph that is not symmetric names it).
__global__ void reorder_degrees(const int64_t *__restrict__ off, const int32_t *__restrict__ list,
                                int64_t np, int64_t n, int64_t *__restrict__ off2, int32_t *__restrict__ lab) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int32_t v = list[p];
    if (p < np) off2[p + 1] = off[v + 1] - off[v];
    lab[p] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off2[0] = 0;
}

// In-place inclusive scan of a[0..n): per-block scan, block totals to sums.
__global__ __launch_bounds__(kScanBlock) void scan_local(int64_t *a, int64_t n, int64_t *sums) {
  __shared__ int64_t part[kScanBlock];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  part[threadIdx.x] = i < n ? a[i] : 0;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const int64_t y = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  if (i < n) a[i] = part[threadIdx.x];
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = part[kScanBlock - 1];
}

// Exclusive scan of sums[0..nb) in one block.
__global__ __launch_bounds__(kScanBlock) void scan_sums(int64_t *sums, int64_t nb) {
  __shared__ int64_t part[kScanBlock];
  const int64_t per = (nb + kScanBlock - 1) / kScanBlock;
  const int64_t lo = threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
  int64_t s = 0;
  for (int64_t b = lo; b < hi; ++b) s += sums[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const int64_t y = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  int64_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
  for (int64_t b = lo; b < hi; ++b) {
    const int64_t c = sums[b];
    sums[b] = run;
    run += c;
  }
}

__global__ __launch_bounds__(kScanBlock) void scan_add(int64_t *a, int64_t n, const int64_t *sums) {
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) a[i] += sums[blockIdx.x];
}

struct CopyArgs {
  const int64_t *off;
  const int32_t *cols;
  const uint32_t *w;
  const int32_t *list;
  const int32_t *old2new;
  const int64_t *off2;
  int32_t *cols2;
  uint32_t *w2;
  // First sweep, folded into the copy: while the labels are still the vertex
  // ids, a row without duplicate entries holds every label once, so its winner
  // is the heaviest entry (smallest id on ties) -- no table, no label gather.
  unsigned long long *first_key;   // per new row: packed argmax key (0: none)
  unsigned long long *hub_rowsum;  // per hub: summed row weight
  unsigned long long *flags;       // bit 0: a row is not strictly increasing
                                   // bit 1: a row's weight sum reaches 2^32
};

// Rows [first, first + count) of the new numbering, G lanes per row (G <= 64
// or the whole block), each lane owning at most K entries of the row (the
// tier bound is G * K) with all its loads issued before any use.
template <int G, int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void reorder_rows(CopyArgs c, int64_t first, int64_t count) {
  constexpr int GPB = BLOCK / G;
  __shared__ unsigned long long red[BLOCK / kWave], red2[BLOCK / kWave];
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  int unsorted = 0, ovf = 0;
  for (int64_t base = (int64_t)blockIdx.x * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
    const int64_t idx = base + g;
    unsigned long long best = 0, rowsum = 0;
    int64_t p = -1, b = 0, e = 0, b2 = 0;
    int32_t v = -1;
    if (idx < count) {
      p = first + idx;
      v = c.list[p];
      b = c.off[v];
      e = c.off[v + 1];
      b2 = c.off2[p];
    }
    int32_t j[K], jn[K];
    uint32_t w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t q = b + lane + (int64_t)k * G;
      const bool in = q < e;
      j[k] = in ? c.cols[q] : -1;
      jn[k] = in && q + 1 < e ? c.cols[q + 1] : 0x7fffffff;
      w[k] = in ? (c.w ? c.w[q] : 1u) : 0u;
    }
    // every old->new lookup is issued before the first store (a store could
    // alias a later lookup's address as far as the compiler knows, which
    // would keep one random gather in flight per lane)
    int32_t nj[K];
#pragma unroll
    for (int k = 0; k < K; ++k) nj[k] = j[k] >= 0 ? c.old2new[j[k]] : 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (j[k] < 0) continue;
      const int64_t q = b + lane + (int64_t)k * G;
      c.cols2[b2 + (q - b)] = nj[k];
      if (c.w) c.w2[b2 + (q - b)] = w[k];
      unsorted |= jn[k] <= j[k];
      rowsum += w[k];
      if (j[k] != v) {
        const unsigned long long key = argmax_key((uint32_t)j[k], w[k]);
        best = key > best ? key : best;
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
      for (int ww = 0; ww < BLOCK / kWave; ++ww) {
        best = red[ww] > best ? red[ww] : best;
        rowsum += red2[ww];
      }
      __syncthreads();
    }
    if (p >= 0 && lane == 0) {
      c.first_key[p] = best;
      ovf |= rowsum >> 32 ? 1 : 0;
    }
  }
  const int any_unsorted = __syncthreads_or(unsorted);
  const int any_ovf = __syncthreads_or(ovf);
  if (threadIdx.x == 0 && (any_unsorted || any_ovf))
    atomicOr(c.flags, (unsigned long long)(any_unsorted ? 1 : 0) | (any_ovf ? 2 : 0));
}

// Hub rows in chunks of kHubChunk entries, one block per chunk; chunk_start
// and chunk_owner are the hub layout (hubs = new ids 0..H-1).  Each lane
// loads its kChunk / 256 entries, then issues all their old->new lookups,
// then stores.  The first-sweep key and weight sum of a hub are combined
// across its chunks.
constexpr int kChunk = kHubChunk;
constexpr int kChunkPerLane = kChunk / 256;
__global__ __launch_bounds__(256) void reorder_hub_rows(CopyArgs c, const int64_t *chunk_start,
                                                        const int32_t *chunk_owner) {
  __shared__ unsigned long long red[256 / kWave], red2[256 / kWave];
  const int64_t ch = blockIdx.x;
  const int64_t p = chunk_owner[ch];
  const int32_t v = c.list[p];
  const int64_t rb = c.off[v], re = c.off[v + 1], b2 = c.off2[p];
  const int64_t b = rb + (ch - chunk_start[p]) * kChunk;
  const int64_t e = b + kChunk < re ? b + kChunk : re;
  unsigned long long best = 0, rowsum = 0;
  int unsorted = 0;
  int32_t j[kChunkPerLane], jn[kChunkPerLane], nj[kChunkPerLane];
  uint32_t w[kChunkPerLane];
#pragma unroll
  for (int k = 0; k < kChunkPerLane; ++k) {
    const int64_t q = b + threadIdx.x + (int64_t)k * 256;
    const bool in = q < e;
    j[k] = in ? c.cols[q] : -1;
    jn[k] = in && q + 1 < re ? c.cols[q + 1] : 0x7fffffff;
    w[k] = in ? (c.w ? c.w[q] : 1u) : 0u;
  }
#pragma unroll
  for (int k = 0; k < kChunkPerLane; ++k) nj[k] = j[k] >= 0 ? c.old2new[j[k]] : 0;
#pragma unroll
  for (int k = 0; k < kChunkPerLane; ++k) {
    if (j[k] < 0) continue;
    const int64_t q = b + threadIdx.x + (int64_t)k * 256;
    c.cols2[b2 + (q - rb)] = nj[k];
    if (c.w) c.w2[b2 + (q - rb)] = w[k];
    unsorted |= jn[k] <= j[k];
    rowsum += w[k];
    if (j[k] != v) {
      const unsigned long long key = argmax_key((uint32_t)j[k], w[k]);
      best = key > best ? key : best;
    }
  }
  best = group_max<kWave>(best);
  rowsum = wave_sum(rowsum);
  if (threadIdx.x % kWave == 0) {
    red[threadIdx.x / kWave] = best;
    red2[threadIdx.x / kWave] = rowsum;
  }
  const int any_unsorted = __syncthreads_or(unsorted);
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; ++w) {
      red[0] = red[w] > red[0] ? red[w] : red[0];
      red2[0] += red2[w];
    }
    if (red[0]) __hip_atomic_fetch_max(&c.first_key[p], red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (red2[0]) __hip_atomic_fetch_add(&c.hub_rowsum[p], red2[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (any_unsorted) atomicOr(c.flags, 1ull);
  }
}

// Applies the folded first sweep (if `apply` and no row failed the strict
// increase test): lab[p] becomes the winner of row p, changes are counted into
// *dn.  Hub weight sums are always checked (bit 1 of flags) and reset.
__global__ __launch_bounds__(256) void first_apply(const unsigned long long *__restrict__ first_key,
                                                   const int32_t *__restrict__ orig, int64_t np,
                                                   unsigned long long *hub_rowsum, int64_t H,
                                                   unsigned long long *flags, int32_t *lab,
                                                   unsigned long long *dn, int apply) {
  __shared__ unsigned long long red[256 / kWave];
  const bool skip = !apply || (*flags & 1ull) != 0;  // uniform
  unsigned long long changes = 0;
  int ovf = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    if (p < H) {
      ovf |= hub_rowsum[p] >> 32 ? 1 : 0;
      hub_rowsum[p] = 0;
    }
    if (skip) continue;
    const unsigned long long key = first_key[p];
    if (key) {
      const uint32_t cstar = key_label(key);
      if ((int32_t)cstar != orig[p]) {
        lab[p] = (int32_t)cstar;
        changes += 1;
      }
    }
  }
  const unsigned long long t = block_sum(changes, red);
  const int any_ovf = __syncthreads_or(ovf);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(dn, t);
    if (any_ovf) atomicOr(flags, 2ull);
  }
}

// Output in old ids: out[list[p]] = val[p] for p < np, out[list[p]] = list[p]
// for the isolated vertices p >= np.
__global__ void reorder_scatter(const int32_t *__restrict__ list, const int32_t *__restrict__ val,
                                int64_t np, int64_t n, int32_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int32_t v = list[p];
    out[v] = p < np ? val[p] : v;
  }
}

int grid_of(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

// Renumbered CSR (off2, cols2, w2) of the np non-isolated vertices and their
// initial labels lab[p] = list[p].  scan_tmp needs plan_blocks(np) + 1 entries.
hipError_t launch_reorder(const int64_t *off, const int32_t *cols, const uint32_t *w, int64_t n,
                          const int32_t *list, const int64_t *tier_count_h, const int64_t *tier_start_h,
                          const int64_t *hub_chunk_start, const int32_t *hub_chunk_owner, int64_t hub_chunks,
                          int32_t *old2new, int64_t *off2, int32_t *cols2, uint32_t *w2, int32_t *lab,
                          int64_t *scan_tmp, unsigned long long *first_key,
                          unsigned long long *hub_rowsum, unsigned long long *flags,
                          unsigned long long *dn0, int apply_first, const TierConfig &cfg, hipStream_t s) {
  const int64_t np = n - tier_count_h[0];
  constexpr int kCap = 256 * 32;
  reorder_invert<<<grid_of(n, 256, kCap), 256, 0, s>>>(list, n, old2new);
  reorder_degrees<<<grid_of(n, 256, kCap), 256, 0, s>>>(off, list, np, n, off2, lab);
  if (np > 0) {
    const int64_t nb = (np + kScanBlock - 1) / kScanBlock;
    scan_local<<<(unsigned)nb, kScanBlock, 0, s>>>(off2 + 1, np, scan_tmp);
    scan_sums<<<1, kScanBlock, 0, s>>>(scan_tmp, nb);
    scan_add<<<(unsigned)nb, kScanBlock, 0, s>>>(off2 + 1, np, scan_tmp);
  }
  CopyArgs c{off, cols, w, list, old2new, off2, cols2, w2, first_key, hub_rowsum, flags};
  const int64_t H = tier_count_h[kNumTiers - 1];
  if (H > 0) launch_fill_u64(reinterpret_cast<uint64_t *>(first_key), 0, H, s);
  for (int t = 1; t < kNumTiers; ++t) {
    const int64_t cnt = tier_count_h[t], first = tier_start_h[t];
    if (cnt <= 0) continue;
    // the copy kernel takes rows up to G * K entries: the smallest that
    // covers the tier's degree bound
    const int64_t d = cfg.bound[t];
    if (t == kNumTiers - 1) {
      if (hub_chunks > 0)
        reorder_hub_rows<<<(unsigned)hub_chunks, 256, 0, s>>>(c, hub_chunk_start, hub_chunk_owner);
    } else if (d <= 8) {
      reorder_rows<1, 256, 8><<<grid_of(cnt, 256, kCap), 256, 0, s>>>(c, first, cnt);
    } else if (d <= 16) {
      reorder_rows<8, 256, 2><<<grid_of(cnt, 32, kCap), 256, 0, s>>>(c, first, cnt);
    } else if (d <= 32) {
      reorder_rows<16, 256, 2><<<grid_of(cnt, 16, kCap), 256, 0, s>>>(c, first, cnt);
    } else if (d <= 64) {
      reorder_rows<32, 256, 2><<<grid_of(cnt, 8, kCap), 256, 0, s>>>(c, first, cnt);
    } else if (d <= 128) {
      reorder_rows<64, 256, 2><<<grid_of(cnt, 4, kCap), 256, 0, s>>>(c, first, cnt);
    } else if (d <= 512) {
      reorder_rows<64, 256, 8><<<grid_of(cnt, 4, kCap), 256, 0, s>>>(c, first, cnt);
    } else if (d <= 2048) {
      reorder_rows<256, 256, 8><<<grid_of(cnt, 1, kCap), 256, 0, s>>>(c, first, cnt);
    } else {
      reorder_rows<1024, 1024, 8><<<grid_of(cnt, 1, kCap), 1024, 0, s>>>(c, first, cnt);
    }
  }
  if (np > 0)
    first_apply<<<grid_of(np, 256, 1024), 256, 0, s>>>(first_key, list, np, hub_rowsum, H, flags, lab, dn0,
                                                       apply_first);
  return hipGetLastError();
}

hipError_t launch_reorder_scatter(const int32_t *list, const int32_t *val, int64_t np, int64_t n,
                                  int32_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  reorder_scatter<<<grid_of(n, 256, 256 * 32), 256, 0, s>>>(list, val, np, n, out);
  return hipGetLastError();
}

}  // namespace gsl
