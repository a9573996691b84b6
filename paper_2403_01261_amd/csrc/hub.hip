// Hub tier of the sweep: vertices of degree above the last level of the tier
// table (4096 by default), too long for one workgroup's LDS table at good
// occupancy.
//
// A hub row is cut into chunks of kHubChunk entries and every chunk gets its
// own workgroup, so one hub keeps many compute units busy.  Partial sums meet
// in a staging area instead of a shared hash table, so no global atomics are
// spent per label:
//   hub_insert : sums the chunk's labels in an LDS table, sorts the distinct
//                (label, sum) pairs by a hash partition of the label (P_k
//                partitions per hub) and stores them, with the partition
//                boundaries, in the chunk's own staging segment;
//   hub_merge  : one workgroup per (hub, partition) sums that partition's pairs
//                from every chunk of the hub in an LDS table and folds the
//                packed argmax key into hub_best[k];
//   hub_decide : one thread per hub compares the winner with C[v];
//   hub_mark   : marks the neighbours of changed hubs, chunk by chunk.
// P_k = ceil(d_k / 2048) (at most kMaxParts), so a partition expects at most
// 2048 distinct labels; a merge table holds 4096 slots and a partition that
// still overflows is redone in 2, 4, ... sub-passes that each keep a hashed
// share of the labels, so every input is handled exactly.  Tables stay at
// 32 KB so several workgroups share a compute unit.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

constexpr int kHubBlock = 256;
constexpr int kHubK = kHubChunk / kHubBlock;  // row entries per lane
constexpr int kTabLog2 = 12;                  // 4096 LDS slots (2 per chunk entry)
constexpr int kTabSlots = 1 << kTabLog2;
constexpr int kMaxParts = kHubMaxParts;
constexpr int kPartSize = 2048;               // expected distinct labels per partition
constexpr int kMergeBlock = 256;
constexpr int kHubFoldRounds = 1;  // label fold rounds per wave before the inserts (as in the tiers)
// Claims before a merge pass gives up and the partition is split into
// sub-passes: at most kHubMergeCapMax, so that a free slot always remains
// (up to kMergeBlock threads may pass the check at once); a smaller cap can
// be set at run time to exercise the sub-pass path on small graphs.
static_assert(kHubMergeCapMax + kMergeBlock < kTabSlots, "a free slot must always remain");
constexpr int kChunkGroup = 1024;                       // chunks whose slices one merge step indexes

static_assert(kHubChunk % kHubBlock == 0, "chunk must split evenly over the block");
static_assert(2 * kHubChunk <= kTabSlots, "insert table must hold every chunk entry");

__device__ __forceinline__ int hub_parts(int64_t d) {
  int64_t p = (d + kPartSize - 1) / kPartSize;
  return (int)(p < 1 ? 1 : (p > kMaxParts ? kMaxParts : p));
}

// Label mixers independent of the Fibonacci slot hash (murmur3 finalizer).
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
__device__ __forceinline__ int part_of(uint32_t label, int P) {
  return (int)(((uint64_t)mix32(label) * (uint64_t)P) >> 32);
}
__device__ __forceinline__ uint32_t sub_of(uint32_t label) { return mix32(label ^ 0x9e3779b9u); }

// Per hub: insert chunks, partitions, histogram entries (chunks * (P + 1)).
__global__ void hub_sizes(const int64_t *__restrict__ off, const int32_t *__restrict__ hubs, int64_t H,
                          int64_t *__restrict__ chunks, int64_t *__restrict__ parts,
                          int64_t *__restrict__ hist) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= H) return;
  const int32_t v = hubs[k];
  const int64_t d = off[v + 1] - off[v];
  const int64_t nc = (d + kHubChunk - 1) / kHubChunk;
  const int P = hub_parts(d);
  chunks[k] = nc;
  parts[k] = P;
  hist[k] = nc * (P + 1);
}

// Exclusive prefix sums of three arrays of H entries (in place, entry H gets
// the total).  One block.
__global__ __launch_bounds__(1024) void hub_scan_prefix(int64_t *a0, int64_t *a1, int64_t *a2, int64_t H) {
  __shared__ int64_t part[1024];
  int64_t *arrs[3] = {a0, a1, a2};
  const int64_t per = (H + 1023) / 1024;
  const int64_t lo = threadIdx.x * per, hi = lo + per < H ? lo + per : H;
  for (int q = 0; q < 3; ++q) {
    int64_t *a = arrs[q];
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t y = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += y;
      __syncthreads();
    }
    int64_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
      const int64_t c = a[i];
      a[i] = run;
      run += c;
    }
    if (threadIdx.x == 1023) a[H] = part[1023];
    __syncthreads();
  }
}

struct HubArgs {
  const int32_t *hubs;           // hub vertex ids (NULL: hub k is vertex k)
  HubLayout L;                   // [H+1] prefix arrays
  unsigned long long *staging;   // chunk c of the batch at (c - chunk_start[k0]) * kHubChunk
  int32_t *hist;                 // partition bounds, relative to hist_start[k0]
  unsigned long long *best;      // [H] packed argmax keys
  unsigned long long *rowsum;    // [H] summed row weights
  int64_t k0, k1;                // hubs of this batch
  int merge_cap;                 // claims before a merge pass splits (1 .. kHubMergeCapMax)
};

// Exclusive scan of a[0..n) (n <= kMaxParts) in LDS by the whole block;
// a[n] receives the total.  `part` needs blockDim.x entries.  Ends with a
// barrier.
template <int BLOCK>
__device__ void block_exclusive_scan(int *a, int n, int *part) {
  const int per = (n + BLOCK - 1) / BLOCK;
  const int lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
  int s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < BLOCK; o <<= 1) {
    const int y = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
  for (int i = lo; i < hi; ++i) {
    const int c = a[i];
    a[i] = run;
    run += c;
  }
  if (threadIdx.x == BLOCK - 1) a[n] = part[BLOCK - 1];
  __syncthreads();
}

// Dynamic LDS: the partition histogram, (largest P of the batch + 1) ints.
__global__ __launch_bounds__(kHubBlock) void hub_insert(SweepArgs a, HubArgs h) {
  __shared__ unsigned long long tab[kTabSlots];
  extern __shared__ int hist[];
  __shared__ int scan_part[kHubBlock];
  __shared__ unsigned long long red[kHubBlock / kWave];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  const int64_t c = h.L.chunk_start[h.k0] + blockIdx.x;
  const int64_t k = h.L.chunk_owner[c];
  const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
  if (!sweep_takes(a, sv, v)) return;  // uniform over the block
  const int64_t rb = a.off[v], re = a.off[v + 1];
  const int P = hub_parts(re - rb);
  const int64_t cl = c - h.L.chunk_start[k];
  const int64_t b = rb + cl * kHubChunk;
  const int64_t e = b + kHubChunk < re ? b + kHubChunk : re;
  for (int s = threadIdx.x; s < kTabSlots; s += kHubBlock) tab[s] = kEmptySlot;
  for (int i = threadIdx.x; i <= P; i += kHubBlock) hist[i] = 0;
  int32_t j[kHubK];
  uint32_t wt[kHubK], lab[kHubK];
#pragma unroll
  for (int q = 0; q < kHubK; ++q) {
    const int64_t p = b + threadIdx.x + (int64_t)q * kHubBlock;
    const bool in = p < e;
    j[q] = in ? a.cols[p] : -1;
    wt[q] = in ? (a.w ? a.w[p] : 1u) : 0u;
  }
#pragma unroll
  for (int q = 0; q < kHubK; ++q) lab[q] = (j[q] >= 0 && j[q] != v) ? (uint32_t)a.C[j[q]] : kNoLabel;
  unsigned long long rs = 0;
#pragma unroll
  for (int q = 0; q < kHubK; ++q) rs += wt[q];
  wave_fold_labels<kHubK>(lab, wt, kHubFoldRounds);  // the whole chunk belongs to one hub
  __syncthreads();  // table and histogram initialised
  int slot[kHubK];
#pragma unroll
  for (int q = 0; q < kHubK; ++q) slot[q] = lab[q] != kNoLabel ? lds_insert(tab, kTabLog2, lab[q], wt[q]) : -1;
  __syncthreads();
  unsigned long long x[kHubK];
  int pp[kHubK], rank[kHubK];
#pragma unroll
  for (int q = 0; q < kHubK; ++q) {
    x[q] = 0;
    pp[q] = 0;
    rank[q] = 0;
    if (slot[q] >= 0) {
      x[q] = tab[slot[q]];
      pp[q] = part_of((uint32_t)(x[q] >> 32), P);
      rank[q] = atomicAdd(&hist[pp[q]], 1);
    }
  }
  __syncthreads();
  block_exclusive_scan<kHubBlock>(hist, P, scan_part);
  unsigned long long *stage = h.staging + (c - h.L.chunk_start[h.k0]) * kHubChunk;
#pragma unroll
  for (int q = 0; q < kHubK; ++q)
    if (slot[q] >= 0) stage[hist[pp[q]] + rank[q]] = x[q];
  int32_t *gh = h.hist + (h.L.hist_start[k] - h.L.hist_start[h.k0]) + cl * (P + 1);
  for (int i = threadIdx.x; i <= P; i += kHubBlock) gh[i] = hist[i];
  const int chunk_records = hist[P];  // written by the scan, read before block_sum's barriers
  rs = block_sum(rs, red);
  if (threadIdx.x == 0) {
    if (rs) __hip_atomic_fetch_add(&h.rowsum[k], rs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (chunk_records)
      __hip_atomic_fetch_add(&h.L.records[k], (unsigned long long)chunk_records, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kMergeBlock) void hub_merge(SweepArgs a, HubArgs h) {
  __shared__ unsigned long long tab[kTabSlots];
  __shared__ int pre[kChunkGroup + 1];
  __shared__ int scan_part[kMergeBlock];
  __shared__ int claimed, overflow;
  __shared__ unsigned long long red[kMergeBlock / kWave];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  const int64_t gp = h.L.part_start[h.k0] + blockIdx.x;
  const int64_t k = h.L.part_owner[gp];
  // The partition count is sized for rows whose labels are all distinct.
  // Workgroup p merges the group of partitions [p * g, (p + 1) * g): g is as
  // many as the hub's records (hub_insert counted them) fill three quarters
  // of a table on average -- all of them once the labels have merged -- and
  // workgroups past the last group return.  A group that still overflows
  // the table falls back to hashed sub-passes below.
  const unsigned long long records = h.L.records[k];
  const int p = (int)(gp - h.L.part_start[k]);
  const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
  const int P = hub_parts(a.off[v + 1] - a.off[v]);
  const unsigned long long fit = (unsigned long long)h.merge_cap * 3 / 4 * (unsigned long long)P;
  const int g = records <= (unsigned long long)h.merge_cap ? P
                : (int)(fit / records < 1 ? 1 : (fit / records > (unsigned long long)P ? P : fit / records));
  if ((int64_t)p * g >= P) return;  // uniform
  if (!sweep_takes(a, sv, v)) return;
  const int64_t c0 = h.L.chunk_start[k], nc = h.L.chunk_start[k + 1] - c0;
  const int32_t *gh = h.hist + (h.L.hist_start[k] - h.L.hist_start[h.k0]);
  const unsigned long long *stage = h.staging + (c0 - h.L.chunk_start[h.k0]) * kHubChunk;
  const int p_lo = p * g, p_hi = p_lo + g < P ? p_lo + g : P;  // partitions merged here
  unsigned long long best = 0;
  for (uint32_t R = 1;; R <<= 1) {
    bool ok = true;
    unsigned long long pass_best = 0;
    for (uint32_t r = 0; r < R && ok; ++r) {
      for (int s = threadIdx.x; s < kTabSlots; s += kMergeBlock) tab[s] = kEmptySlot;
      if (threadIdx.x == 0) {
        claimed = 0;
        overflow = 0;
      }
      __syncthreads();
      for (int64_t g0 = 0; g0 < nc; g0 += kChunkGroup) {
        const int gn = (int)(nc - g0 < kChunkGroup ? nc - g0 : kChunkGroup);
        for (int i = threadIdx.x; i < gn; i += kMergeBlock) {
          const int32_t *hc = gh + (g0 + i) * (P + 1);
          pre[i] = hc[p_hi] - hc[p_lo];
        }
        __syncthreads();
        block_exclusive_scan<kMergeBlock>(pre, gn, scan_part);
        const int total = pre[gn];
        for (int t = threadIdx.x; t < total; t += kMergeBlock) {
          int lo = 0, hi = gn;  // chunk i with pre[i] <= t < pre[i + 1]
          while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (pre[mid] <= t)
              lo = mid;
            else
              hi = mid;
          }
          const int32_t *hc = gh + (g0 + lo) * (P + 1);
          const unsigned long long xv = stage[(g0 + lo) * kHubChunk + hc[p_lo] + (t - pre[lo])];
          const uint32_t label = (uint32_t)(xv >> 32);
          if (R > 1 && (sub_of(label) & (R - 1)) != r) continue;
          if (__hip_atomic_load(&overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) continue;
          if (__hip_atomic_load(&claimed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= h.merge_cap) {
            overflow = 1;
            continue;
          }
          if (lds_insert(tab, kTabLog2, label, (uint32_t)xv) >= 0) atomicAdd(&claimed, 1);
        }
        __syncthreads();
      }
      if (overflow) {
        ok = false;  // uniform: read after the barrier
      } else {
        for (int s = threadIdx.x; s < kTabSlots; s += kMergeBlock) {
          const unsigned long long xv = tab[s];
          if (xv != kEmptySlot) {
            const unsigned long long key = argmax_key((uint32_t)(xv >> 32), (uint32_t)xv);
            pass_best = key > pass_best ? key : pass_best;
          }
        }
      }
      __syncthreads();
    }
    if (ok) {
      best = pass_best;
      break;
    }
  }
  best = group_max<kWave>(best);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < kMergeBlock / kWave; ++w) m = red[w] > m ? red[w] : m;
    if (m) __hip_atomic_fetch_max(&h.best[k], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(256) void hub_decide(SweepArgs a, HubArgs h) {
  __shared__ unsigned long long red[256 / kWave];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  LocalCounts lc;
  const int64_t k = h.k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < h.k1) {
    const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
    if (sweep_takes(a, sv, v)) {
      const unsigned long long best = h.best[k];
      const unsigned long long rs = h.rowsum[k];
      h.best[k] = 0;
      h.rowsum[k] = 0;
      h.L.records[k] = 0;
      lc.processed = 1;
      lc.edges = (unsigned long long)(a.off[v + 1] - a.off[v]);
      lc.overflow = rs >> 32 ? 1 : 0;
      // A row whose weights sum to 2^32 or more may have carried a sum into
      // the label half of a packed table slot: no change is recorded (the
      // call fails with the overflow).
      if (best && !(rs >> 32)) {
        const uint32_t cstar = key_label(best);
        if (cstar != (uint32_t)a.C[v]) {
          if (a.inplace)
            __hip_atomic_store(const_cast<int32_t *>(a.C) + v, (int32_t)cstar, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          else
            a.Cn[v] = (int32_t)cstar;
          a.chg[v] = 1;
          lc.dn = 1;
          if (sv.mark) lc.marked = lc.edges;  // hub_mark flags the whole row
        }
      }
    }
  }
  const unsigned long long dn = block_sum(lc.dn, red);
  const unsigned long long pr = block_sum(lc.processed, red);
  const unsigned long long ed = block_sum(lc.edges, red);
  const unsigned long long ov = block_sum(lc.overflow, red);
  const unsigned long long mk = block_sum(lc.marked, red);
  if (threadIdx.x == 0) {
    if (mk) atomicAdd(a.tier + 3, mk);
    if (dn) {
      atomicAdd(a.dn + sv.it, dn);
      atomicAdd(a.tier + 2, dn);
    }
    if (pr) {
      atomicAdd(a.processed + sv.it, pr);
      atomicAdd(a.tier + 0, pr);
    }
    if (ed) {
      atomicAdd(a.edges + sv.it, ed);
      atomicAdd(a.tier + 1, ed);
    }
    if (ov) atomicAdd(a.overflow, ov);
  }
}

__global__ __launch_bounds__(kHubBlock) void hub_mark(SweepArgs a, HubArgs h) {
  SweepView sv;
  if (!sweep_view(a, sv) || !sv.mark) return;
  const int64_t c = h.L.chunk_start[h.k0] + blockIdx.x;
  const int64_t k = h.L.chunk_owner[c];
  const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
  if (!a.chg[v]) return;  // uniform: only hubs changed in this sweep
  const int64_t rb = a.off[v], re = a.off[v + 1];
  const int64_t b = rb + (c - h.L.chunk_start[k]) * kHubChunk;
  const int64_t e = b + kHubChunk < re ? b + kHubChunk : re;
  for (int64_t p = b + threadIdx.x; p < e; p += kHubBlock) {
    const int32_t jj = a.cols[p];
    if (!sv.nact[jj]) sv.nact[jj] = 1;
  }
}

// Block per hub (grid-stride): the hub's chunks and partitions name it as
// their owner, and its record count starts at zero.
__global__ __launch_bounds__(256) void hub_owners(HubLayout L, int64_t H) {
  for (int64_t k = blockIdx.x; k < H; k += gridDim.x) {
    const int64_t c0 = L.chunk_start[k], c1 = L.chunk_start[k + 1];
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) L.chunk_owner[c] = (int32_t)k;
    const int64_t p0 = L.part_start[k], p1 = L.part_start[k + 1];
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) L.part_owner[p] = (int32_t)k;
    if (threadIdx.x == 0) L.records[k] = 0;
  }
}

}  // namespace

hipError_t launch_hub_owners(HubLayout L, int64_t H, hipStream_t s) {
  if (H <= 0) return hipSuccess;
  hub_owners<<<(unsigned)(H < 65536 ? H : 65536), 256, 0, s>>>(L, H);
  return hipGetLastError();
}

hipError_t launch_hub_layout(const int64_t *off, const int32_t *hubs, int64_t H, HubLayout L,
                             hipStream_t s) {
  if (H <= 0) return hipSuccess;
  hub_sizes<<<(unsigned)((H + 255) / 256), 256, 0, s>>>(off, hubs, H, L.chunk_start, L.part_start,
                                                        L.hist_start);
  hub_scan_prefix<<<1, 1024, 0, s>>>(L.chunk_start, L.part_start, L.hist_start, H);
  return hipGetLastError();
}

// The hub kernels for hubs [k0, k1): stage 0 is hub_insert, stage 1 the
// merge, decision and marking.  Host copies of the prefix arrays give the grid
// sizes without a device round trip.
hipError_t launch_hub_sweep(const SweepArgs &a, const int32_t *hubs, HubLayout L,
                            const int64_t *chunk_start_h, const int64_t *part_start_h,
                            unsigned long long *staging, int32_t *hist, unsigned long long *best,
                            unsigned long long *rowsum, int64_t k0, int64_t k1, int max_parts,
                            int merge_cap, int stage, hipStream_t s) {
  if (k1 <= k0) return hipSuccess;
  if (merge_cap < 1 || merge_cap > kHubMergeCapMax) return hipErrorInvalidValue;
  HubArgs h{hubs, L, staging, hist, best, rowsum, k0, k1, merge_cap};
  const int64_t chunks = chunk_start_h[k1] - chunk_start_h[k0];
  const int64_t parts = part_start_h[k1] - part_start_h[k0];
  if (stage == 0) {
    hub_insert<<<(unsigned)chunks, kHubBlock, (size_t)(max_parts + 1) * sizeof(int), s>>>(a, h);
    return hipGetLastError();
  }
  hub_merge<<<(unsigned)parts, kMergeBlock, 0, s>>>(a, h);
  hub_decide<<<(unsigned)((k1 - k0 + 255) / 256), 256, 0, s>>>(a, h);
  hub_mark<<<(unsigned)chunks, kHubBlock, 0, s>>>(a, h);  // returns at once unless marking
  return hipGetLastError();
}

}  // namespace gsl
