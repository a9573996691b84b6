// Hub tier of the sweep: vertices whose row is longer than one workgroup's LDS
// table can take (degree > 8192).
//
// A hub row is cut into chunks of kHubChunk entries and every chunk gets its
// own workgroup, so one hub keeps many compute units busy:
//   hub_insert : sums the chunk's labels in an LDS table, then adds each
//                distinct (label, sum) into the hub's table in global memory
//                (agent-scope atomics; the LDS pass removes repeated labels
//                before they reach global memory);
//   hub_scan   : reads every hub table in chunks of kScanChunk slots, clears
//                them and folds the packed argmax keys into hub_best[k];
//   hub_decide : one thread per hub compares the winning label with C[v] and
//                records the change;
//   hub_mark   : marks the neighbours of changed hubs, chunk by chunk.
// The per-hub layout (chunk, table and scan-chunk prefix sums) is built once
// per call by hub_sizes + hub_scan_prefix.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

constexpr int kHubBlock = 1024;
constexpr int kHubK = 8;
constexpr int kHubChunk = kHubBlock * kHubK;  // row entries per insert workgroup
constexpr int kHubLog2S = 14;                 // LDS slots: 2 per chunk entry
constexpr int kScanBlock = 256;
constexpr int kScanChunk = kScanBlock * 16;   // table slots per scan workgroup

// Largest k with start[k] <= x, for k in [lo, hi).
__device__ __forceinline__ int64_t owner(const int64_t *start, int64_t lo, int64_t hi, int64_t x) {
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (start[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Adds (label, w) to a global table, probing linearly from slot h.
__device__ __forceinline__ void global_add_from(unsigned long long *tab, uint32_t mask, uint32_t h,
                                                uint32_t label, uint32_t w) {
  const unsigned long long mine = ((unsigned long long)label << 32) | w;
  for (;;) {
    unsigned long long expected = kEmptySlot;
    if (__hip_atomic_compare_exchange_strong(&tab[h], &expected, mine, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
    if ((uint32_t)(expected >> 32) == label) {
      __hip_atomic_fetch_add(&tab[h], (unsigned long long)w, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    h = (h + 1u) & mask;
  }
}

__device__ __forceinline__ int hub_log2(int64_t d) { return ceil_log2((uint64_t)(2 * (d > 0 ? d : 1))); }

// Per hub: insert chunks, table slots, scan chunks.
__global__ void hub_sizes(const int64_t *__restrict__ off, const int32_t *__restrict__ hubs, int64_t H,
                          int64_t *__restrict__ chunks, int64_t *__restrict__ slots,
                          int64_t *__restrict__ tchunks) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= H) return;
  const int32_t v = hubs[k];
  const int64_t d = off[v + 1] - off[v];
  const int64_t s = (int64_t)1 << hub_log2(d);
  chunks[k] = (d + kHubChunk - 1) / kHubChunk;
  slots[k] = s;
  tchunks[k] = (s + kScanChunk - 1) / kScanChunk;
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
  const int32_t *hubs;        // hub vertex ids (NULL: hub k is vertex k)
  const int64_t *chunk_start; // [H+1]
  const int64_t *tab_start;   // [H+1]
  const int64_t *tchunk_start;// [H+1]
  unsigned long long *tab;    // table pool; hub k of the batch at tab_start[k] - tab_start[k0]
  unsigned long long *best;   // [H] packed argmax keys
  unsigned long long *rowsum; // [H] summed row weights
  int64_t k0, k1;             // hubs of this batch
};

__global__ __launch_bounds__(kHubBlock) void hub_insert(SweepArgs a, HubArgs h) {
  __shared__ unsigned long long tab[1 << kHubLog2S];
  __shared__ unsigned long long red[kHubBlock / kWave];
  const int64_t c = h.chunk_start[h.k0] + blockIdx.x;
  const int64_t k = owner(h.chunk_start, h.k0, h.k1, c);
  const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
  if (!a.dense && !a.act[v]) return;  // uniform over the block
  for (int s = threadIdx.x; s < (1 << kHubLog2S); s += kHubBlock) tab[s] = kEmptySlot;
  const int64_t rb = a.off[v], re = a.off[v + 1];
  const int64_t b = rb + (c - h.chunk_start[k]) * kHubChunk;
  const int64_t e = b + kHubChunk < re ? b + kHubChunk : re;
  int32_t j[kHubK];
  uint32_t wt[kHubK], lab[kHubK];
  int slot[kHubK];
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
  __syncthreads();  // table initialised
#pragma unroll
  for (int q = 0; q < kHubK; ++q) slot[q] = lab[q] != kNoLabel ? lds_insert(tab, kHubLog2S, lab[q], wt[q]) : -1;
  __syncthreads();
  const int log2s = hub_log2(re - rb);
  const uint32_t gmask = (1u << log2s) - 1u;
  unsigned long long *gt = h.tab + (h.tab_start[k] - h.tab_start[h.k0]);
  // All first-probe compare-and-swaps of a thread are issued together; only
  // the (rare) collisions walk on one by one.
  unsigned long long x[kHubK], prev[kHubK];
  uint32_t gh[kHubK];
#pragma unroll
  for (int q = 0; q < kHubK; ++q) {
    x[q] = slot[q] >= 0 ? tab[slot[q]] : kEmptySlot;
    gh[q] = slot_hash((uint32_t)(x[q] >> 32), log2s);
  }
#pragma unroll
  for (int q = 0; q < kHubK; ++q) {
    prev[q] = kEmptySlot;
    if (slot[q] >= 0)
      __hip_atomic_compare_exchange_strong(&gt[gh[q]], &prev[q], x[q], __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int q = 0; q < kHubK; ++q) {
    if (slot[q] < 0 || prev[q] == kEmptySlot) continue;  // claimed on the first probe
    const uint32_t label = (uint32_t)(x[q] >> 32), w = (uint32_t)x[q];
    if ((uint32_t)(prev[q] >> 32) == label) {
      __hip_atomic_fetch_add(&gt[gh[q]], (unsigned long long)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    global_add_from(gt, gmask, (gh[q] + 1u) & gmask, label, w);
  }
  rs = block_sum(rs, red);
  if (threadIdx.x == 0 && rs)
    __hip_atomic_fetch_add(&h.rowsum[k], rs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kScanBlock) void hub_scan(SweepArgs a, HubArgs h) {
  __shared__ unsigned long long red[kScanBlock / kWave];
  const int64_t tc = h.tchunk_start[h.k0] + blockIdx.x;
  const int64_t k = owner(h.tchunk_start, h.k0, h.k1, tc);
  const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
  if (!a.dense && !a.act[v]) return;
  const int64_t base = h.tab_start[k] - h.tab_start[h.k0];
  const int64_t s0 = (tc - h.tchunk_start[k]) * kScanChunk;
  const int64_t size = h.tab_start[k + 1] - h.tab_start[k];
  const int64_t s1 = s0 + kScanChunk < size ? s0 + kScanChunk : size;
  unsigned long long best = 0;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += kScanBlock) {
    unsigned long long *slot = h.tab + base + s;
    const unsigned long long x = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (x != kEmptySlot) {
      const unsigned long long key = argmax_key((uint32_t)(x >> 32), (uint32_t)x);
      best = key > best ? key : best;
      __hip_atomic_store(slot, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  best = group_max<kWave>(best);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) m = red[w] > m ? red[w] : m;
    if (m) __hip_atomic_fetch_max(&h.best[k], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(256) void hub_decide(SweepArgs a, HubArgs h) {
  __shared__ unsigned long long red[256 / kWave];
  LocalCounts lc;
  const int64_t k = h.k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < h.k1) {
    const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
    if (a.dense || a.act[v]) {
      const unsigned long long best = h.best[k];
      const unsigned long long rs = h.rowsum[k];
      h.best[k] = 0;
      h.rowsum[k] = 0;
      lc.processed = 1;
      lc.edges = (unsigned long long)(a.off[v + 1] - a.off[v]);
      lc.overflow = rs >> 32 ? 1 : 0;
      if (best) {
        const uint32_t cstar = key_label(best);
        if (cstar != (uint32_t)a.C[v]) {
          a.Cn[v] = (int32_t)cstar;
          a.chg[v] = 1;
          lc.dn = 1;
          if (a.mark) lc.marked = lc.edges;  // hub_mark flags the whole row
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
      atomicAdd(a.dn, dn);
      atomicAdd(a.tier + 2, dn);
    }
    if (pr) {
      atomicAdd(a.processed, pr);
      atomicAdd(a.tier + 0, pr);
    }
    if (ed) {
      atomicAdd(a.edges, ed);
      atomicAdd(a.tier + 1, ed);
    }
    if (ov) atomicAdd(a.overflow, ov);
  }
}

__global__ __launch_bounds__(kHubBlock) void hub_mark(SweepArgs a, HubArgs h) {
  const int64_t c = h.chunk_start[h.k0] + blockIdx.x;
  const int64_t k = owner(h.chunk_start, h.k0, h.k1, c);
  const int32_t v = h.hubs ? h.hubs[k] : (int32_t)k;
  if (!a.chg[v]) return;  // uniform: only hubs changed in this sweep
  const int64_t rb = a.off[v], re = a.off[v + 1];
  const int64_t b = rb + (c - h.chunk_start[k]) * kHubChunk;
  const int64_t e = b + kHubChunk < re ? b + kHubChunk : re;
  for (int64_t p = b + threadIdx.x; p < e; p += kHubBlock) {
    const int32_t jj = a.cols[p];
    if (!a.nact[jj]) a.nact[jj] = 1;
  }
}

}  // namespace

hipError_t launch_hub_layout(const int64_t *off, const int32_t *hubs, int64_t H, int64_t *chunk_start,
                             int64_t *tab_start, int64_t *tchunk_start, hipStream_t s) {
  if (H <= 0) return hipSuccess;
  hub_sizes<<<(unsigned)((H + 255) / 256), 256, 0, s>>>(off, hubs, H, chunk_start, tab_start, tchunk_start);
  hub_scan_prefix<<<1, 1024, 0, s>>>(chunk_start, tab_start, tchunk_start, H);
  return hipGetLastError();
}

// The hub kernels for hubs [k0, k1): stage 0 is hub_insert, stage 1 the
// scan, decision and marking.  Host arrays give the prefix sums so grid sizes
// are known without a device round trip.
hipError_t launch_hub_sweep(const SweepArgs &a, const int32_t *hubs, const int64_t *chunk_start,
                            const int64_t *tab_start, const int64_t *tchunk_start,
                            const int64_t *chunk_start_h, const int64_t *tchunk_start_h,
                            unsigned long long *tab, unsigned long long *best,
                            unsigned long long *rowsum, int64_t k0, int64_t k1, int stage,
                            hipStream_t s) {
  if (k1 <= k0) return hipSuccess;
  HubArgs h{hubs, chunk_start, tab_start, tchunk_start, tab, best, rowsum, k0, k1};
  const int64_t chunks = chunk_start_h[k1] - chunk_start_h[k0];
  const int64_t tchunks = tchunk_start_h[k1] - tchunk_start_h[k0];
  if (stage == 0) {
    hub_insert<<<(unsigned)chunks, kHubBlock, 0, s>>>(a, h);
    return hipGetLastError();
  }
  hub_scan<<<(unsigned)tchunks, kScanBlock, 0, s>>>(a, h);
  hub_decide<<<(unsigned)((k1 - k0 + 255) / 256), 256, 0, s>>>(a, h);
  if (a.mark) hub_mark<<<(unsigned)chunks, kHubBlock, 0, s>>>(a, h);
  return hipGetLastError();
}

}  // namespace gsl
