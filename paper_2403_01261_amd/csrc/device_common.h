// Device helpers shared by the kernels: label hash tables, packed argmax keys,
// wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gsl {

constexpr int kWave = 64;

// A hash-table slot packs (label << 32) | summed_weight.  Labels are < 2^31,
// so the all-ones label marks an empty slot.
constexpr unsigned long long kEmptySlot = 0xFFFFFFFF00000000ull;
constexpr uint32_t kNoLabel = 0xFFFFFFFFu;

// Argmax key of a (label, weight) pair: larger weight first, then smaller
// label.  0 means "no candidate" (a real key has ~label >= 2^31).
__device__ __forceinline__ unsigned long long argmax_key(uint32_t label, uint32_t weight) {
  return ((unsigned long long)weight << 32) | (unsigned long long)(~label);
}
__device__ __forceinline__ uint32_t key_label(unsigned long long key) { return ~(uint32_t)key; }

// Fibonacci hashing of a label onto 2^log2s slots (log2s >= 1).
__device__ __forceinline__ uint32_t slot_hash(uint32_t label, int log2s) {
  return (label * 2654435761u) >> (32 - log2s);
}

__device__ __forceinline__ int ceil_log2(uint64_t x) {  // x >= 1
  return x <= 1 ? 0 : 64 - __clzll((long long)(x - 1));
}

// Table size (log2) for a row of d entries: at least 2d slots, clamped.
__device__ __forceinline__ int table_log2(int64_t d, int lo, int hi) {
  int l = ceil_log2((uint64_t)(d > 0 ? 2 * d : 2));
  return l < lo ? lo : (l > hi ? hi : l);
}

// Adds weight w to label `label` in an LDS open-addressing table of 2^log2s
// slots (linear probing).  The table must have a free slot for every distinct
// label inserted.  A slot's label never changes once claimed, so a stale read
// can only cost a failed compare-and-swap.
__device__ __forceinline__ void lds_table_add(unsigned long long *tab, int log2s, uint32_t label,
                                              uint32_t w) {
  const uint32_t mask = (1u << log2s) - 1u;
  uint32_t h = slot_hash(label, log2s);
  const unsigned long long mine = ((unsigned long long)label << 32) | w;
  for (;;) {
    const unsigned long long cur = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
    if ((uint32_t)(cur >> 32) == label) {
      atomicAdd(&tab[h], (unsigned long long)w);
      return;
    }
    if (cur == kEmptySlot) {
      const unsigned long long prev = atomicCAS(&tab[h], kEmptySlot, mine);
      if (prev == kEmptySlot) return;
      if ((uint32_t)(prev >> 32) == label) {
        atomicAdd(&tab[h], (unsigned long long)w);
        return;
      }
    }
    h = (h + 1u) & mask;
  }
}

// Adds (label, w) to an LDS table with a compare-and-swap first: returns the
// slot index if this call claimed a new slot for `label`, -1 if the label was
// already present (its weight was added).  The table must keep a free slot
// for every distinct label inserted.
__device__ __forceinline__ int lds_insert(unsigned long long *tab, int log2s, uint32_t label,
                                          uint32_t w) {
  const uint32_t mask = (1u << log2s) - 1u;
  uint32_t h = slot_hash(label, log2s);
  const unsigned long long mine = ((unsigned long long)label << 32) | w;
  for (;;) {
    const unsigned long long prev = atomicCAS(&tab[h], kEmptySlot, mine);
    if (prev == kEmptySlot) return (int)h;
    if ((uint32_t)(prev >> 32) == label) {
      atomicAdd(&tab[h], (unsigned long long)w);
      return -1;
    }
    h = (h + 1u) & mask;
  }
}

// Same on a global-memory table private to one workgroup: workgroup-scope
// atomics (performed in the L2 of the workgroup's XCD).
__device__ __forceinline__ void global_table_add(unsigned long long *tab, int log2s, uint32_t label,
                                                 uint32_t w) {
  const uint32_t mask = (1u << log2s) - 1u;
  uint32_t h = slot_hash(label, log2s);
  const unsigned long long mine = ((unsigned long long)label << 32) | w;
  for (;;) {
    unsigned long long cur = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(cur >> 32) == label) {
      __hip_atomic_fetch_add(&tab[h], (unsigned long long)w, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    if (cur == kEmptySlot) {
      unsigned long long expected = kEmptySlot;
      if (__hip_atomic_compare_exchange_strong(&tab[h], &expected, mine, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
        return;
      if ((uint32_t)(expected >> 32) == label) {
        __hip_atomic_fetch_add(&tab[h], (unsigned long long)w, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
      }
    }
    h = (h + 1u) & mask;
  }
}

// Folds repeated labels of one wavefront before they reach the LDS table
// (every lane of the wave must work on the same table).  Up to `rounds`
// times: take the label of the first entry not yet folded, sum the weights of
// every entry of the wave with that label into that entry and drop the
// others.  On power-law graphs most entries of a long row carry a few labels
// after the first sweeps; without this every one of them is an atomic on the
// same LDS address.  Stops at the first label that occurs only once.
// Weights of dropped entries stay in the caller's row sum.
template <int K>
__device__ __forceinline__ void wave_fold_labels(uint32_t (&lab)[K], uint32_t (&wt)[K], int rounds) {
  const int wl = threadIdx.x % kWave;
  bool led[K];
#pragma unroll
  for (int k = 0; k < K; ++k) led[k] = false;
  for (int r = 0; r < rounds; ++r) {
    int kk = -1, leader = -1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const unsigned long long b = __ballot(lab[k] != kNoLabel && !led[k]);
      if (kk < 0 && b) {
        kk = k;
        leader = __ffsll((long long)b) - 1;
      }
    }
    if (kk < 0) return;  // uniform: nothing left in the wave
    uint32_t mine = kNoLabel;
#pragma unroll
    for (int k = 0; k < K; ++k) mine = k == kk ? lab[k] : mine;
    const uint32_t L = (uint32_t)__shfl((int)mine, leader);
    int count = 0;
    unsigned long long local = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool m = lab[k] == L;
      count += __popcll(__ballot(m));
      local += m ? wt[k] : 0u;
    }
    if (count < 2) return;  // uniform: the most common labels are gone
    unsigned long long sum = local;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, kWave);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (lab[k] != L) continue;
      if (wl == leader && k == kk) {
        wt[k] = (uint32_t)sum;  // >= 2^32 only when the row sum overflows, which is reported
        led[k] = true;
      } else {
        lab[k] = kNoLabel;
        wt[k] = 0;
      }
    }
  }
}

// Max over the G lanes of a group (G a power of two <= 64, groups aligned).
template <int G>
__device__ __forceinline__ unsigned long long group_max(unsigned long long x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, G);
    x = y > x ? y : x;
  }
  return x;
}

// Sum over the G lanes of a group.
template <int G>
__device__ __forceinline__ unsigned long long group_sum(unsigned long long x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
  return x;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Block-wide sum; the result is valid in thread 0.  `red` needs
// blockDim.x / 64 entries.  Contains __syncthreads.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long x,
                                                        unsigned long long *red) {
  x = wave_sum(x);
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) red[wid] = x;
  __syncthreads();
  unsigned long long t = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) t += red[k];
  return t;
}

// Batcher's odd-even merge sort of D register values (D a power of two):
// a sorting network, so the compare-exchange sequence is the same for every
// input and every index is a compile-time constant once unrolled (19, 63 and
// 191 compare-exchanges for D = 8, 16, 32).  Labels end up ascending; with
// W, each weight moves with its label.
template <int D, bool W>
__device__ __forceinline__ void sort_by_label(uint32_t (&l)[D], uint32_t (&w)[D]) {
#pragma unroll
  for (int p = 1; p < D; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < D; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i) {
          const int x = i + j, y = i + j + k;
          if (y < D && x / (2 * p) == y / (2 * p)) {
            if constexpr (W) {
              const bool s = l[x] > l[y];
              const uint32_t lx = l[x], wx = w[x];
              l[x] = s ? l[y] : lx;
              l[y] = s ? lx : l[y];
              w[x] = s ? w[y] : wx;
              w[y] = s ? wx : w[y];
            } else {
              const uint32_t lo = l[x] < l[y] ? l[x] : l[y], hi = l[x] < l[y] ? l[y] : l[x];
              l[x] = lo;
              l[y] = hi;
            }
          }
        }
}

// Per-thread sweep counters, reduced once per block at kernel end.
struct LocalCounts {
  unsigned long long dn = 0, processed = 0, edges = 0, overflow = 0, marked = 0;
};

}  // namespace gsl
