// Degree bucketing: a stable partition of the vertex ids by degree tier.
//
// The paper spreads vertices over CPU threads with per-thread hashtables
// (Alg. 3, Sec. 5.1.2); on the GPU the work unit must match the row length
// instead.  plan_count counts the vertices and row entries of each tier in
// each block of 1024 vertices, plan_scan turns the counts into per-block bases
// and tier starts, and plan_scatter writes every vertex id into its tier's
// segment of `list`, ascending within each tier.  Tiers are laid out from the
// longest rows down (hubs first, isolated vertices last), so `list` doubles as
// a degree-ordered renumbering of the graph.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

constexpr int kPlanBlock = 1024;

__device__ __forceinline__ int tier_of(int64_t d, const TierBounds &tb) {
  if (d <= 0) return 0;
#pragma unroll
  for (int t = 1; t < kNumTiers - 1; ++t)
    if (d <= tb.b[t]) return t;
  return kNumTiers - 1;
}

__global__ __launch_bounds__(kPlanBlock) void plan_count(const int64_t *__restrict__ off, int64_t n,
                                                         int64_t *__restrict__ blk_counts,
                                                         Counters *ctr, TierBounds tb) {
  __shared__ int cnt[kNumTiers];
  __shared__ unsigned long long ecnt[kNumTiers];
  __shared__ unsigned long long dmax[kPlanBlock / kWave];
  if (threadIdx.x < kNumTiers) {
    cnt[threadIdx.x] = 0;
    ecnt[threadIdx.x] = 0;
  }
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * kPlanBlock + threadIdx.x;
  int64_t d = 0;
  if (v < n) {
    d = off[v + 1] - off[v];
    const int t = tier_of(d, tb);
    atomicAdd(&cnt[t], 1);
    if (d > 0) atomicAdd(&ecnt[t], (unsigned long long)d);
  }
  unsigned long long m = (unsigned long long)(d > 0 ? d : 0);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(m, o, kWave);
    m = y > m ? y : m;
  }
  if (threadIdx.x % kWave == 0) dmax[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x < kNumTiers) {
    blk_counts[(int64_t)blockIdx.x * kNumTiers + threadIdx.x] = cnt[threadIdx.x];
    if (ecnt[threadIdx.x])
      atomicAdd(reinterpret_cast<unsigned long long *>(&ctr->tier_edges[threadIdx.x]), ecnt[threadIdx.x]);
  }
  if (threadIdx.x == 0) {
    unsigned long long mm = 0;
    for (int k = 0; k < kPlanBlock / kWave; ++k) mm = dmax[k] > mm ? dmax[k] : mm;
    atomicMax(&ctr->max_degree, (uint64_t)mm);
  }
}

// One block: exclusive scan of blk_counts over blocks for every tier (in
// place), tier totals and tier starts (tiers laid out in order 9..0).
__global__ __launch_bounds__(kPlanBlock) void plan_scan(int64_t *__restrict__ blk_counts,
                                                        int64_t nblk, Counters *ctr) {
  __shared__ int64_t part[kPlanBlock];
  __shared__ int64_t totals[kNumTiers];
  const int64_t per = (nblk + kPlanBlock - 1) / kPlanBlock;
  const int64_t lo = threadIdx.x * per, hi = lo + per < nblk ? lo + per : nblk;
  for (int t = 0; t < kNumTiers; ++t) {
    int64_t s = 0;
    for (int64_t b = lo; b < hi; ++b) s += blk_counts[b * kNumTiers + t];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the per-thread sums.
    for (int o = 1; o < kPlanBlock; o <<= 1) {
      const int64_t y = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += y;
      __syncthreads();
    }
    int64_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int64_t b = lo; b < hi; ++b) {
      const int64_t c = blk_counts[b * kNumTiers + t];
      blk_counts[b * kNumTiers + t] = run;
      run += c;
    }
    if (threadIdx.x == kPlanBlock - 1) totals[t] = part[kPlanBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int64_t start = 0;
    for (int t = kNumTiers - 1; t >= 0; --t) {
      ctr->tier_count[t] = totals[t];
      ctr->tier_start[t] = start;
      start += totals[t];
    }
  }
}

__global__ __launch_bounds__(kPlanBlock) void plan_scatter(const int64_t *__restrict__ off, int64_t n,
                                                           const int64_t *__restrict__ blk_base,
                                                           const Counters *ctr,
                                                           int32_t *__restrict__ list, TierBounds tb) {
  constexpr int W = kPlanBlock / kWave;
  __shared__ int wcnt[W][kNumTiers];
  const int64_t v = (int64_t)blockIdx.x * kPlanBlock + threadIdx.x;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  int t = -1;
  if (v < n) t = tier_of(off[v + 1] - off[v], tb);
  const unsigned long long below = (1ull << lane) - 1ull;
  int rank = 0;
#pragma unroll
  for (int k = 0; k < kNumTiers; ++k) {
    const unsigned long long m = __ballot(t == k);
    if (t == k) rank = __popcll(m & below);
    if (lane == 0) wcnt[wid][k] = __popcll(m);
  }
  __syncthreads();
  if (t >= 0) {
    int before = 0;
    for (int w = 0; w < wid; ++w) before += wcnt[w][t];
    const int64_t pos = ctr->tier_start[t] + blk_base[(int64_t)blockIdx.x * kNumTiers + t] + before + rank;
    list[pos] = (int32_t)v;
  }
}

}  // namespace

int64_t plan_blocks(int64_t n) { return (n + kPlanBlock - 1) / kPlanBlock; }

// list receives every vertex grouped by tier (9 first, 0 last); entry
// tier_start[t] is the first vertex of tier t.
hipError_t launch_plan(const int64_t *off, int64_t n, int32_t *list, int64_t *blk_counts,
                       Counters *ctr, const TierConfig &cfg, hipStream_t s) {
  const int64_t nblk = plan_blocks(n);
  if (nblk <= 0) return hipSuccess;
  TierBounds tb;
  for (int t = 0; t < kNumTiers; ++t) tb.b[t] = cfg.bound[t];
  plan_count<<<(unsigned)nblk, kPlanBlock, 0, s>>>(off, n, blk_counts, ctr, tb);
  plan_scan<<<1, kPlanBlock, 0, s>>>(blk_counts, nblk, ctr);
  plan_scatter<<<(unsigned)nblk, kPlanBlock, 0, s>>>(off, n, blk_counts, ctr, list, tb);
  return hipGetLastError();
}

}  // namespace gsl
