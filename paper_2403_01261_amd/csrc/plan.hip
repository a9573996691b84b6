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
  const int lane = threadIdx.x % kWave;
  int64_t d = 0;
  int t = -1;
  if (v < n) {
    d = off[v + 1] - off[v];
    t = tier_of(d, tb);
  }
  // Per wave: one LDS add per tier present (ballot), with the wave's sum of
  // the degrees of that tier -- not one contended LDS atomic per vertex.
  for (int k = 0; k < kNumTiers; ++k) {
    const unsigned long long m = __ballot(t == k);
    if (!m) continue;
    unsigned long long e = t == k && d > 0 ? (unsigned long long)d : 0ull;
    e = wave_sum(e);
    if (lane == 0) {
      atomicAdd(&cnt[k], __popcll(m));
      if (e) atomicAdd(&ecnt[k], e);
    }
  }
  unsigned long long mx = (unsigned long long)(d > 0 ? d : 0);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(mx, o, kWave);
    mx = y > mx ? y : mx;
  }
  if (lane == 0) dmax[threadIdx.x / kWave] = mx;
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

// The scan of blk_counts ([block][tier], exclusive over blocks for every
// tier) in three steps: plan_scan_sums totals each group of kPlanBlock
// blocks, plan_scan (one workgroup) scans the group totals and sets the tier
// totals and starts, plan_scan_add scans inside each group from its base.
__global__ __launch_bounds__(kPlanBlock) void plan_scan_sums(const int64_t *__restrict__ blk, int64_t nblk,
                                                             int64_t *__restrict__ grp) {
  __shared__ int64_t ws[kPlanBlock / kWave][kNumTiers];
  const int64_t i = (int64_t)blockIdx.x * kPlanBlock + threadIdx.x;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int t = 0; t < kNumTiers; ++t) {
    unsigned long long x = i < nblk ? (unsigned long long)blk[i * kNumTiers + t] : 0ull;
    x = wave_sum(x);
    if (lane == 0) ws[wid][t] = (int64_t)x;
  }
  __syncthreads();
  if (threadIdx.x < kNumTiers) {
    int64_t sum = 0;
    for (int w = 0; w < kPlanBlock / kWave; ++w) sum += ws[w][threadIdx.x];
    grp[(int64_t)blockIdx.x * kNumTiers + threadIdx.x] = sum;
  }
}

__global__ __launch_bounds__(kPlanBlock) void plan_scan_add(int64_t *__restrict__ blk, int64_t nblk,
                                                            const int64_t *__restrict__ grp) {
  __shared__ int64_t ws[kPlanBlock / kWave][kNumTiers];
  const int64_t i = (int64_t)blockIdx.x * kPlanBlock + threadIdx.x;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  int64_t x[kNumTiers], incl[kNumTiers];
#pragma unroll
  for (int t = 0; t < kNumTiers; ++t) {
    x[t] = i < nblk ? blk[i * kNumTiers + t] : 0;
    incl[t] = x[t];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(incl[t], o, kWave);
      incl[t] += lane >= o ? y : 0;
    }
    if (lane == kWave - 1) ws[wid][t] = incl[t];
  }
  __syncthreads();
  if (i < nblk) {
#pragma unroll
    for (int t = 0; t < kNumTiers; ++t) {
      int64_t base = grp[(int64_t)blockIdx.x * kNumTiers + t];
      for (int w = 0; w < wid; ++w) base += ws[w][t];
      blk[i * kNumTiers + t] = base + incl[t] - x[t];
    }
  }
}

// One block: exclusive scan of the group totals over groups for every tier
// (in place), tier totals and tier starts (tiers laid out in order 9..0).
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

int64_t plan_scratch(int64_t n) {
  const int64_t nblk = plan_blocks(n);
  return (nblk + plan_blocks(nblk)) * kNumTiers;
}

// list receives every vertex grouped by tier (9 first, 0 last); entry
// tier_start[t] is the first vertex of tier t.
hipError_t launch_plan(const int64_t *off, int64_t n, int32_t *list, int64_t *blk_counts,
                       Counters *ctr, const TierConfig &cfg, hipStream_t s) {
  const int64_t nblk = plan_blocks(n);
  if (nblk <= 0) return hipSuccess;
  TierBounds tb;
  for (int t = 0; t < kNumTiers; ++t) tb.b[t] = cfg.bound[t];
  const int64_t ngrp = plan_blocks(nblk);
  int64_t *grp = blk_counts + nblk * kNumTiers;  // group totals (plan_scratch)
  plan_count<<<(unsigned)nblk, kPlanBlock, 0, s>>>(off, n, blk_counts, ctr, tb);
  plan_scan_sums<<<(unsigned)ngrp, kPlanBlock, 0, s>>>(blk_counts, nblk, grp);
  plan_scan<<<1, kPlanBlock, 0, s>>>(grp, ngrp, ctr);
  plan_scan_add<<<(unsigned)ngrp, kPlanBlock, 0, s>>>(blk_counts, nblk, grp);
  plan_scatter<<<(unsigned)nblk, kPlanBlock, 0, s>>>(off, n, blk_counts, ctr, list, tb);
  return hipGetLastError();
}

}  // namespace gsl
