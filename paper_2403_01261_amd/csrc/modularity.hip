// Modularity of a labelling (Eq. 1, second form) with exact integer sums.
//
//   2m      = sum of w over all CSR entries
//   I       = sum of w over entries (i, j) with C_i == C_j      (= sum_c sigma_c)
//   Sigma_c = sum of w over entries (i, j) with C_i == c
//   S2      = sum_c Sigma_c^2                                    (128-bit)
//   Q       = I / 2m - S2 / (2m)^2, each operation IEEE double, round to nearest
//
// Integer sums are order independent, so Q does not depend on the schedule.
#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

constexpr int kModBlock = 256;
constexpr int kShortRow = 32;

// Per vertex: K_i and the intra-community weight.  Rows up to kShortRow are
// scanned by their own thread; longer rows are collected by ballot and scanned
// by the whole wavefront.
__global__ __launch_bounds__(kModBlock) void mod_rows(const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ cols,
                                                      const uint32_t *__restrict__ w, int64_t n,
                                                      const int32_t *__restrict__ C,
                                                      unsigned long long *sigma_tot, Counters *ctr) {
  __shared__ unsigned long long red[kModBlock / kWave];
  const int lane = threadIdx.x % kWave;
  unsigned long long my_two_m = 0, my_intra = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t b = 0, e = 0;
    int32_t c = 0;
    if (v < n) {
      b = off[v];
      e = off[v + 1];
      c = C[v];
    }
    const bool longrow = v < n && e - b > kShortRow;
    if (v < n && !longrow) {
      unsigned long long k = 0, in = 0;
      for (int64_t p = b; p < e; ++p) {
        const unsigned long long we = w ? w[p] : 1u;
        k += we;
        if (C[cols[p]] == c) in += we;
      }
      my_two_m += k;
      my_intra += in;
      if (k) atomicAdd(&sigma_tot[c], k);
    }
    unsigned long long pending = __ballot(longrow);
    while (pending) {
      const int src = __ffsll((long long)pending) - 1;
      pending &= pending - 1;
      const int64_t vb = __shfl(b, src, kWave), ve = __shfl(e, src, kWave);
      const int32_t vc = __shfl(c, src, kWave);
      unsigned long long k = 0, in = 0;
      for (int64_t p = vb + lane; p < ve; p += kWave) {
        const unsigned long long we = w ? w[p] : 1u;
        k += we;
        if (C[cols[p]] == vc) in += we;
      }
      k = wave_sum(k);
      in = wave_sum(in);
      if (lane == 0) {
        my_two_m += k;
        my_intra += in;
        if (k) atomicAdd(&sigma_tot[vc], k);
      }
    }
  }
  const unsigned long long t2 = block_sum(my_two_m, red);
  const unsigned long long ti = block_sum(my_intra, red);
  if (threadIdx.x == 0) {
    if (t2) atomicAdd(reinterpret_cast<unsigned long long *>(&ctr->two_m), t2);
    if (ti) atomicAdd(reinterpret_cast<unsigned long long *>(&ctr->intra), ti);
  }
}

struct U128 {
  unsigned long long lo, hi;
};

__device__ __forceinline__ U128 add128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
  return r;
}

__device__ __forceinline__ U128 shfl_xor128(U128 x, int o) {
  U128 r;
  r.lo = __shfl_xor(x.lo, o, kWave);
  r.hi = __shfl_xor(x.hi, o, kWave);
  return r;
}

// Per-block partial of sum_c Sigma_c^2 (128-bit) -> partials[2 * block].
__global__ __launch_bounds__(kModBlock) void mod_squares(const unsigned long long *__restrict__ sig,
                                                         int64_t n,
                                                         unsigned long long *__restrict__ partials) {
  __shared__ U128 red[kModBlock / kWave];
  U128 acc = {0, 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    const unsigned long long s = sig[c];
    U128 sq = {s * s, __umul64hi(s, s)};
    acc = add128(acc, sq);
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc = add128(acc, shfl_xor128(acc, o));
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    U128 t = {0, 0};
    for (int k = 0; k < kModBlock / kWave; ++k) t = add128(t, red[k]);
    partials[2 * blockIdx.x] = t.lo;
    partials[2 * blockIdx.x + 1] = t.hi;
  }
}

// Correctly rounded (to nearest even) conversion of a 128-bit unsigned integer.
__device__ __forceinline__ double u128_to_double(unsigned long long hi, unsigned long long lo) {
  if (hi == 0) return (double)lo;
  const int s = __clzll((long long)hi);
  unsigned long long top = s ? (hi << s) | (lo >> (64 - s)) : hi;
  const unsigned long long rest = s ? lo << s : lo;
  top |= rest ? 1ull : 0ull;  // sticky bit: below the rounding position
  return ldexp((double)top, 64 - s);
}

__global__ void mod_finish(const unsigned long long *__restrict__ partials, int nparts,
                           Counters *ctr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  U128 t = {0, 0};
  for (int k = 0; k < nparts; ++k) t = add128(t, U128{partials[2 * k], partials[2 * k + 1]});
  ctr->s2_lo = t.lo;
  ctr->s2_hi = t.hi;
  const unsigned long long two_m = ctr->two_m, I = ctr->intra;
  if (two_m == 0) {
    ctr->q = 0.0;
    return;
  }
  const double M = (double)two_m;
  const double a = __ddiv_rn((double)I, M);
  const double b = __ddiv_rn(u128_to_double(t.hi, t.lo), __dmul_rn(M, M));
  ctr->q = __dsub_rn(a, b);
}

}  // namespace

hipError_t launch_modularity(const int64_t *off, const int32_t *cols, const uint32_t *w, int64_t n,
                             const int32_t *labels, unsigned long long *sigma_tot,
                             unsigned long long *partials, int partial_blocks, Counters *ctr,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + kModBlock - 1) / kModBlock;
  if (g > 256 * 16) g = 256 * 16;
  mod_rows<<<(unsigned)g, kModBlock, 0, s>>>(off, cols, w, n, labels, sigma_tot, ctr);
  int64_t g2 = (n + kModBlock - 1) / kModBlock;
  if (g2 > partial_blocks) g2 = partial_blocks;
  mod_squares<<<(unsigned)g2, kModBlock, 0, s>>>(sigma_tot, n, partials);
  mod_finish<<<1, 64, 0, s>>>(partials, (int)g2, ctr);
  return hipGetLastError();
}

}  // namespace gsl
