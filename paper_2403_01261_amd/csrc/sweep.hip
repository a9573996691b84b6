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
// row's total weight reaches 2^32 and raises `overflow` otherwise (such a
// row records no change, so no label outside [0, n) ever reaches C).
#include <utility>

#include "device_common.h"
#include "gsl_internal.h"

namespace gsl {

namespace {

// Repeated labels folded per wave before the LDS inserts (wave_fold_labels):
// a single pass, for the wave's most common label.  Measured on rmat-s26 /
// rmat-s22 (ms per call): no fold 207 / 9.33, a single pass 196 / 8.71, two
// passes 196 / 8.82, four 198 / 8.89, eight 197.5 on rmat-s26.
constexpr int kFoldRounds = 1;

__device__ __forceinline__ void record_change(const SweepArgs &a, int32_t v, uint32_t cstar,
                                              LocalCounts &lc) {
  if (a.inplace)
    __hip_atomic_store(const_cast<int32_t *>(a.C) + v, (int32_t)cstar, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  else
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
// Thread-per-vertex variants: one thread per vertex, degree <= D (the first
// level by default, any level that fits).  The row's labels (and weights)
// stay in registers.  A sorting network puts equal labels next to each
// other, and one pass over the sorted runs keeps the running sum of each run
// and the largest argmax key seen.  A run's partial sums never exceed its
// total, so the largest key is that of the label with the largest total (the
// smallest such label on ties, which the key orders first).  Entries j == i
// and the padding beyond the row carry the no-label value, which sorts last
// and never becomes a candidate.  W: weighted rows; without it every entry
// weighs 1.
//
// The sweep waits on its vector memory instructions (row loads and label
// gathers, one lane access each): with V4 a row comes in as 16-byte words
// (load_row), each label is loaded into the register that held its column,
// and with O32 (fewer than 2^30 vertices) the gather address is the label
// array's base plus a 32-bit byte offset, which needs no 64-bit address
// registers.  A sparse sweep after few changes walks the frontier instead of
// the tier list.
// ---------------------------------------------------------------------------
__device__ const int32_t kZeroI32 = 0;
__device__ const uint8_t kZeroU8 = 0;

template <bool O32>
__device__ __forceinline__ uint32_t gather_label(const int32_t *__restrict__ C, int32_t c) {
  if constexpr (O32)
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(C) + ((uint32_t)c << 2));
  else
    return (uint32_t)C[c];
}

// Row entries [b, b + d) of a 4-byte array into r[0..D), `fill` beyond d.
// V4: 16-byte loads of the aligned words that cover the row -- at most
// D / 4 + 1 loads instead of D, vector memory instructions being what the
// thread-per-vertex sweep waits on -- then shifted into place in registers.
// Only words that hold an entry of the row are loaded, and an aligned 16-byte
// word lies within one page (the page of that entry), so no load reaches
// unmapped memory.  V4 needs a 16-byte aligned array.  Register indices are
// template constants (index sequences rather than loops), so the words stay
// in registers.
template <int... Q>
__device__ __forceinline__ void load_words(const uint4 *__restrict__ p, int lim, uint32_t fill, uint32_t *t,
                                           std::integer_sequence<int, Q...>) {
  ((t[4 * Q] = fill, t[4 * Q + 1] = fill, t[4 * Q + 2] = fill, t[4 * Q + 3] = fill), ...);
  ([&] {
    if (4 * Q < lim) {
      const uint4 v = p[Q];
      t[4 * Q] = v.x;
      t[4 * Q + 1] = v.y;
      t[4 * Q + 2] = v.z;
      t[4 * Q + 3] = v.w;
    }
  }(), ...);
}

// Word K + sh of t (sh in 0..3).  The empty asm hands the selects plain
// register values: a select between two array elements would otherwise
// become a load through a selected address, which keeps the array in
// scratch memory.
template <int K>
__device__ __forceinline__ uint32_t shifted_word(const uint32_t *t, int sh, int d, uint32_t fill) {
  uint32_t c0 = t[K], c1 = t[K + 1], c2 = t[K + 2], c3 = t[K + 3];
  asm("" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3));
  const uint32_t lo = (sh & 1) ? c1 : c0, hi = (sh & 1) ? c3 : c2;
  return K < d ? ((sh & 2) ? hi : lo) : fill;
}

template <int... K>
__device__ __forceinline__ void shift_words(const uint32_t *t, int sh, int d, uint32_t fill, uint32_t *r,
                                            std::integer_sequence<int, K...>) {
  ((r[K] = shifted_word<K>(t, sh, d, fill)), ...);
}

template <int D, bool V4>
__device__ __forceinline__ void load_row(const uint32_t *__restrict__ x, int64_t b, int d, uint32_t fill,
                                         uint32_t (&r)[D]) {
  if constexpr (!V4) {
#pragma unroll
    for (int k = 0; k < D; ++k) r[k] = k < d ? x[b + k] : fill;
  } else {
    constexpr int Q = D / 4 + 1;
    const int64_t b4 = b & ~int64_t(3);
    const int sh = (int)(b - b4);
    uint32_t t[4 * Q];
    load_words(reinterpret_cast<const uint4 *>(x + b4), sh + d, fill, t, std::make_integer_sequence<int, Q>{});
    shift_words(t, sh, d, fill, r, std::make_integer_sequence<int, D>{});
  }
}

// One listed vertex v that takes part in the sweep.
template <int D, bool W, bool O32, bool V4>
__device__ __forceinline__ void thread_vertex(const SweepArgs &a, const SweepView &sv, int32_t v, LocalCounts &lc) {
  // Everything that depends on v alone is loaded at once (absent arrays read
  // constants instead of branching: a branch would make the wave wait for
  // every load issued before it), so a vertex of a dense sweep waits for four
  // dependent loads before its gathers instead of six.
  const int32_t *gp = a.gid ? a.gid + v : &kZeroI32;
  const int64_t b = a.off[v];
  const int d = (int)(a.off[v + 1] - b);
  const int32_t g = *gp;
  const uint32_t own = (uint32_t)a.C[v];
  const uint8_t *dp = a.gdone ? a.gdone + g : &kZeroU8;
  if (*dp) return;
  uint32_t lab[D], w[D];
  load_row<D, V4>(reinterpret_cast<const uint32_t *>(a.cols), b, d, (uint32_t)v, lab);
#pragma unroll
  for (int k = 0; k < D; ++k) lab[k] = lab[k] != (uint32_t)v ? gather_label<O32>(a.C, (int32_t)lab[k]) : kNoLabel;
  unsigned long long rowsum = (unsigned long long)d;
  if constexpr (W) {
    rowsum = 0;
    load_row<D, V4>(a.w, b, d, 0u, w);
#pragma unroll
    for (int k = 0; k < D; ++k) rowsum += w[k];
  }
  sort_by_label<D, W>(lab, w);
  unsigned long long best = 0;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t wk = W ? w[k] : 1u;
    s = (k > 0 && lab[k] == lab[k - 1]) ? s + wk : wk;
    const unsigned long long key = lab[k] != kNoLabel ? argmax_key(lab[k], s) : 0ull;
    best = key > best ? key : best;
  }
  lc.processed += 1;
  lc.edges += (unsigned long long)d;
  lc.overflow += rowsum >> 32 ? 1 : 0;
  if (best && !(rowsum >> 32)) {
    const uint32_t cstar = key_label(best);
    if (cstar != own) {
      record_change(a, v, cstar, lc);
      if (sv.mark) {
        // the row again (just read, so mostly from cache) for the flags
        for (int k = 0; k < d; ++k) {
          const int32_t j = a.cols[b + k];
          if (!sv.nact[j]) sv.nact[j] = 1;
        }
        lc.marked += (unsigned long long)d;
      }
    }
  }
}

// The thread's next kAhead grid-stride entries are listed, and in a sparse
// sweep their one-byte flags read, all at once before any of them is
// processed: a sparse sweep late in the loop is mostly this scan, and one
// round trip then covers kAhead entries (4,096-graph batch: 119.3 -> 117.9 ms
// per call).
constexpr int kAhead = 4;

template <int D, bool W, bool O32, bool V4>
__global__ __launch_bounds__(256) void sweep_thread(SweepArgs a, const int32_t *__restrict__ list,
                                                    int64_t first, int64_t count) {
  __shared__ unsigned long long red[256 / kWave];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  LocalCounts lc;
  // a sparse sweep with a frontier walks the frontier instead of the tier
  const bool front = !sv.dense && sv.front && a.fcount;
  if (front) {
    list = a.flist;
    count = *a.fcount;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx0 < count; idx0 += kAhead * stride) {
    int32_t vv[kAhead];
    bool take[kAhead];
#pragma unroll
    for (int k = 0; k < kAhead; ++k) {
      const int64_t idx = idx0 + (int64_t)k * stride;
      vv[k] = idx < count ? (list ? list[first + idx] : (int32_t)(first + idx)) : -1;
    }
#pragma unroll
    for (int k = 0; k < kAhead; ++k) take[k] = vv[k] >= 0 && (sv.dense || front || sv.act[vv[k]]);
#pragma unroll 1
    for (int k = 0; k < kAhead; ++k)
      if (take[k]) thread_vertex<D, W, O32, V4>(a, sv, vv[k], lc);
  }
  flush_counts(a, lc, red);
}

template <int D, bool V4>
void launch_thread_rows(const SweepArgs &a, const int32_t *list, int64_t first, int64_t count, int grid,
                        hipStream_t s) {
  const bool o32 = a.n < (int64_t(1) << 30);
  if (a.w) {
    if (o32)
      sweep_thread<D, true, true, V4><<<grid, 256, 0, s>>>(a, list, first, count);
    else
      sweep_thread<D, true, false, V4><<<grid, 256, 0, s>>>(a, list, first, count);
  } else {
    if (o32)
      sweep_thread<D, false, true, V4><<<grid, 256, 0, s>>>(a, list, first, count);
    else
      sweep_thread<D, false, false, V4><<<grid, 256, 0, s>>>(a, list, first, count);
  }
}

// 16-byte row loads when the column (and weight) arrays are 16-byte aligned
// (the library's own copies always are; a caller's array may not be).
template <int D>
void launch_thread(const SweepArgs &a, const int32_t *list, int64_t first, int64_t count, int grid,
                   hipStream_t s) {
  if (((uintptr_t)a.cols & 15) == 0 && ((uintptr_t)a.w & 15) == 0)
    launch_thread_rows<D, true>(a, list, first, count, grid, s);
  else
    launch_thread_rows<D, false>(a, list, first, count, grid, s);
}

// ---------------------------------------------------------------------------
// Tiers 2-7: a group of G lanes per vertex -- a slice of a wavefront (G <= 64)
// or the whole workgroup (G == BLOCK) -- with a private LDS table of up to
// 2^LOG2S slots.  Every lane owns at most K row entries (the tier bound is
// G * K), loads them all before inserting, and remembers the slots it
// claimed: after the barrier the claimers read the final sums of their own
// slots (the argmax candidates) and clear them, so no lane scans empty slots.
//
// The block walks the tier in windows of `win` list entries (a multiple of
// the groups per block, at most BLOCK): one thread per entry decides whether
// the vertex takes part in this sweep (pruning flag, stopped graph of a
// batch), the taken vertices are packed into LDS in list order, and the
// groups then work through the packed vertices only.  A sparse sweep thus
// costs one flag check per thread instead of one per group, and one after
// few changes walks the frontier (every entry taken).  All groups of a block
// move through the insert / read phases together.
// ---------------------------------------------------------------------------
template <int G, int LOG2S, int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void sweep_lds(SweepArgs a, const int32_t *__restrict__ list,
                                                   int64_t first, int64_t count, int win) {
  static_assert(G <= 64 || G == BLOCK, "group is a wave slice or the block");
  constexpr int GPB = BLOCK / G;
  constexpr int S = 1 << LOG2S;
  constexpr int NW = BLOCK / kWave;
  __shared__ unsigned long long tab[GPB * S];
  __shared__ unsigned long long red[NW];
  __shared__ unsigned long long red2[NW];
  __shared__ int32_t q[BLOCK];
  __shared__ int64_t qb[BLOCK], qe[BLOCK];  // row bounds of the packed vertices
  __shared__ int wcnt[NW];
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  for (int s = threadIdx.x; s < GPB * S; s += BLOCK) tab[s] = kEmptySlot;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int wid = threadIdx.x / kWave, wl = threadIdx.x % kWave;
  unsigned long long *T = tab + g * S;
  LocalCounts lc;
  // a sparse sweep with a frontier walks the frontier instead of the tier
  if (!sv.dense && sv.front && a.fcount) {
    list = a.flist;
    count = *a.fcount;
  }
  for (int64_t w0 = (int64_t)blockIdx.x * win; w0 < count; w0 += (int64_t)gridDim.x * win) {
    // pack the taken vertices of the window with their row bounds (loaded
    // here, all at once, instead of one dependent load per group round)
    int32_t u = -1;
    int64_t ub = 0, ue = 0;
    if (threadIdx.x < win && w0 + threadIdx.x < count) {
      u = list ? list[first + w0 + threadIdx.x] : (int32_t)(first + w0 + threadIdx.x);
      if (!sweep_takes(a, sv, u)) u = -1;
      if (u >= 0) {
        ub = a.off[u];
        ue = a.off[u + 1];
      }
    }
    const unsigned long long m = __ballot(u >= 0);
    if (wl == 0) wcnt[wid] = __popcll(m);
    __syncthreads();
    int pos = __popcll(m & ((1ull << wl) - 1ull)), total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      pos += w < wid ? wcnt[w] : 0;
      total += wcnt[w];
    }
    if (u >= 0) {
      q[pos] = u;
      qb[pos] = ub;
      qe[pos] = ue;
    }
    __syncthreads();
    for (int r0 = 0; r0 < total; r0 += GPB) {
      const int32_t v = r0 + g < total ? q[r0 + g] : -1;
      int64_t b = 0, e = 0;
      int log2s = 1;
      if (v >= 0) {
        b = qb[r0 + g];
        e = qe[r0 + g];
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
      if constexpr (G >= kWave) wave_fold_labels<K>(lab, wt, kFoldRounds);  // one vertex per wave
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
        if (wl == 0) {
          red[wid] = best;
          red2[wid] = rowsum;
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
        // A row whose weights sum to 2^32 or more may have carried a sum
        // into the label half of a packed slot: nothing is recorded for it
        // (the call fails with the overflow).
        if (best && !(rowsum >> 32)) {
          const uint32_t cstar = key_label(best);
          if (cstar != (uint32_t)a.C[v]) {
            if (lane == 0) record_change(a, v, cstar, lc);
            if (sv.mark) {
#pragma unroll
              for (int k = 0; k < K; ++k)
                if (j[k] >= 0) {
                  if (!sv.nact[j[k]]) sv.nact[j[k]] = 1;
                  lc.marked += 1;
                }
            }
          }
        }
      }
      __syncthreads();
    }
  }
  flush_counts(a, lc, red);
}

// Copies the new label of every changed vertex into C, clears chg and, when
// requested, clears the active flags consumed by the sweep.  Four vertices per
// thread; the flag arrays are padded to a multiple of 4 bytes.  With 16-byte
// aligned label arrays (the library's own always are) a quad's labels (and
// graph ids) move as one 16-byte load and store: the changed labels are
// blended into the quad's current ones.  A quad whose last vertices lie past
// n is copied label by label (the arrays hold n labels).
__global__ __launch_bounds__(256) void apply_changes(SweepArgs a, int32_t *__restrict__ C, int64_t n,
                                                     unsigned long long *__restrict__ gdn) {
  SweepView sv;
  if (!sweep_view(a, sv)) return;
  const int32_t *__restrict__ Cn = a.Cn;
  uint8_t *__restrict__ chg = a.chg;
  uint8_t *act_clear = sv.dense ? nullptr : const_cast<uint8_t *>(sv.act);
  const int64_t quads = (n + 3) / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int wl = threadIdx.x % kWave;
  const bool v4 = ((uintptr_t)C & 15) == 0 && ((uintptr_t)Cn & 15) == 0 && ((uintptr_t)a.gid & 15) == 0;
  // uniform trip count per block, so the per-graph counting below can use
  // whole-wave reductions
  for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x; q0 < quads; q0 += stride) {
    const int64_t q = q0 + threadIdx.x;
    uint32_t word = 0;
    if (q < quads) {
      word = reinterpret_cast<uint32_t *>(chg)[q];
      if (act_clear) reinterpret_cast<uint32_t *>(act_clear)[q] = 0u;
    }
    int32_t gq = -1;
    unsigned long long cnt = 0;
    if (word) {
      reinterpret_cast<uint32_t *>(chg)[q] = 0u;
      const bool whole = v4 && 4 * q + 4 <= n;
      int32_t gg[4] = {0, 0, 0, 0};
      if (whole && gdn) {
        const int4 g4 = reinterpret_cast<const int4 *>(a.gid)[q];
        gg[0] = g4.x;
        gg[1] = g4.y;
        gg[2] = g4.z;
        gg[3] = g4.w;
      }
      if (whole && !a.inplace) {
        const int4 cn = reinterpret_cast<const int4 *>(Cn)[q];
        int4 c = reinterpret_cast<const int4 *>(C)[q];
        if (word & 0xffu) c.x = cn.x;
        if (word & 0xff00u) c.y = cn.y;
        if (word & 0xff0000u) c.z = cn.z;
        if (word & 0xff000000u) c.w = cn.w;
        reinterpret_cast<int4 *>(C)[q] = c;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((word >> (8 * k)) & 0xffu) {
          const int64_t v = 4 * q + k;
          if (!whole && !a.inplace) C[v] = Cn[v];
          if (gdn) {
            const int32_t g = whole ? gg[k] : a.gid[v];
            if (gq < 0) gq = g;
            if (g == gq)
              cnt += 1;
            else
              atomicAdd(&gdn[g], 1ull);  // quad straddles two graphs
          }
        }
    }
    if (!gdn) continue;
    // changes per graph: one atomic per run of lanes with the same graph
    unsigned long long pending = __ballot(cnt > 0);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int32_t lg = __shfl(gq, leader);
      const bool same = cnt > 0 && gq == lg;
      const unsigned long long sum = wave_sum(same ? cnt : 0ull);
      if (wl == leader) atomicAdd(&gdn[lg], sum);
      pending &= ~__ballot(same);
    }
  }
}

// Frontier of a sparse sweep (see launch_frontier): one thread per vertex of
// a 1,024-vertex chunk, ranks within the chunk by ballot per tier, one atomic
// per tier and chunk.  The grid is capped (chunks in a grid-stride loop), so
// the launch costs little in the sweeps that do not build one.
constexpr int kFrontierBlock = 1024;
constexpr int kFrontierGrid = 1024;

__global__ __launch_bounds__(kFrontierBlock) void frontier_build(SweepArgs a, int64_t n, TierBounds tb,
                                                                 TierBounds start, int32_t *__restrict__ flist,
                                                                 int64_t *__restrict__ fcount) {
  constexpr int W = kFrontierBlock / kWave;
  __shared__ int wcnt[W][kNumTiers];
  __shared__ unsigned long long base[kNumTiers];
  SweepView sv;
  if (!sweep_view(a, sv) || sv.dense || !sv.front) return;  // uniform
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t c0 = (int64_t)blockIdx.x * kFrontierBlock; c0 < n; c0 += (int64_t)gridDim.x * kFrontierBlock) {
    const int64_t v = c0 + threadIdx.x;
    int t = -1;
    if (v < n && sv.act[v] && !(a.gid && a.gdone[a.gid[v]])) {
      t = tier_of(a.off[v + 1] - a.off[v], tb);
      if (t == 0 || t == kNumTiers - 1) t = -1;  // no entries / a hub (the hub kernels read the flags)
    }
    int rank = 0;
#pragma unroll
    for (int k = 1; k < kNumTiers - 1; ++k) {
      const unsigned long long m = __ballot(t == k);
      if (t == k) rank = __popcll(m & below);
      if (lane == 0) wcnt[wid][k] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x > 0 && threadIdx.x < kNumTiers - 1) {
      int total = 0;
      for (int w = 0; w < W; ++w) total += wcnt[w][threadIdx.x];
      base[threadIdx.x] = total ? atomicAdd(reinterpret_cast<unsigned long long *>(&fcount[threadIdx.x]),
                                            (unsigned long long)total)
                                : 0ull;
    }
    __syncthreads();
    if (t >= 0) {
      int before = 0;
      for (int w = 0; w < wid; ++w) before += wcnt[w][t];
      flist[start.b[t] + (int64_t)base[t] + before + rank] = (int32_t)v;
    }
    __syncthreads();  // wcnt and base are rewritten by the next chunk
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

// Window of list entries per block iteration for a tier of `count` vertices
// handled by groups of G lanes: as large as the block (one flag check per
// thread), but small enough that the tier still spreads over about
// kMaxTierGrid blocks.
int window_for(int64_t count, int gpb, int block) {
  const int64_t per_block = (count + kMaxTierGrid - 1) / kMaxTierGrid;
  int64_t win = (per_block + gpb - 1) / gpb * gpb;
  if (win < gpb) win = gpb;
  if (win > block) win = block;
  return (int)win;
}

template <int G, int LOG2S, int BLOCK, int K>
int launch_lds(const SweepArgs &a, const int32_t *list, int64_t first, int64_t count, hipStream_t s) {
  const int win = window_for(count, BLOCK / G, BLOCK);
  const int grid = grid_for(count, win, kMaxTierGrid);
  sweep_lds<G, LOG2S, BLOCK, K><<<grid, BLOCK, 0, s>>>(a, list, first, count, win);
  return grid;
}

}  // namespace

hipError_t launch_sweep_tier(int variant, const SweepArgs &a, const int32_t *list, int64_t first,
                             int64_t count, int *grid_out, hipStream_t s) {
  *grid_out = 0;
  if (count <= 0) return hipSuccess;
  int grid = 0;
  switch (variant) {
    case 0:
      grid = grid_for(count, 256, kMaxTierGrid);
      launch_thread<8>(a, list, first, count, grid, s);
      break;
    case 15:
      grid = grid_for(count, 256, kMaxTierGrid);
      launch_thread<16>(a, list, first, count, grid, s);
      break;
    case 16:
      grid = grid_for(count, 256, kMaxTierGrid);
      launch_thread<32>(a, list, first, count, grid, s);
      break;
    case 1: grid = launch_lds<8, 5, 256, 2>(a, list, first, count, s); break;
    case 2: grid = launch_lds<4, 5, 256, 4>(a, list, first, count, s); break;
    case 3: grid = launch_lds<16, 6, 256, 2>(a, list, first, count, s); break;
    case 4: grid = launch_lds<8, 6, 256, 4>(a, list, first, count, s); break;
    case 5: grid = launch_lds<32, 7, 256, 2>(a, list, first, count, s); break;
    case 6: grid = launch_lds<16, 7, 256, 4>(a, list, first, count, s); break;
    case 7: grid = launch_lds<64, 8, 256, 2>(a, list, first, count, s); break;
    case 8: grid = launch_lds<32, 8, 256, 4>(a, list, first, count, s); break;
    case 9: grid = launch_lds<64, 10, 256, 8>(a, list, first, count, s); break;
    case 10: grid = launch_lds<128, 10, 128, 4>(a, list, first, count, s); break;
    case 11: grid = launch_lds<256, 12, 256, 8>(a, list, first, count, s); break;
    case 12: grid = launch_lds<512, 12, 512, 4>(a, list, first, count, s); break;
    case 13: grid = launch_lds<512, 13, 512, 8>(a, list, first, count, s); break;
    case 14: grid = launch_lds<1024, 14, 1024, 8>(a, list, first, count, s); break;
    case 17: grid = launch_lds<256, 11, 256, 4>(a, list, first, count, s); break;
    case 18:
      grid = grid_for(count, 256, kMaxTierGrid);
      launch_thread<64>(a, list, first, count, grid, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  *grid_out = grid;
  return hipGetLastError();
}

namespace {
__global__ void reduce_counts(const unsigned long long *__restrict__ part, TierGrids g,
                              unsigned long long (*tier_stats)[4], const SweepCtrl *ctrl,
                              unsigned long long *dn, unsigned long long *processed,
                              unsigned long long *edges, unsigned long long *overflow) {
  __shared__ unsigned long long red[256 / kWave];
  const int t = blockIdx.x;
  const int nb = g.g[t];
  if (nb <= 0 || ctrl->done) return;
  const int it = ctrl->it;
  dn += it;
  processed += it;
  edges += it;
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
                                unsigned long long (*tier_stats)[4], const SweepCtrl *ctrl,
                                unsigned long long *dn, unsigned long long *processed,
                                unsigned long long *edges, unsigned long long *overflow, hipStream_t s) {
  reduce_counts<<<kNumTiers, 256, 0, s>>>(part, g, tier_stats, ctrl, dn, processed, edges, overflow);
  return hipGetLastError();
}

hipError_t launch_frontier(const SweepArgs &a, int64_t n, const TierConfig &cfg, const int64_t *tier_start_h,
                           int32_t *flist, int64_t *fcount, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  TierBounds tb, start;
  for (int t = 0; t < kNumTiers; ++t) {
    tb.b[t] = cfg.bound[t];
    start.b[t] = tier_start_h[t];
  }
  const int64_t chunks = (n + kFrontierBlock - 1) / kFrontierBlock;
  frontier_build<<<(unsigned)(chunks < kFrontierGrid ? chunks : kFrontierGrid), kFrontierBlock, 0, s>>>(
      a, n, tb, start, flist, fcount);
  return hipGetLastError();
}

hipError_t launch_apply(const SweepArgs &a, int32_t *C, int64_t n, int64_t *gdn, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  apply_changes<<<grid_for((n + 3) / 4, 256, 256 * 32), 256, 0, s>>>(
      a, C, n, reinterpret_cast<unsigned long long *>(gdn));
  return hipGetLastError();
}

namespace {

// After a sweep: stop on overflow, convergence or the iteration cap; choose
// the next sweep's mode.  A sweep marks neighbours only when the previous one
// changed at most n/8 vertices; the sweep after a non-marking sweep runs
// dense (pruning is exact, so processing extra vertices changes nothing).
__global__ void sweep_end(SweepCtrl *c, const unsigned long long *dn, unsigned long long *marked_sweeps,
                          const unsigned long long *overflow, int64_t *fcount, int64_t *ftotal) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || c->done) return;
  const unsigned long long d = dn[c->it];
  marked_sweeps[c->it] = (unsigned long long)c->mark;
  const int marked = c->mark;
  c->it += 1;
  if (*overflow) {
    c->error = 1;
    c->done = 1;
    return;
  }
  bool stop = c->it >= c->max_iters;
  if (c->graphs > 0) {
    stop = stop || c->active == 0;
    c->active = 0;
  } else {
    stop = stop || (int64_t)d <= c->limit;
  }
  c->done = stop ? 1 : 0;
  c->dense = (c->prune && marked) ? 0 : 1;
  c->mark = (c->prune && (int64_t)d * 8 <= c->n) ? 1 : 0;
  // After a sweep with few changes the next sweep's active vertices are few
  // too: a frontier of them beats scanning the tier lists (a sweep that
  // changed a quarter of the vertices, as on road graphs, keeps the scan).
  c->front = (int64_t)d * 16 <= c->n ? 1 : 0;
  if (fcount)
    for (int t = 0; t < kNumTiers; ++t) {
      if (ftotal) ftotal[t] += fcount[t];
      fcount[t] = 0;
    }
}

// Sets up the loop state before the first sweep.  When the renumbering copy
// already ran sweep 0 (first_flags bit 0 clear: every row strictly
// increasing), the loop resumes at sweep 1 with that sweep's change count.
__global__ void loop_init(SweepCtrl *c, const unsigned long long *first_flags, unsigned long long *dn,
                          unsigned long long *marked_sweeps, int check_overflow) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  c->it = 0;
  c->error = 0;
  c->active = 0;
  c->dense = 1;
  c->mark = 0;
  c->front = 0;
  c->done = c->max_iters <= 0 ? 1 : 0;
  if (!first_flags || c->max_iters <= 0) return;
  const unsigned long long ff = *first_flags;
  if (ff & 1ull) {
    dn[0] = 0;
    return;
  }
  marked_sweeps[0] = 0;
  c->it = 1;
  if (check_overflow && (ff & 2ull)) {
    c->error = 1;
    c->done = 1;
    return;
  }
  const int64_t d = (int64_t)dn[0];
  c->done = (d <= c->limit || c->max_iters <= 1) ? 1 : 0;
  c->mark = (c->prune && d * 8 <= c->n) ? 1 : 0;
}

// Largest dN with dN / n <= tolerance in IEEE double (n > 0); the same
// search as the host's gsl_convergence_limit.
__device__ int64_t conv_limit(int64_t n, double tol) {
  const double dn = (double)n;
  int64_t k = (int64_t)floor(__dmul_rn(tol, dn));
  if (k < 0) k = 0;
  if (k > n) k = n;
  while (k > 0 && !(__ddiv_rn((double)k, dn) <= tol)) --k;
  while (k < n && __ddiv_rn((double)(k + 1), dn) <= tol) ++k;
  return k;
}

// Block per graph of a batch: graph id of each vertex, convergence limit,
// sweep count and stop flag (graphs without vertices, or max_iters 0, never
// run).
__global__ __launch_bounds__(256) void batch_init(const int64_t *__restrict__ vtx_base, int64_t graphs,
                                                  int32_t max_iters, double tol, int32_t *__restrict__ gid,
                                                  int64_t *__restrict__ glimit, int32_t *__restrict__ giters,
                                                  uint8_t *__restrict__ gdone, int64_t *__restrict__ gdn) {
  for (int64_t g = blockIdx.x; g < graphs; g += gridDim.x) {
    const int64_t b = vtx_base[g], e = vtx_base[g + 1];
    for (int64_t v = b + threadIdx.x; v < e; v += blockDim.x) gid[v] = (int32_t)g;
    if (threadIdx.x == 0) {
      glimit[g] = e > b ? conv_limit(e - b, tol) : 0;
      giters[g] = 0;
      gdn[g] = 0;
      gdone[g] = (e <= b || max_iters <= 0) ? 1 : 0;
    }
  }
}

// Thread per graph: count the sweep, stop graphs that converged or reached
// the cap, add the graphs still running to ctrl->active and clear the
// per-graph change counts for the next sweep.
__global__ __launch_bounds__(256) void graph_end(SweepCtrl *c, int64_t *__restrict__ gdn,
                                                 const int64_t *__restrict__ glimit, int32_t *giters,
                                                 uint8_t *gdone, int64_t graphs) {
  __shared__ unsigned long long red[256 / kWave];
  if (c->done) return;
  unsigned long long running = 0;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < graphs && !gdone[g]) {
    const int32_t it = giters[g] + 1;
    giters[g] = it;
    if (gdn[g] <= glimit[g] || it >= c->graph_max_iters)
      gdone[g] = 1;
    else
      running = 1;
    gdn[g] = 0;
  }
  running = block_sum(running, red);
  if (threadIdx.x == 0 && running) atomicAdd(reinterpret_cast<unsigned long long *>(&c->active), running);
}

}  // namespace

hipError_t launch_sweep_end(SweepCtrl *ctrl, const unsigned long long *dn, unsigned long long *marked_sweeps,
                            const unsigned long long *overflow, hipStream_t s, int64_t *fcount,
                            int64_t *ftotal) {
  sweep_end<<<1, 64, 0, s>>>(ctrl, dn, marked_sweeps, overflow, fcount, ftotal);
  return hipGetLastError();
}

hipError_t launch_loop_init(SweepCtrl *ctrl, const unsigned long long *first_flags, unsigned long long *dn,
                            unsigned long long *marked_sweeps, int check_overflow, hipStream_t s) {
  loop_init<<<1, 64, 0, s>>>(ctrl, first_flags, dn, marked_sweeps, check_overflow);
  return hipGetLastError();
}

hipError_t launch_batch_init(const int64_t *vtx_base, int64_t graphs, int32_t max_iters, double tol,
                             int32_t *gid, int64_t *glimit, int32_t *giters, uint8_t *gdone, int64_t *gdn,
                             hipStream_t s) {
  if (graphs <= 0) return hipSuccess;
  batch_init<<<grid_for(graphs, 1, 256 * 16), 256, 0, s>>>(vtx_base, graphs, max_iters, tol, gid, glimit,
                                                          giters, gdone, gdn);
  return hipGetLastError();
}

hipError_t launch_graph_end(SweepCtrl *ctrl, int64_t *gdn, const int64_t *glimit, int32_t *giters,
                            uint8_t *gdone, int64_t graphs, hipStream_t s) {
  if (graphs <= 0) return hipSuccess;
  graph_end<<<grid_for(graphs, 256, 1 << 20), 256, 0, s>>>(ctrl, gdn, glimit, giters, gdone, graphs);
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
