// Internal declarations shared by the HIP translation units of libgsl_lpa.so.
// Not part of the public ABI (that is include/gsl_lpa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gsl {

// ----------------------------------------------------------------------------
// Degree tiers.  Every vertex with degree d > 0 is processed by the kernel of
// the smallest tier whose bound is >= d; tier 0 holds isolated vertices, which
// never change label.  Tiers 1 - 7 (the seven levels of the tier table) each
// run one sweep variant of the menu below:
//   thread per vertex : labels held in registers and sorted (variants 0, 15,
//                       16, 18)
//   G lanes per vertex: an LDS hash table per group, or per workgroup when
//                       the group is the whole workgroup
//   tier 8 (hub)      : rows above the last level's bound, cut into chunks,
//                       one workgroup per chunk, partial sums merged per hash
//                       partition (hub.hip)
// ----------------------------------------------------------------------------
constexpr int kNumTiers = 9;
constexpr int kHubTier = 8;

// Sweep kernel variants a tier can use: a thread per vertex (variant 0) or a
// group of G lanes with K entries per lane and a 2^LOG2S-slot LDS table, in
// blocks of BLOCK threads.  A variant takes rows of up to G * K entries.
struct SweepVariant {
  int group, log2s, block, per_lane;
};
constexpr int kNumVariants = 19;
constexpr SweepVariant kVariants[kNumVariants] = {
    {1, 0, 256, 8},     // 0: thread per vertex, row in registers (d <= 8)
    {8, 5, 256, 2},     // 1: d <= 16
    {4, 5, 256, 4},     // 2: d <= 16
    {16, 6, 256, 2},    // 3: d <= 32
    {8, 6, 256, 4},     // 4: d <= 32
    {32, 7, 256, 2},    // 5: d <= 64
    {16, 7, 256, 4},    // 6: d <= 64
    {64, 8, 256, 2},    // 7: d <= 128
    {32, 8, 256, 4},    // 8: d <= 128
    {64, 10, 256, 8},   // 9: d <= 512
    {128, 10, 128, 4},  // 10: d <= 512, one 128-thread workgroup per vertex
    {256, 12, 256, 8},  // 11: d <= 2048, one workgroup per vertex
    {512, 12, 512, 4},  // 12: d <= 2048, one 512-thread workgroup per vertex
    {512, 13, 512, 8},  // 13: d <= 4096 (64 KB table)
    {1024, 14, 1024, 8},  // 14: d <= 8192 (128 KB table, one workgroup per CU)
    {1, 0, 256, 16},    // 15: thread per vertex, d <= 16
    {1, 0, 256, 32},    // 16: thread per vertex, d <= 32
    {256, 11, 256, 4},  // 17: d <= 1024, one workgroup per vertex (16 KB table)
    {1, 0, 256, 64},    // 18: thread per vertex, d <= 64
};
constexpr int64_t variant_capacity(int v) { return (int64_t)kVariants[v].group * kVariants[v].per_lane; }

// Degree tiers of one call: tier t (1..7) takes degrees (bound[t-1],
// bound[t]] with sweep variant variant[t]; tier 0 is degree 0 and tier 8
// (hubs) every degree above bound[7].
struct TierConfig {
  int64_t bound[kNumTiers];
  int variant[kNumTiers];
};
// Default levels: a thread per vertex up to degree 32, then groups of 16,
// 32 and 64 lanes, 256-lane workgroups up to 1024 (2,048-slot table) and
// 2048 (4,096 slots), and a 512-lane workgroup up to 4096; hubs above.
constexpr TierConfig kDefaultTiers = {{0, 32, 64, 128, 512, 1024, 2048, 4096, (int64_t)0x7fffffffffffffffLL},
                                      {0, 16, 6, 8, 9, 17, 11, 13, 0}};
// The fp32-weight kernels are instantiated for these bounds only.
constexpr TierConfig kF32Tiers = {{0, 8, 16, 32, 64, 128, 512, 2048, (int64_t)0x7fffffffffffffffLL},
                                  {0, 0, 1, 3, 5, 7, 9, 11, 0}};
// Bounds as a kernel argument.
struct TierBounds {
  int64_t b[kNumTiers];
};

// Tier of a row of d entries: 0 empty, t for the first bound b[t] >= d
// (t = 1 .. kNumTiers - 2), kNumTiers - 1 (hubs) above the last.
__host__ __device__ __forceinline__ int tier_of(int64_t d, const TierBounds &tb) {
  if (d <= 0) return 0;
  for (int t = 1; t < kNumTiers - 1; ++t)
    if (d <= tb.b[t]) return t;
  return kNumTiers - 1;
}

// Device-side counters; one block of memory zeroed at the start of every call.
struct Counters {
  int64_t tier_count[16];   // vertices per tier
  int64_t tier_start[16];   // first index of each tier in the vertex list
  uint64_t max_degree;
  uint64_t overflow;        // set when a row's weight sum reaches 2^32
  uint64_t split_changed;   // hook round: nonzero if any union happened
  uint64_t bad_label;       // set when an input label is outside [0, n)
  uint64_t first_flags;     // folded first sweep: bit 0 unsorted row, bit 1 overflow
  uint64_t two_m, intra;    // modularity integer parts
  uint64_t s2_lo, s2_hi;
  double q;
  uint64_t pad[3];
  int64_t tier_edges[16];   // row entries per tier
  int64_t fcount[16];       // sparse sweeps: active vertices of each tier (the frontier)
  int64_t ftotal[16];       // frontier entries per tier, summed over the sweeps
  // per tier, summed over sweeps: processed, edges, changed, marked
  unsigned long long tier_stats[kNumTiers][4];
  // followed by per-sweep arrays dn[max_iters], processed[], edges[], marked[]
};

// Loop state kept on the device, so a whole sequence of sweeps can be
// enqueued (or captured in a graph) without the host reading anything back:
// every sweep kernel returns at once when `done` is set, and sweep_end
// advances the state after each sweep.
struct SweepCtrl {
  int32_t it;          // index of the sweep about to run
  int32_t done;        // converged, iteration cap reached, or error
  int32_t dense;       // this sweep processes every listed vertex
  int32_t mark;        // this sweep marks the neighbours of changed vertices
  int32_t max_iters;
  int32_t prune;
  int32_t error;       // 1: a row's weight sum reached 2^32
  int32_t graph_max_iters;  // batches: each graph's own sweep cap (a session's sweeps outrun any graph's)
  int64_t limit;       // largest dN that counts as converged (one graph)
  int64_t n;           // vertices, for the marking heuristic
  int64_t graphs;      // 0: one graph; else graphs of a batch
  int64_t active;      // graphs still running after the last sweep (batch)
  int32_t front;       // this sweep (when sparse) walks a frontier: the last one changed at most n/16
  int32_t pad;
};

// Arguments common to every sweep kernel.
struct SweepArgs {
  const int64_t *off;
  const int32_t *cols;
  const uint32_t *w;      // NULL: unit weights
  const int32_t *C;       // labels read by this sweep
  int32_t *Cn;            // new label of each changed vertex
  uint8_t *chg;           // 1 where the vertex changed in this sweep
  uint8_t *act0, *act1;   // active flags: sweep t reads act[t & 1], marks act[(t + 1) & 1]
  const SweepCtrl *ctrl;  // loop state (dense / mark / it / done)
  // Per-sweep counters (indexed by ctrl->it) and the overflow flag.
  unsigned long long *dn, *processed, *edges, *marked_sweeps, *overflow;
  unsigned long long *tier;  // this tier's [processed, edges, changed, marked]
  // Per-block count records of the tier kernels (kCountFields per block);
  // summed by launch_reduce_counts instead of contended global atomics.
  unsigned long long *part;
  // Batches: graph of every vertex and the graphs that have stopped (NULL
  // for a single graph).
  const int32_t *gid;
  const uint8_t *gdone;
  // 1: asynchronous sweeps -- a changed label is written straight into C,
  // so vertices later in the same sweep may already read it (the paper's
  // in-place lpaMove); results then depend on timing.
  int32_t inplace;
  int64_t n;  // vertices (labels C[0..n))
  // Frontier of a sparse sweep: this tier's taking part vertices are
  // flist[first + i], i < *fcount (the tier's own range of the list layout).
  // fcount NULL: the tier list is scanned against the active flags.
  const int32_t *flist;
  const int64_t *fcount;
};

// What a sweep kernel needs from the loop state.
struct SweepView {
  int it, dense, mark, front;
  const uint8_t *act;
  uint8_t *nact;
};

__device__ __forceinline__ bool sweep_view(const SweepArgs &a, SweepView &v) {
  const SweepCtrl *c = a.ctrl;
  if (c->done) return false;
  v.it = c->it;
  v.dense = c->dense;
  v.mark = c->mark;
  v.front = c->front;
  v.act = (v.it & 1) ? a.act1 : a.act0;
  v.nact = (v.it & 1) ? a.act0 : a.act1;
  return true;
}

// Vertex v takes part in this sweep.
__device__ __forceinline__ bool sweep_takes(const SweepArgs &a, const SweepView &sv, int32_t v) {
  if (a.gid && a.gdone[a.gid[v]]) return false;
  return sv.dense || sv.act[v];
}

constexpr int kCountFields = 5;        // dn, processed, edges, marked, overflow
constexpr int kMaxTierGrid = 256 * 16; // largest grid of a tier kernel

struct TierGrids {
  int g[kNumTiers];
};

// ---- launchers (stream-ordered, no synchronisation) ----
hipError_t launch_plan(const int64_t *off, int64_t n, int32_t *list, int64_t *blk_counts,
                       Counters *ctr, const TierConfig &cfg, hipStream_t s);
int64_t plan_blocks(int64_t n);
// Entries of the plan's scratch array (blk_counts) for n vertices.
int64_t plan_scratch(int64_t n);

// Sweep kernel of one tier with the given variant (kVariants index).
hipError_t launch_sweep_tier(int variant, const SweepArgs &a, const int32_t *list, int64_t first,
                             int64_t count, int *grid_out, hipStream_t s);
// Sums the per-block records of tier t (part + t * kMaxTierGrid * kCountFields,
// g.g[t] blocks) into the tier and sweep counters.
hipError_t launch_reduce_counts(const unsigned long long *part, TierGrids g,
                                unsigned long long (*tier_stats)[4], const SweepCtrl *ctrl,
                                unsigned long long *dn, unsigned long long *processed,
                                unsigned long long *edges, unsigned long long *overflow, hipStream_t s);
// Hub tier layout: rows cut into chunks of kHubChunk entries; prefix sums
// over the hubs (H + 1 entries each) of their chunks, hash partitions and
// partition-boundary records (chunks * (partitions + 1)).
constexpr int kHubChunk = 2048;
// Most hash partitions of one hub row.
constexpr int kHubMaxParts = 8192;
// Merge table claims before a hub partition is re-merged in hashed
// sub-passes (the largest value; see hub.hip).
constexpr int kHubMergeCapMax = 4096 - 256 - 1;
struct HubLayout {
  int64_t *chunk_start;
  int64_t *part_start;
  int64_t *hist_start;
  int32_t *chunk_owner;          // [total chunks] hub of each chunk
  int32_t *part_owner;           // [total partitions] hub of each partition
  unsigned long long *records;   // [H] (label, sum) records staged in the current sweep
};
// Chunk and partition prefix sums of the hubs (owners and records are filled
// by launch_hub_owners once the host has sized them).
hipError_t launch_hub_layout(const int64_t *off, const int32_t *hubs, int64_t H, HubLayout L,
                             hipStream_t s);
// chunk_owner / part_owner from the prefix sums; records cleared.
hipError_t launch_hub_owners(HubLayout L, int64_t H, hipStream_t s);
hipError_t launch_hub_sweep(const SweepArgs &a, const int32_t *hubs, HubLayout L,
                            const int64_t *chunk_start_h, const int64_t *part_start_h,
                            unsigned long long *staging, int32_t *hist, unsigned long long *best,
                            unsigned long long *rowsum, int64_t k0, int64_t k1, int max_parts,
                            int merge_cap, int stage, hipStream_t s);
// Copies changed labels into C and clears the consumed flags (this sweep's
// active flags when it was sparse).  Batches (gdn != NULL): also adds each
// graph's changes to gdn[graph].
hipError_t launch_apply(const SweepArgs &a, int32_t *C, int64_t n, int64_t *gdn, hipStream_t s);
// Sparse sweeps that follow a sweep with few changes only (the kernel reads
// the loop state): the frontier of the sweep about to run -- each vertex of
// [0, n) whose active flag is set, whose row is not empty and not a hub's, and
// whose graph still runs -- into its tier's range [tier_start[t], +count) of
// flist, the counts added to fcount[t] (which the sweep_end before cleared,
// and the sweep_end after adds to the per-tier totals).
// Other sweeps return at once.
hipError_t launch_frontier(const SweepArgs &a, int64_t n, const TierConfig &cfg, const int64_t *tier_start_h,
                           int32_t *flist, int64_t *fcount, hipStream_t s);
// Advances the loop state after a sweep.
hipError_t launch_sweep_end(SweepCtrl *ctrl, const unsigned long long *dn, unsigned long long *marked_sweeps,
                            const unsigned long long *overflow, hipStream_t s,
                            int64_t *fcount = nullptr, int64_t *ftotal = nullptr);
// Loop state before the first sweep; first_flags (NULL unless renumbered)
// tells whether the renumbering copy already ran sweep 0.
hipError_t launch_loop_init(SweepCtrl *ctrl, const unsigned long long *first_flags, unsigned long long *dn,
                            unsigned long long *marked_sweeps, int check_overflow, hipStream_t s);
// ---- fp32 weights summed in fp64 (sweep_f32.hip); SweepArgs::w holds floats ----
hipError_t launch_sweep_tier_f32(int tier, const SweepArgs &a, const int32_t *list, int64_t first, int64_t count,
                                 int *grid_out, hipStream_t s);
// Hub tier: per-chunk LDS sums folded into a global table per hub
// (hub_f32_slots(chunks) slots in total, empty before the first sweep and
// left empty by every sweep).
hipError_t launch_hub_f32(const SweepArgs &a, const int32_t *hubs, const int64_t *chunk_start, int64_t H,
                          int64_t chunks, uint32_t *gkeys, double *gsums, hipStream_t s);
int64_t hub_f32_slots(int64_t chunks);
hipError_t launch_hub_f32_clear(uint32_t *gkeys, double *gsums, int64_t slots, hipStream_t s);
// *bad |= 1 if a weight is negative, NaN or infinite.
hipError_t launch_check_f32(const float *w, int64_t nnz, unsigned long long *bad, hipStream_t s);
// Batches: graph id per vertex, per-graph limits, sweep counts and stop flags.
hipError_t launch_batch_init(const int64_t *vtx_base, int64_t graphs, int32_t max_iters, double tol,
                             int32_t *gid, int64_t *glimit, int32_t *giters, uint8_t *gdone, int64_t *gdn,
                             hipStream_t s);
// Batches: per-graph stop decisions after apply (before sweep_end); clears gdn.
hipError_t launch_graph_end(SweepCtrl *ctrl, int64_t *gdn, const int64_t *glimit, int32_t *giters,
                            uint8_t *gdone, int64_t graphs, hipStream_t s);
// ---- batches (batch.hip) ----
// One graph of a batch given as its own arrays; the same layout as gsl_graph
// in the public header.
struct GraphDesc {
  const int64_t *offsets;
  const int32_t *cols;
  const uint32_t *weights;
  int32_t *labels_out;
  int64_t n;
};
// Sets *bad when vtx_base / edge_base ([G + 1] each) do not start at 0, end
// at N / nnz and stay non-decreasing.
hipError_t launch_check_bases(const int64_t *vtx_base, const int64_t *edge_base, int64_t G, int64_t N,
                              int64_t nnz, unsigned long long *bad, hipStream_t s);
// out[e] = cols[e] + vtx_base[graph of entry e].
hipError_t launch_globalize_cols(const int32_t *cols, const int64_t *edge_base, const int64_t *vtx_base,
                                 int64_t G, int64_t nnz, int32_t *out, hipStream_t s);
// cnt[g] = offsets[n] - offsets[0] of graph g, -1 if its offsets decrease.
hipError_t launch_graph_entries(const GraphDesc *d, int64_t G, int64_t *cnt, hipStream_t s);
// Separate graphs -> one global CSR (off [N + 1], cols [nnz], w [nnz] or NULL),
// vertex ids shifted by vshift and entry positions by eshift (the position
// of the gathered block in a larger array; 0 for a batch of its own).  An
// entry outside [0, n_g) sets bad[g] and is replaced by local vertex 0.
hipError_t launch_gather(const GraphDesc *d, const int64_t *vtx_base, const int64_t *edge_base, int64_t G,
                         int64_t N, int64_t nnz, int64_t vshift, int64_t eshift, int64_t *off, int32_t *cols,
                         uint32_t *w, uint32_t *bad, hipStream_t s);
// ---- sessions: graphs joining and leaving a resident batch between sweeps ----
// One graph of a session: vertices [vb, vb + n) and entries [eb, eb + nnz) of
// the arena, its slot, its convergence limit, its output, and (compaction)
// its new position.
struct SessionRange {
  int64_t vb, n, eb, nnz;
  int64_t new_vb, new_eb;
  int64_t limit;
  int32_t *labels_out;
  int32_t slot, pad;
};
hipError_t launch_session_admit(const SessionRange *r, int64_t count, int32_t *gid, int32_t *lab, uint8_t *act0,
                                uint8_t *act1, hipStream_t s);
hipError_t launch_session_slots(const SessionRange *r, int64_t count, int32_t max_iters, double tol, int64_t *glimit,
                                int32_t *giters, uint8_t *gdone, int64_t *gdn, hipStream_t s);
hipError_t launch_session_split_labels(const int32_t *lab, const int32_t *gid, const uint8_t *sel, int64_t n,
                                       int32_t *out, hipStream_t s);
hipError_t launch_session_finish(const SessionRange *r, int64_t count, const int32_t *split, int32_t *gid,
                                 int32_t dead, hipStream_t s);
hipError_t launch_session_move(const SessionRange *r, int64_t count, const int64_t *off, const int32_t *cols,
                               const uint32_t *w, const int32_t *lab, int64_t *off2, int32_t *cols2, uint32_t *w2,
                               int32_t *lab2, int32_t *gid, uint8_t *act0, uint8_t *act1, hipStream_t s);
// One graph: *bad |= 1 if offsets[0] != 0 or offsets decrease, |= 2 if a
// column is outside [0, n).
hipError_t launch_check_graph(const int64_t *off, const int32_t *cols, int64_t n, int64_t nnz,
                              unsigned long long *bad, hipStream_t s);
// lab[v] -= vtx_base[graph of v].
hipError_t launch_localize(int32_t *lab, const int64_t *vtx_base, int64_t G, int64_t N, hipStream_t s);
// d[g].labels_out[i] = lab[vtx_base[g] + i] for graphs with bad[g] == 0.
hipError_t launch_scatter_labels(const GraphDesc *d, const int32_t *lab, const int64_t *vtx_base,
                                 const uint32_t *bad, int64_t G, int64_t N, hipStream_t s);

hipError_t launch_init_labels(int32_t *C, int32_t *Cn, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t count, hipStream_t s);

// Alg. 2 split by union-find.  With gid / sel (batches), the first linking
// pass skips the rows of graphs g with sel[g] == 0: a caller that gives those
// vertices their own ids as labels keeps them singletons at the cost of a
// flag check.
hipError_t launch_split(const int64_t *off, const int32_t *cols, int64_t n, const int32_t *C,
                        int32_t *parent, int32_t *out, const int32_t *list,
                        const int64_t *tier_count_host, const int64_t *tier_start_host,
                        const int32_t *orig, int32_t *minorig, int64_t n_total, int32_t *rep,
                        unsigned long long *cp, const TierConfig &cfg, hipStream_t s,
                        const int32_t *gid = nullptr, const uint8_t *sel = nullptr);
// Alg. 1 split (min-label propagation on intra-community entries): labels
// and flags initialised by launch_split_lp_init (f0 all set, f1 clear; NULL
// flags for LP without pruning), then rounds until *changed stays 0.
hipError_t launch_split_lp_init(int32_t *lab, uint8_t *f0, uint8_t *f1, int64_t n, hipStream_t s);
hipError_t launch_split_lp_round(const int64_t *off, const int32_t *cols, int64_t n, const int32_t *C,
                                 int32_t *lab, const int32_t *list, const int64_t *tier_count_host,
                                 const int64_t *tier_start_host, const TierConfig &cfg, uint8_t *fin,
                                 uint8_t *fout, unsigned long long *changed, hipStream_t s);
// Alg. 4 from split labels comp (smallest id of each piece): pieces[c] =
// number of pieces of community c, D[c] = pieces[c] > 1 (D may be NULL),
// *count += number of such communities.
hipError_t launch_disconnected(const int32_t *labels, const int32_t *comp, int64_t n, int32_t *pieces,
                               uint8_t *D, unsigned long long *count, hipStream_t s);
hipError_t launch_reorder(const int64_t *off, const int32_t *cols, const uint32_t *w, int64_t n,
                          const int32_t *list, const int64_t *tier_count_h, const int64_t *tier_start_h,
                          const int64_t *hub_chunk_start, const int32_t *hub_chunk_owner, int64_t hub_chunks,
                          int32_t *old2new,
                          int64_t *off2, int32_t *cols2, uint32_t *w2, int32_t *lab,
                          int64_t *scan_tmp, unsigned long long *first_key,
                          unsigned long long *hub_rowsum, unsigned long long *flags,
                          unsigned long long *dn0, int apply_first, const TierConfig &cfg, hipStream_t s);
hipError_t launch_reorder_scatter(const int32_t *list, const int32_t *val, int64_t np, int64_t n,
                                  int32_t *out, hipStream_t s);
hipError_t launch_check_labels(const int32_t *labels, int64_t n, unsigned long long *bad,
                               hipStream_t s);

hipError_t launch_modularity(const int64_t *off, const int32_t *cols, const uint32_t *w, int64_t n,
                             const int32_t *labels, unsigned long long *sigma_tot,
                             unsigned long long *partials, int partial_blocks, Counters *ctr,
                             hipStream_t s);

}  // namespace gsl
