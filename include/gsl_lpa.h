/*
 * gsl_lpa.h -- C ABI of the MI355X (gfx950) GSL-LPA library, libgsl_lpa.so.
 *
 * GSL-LPA (Sahu, arXiv:2403.01261) is label-propagation community detection
 * followed by a split pass that breaks every internally-disconnected community
 * into its connected pieces.  The library runs every step in HIP kernels.
 *
 * Conventions shared by all entry points
 * -------------------------------------
 *  - Graphs are CSR: offsets int64[n+1] (offsets[0] == 0, non-decreasing),
 *    cols int32[nnz] with nnz = offsets[n] and 0 <= cols[e] < n, weights
 *    uint32[nnz] or NULL meaning every weight is 1.  The graph must be
 *    symmetric: an entry (i, j, w) implies an entry (j, i, w) (the paper
 *    adds reverse edges, Sec. 5.1.3).  This is the caller's promise; it is not
 *    checked.  Rows need not be sorted; self loops and duplicate entries are
 *    allowed (a self loop never votes, duplicates add their weights).
 *  - Every array argument is a DEVICE pointer on the current HIP device,
 *    allocated and owned by the caller.  Outputs must not alias inputs.
 *  - Vertex ids and labels are int32: 0 <= n < 2^31.
 *  - Work is enqueued on the stream given to gsl_set_stream (default: the
 *    null stream) and every call returns only after that work has finished.
 *  - Scratch memory is owned by the library, cached per device and grown on
 *    demand; gsl_release() frees it.
 *  - Calls return a gsl_status.  No C++ exception crosses the ABI.  On error
 *    gsl_last_error() returns a message for the calling thread; outputs are
 *    unspecified.
 *  - Calls without a context argument share one scratch cache per device
 *    and are serialised by a process-wide lock.  Calls on different
 *    gsl_context objects (gsl_lpa_graphs) have their own scratch and stream
 *    and may run at the same time from different host threads; their work
 *    then overlaps on the device.
 */
#ifndef GSL_LPA_H
#define GSL_LPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gsl_status {
  GSL_OK = 0,
  GSL_EINVAL = -1,    /* bad argument (size, range, NULL where not allowed) */
  GSL_ENOMEM = -2,    /* device allocation of scratch failed */
  GSL_EDEVICE = -3,   /* a HIP runtime call failed; see gsl_last_error() */
  GSL_EOVERFLOW = -4, /* a row's summed weight reaches 2^32 (see gsl_lpa) */
  GSL_EAGAIN = -5     /* no room in a session right now (see gsl_session_add) */
} gsl_status;

#define GSL_STATS_MAX_ITERS 64
#define GSL_STATS_TIERS 10

typedef struct gsl_options {
  int32_t prune;  /* nonzero (default 1): pruning, Alg. 3 -- only vertices with a
                     neighbour that changed in the previous sweep are processed.
                     Results are identical either way; it only saves work. */
  int32_t split;  /* nonzero (default 1): run the split pass (Alg. 2) after the
                     sweeps, as GSL-LPA does; 0 returns the raw LPA labels. */
  int32_t timing; /* nonzero: fill the ms_* fields of gsl_stats (records HIP
                     events between phases). */
  int32_t layout; /* 0 (default): automatic; 1: always sweep a degree-ordered
                     renumbered copy of the graph (hubs first), which packs
                     the labels of high-degree vertices together; 2: never.
                     The copy costs nnz * 4 (+ nnz * 4 with weights) bytes of
                     device memory.  Results are identical either way. */
  int32_t async_sweeps; /* nonzero: asynchronous sweeps as the paper's lpaMove
                     runs them (Alg. 3) -- a changed label is written in
                     place at once, so later vertices of the same sweep may
                     see it.  Results then depend on scheduling (not bit-exact
                     run to run); the split still leaves no disconnected
                     community.  Default 0: synchronous sweeps. */
} gsl_options;

typedef struct gsl_stats {
  int32_t iterations;                       /* sweeps performed */
  int32_t split_rounds;                     /* hook rounds of the split */
  int64_t changed[GSL_STATS_MAX_ITERS];     /* dN of each sweep (Alg. 3) */
  int64_t processed[GSL_STATS_MAX_ITERS];   /* vertices scanned in each sweep */
  int64_t edges[GSL_STATS_MAX_ITERS];       /* row entries scanned in each sweep */
  int64_t marked[GSL_STATS_MAX_ITERS];      /* 1 if the sweep marked neighbours */
  int64_t nnz;                              /* offsets[n] */
  int64_t max_degree;
  float ms_plan, ms_sweeps, ms_split, ms_total;
  float ms_sweep[GSL_STATS_MAX_ITERS];
  /* Per degree tier (index 0 = isolated vertices, 1..7 = the levels of the
   * tier table in order of increasing degree, 8 = hub rows, longer than the
   * last level's bound; index 9 is unused), summed over all sweeps of the
   * call. */
  int64_t tier_vertices[GSL_STATS_TIERS];   /* vertices in the tier */
  int64_t tier_launches[GSL_STATS_TIERS];   /* sweep kernel launches */
  int64_t tier_processed[GSL_STATS_TIERS];  /* vertices scanned */
  int64_t tier_edges[GSL_STATS_TIERS];      /* row entries scanned */
  int64_t tier_changed[GSL_STATS_TIERS];    /* vertices that changed label */
  int64_t tier_marked[GSL_STATS_TIERS];     /* neighbour flags written */
  int64_t tier_sparse[GSL_STATS_TIERS];     /* launches that scanned the tier against the active flags */
  int32_t renumbered;                       /* 1 if the sweeps ran on the renumbered copy */
  float ms_reorder;                         /* time to build that copy (timing != 0) */
  float ms_hub_finish;                      /* hub table scan, decision, marking */
  float ms_tier[GSL_STATS_TIERS];           /* kernel time (timing != 0) */
  /* Sparse sweeps after a sweep with few changes walk a frontier of the
   * active vertices instead of scanning the tier: */
  int64_t tier_frontier[GSL_STATS_TIERS];        /* such launches */
  int64_t tier_frontier_listed[GSL_STATS_TIERS]; /* frontier entries they walked */
} gsl_stats;

/*
 * gsl_lpa -- GSL-LPA (Alg. 3): label-propagation sweeps, then the split.
 *
 * Labels start as C[i] = i.  Each sweep gives every processed vertex i the
 * label c maximising sum_{j in row i, j != i, C[j] = c} w_ij (Eq. 2), the
 * smallest such label on ties; a vertex with no entry j != i keeps its label.
 * Sweeps are synchronous: all vertices read the labels of the previous sweep.
 * dN counts the vertices whose label changed; the loop stops after max_iters
 * sweeps or as soon as dN / n <= tolerance (evaluated exactly as that double
 * comparison).  Finally the split (Alg. 2) relabels every vertex with the
 * smallest vertex id of its connected piece inside its community, so no
 * output community is internally disconnected.
 *
 *   offsets, cols, weights, n : graph (see conventions); weights may be NULL
 *   max_iters  : MAX_ITERATIONS, >= 0
 *   tolerance  : tau, 0 <= tolerance <= 1
 *   labels_out : int32[n] device array receiving the labels
 *
 * Returns GSL_EOVERFLOW when some vertex's summed row weight is >= 2^32 (label
 * weights are summed exactly in 32-bit integers).  n == 0 is a no-op.
 */
int gsl_lpa(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
            int32_t max_iters, double tolerance, int32_t *labels_out);

/*
 * gsl_lpa_ex -- gsl_lpa with options (NULL: defaults {1, 1, 0, 0, 0}) and optional
 * statistics (stats may be NULL; per-sweep arrays hold the first
 * GSL_STATS_MAX_ITERS sweeps).
 */
int gsl_lpa_ex(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
               int32_t max_iters, double tolerance, const gsl_options *opt, gsl_stats *stats,
               int32_t *labels_out);

/*
 * gsl_lpa_noalloc -- gsl_lpa for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and the same labels as gsl_lpa, computed by
 * the same kernels (pruning on, split on, the graph's own vertex order), with
 * every scratch buffer carved from one static device array of
 * GSL_NOALLOC_SCRATCH_BYTES per device (its address is looked up once per
 * device, on the first call there; the array is held until the process ends).
 * The call allocates nothing: no hipMalloc, hipFree, host pinning, events or
 * graphs; it reads small results back through pageable host memory.
 *
 * Limits (GSL_EINVAL beyond them, before any device work): n at most
 * GSL_NOALLOC_MAX_VERTICES, max_iters at most GSL_NOALLOC_MAX_ITERS, at most
 * GSL_NOALLOC_MAX_HUBS rows above the last tier bound, and no such row longer
 * than 2^20 entries.  Every call on a device shares that device's array, and
 * each call leaves its contents behind (every buffer is re-initialised before
 * use).  Calls that overlapped on one device would race on it; the library
 * lock serialises the calls of one process and each process has its own
 * array.  gsl_set_tiers and gsl_set_hub_limits apply as for gsl_lpa.
 */
#define GSL_NOALLOC_MAX_VERTICES (1 << 20)
#define GSL_NOALLOC_MAX_ITERS 256
#define GSL_NOALLOC_MAX_HUBS 16384
#define GSL_NOALLOC_SCRATCH_BYTES (48 << 20)
int gsl_lpa_noalloc(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
                    int32_t max_iters, double tolerance, int32_t *labels_out);

/*
 * gsl_lpa_f32 -- gsl_lpa_ex with fp32 weights summed in fp64, the paper's
 * precision (Sec. 5.1.2).  weights: float[nnz] DEVICE array, every value
 * finite and >= 0 (else GSL_EINVAL), or NULL (unit weights, identical to
 * gsl_lpa_ex).  The label rule is unchanged: largest summed weight, smallest
 * label on ties.  Sums are formed with atomics in an order that varies, so a
 * sum may differ in its last bits from the entry-order sum when weights span
 * more than 2^29 in magnitude; only exact ties can then resolve differently
 * (results are bit-exact whenever every partial sum is exact in fp64, e.g.
 * weights that are multiples of a common power of two).  The degree tiers are
 * the defaults (gsl_set_tiers does not apply).
 */
int gsl_lpa_f32(const int64_t *offsets, const int32_t *cols, const float *weights, int64_t n, int32_t max_iters,
                double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *labels_out);

/*
 * gsl_split -- the split pass alone (Alg. 2; Alg. 1 reaches the same fixed
 * point): labels_out[i] = the smallest vertex id v such that v and i are joined
 * by a path whose vertices all carry label labels_in[i].
 *
 *   labels_in  : int32[n] device array, each value in [0, n)
 *   labels_out : int32[n] device array
 * Returns GSL_EINVAL if a label is outside [0, n).
 */
int gsl_split(const int64_t *offsets, const int32_t *cols, int64_t n, const int32_t *labels_in,
              int32_t *labels_out);

/*
 * gsl_split_ex -- gsl_split with a choice of technique.  All give the same
 * labels (the smallest vertex id of each connected piece of each community);
 * they differ in speed:
 *   GSL_SPLIT_UNION_FIND  lock-free union-find in Afforest edge order (what
 *                         gsl_split and gsl_lpa use);
 *   GSL_SPLIT_LP          Alg. 1: min-label propagation over intra-community
 *                         entries, every vertex every round, until no label
 *                         changes (rounds grow with the pieces' diameter);
 *   GSL_SPLIT_LPP         Alg. 1 with pruning: a vertex is processed only if
 *                         a same-community neighbour changed in the previous
 *                         round (frontier-driven, the GPU form of Alg. 2's
 *                         BFS).
 *   rounds_out : HOST, propagation rounds (1 for union-find); may be NULL
 *   ms_out     : HOST, device time of the split in ms; may be NULL
 */
#define GSL_SPLIT_UNION_FIND 0
#define GSL_SPLIT_LP 1
#define GSL_SPLIT_LPP 2
int gsl_split_ex(const int64_t *offsets, const int32_t *cols, int64_t n, const int32_t *labels_in,
                 int32_t *labels_out, int32_t technique, int32_t *rounds_out, float *ms_out);

/*
 * gsl_disconnected -- the disconnected-community check (Alg. 4): a community
 * (the vertices sharing one label) is disconnected when its vertices are not
 * all joined by paths whose vertices all carry that label.
 *
 *   labels    : int32[n] device array, each value in [0, n)
 *   flags_out : uint8[n] DEVICE array indexed by label: 1 if that community
 *               is disconnected, else 0 (labels no vertex carries get 0);
 *               may be NULL
 *   count_out : HOST pointer receiving the number of disconnected
 *               communities; may be NULL
 * Returns GSL_EINVAL if a label is outside [0, n).  After gsl_lpa with the
 * split the count is 0; on raw LPA labels (split = 0) it measures what the
 * split repairs.
 */
int gsl_disconnected(const int64_t *offsets, const int32_t *cols, int64_t n, const int32_t *labels,
                     uint8_t *flags_out, int64_t *count_out);

/*
 * gsl_modularity -- modularity Q of a labelling (Eq. 1, second form):
 *   Q = sum_c [ sigma_c / 2m - (Sigma_c / 2m)^2 ]
 * where sigma_c sums w over CSR entries (i, j) with C_i = C_j = c, Sigma_c
 * sums w over entries with C_i = c and 2m sums w over all entries.  The sums
 * are exact integers; Q = I/2m - S2/(2m)^2 with I = sum sigma_c and
 * S2 = sum Sigma_c^2 is evaluated once in IEEE double precision.  Q = 0 when
 * 2m = 0.
 *
 *   labels : int32[n] device array, each value in [0, n)
 *   q_out  : HOST pointer receiving Q
 */
int gsl_modularity(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
                   const int32_t *labels, double *q_out);

/*
 * gsl_lpa_batched -- GSL-LPA on a batch of independent graphs in one run.
 *
 * Every graph gets exactly the result gsl_lpa would give it alone: its own
 * sweeps, its own convergence test dN_g / n_g <= tolerance and its own sweep
 * count (a graph that has stopped takes no further part), then the split.
 * The batch is one concatenated CSR with LOCAL vertex ids:
 *
 *   num_graphs : G >= 0
 *   vtx_base   : int64[G+1]; graph g owns rows [vtx_base[g], vtx_base[g+1]),
 *                vtx_base[0] == 0, non-decreasing, N = vtx_base[G] < 2^31
 *   edge_base  : int64[G+1]; graph g owns entries [edge_base[g],
 *                edge_base[g+1]), edge_base[0] == 0, non-decreasing,
 *                edge_base[g] == offsets[vtx_base[g]]
 *   offsets    : int64[N+1], positions in the concatenated cols array
 *   cols       : int32[nnz], graph g's entries in [0, n_g) (local ids)
 *   weights    : uint32[nnz] or NULL (every weight 1)
 *   labels_out : int32[N]; graph g's labels (local ids) at vtx_base[g] ...
 *
 * Base arrays that do not start at 0, end at N and offsets[N], or decrease
 * give GSL_EINVAL (checked on the device).  The library builds a global-id
 * copy of cols (nnz * 4 bytes of scratch).
 */
int gsl_lpa_batched(int64_t num_graphs, const int64_t *vtx_base, const int64_t *edge_base,
                    const int64_t *offsets, const int32_t *cols, const uint32_t *weights,
                    int32_t max_iters, double tolerance, int32_t *labels_out);

/*
 * gsl_lpa_batched_ex -- gsl_lpa_batched with options (the layout field is
 * ignored: batches keep their vertex order), statistics of the whole batch
 * (iterations = the largest per-graph sweep count) and iterations_out, an
 * int32[G] DEVICE array receiving each graph's sweep count (may be NULL).
 */
int gsl_lpa_batched_ex(int64_t num_graphs, const int64_t *vtx_base, const int64_t *edge_base,
                       const int64_t *offsets, const int32_t *cols, const uint32_t *weights,
                       int32_t max_iters, double tolerance, const gsl_options *opt,
                       gsl_stats *stats, int32_t *labels_out, int32_t *iterations_out);

/* One graph of a batch of separate graphs; all pointers are device pointers.
 * Row v's entries are cols[offsets[v] .. offsets[v+1]) (offsets[0] need not
 * be 0), with local ids in [0, n). */
typedef struct gsl_graph {
  const int64_t *offsets;  /* int64[n+1] (may be NULL when n == 0) */
  const int32_t *cols;
  const uint32_t *weights; /* NULL: every weight 1 */
  int32_t *labels_out;     /* int32[n] */
  int64_t n;
} gsl_graph;

/* A context: scratch memory and a stream of its own (created non-blocking, at
 * default priority, on the current device). */
typedef struct gsl_context gsl_context;

int gsl_context_create(gsl_context **out);
/* Waits for the context's stream, frees its scratch (and its stream unless
 * one was set with gsl_context_set_stream). */
void gsl_context_destroy(gsl_context *ctx);
/* Use a caller-owned stream (hipStream_t) from now on. */
int gsl_context_set_stream(gsl_context *ctx, void *hip_stream);
/* The context's stream (hipStream_t). */
void *gsl_context_stream(gsl_context *ctx);

/*
 * gsl_lpa_graphs -- gsl_lpa_batched for G graphs held in separate arrays
 * (host array graphs[G] of descriptors), run in one batch on the context
 * (NULL: the shared per-device scratch and the gsl_set_stream stream).  The
 * library gathers the graphs into one global CSR (offsets, cols and, if any
 * graph has weights, weights: (N + 1) * 8 + nnz * 4 (* 2) bytes of scratch)
 * and writes each graph's labels to its labels_out.  Synchronous like every
 * call.
 *
 *   iterations_out : HOST int32[G], each graph's sweep count (may be NULL)
 *   status_out     : HOST int32[G] (may be NULL).  A graph whose offsets
 *                    decrease or whose cols leave [0, n) is checked on the
 *                    device while it is gathered; it gets GSL_EINVAL here,
 *                    its labels_out is left untouched, and the other graphs
 *                    still get their results.  With status_out == NULL such
 *                    a graph makes the call return GSL_EINVAL instead (the
 *                    other graphs' labels are still written).
 * A weight overflow (GSL_EOVERFLOW) fails the whole call.
 */
int gsl_lpa_graphs(gsl_context *ctx, int64_t num_graphs, const gsl_graph *graphs, int32_t max_iters,
                   double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *iterations_out,
                   int32_t *status_out);

/*
 * Sessions: continuous batching.  A session keeps a batch of graphs resident
 * on the device and runs their sweeps; graphs join it and leave it between
 * sweeps, so a graph submitted while others are running starts with the very
 * next sweep instead of waiting for a whole batch to drain.  Every graph gets
 * exactly what gsl_lpa would give it alone (its own sweeps, its own
 * convergence test dN_g / n_g <= tolerance and sweep count, then the split of
 * Alg. 2), whatever else shares the session and whenever it joined.
 *
 * A session owns a stream (non-blocking, default priority) and device memory
 * for at most max_vertices vertices and max_entries CSR entries of graphs
 * running at once (held twice, so that the graphs still running can be moved
 * together when finished graphs leave gaps) and max_graphs graphs.  Calls on
 * one session are serialised; calls on different sessions may overlap on the
 * device.
 */
typedef struct gsl_session gsl_session;

/* Device bytes a session of this capacity holds (an upper bound for the hub
 * tier's buffers, which grow with the hub rows present); -1 for a bad
 * capacity.  Host-only. */
int64_t gsl_session_bytes(int64_t max_vertices, int64_t max_entries, int32_t max_graphs, int32_t weighted);

/* New session on the current device.  weighted: graphs may carry uint32
 * weights (else every graph must pass NULL weights).  max_iters and
 * tolerance apply to every graph, as in gsl_lpa. */
int gsl_session_create(int64_t max_vertices, int64_t max_entries, int32_t max_graphs, int32_t max_iters,
                       double tolerance, int32_t weighted, gsl_session **out);
/* Waits for the session's stream and frees everything; unfinished graphs'
 * outputs are left untouched. */
void gsl_session_destroy(gsl_session *s);
/* The session's stream (hipStream_t). */
void *gsl_session_stream(gsl_session *s);

/*
 * gsl_session_add -- admits graphs (host array graphs[num_graphs] of device
 * descriptors, local ids, as for gsl_lpa_graphs) in order.  For each graph:
 *   status_out[g] = GSL_OK     admitted; tickets_out[g] names it in the
 *                              results of gsl_session_step (an empty graph
 *                              needs no sweep: ticket -1, nothing to write)
 *                   GSL_EAGAIN no room right now (vertices, entries or graph
 *                              slots of the session are taken): submit again
 *                              after a step has finished some graphs; every
 *                              later graph of the call gets GSL_EAGAIN too
 *                   GSL_EINVAL decreasing offsets, an entry outside [0, n),
 *                              weights in an unweighted session, or a graph
 *                              larger than the session could ever hold
 * The graph's arrays are copied into the session before the call returns;
 * the caller may reuse them at once, but labels_out must stay valid until
 * the graph's ticket has come back from gsl_session_step.
 */
int gsl_session_add(gsl_session *s, int64_t num_graphs, const gsl_graph *graphs, int64_t *tickets_out,
                    int32_t *status_out);

/*
 * gsl_session_step -- runs up to `sweeps` (1 .. 64) synchronous sweeps of
 * every graph in the session (Alg. 3, each graph on its own, as in
 * gsl_lpa_batched), then the split of every graph that has stopped, whose
 * labels (local ids) go to its labels_out.  Returns when that is done.
 *   done_tickets     : HOST int64[capacity], tickets of the graphs finished
 *                      by this call (at most capacity; others finish in a
 *                      later call)
 *   done_iterations  : HOST int32[capacity] (may be NULL), their sweep counts
 *   done_count       : HOST, how many were written
 * GSL_EOVERFLOW when a row's summed weight reaches 2^32; the session's
 * running graphs are then lost (destroy it).
 */
int gsl_session_step(gsl_session *s, int32_t sweeps, int64_t capacity, int64_t *done_tickets,
                     int32_t *done_iterations, int64_t *done_count);

/* Graphs running, their vertices and entries, free capacity, device bytes
 * held (any pointer may be NULL). */
int gsl_session_info(gsl_session *s, int64_t *live_graphs, int64_t *live_vertices, int64_t *live_entries,
                     int64_t *free_vertices, int64_t *free_entries, int64_t *device_bytes);

/*
 * gsl_graphs_bytes -- host-only: an upper bound of the device scratch that a
 * gsl_lpa_graphs call on `graphs` graphs with n vertices and nnz entries in
 * all (weighted or not, max_iters sweeps) adds to its context's cache (for a
 * server's memory budget); -1 for bad arguments.
 */
int64_t gsl_graphs_bytes(int64_t n, int64_t nnz, int64_t graphs, int32_t weighted, int32_t max_iters);

/*
 * gsl_check_graph -- checks a CSR on the device: offsets[0] == 0, offsets
 * non-decreasing, every column in [0, n).  Returns GSL_OK or GSL_EINVAL (the
 * message names the defect).  Symmetry is not checked.  Every other entry
 * point assumes these properties without checking them (except
 * gsl_lpa_graphs, above); a server that accepts graphs from elsewhere calls
 * this first.
 */
int gsl_check_graph(const int64_t *offsets, const int32_t *cols, int64_t n);

/*
 * gsl_convergence_limit -- host-only helper: the largest k in [0, n] with
 * (double)k / (double)n <= tolerance (0 for n == 0, -1 for a tolerance
 * outside [0, 1]).  The device loop stops when dN <= this limit, which is the
 * same test as dN / n <= tolerance (Alg. 3) because correctly rounded
 * division is monotone in k.
 */
int64_t gsl_convergence_limit(int64_t n, double tolerance);

/*
 * Degree tiers (the launch plan).  Vertices are bucketed by degree into
 * GSL_TIER_LEVELS levels plus degree 0 (never processed) and hubs (every
 * degree above the last level, processed chunk-wise).  Level l takes the
 * degrees (max_degree[l-1], max_degree[l]] and runs the sweep kernel
 * `variant`.  Variants differ in lanes per vertex, entries per lane, LDS
 * table size and workgroup size (gsl_tier_variant); a variant takes rows of
 * up to `capacity` entries; any variant may serve any level.  The choice
 * changes speed, never results.
 */
#define GSL_TIER_LEVELS 7
typedef struct gsl_tier {
  int32_t max_degree; /* non-decreasing over the levels, <= the variant's capacity */
  int32_t variant;
} gsl_tier;
typedef struct gsl_variant_info {
  int32_t group;      /* lanes per vertex (1: a thread per vertex) */
  int32_t table_log2; /* LDS table of 2^table_log2 slots per group */
  int32_t block;      /* threads per workgroup */
  int32_t per_lane;   /* row entries each lane holds */
  int32_t capacity;   /* largest degree: group * per_lane */
} gsl_variant_info;

/* Sets the tiers of all later calls in this process (levels[GSL_TIER_LEVELS];
 * NULL restores the defaults: bounds 32/64/128/512/1024/2048/4096 with
 * variants 16/6/8/9/17/11/13).  GSL_EINVAL for an
 * invalid table (nothing changes).  gsl_lpa_f32 always runs the bounds
 * 8/16/32/64/128/512/2048. */
int gsl_set_tiers(const gsl_tier *levels);
/* Current tiers into levels_out[GSL_TIER_LEVELS]. */
int gsl_get_tiers(gsl_tier *levels_out);
/* Shape of sweep variant `variant` (0 .. until GSL_EINVAL). */
int gsl_tier_variant(int32_t variant, gsl_variant_info *info);

/*
 * gsl_set_hub_limits -- limits of the hub tier (rows longer than the last
 * level's bound) for all later calls in this process.  Hub rows are summed
 * chunk by chunk into a staging area of (label, sum) records, one batch of
 * hubs at a time, and the records of each hash partition of a hub are then
 * merged in a 4,096-slot table; a partition with more distinct labels than
 * the table takes is merged again in 2, 4, ... hashed sub-passes.  Neither
 * limit changes results, only memory use and speed.
 *   staging_bytes : device bytes of staging per hub batch (a hub batch always
 *                   holds at least one hub); 0 restores the default 4 GiB,
 *                   else at least 16,384
 *   merge_claims  : distinct labels one merge pass accepts before the
 *                   partition is split into sub-passes, in [1, 3839];
 *                   0 restores the default 3839
 * GSL_EINVAL outside these ranges (nothing changes).
 */
int gsl_set_hub_limits(int64_t staging_bytes, int32_t merge_claims);

/* Stream for all subsequent calls of this process (a hipStream_t; NULL = the
 * null stream). */
int gsl_set_stream(void *hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char *gsl_last_error(void);

/* Frees the cached scratch memory of every device. */
void gsl_release(void);

/* Library version string. */
const char *gsl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSL_LPA_H */
