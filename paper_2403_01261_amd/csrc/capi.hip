// C ABI of libgsl_lpa.so (declared in include/gsl_lpa.h): argument checks,
// per-device scratch cache and the host loop that enqueues the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gsl_lpa.h"
#include "gsl_internal.h"

// Scratch of gsl_lpa_noalloc: one array per device, loaded with the code
// object and held until the process ends.  Host code never uses this name as
// an address (it is a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, in noalloc_setup.
static __device__ __align__(256) unsigned char scratch[GSL_NOALLOC_SCRATCH_BYTES];

namespace {

using gsl::Counters;

thread_local std::string g_err;
hipStream_t g_stream = nullptr;
std::mutex g_mu;
// Degree tiers used by every call (gsl_set_tiers); read once per call.
std::mutex g_tier_mu;
gsl::TierConfig g_tiers = gsl::kDefaultTiers;

// Hub tier limits (gsl_set_hub_limits): staging bytes per hub batch and
// merge-table claims before a partition is re-merged in sub-passes.
constexpr int64_t kDefaultHubStagingBytes = (int64_t)4 << 30;
struct HubLimits {
  int64_t staging_bytes = kDefaultHubStagingBytes;
  int32_t merge_cap = gsl::kHubMergeCapMax;
};
HubLimits g_hub_limits;

gsl::TierConfig current_tiers() {
  std::lock_guard<std::mutex> lk(g_tier_mu);
  return g_tiers;
}

HubLimits current_hub_limits() {
  std::lock_guard<std::mutex> lk(g_tier_mu);
  return g_hub_limits;
}

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return fail(GSL_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),      \
                  __FILE__, __LINE__);                                                     \
  } while (0)

// Scratch cached per device; grown on demand, freed by gsl_release().
struct Scratch {
  // Carved once from the no-alloc region (gsl_lpa_noalloc): every buffer is
  // preset at its largest size, so a call that needs more fails instead of
  // allocating.
  bool fixed = false;
  int64_t n_cap = -1;
  int32_t *Cn = nullptr;
  uint8_t *chg = nullptr;
  uint8_t *act[2] = {nullptr, nullptr};
  int32_t *list = nullptr;
  int32_t *parent = nullptr;
  int32_t *rep = nullptr;  // split: representative component per community
  int64_t *blk_counts = nullptr;
  unsigned long long *sigma = nullptr;
  unsigned long long *partials = nullptr;
  int partial_blocks = 0;
  unsigned long long *tier_part = nullptr;  // per-block count records of the tier kernels
  int64_t ctr_bytes = 0;
  Counters *ctr = nullptr;
  Counters *ctr_host = nullptr;  // pinned mirror (with the per-sweep arrays)
  // pinned staging for small device-to-host reads (a pageable destination
  // makes every copy a synchronous round trip): kPinSmall words, then the
  // hub layout
  int64_t *pin = nullptr;
  int64_t pin_cap = 0;
  // hub tier layout (prefix sums over the hubs of the current graph)
  int64_t hub_cap = 0;
  int64_t *hub_chunk_start = nullptr, *hub_part_start = nullptr, *hub_hist_start = nullptr;
  unsigned long long *hub_best = nullptr, *hub_rowsum = nullptr, *hub_records = nullptr;
  int32_t *hub_chunk_owner = nullptr, *hub_part_owner = nullptr;  // hub of every chunk / partition
  int64_t hub_chunk_owner_cap = 0, hub_part_owner_cap = 0;
  unsigned long long *hub_staging = nullptr;  // (label, sum) pairs of one batch
  int32_t *hub_hist = nullptr;                // partition bounds of one batch
  int64_t hub_staging_cap = 0, hub_hist_cap = 0;
  std::vector<int64_t> h_chunk, h_part, h_hist;  // host copies of the prefix sums
  std::vector<int> hub_max_parts;                // largest partition count per batch
  std::vector<std::pair<int64_t, int64_t>> hub_batches;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_reorder = nullptr;
  std::vector<hipEvent_t> pool;  // per-launch timing events
  // degree-ordered renumbered copy of the graph
  int32_t *old2new = nullptr, *lab2 = nullptr, *minorig = nullptr;
  unsigned long long *first_key = nullptr;
  int64_t *off2 = nullptr;
  int64_t copy_n_cap = -1, copy_nnz_cap = -1;
  int32_t *cols2 = nullptr;
  uint32_t *w2 = nullptr;
  bool w2_ok = false;
  // device loop state and the cached loop graph
  gsl::SweepCtrl *ctrl = nullptr;
  hipGraphExec_t loop_exec = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the loop graph is captured on
  std::vector<uint64_t> loop_key;
  // chunked loop launches: the stop flag after each chunk (pinned host
  // memory) and the events the host waits on
  int32_t *done_host = nullptr;
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  // batches: graph of every vertex, per-graph limits / counts / flags, the
  // base arrays and descriptors of separate graphs, and the global copy
  int64_t batch_n_cap = -1, batch_g_cap = -1;
  int32_t *gid = nullptr, *giters = nullptr;
  int64_t *glimit = nullptr, *gdn = nullptr;
  uint8_t *gdone = nullptr;
  int64_t *gvb = nullptr, *geb = nullptr, *gcnt = nullptr;
  gsl::GraphDesc *gdesc = nullptr;
  unsigned long long *gbad = nullptr;
  uint32_t *gflag = nullptr;  // per-graph: entry outside the graph's range
  // fp32 weights: global hub tables (keys, fp64 sums)
  uint32_t *fkeys = nullptr;
  double *fsums = nullptr;
  int64_t fslots_cap = -1;
  int32_t *glab = nullptr;
  int64_t *goff = nullptr;
  int64_t gcols_cap = -1, gw_cap = -1, goff_cap = -1, batch_glab_cap = -1;
  int32_t *gcols = nullptr;
  uint32_t *gw = nullptr;
};

}  // namespace

// A context: its own scratch and stream, so calls on different contexts (from
// different host threads) run concurrently on the device.
struct gsl_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::mutex mu;
  Scratch s;
};

namespace {
// One graph of a session (host side).
struct SessionSlot {
  bool live = false;
  int64_t ticket = -1;
  int64_t vb = 0, n = 0, eb = 0, nnz = 0, limit = 0;
  int32_t *labels_out = nullptr;
};
constexpr int kSessionSweepCap = 64;  // most sweeps one gsl_session_step runs
// Dead space a session keeps before it compacts at the start of a step.
constexpr int64_t kSessionCompactVertices = 1 << 16, kSessionCompactEntries = 1 << 20;
}  // namespace

// A session: a resident batch (the arena) that graphs join and leave between
// sweeps.  Every live graph owns a vertex range and an entry range of the
// arena, holds global ids there, and runs exactly the sweeps it would run
// alone; a finished graph's ranges stay as dead space (vertices of the dead
// slot, never processed) until a compaction moves the live graphs together.
struct gsl_session {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  Scratch s;
  int64_t cap_v = 0, cap_e = 0;
  int32_t cap_g = 0;
  int32_t max_iters = 20;
  double tol = 0.05;
  bool weighted = false;
  int cur = 0;  // arena buffer in use (the other is the compaction target)
  int64_t *off[2] = {nullptr, nullptr};
  int32_t *cols[2] = {nullptr, nullptr};
  uint32_t *w[2] = {nullptr, nullptr};
  int32_t *lab[2] = {nullptr, nullptr};
  int32_t *split_in = nullptr, *split_out = nullptr;
  uint8_t *sel = nullptr;             // [cap_g + 1] graphs finishing in this step
  gsl::SessionRange *ranges = nullptr;  // [cap_g] range records for the kernels
  int64_t vtop = 0, etop = 0;         // arena in use: [0, vtop) vertices, [0, etop) entries
  int64_t live_v = 0, live_e = 0;
  std::vector<SessionSlot> slot;
  std::vector<int32_t> free_slot;
  int64_t next_ticket = 0;
  bool dirty = true;                  // the arena changed since the last plan
  gsl::Counters plan{};
  gsl::SweepCtrl ctrl{};              // loop state carried from step to step
  int64_t bytes = 0;                  // device bytes allocated at creation
};

namespace {

// Returns event k of the pool, creating events on demand.
hipEvent_t pool_event(Scratch &s, size_t k) {
  while (s.pool.size() <= k) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s.pool.push_back(e);
  }
  return s.pool[k];
}

std::map<int, Scratch> g_scratch;

void free_scratch(Scratch &s) {
  hipFree(s.Cn);
  hipFree(s.chg);
  hipFree(s.act[0]);
  hipFree(s.act[1]);
  hipFree(s.list);
  hipFree(s.parent);
  hipFree(s.rep);
  hipFree(s.blk_counts);
  hipFree(s.sigma);
  hipFree(s.partials);
  hipFree(s.tier_part);
  hipFree(s.ctr);
  hipFree(s.hub_chunk_start);
  hipFree(s.hub_part_start);
  hipFree(s.hub_hist_start);
  hipFree(s.hub_best);
  hipFree(s.hub_rowsum);
  hipFree(s.hub_records);
  hipFree(s.hub_chunk_owner);
  hipFree(s.hub_part_owner);
  hipFree(s.hub_staging);
  hipFree(s.hub_hist);
  if (s.ctr_host) hipHostFree(s.ctr_host);
  if (s.pin) hipHostFree(s.pin);
  for (auto &e : s.ev)
    if (e) hipEventDestroy(e);
  for (auto &e : s.pool) hipEventDestroy(e);
  if (s.ev_reorder) hipEventDestroy(s.ev_reorder);
  if (s.loop_exec) hipGraphExecDestroy(s.loop_exec);
  if (s.cap_stream) hipStreamDestroy(s.cap_stream);
  if (s.done_host) hipHostFree(s.done_host);
  for (auto &e : s.chunk_ev)
    if (e) hipEventDestroy(e);
  hipFree(s.ctrl);
  hipFree(s.gid);
  hipFree(s.giters);
  hipFree(s.glimit);
  hipFree(s.gdn);
  hipFree(s.gdone);
  hipFree(s.gvb);
  hipFree(s.geb);
  hipFree(s.gcnt);
  hipFree(s.gdesc);
  hipFree(s.gbad);
  hipFree(s.gflag);
  hipFree(s.fkeys);
  hipFree(s.fsums);
  hipFree(s.glab);
  hipFree(s.goff);
  hipFree(s.gcols);
  hipFree(s.gw);
  hipFree(s.old2new);
  hipFree(s.lab2);
  hipFree(s.minorig);
  hipFree(s.first_key);
  hipFree(s.off2);
  hipFree(s.cols2);
  hipFree(s.w2);
  s = Scratch();
}

template <class T>
hipError_t dmalloc(T **p, int64_t count) {
  return hipMalloc(reinterpret_cast<void **>(p), (size_t)(count > 0 ? count : 1) * sizeof(T));
}

// Makes sure per-vertex scratch holds n vertices and the counters block holds
// max_iters sweeps.
// Loop graphs of graphs with at least kChunkMinEntries row entries hold
// kChunkSweeps sweeps and are launched chunk by chunk (see lpa_impl).
constexpr int64_t kChunkMinEntries = int64_t(1) << 23;
constexpr int kChunkSweeps = 2;
// Most kernel launches one captured loop graph holds.  Every hub batch adds
// four launches to a sweep, so many hubs over a small staging area make wide
// sweeps: a 20-sweep graph of about 2 * 10^5 chained launches has ended the
// process inside the call where one of 4 * 10^4 ran.  Wider loops capture
// fewer sweeps per graph, and a sweep wider than this is launched directly.
constexpr int64_t kMaxGraphLaunches = 1 << 14;
// Fewest vertices of a sweep that walks a frontier in its sparse sweeps.
constexpr int64_t kFrontierMinVertices = int64_t(1) << 20;

int ensure_scratch(Scratch &s, int64_t n, int32_t max_iters) {
  const int64_t need = (int64_t)sizeof(Counters) + 4 * (int64_t)sizeof(uint64_t) * (max_iters > 0 ? max_iters : 1);
  if (s.fixed) {
    if (n > s.n_cap || need > s.ctr_bytes)
      return fail(GSL_EINVAL, "%lld vertices / %d sweeps exceed the no-alloc scratch", (long long)n, max_iters);
    return GSL_OK;
  }
  if (n > s.n_cap) {
    const int64_t cap = n;
    hipFree(s.Cn);
    hipFree(s.chg);
    hipFree(s.act[0]);
    hipFree(s.act[1]);
    hipFree(s.list);
    hipFree(s.parent);
    hipFree(s.rep);
    hipFree(s.blk_counts);
    hipFree(s.sigma);
    s.Cn = nullptr; s.chg = nullptr; s.act[0] = s.act[1] = nullptr; s.list = nullptr;
    s.parent = nullptr; s.rep = nullptr; s.blk_counts = nullptr; s.sigma = nullptr;
    s.n_cap = -1;
    const int64_t flag_bytes = (cap + 3) / 4 * 4 + 16;
    if (dmalloc(&s.Cn, cap) != hipSuccess || dmalloc(&s.chg, flag_bytes) != hipSuccess ||
        dmalloc(&s.act[0], flag_bytes) != hipSuccess || dmalloc(&s.act[1], flag_bytes) != hipSuccess ||
        dmalloc(&s.list, cap) != hipSuccess || dmalloc(&s.parent, cap) != hipSuccess ||
        dmalloc(&s.rep, cap) != hipSuccess ||
        dmalloc(&s.blk_counts, gsl::plan_scratch(cap)) != hipSuccess ||
        dmalloc(&s.sigma, cap) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "device allocation of scratch for %lld vertices failed", (long long)n);
    }
    s.n_cap = cap;
  }
  if (!s.partials) {
    s.partial_blocks = 4096;
    if (dmalloc(&s.partials, 2 * (int64_t)s.partial_blocks) != hipSuccess ||
        dmalloc(&s.tier_part, (int64_t)gsl::kNumTiers * gsl::kMaxTierGrid * gsl::kCountFields) != hipSuccess)
      return fail(GSL_ENOMEM, "device allocation failed");
  }
  if (!s.ctrl && dmalloc(&s.ctrl, 1) != hipSuccess) return fail(GSL_ENOMEM, "device allocation failed");
  if (need > s.ctr_bytes) {
    hipFree(s.ctr);
    if (s.ctr_host) hipHostFree(s.ctr_host);
    s.ctr = nullptr;
    s.ctr_host = nullptr;
    s.ctr_bytes = 0;
    if (hipMalloc(reinterpret_cast<void **>(&s.ctr), (size_t)need) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&s.ctr_host), (size_t)need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "counter allocation failed");
    }
    s.ctr_bytes = need;
  }
  return GSL_OK;
}

// The phase events (timing mode, split timing).
int ensure_events(Scratch &s) {
  if (!s.ev[0])
    for (auto &e : s.ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(GSL_EDEVICE, "hipEventCreate failed");
  return GSL_OK;
}


unsigned long long *sweep_array(Counters *c, int which, int32_t max_iters) {
  auto *base = reinterpret_cast<unsigned long long *>(c + 1);
  return base + (size_t)which * (size_t)(max_iters > 0 ? max_iters : 1);
}

int get_scratch(Scratch **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  *out = &g_scratch[dev];
  return GSL_OK;
}

bool bad_tolerance(double t) { return !(t >= 0.0 && t <= 1.0); }

constexpr int64_t kPinSmall = 16;  // words of Scratch::pin before the hub layout

// Pinned host staging of at least `words` int64 words.
int ensure_pinned(Scratch &s, int64_t words) {
  if (words <= s.pin_cap) return GSL_OK;
  if (s.fixed) return fail(GSL_EINVAL, "the graph has more hub rows than the no-alloc scratch holds");
  if (s.pin) hipHostFree(s.pin);
  s.pin = nullptr;
  s.pin_cap = 0;
  const int64_t cap = words < 4096 ? 4096 : words;
  if (hipHostMalloc(reinterpret_cast<void **>(&s.pin), (size_t)cap * sizeof(int64_t), hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipGetLastError();
    s.pin = nullptr;
    return fail(GSL_ENOMEM, "pinned host allocation failed");
  }
  s.pin_cap = cap;
  return GSL_OK;
}

// Reads offsets[0] and offsets[n]; checks offsets[0] == 0 and nnz >= 0.
int read_nnz(const int64_t *offsets, int64_t n, int64_t *nnz, hipStream_t st) {
  int64_t ends[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&ends[1], offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ends[0] != 0) return fail(GSL_EINVAL, "offsets[0] must be 0 (got %lld)", (long long)ends[0]);
  if (ends[1] < 0) return fail(GSL_EINVAL, "offsets[n] must be >= 0");
  *nnz = ends[1];
  return GSL_OK;
}

// Runs the degree plan and copies the counters block to the host mirror;
// with `ends` (2 words of pinned host memory) also offsets[0] and offsets[n],
// in the same round trip.  The plan reads offsets only, so it may run before
// they are validated.
int run_plan(Scratch &s, const int64_t *offsets, int64_t n, const gsl::TierConfig &cfg, hipStream_t st,
             int64_t *ends = nullptr) {
  HIP_TRY(gsl::launch_fill_u64(reinterpret_cast<uint64_t *>(s.ctr), 0, s.ctr_bytes / 8, st));
  HIP_TRY(gsl::launch_plan(offsets, n, s.list, s.blk_counts, s.ctr, cfg, st));
  HIP_TRY(hipMemcpyAsync(s.ctr_host, s.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  if (ends) {
    HIP_TRY(hipMemcpyAsync(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&ends[1], offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return GSL_OK;
}

// Builds the hub layout of the current graph and splits the hubs into
// batches whose staging area fits kHubStagingBytes (at least one hub each).
int prepare_hubs(Scratch &s, const int64_t *offsets, const int32_t *hubs, int64_t H, int64_t staging_bytes,
                 hipStream_t st) {
  s.hub_batches.clear();
  if (H <= 0) return GSL_OK;
  if (H > s.hub_cap) {
    if (s.fixed) return fail(GSL_EINVAL, "%lld hub rows exceed the no-alloc scratch", (long long)H);
    hipFree(s.hub_chunk_start);
    hipFree(s.hub_part_start);
    hipFree(s.hub_hist_start);
    hipFree(s.hub_best);
    hipFree(s.hub_rowsum);
    hipFree(s.hub_records);
    s.hub_chunk_start = s.hub_part_start = s.hub_hist_start = nullptr;
    s.hub_best = s.hub_rowsum = s.hub_records = nullptr;
    s.hub_cap = 0;
    if (dmalloc(&s.hub_chunk_start, H + 1) != hipSuccess || dmalloc(&s.hub_part_start, H + 1) != hipSuccess ||
        dmalloc(&s.hub_hist_start, H + 1) != hipSuccess || dmalloc(&s.hub_best, H) != hipSuccess ||
        dmalloc(&s.hub_rowsum, H) != hipSuccess || dmalloc(&s.hub_records, H) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "hub layout allocation failed");
    }
    s.hub_cap = H;
  }
  HIP_TRY(gsl::launch_fill_u64(reinterpret_cast<uint64_t *>(s.hub_best), 0, H, st));
  HIP_TRY(gsl::launch_fill_u64(reinterpret_cast<uint64_t *>(s.hub_rowsum), 0, H, st));
  gsl::HubLayout L{s.hub_chunk_start, s.hub_part_start, s.hub_hist_start, nullptr, nullptr, s.hub_records};
  HIP_TRY(gsl::launch_hub_layout(offsets, hubs, H, L, st));
  int rc = ensure_pinned(s, kPinSmall + 3 * (H + 1));
  if (rc) return rc;
  int64_t *ph = s.pin + kPinSmall;
  HIP_TRY(hipMemcpyAsync(ph, s.hub_chunk_start, (size_t)(H + 1) * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(ph + (H + 1), s.hub_part_start, (size_t)(H + 1) * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(ph + 2 * (H + 1), s.hub_hist_start, (size_t)(H + 1) * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  s.h_chunk.assign(ph, ph + (H + 1));
  s.h_part.assign(ph + (H + 1), ph + 2 * (H + 1));
  s.h_hist.assign(ph + 2 * (H + 1), ph + 3 * (H + 1));
  // the hub of every chunk and partition (one load in the kernels instead of
  // a binary search over the hubs)
  const int64_t total_chunks = s.h_chunk[(size_t)H], total_parts = s.h_part[(size_t)H];
  if (total_chunks > s.hub_chunk_owner_cap || total_parts > s.hub_part_owner_cap) {
    if (s.fixed) return fail(GSL_EINVAL, "%lld hub chunks exceed the no-alloc scratch", (long long)total_chunks);
    hipFree(s.hub_chunk_owner);
    hipFree(s.hub_part_owner);
    s.hub_chunk_owner = s.hub_part_owner = nullptr;
    s.hub_chunk_owner_cap = s.hub_part_owner_cap = 0;
    if (dmalloc(&s.hub_chunk_owner, total_chunks) != hipSuccess || dmalloc(&s.hub_part_owner, total_parts) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "hub owner allocation failed");
    }
    s.hub_chunk_owner_cap = total_chunks;
    s.hub_part_owner_cap = total_parts;
  }
  L.chunk_owner = s.hub_chunk_owner;
  L.part_owner = s.hub_part_owner;
  HIP_TRY(gsl::launch_hub_owners(L, H, st));
  const int64_t chunk_cap = staging_bytes / ((int64_t)gsl::kHubChunk * 8);
  int64_t k0 = 0;
  for (int64_t k = 0; k < H; ++k) {
    if (k > k0 && s.h_chunk[(size_t)k + 1] - s.h_chunk[(size_t)k0] > chunk_cap) {
      s.hub_batches.push_back({k0, k});
      k0 = k;
    }
  }
  s.hub_batches.push_back({k0, H});
  s.hub_max_parts.clear();
  for (auto &bt : s.hub_batches) {
    int64_t m = 1;
    for (int64_t k = bt.first; k < bt.second; ++k) {
      const int64_t P = s.h_part[(size_t)k + 1] - s.h_part[(size_t)k];
      m = P > m ? P : m;
    }
    s.hub_max_parts.push_back((int)m);
  }
  int64_t need_chunks = 0, need_hist = 0;
  for (auto &bt : s.hub_batches) {
    const int64_t c = s.h_chunk[(size_t)bt.second] - s.h_chunk[(size_t)bt.first];
    const int64_t h = s.h_hist[(size_t)bt.second] - s.h_hist[(size_t)bt.first];
    need_chunks = c > need_chunks ? c : need_chunks;
    need_hist = h > need_hist ? h : need_hist;
  }
  const int64_t need_staging = need_chunks * gsl::kHubChunk;
  if (s.fixed && (need_staging > s.hub_staging_cap || need_hist > s.hub_hist_cap))
    return fail(GSL_EINVAL, "a hub row of %lld chunks exceeds the no-alloc staging area", (long long)need_chunks);
  if (need_staging > s.hub_staging_cap) {
    hipFree(s.hub_staging);
    s.hub_staging = nullptr;
    s.hub_staging_cap = 0;
    if (dmalloc(&s.hub_staging, need_staging) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "hub staging allocation (%lld pairs) failed", (long long)need_staging);
    }
    s.hub_staging_cap = need_staging;
  }
  if (need_hist > s.hub_hist_cap) {
    hipFree(s.hub_hist);
    s.hub_hist = nullptr;
    s.hub_hist_cap = 0;
    if (dmalloc(&s.hub_hist, need_hist) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "hub partition records allocation failed");
    }
    s.hub_hist_cap = need_hist;
  }
  return GSL_OK;
}

// Space for the renumbered copy: n vertices, nnz entries (weights if asked).
int ensure_copy(Scratch &s, int64_t n, int64_t nnz, bool weighted) {
  if (n > s.copy_n_cap) {
    hipFree(s.old2new);
    hipFree(s.lab2);
    hipFree(s.minorig);
    hipFree(s.first_key);
    hipFree(s.off2);
    s.old2new = s.lab2 = s.minorig = nullptr;
    s.first_key = nullptr;
    s.off2 = nullptr;
    s.copy_n_cap = -1;
    if (dmalloc(&s.old2new, n) != hipSuccess || dmalloc(&s.lab2, n) != hipSuccess ||
        dmalloc(&s.minorig, n) != hipSuccess || dmalloc(&s.off2, n + 1) != hipSuccess ||
        dmalloc(&s.first_key, n) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "allocation of the renumbered copy (%lld vertices) failed", (long long)n);
    }
    s.copy_n_cap = n;
  }
  if (nnz > s.copy_nnz_cap || (weighted && !s.w2_ok)) {
    hipFree(s.cols2);
    hipFree(s.w2);
    s.cols2 = nullptr;
    s.w2 = nullptr;
    s.w2_ok = false;
    s.copy_nnz_cap = -1;
    const int64_t cap = nnz > s.copy_nnz_cap ? nnz : s.copy_nnz_cap;
    if (dmalloc(&s.cols2, cap) != hipSuccess || (weighted && dmalloc(&s.w2, cap) != hipSuccess)) {
      (void)hipGetLastError();
      hipFree(s.cols2);
      s.cols2 = nullptr;
      return fail(GSL_ENOMEM, "allocation of the renumbered copy (%lld entries) failed", (long long)nnz);
    }
    s.copy_nnz_cap = cap;
    s.w2_ok = weighted;
  }
  return GSL_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// A batch of independent graphs laid out as one graph with global ids (see
// gsl_lpa_batched); NULL for a single graph.
struct Batch {
  int64_t graphs;
  const int64_t *vtx_base;         // device [graphs + 1]
  int32_t *iters_dev;              // per-graph sweep counts out (device) or NULL
  int32_t *iters_host;             // per-graph sweep counts out (host) or NULL
  const gsl::GraphDesc *scatter;   // separate graphs: descriptors of the outputs, else NULL
  const uint32_t *flags;           // separate graphs: per-graph bad-entry flags (device)
  uint32_t *flags_host;            // copy of those flags (host) or NULL
};

// One timing record: an event pair around a launch of tier `tier` in sweep
// `sweep` (kind 0: the tier kernel, 1: the hub finishing kernels).
struct Launch {
  int tier, sweep, kind;
  size_t ev;
};

// f32: `weights` holds fp32 values (summed in fp64) instead of uint32.
int lpa_impl(Scratch &s, hipStream_t st, const int64_t *offsets, const int32_t *cols, const uint32_t *weights,
             int64_t n, int32_t max_iters, double tolerance, const gsl_options *opt, gsl_stats *stats,
             int32_t *labels_out, const Batch *batch = nullptr, bool f32 = false) {
  gsl_options o = {1, 1, 0, 0, 0};
  if (opt) o = *opt;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n = %lld out of range", (long long)n);
  if (max_iters < 0) return fail(GSL_EINVAL, "max_iters must be >= 0");
  if (bad_tolerance(tolerance)) return fail(GSL_EINVAL, "tolerance must be in [0, 1]");
  if (n == 0) return GSL_OK;
  if (!offsets || !labels_out) return fail(GSL_EINVAL, "offsets and labels_out must not be NULL");
  int rc = GSL_OK;
  if ((rc = ensure_pinned(s, kPinSmall))) return rc;
  if ((rc = ensure_scratch(s, n, max_iters))) return rc;
  // fp32 weights run fixed tiers (their kernels are instantiated for those
  // bounds only)
  const gsl::TierConfig cfg = f32 ? gsl::kF32Tiers : current_tiers();
  const HubLimits hub_lim = current_hub_limits();
  if (o.timing) {
    if (s.fixed) return fail(GSL_EINVAL, "timing is not available without allocation");
    if ((rc = ensure_events(s))) return rc;
    HIP_TRY(hipEventRecord(s.ev[0], st));
  }
  if ((rc = run_plan(s, offsets, n, cfg, st, s.pin))) return rc;
  if (s.pin[0] != 0) return fail(GSL_EINVAL, "offsets[0] must be 0 (got %lld)", (long long)s.pin[0]);
  if (s.pin[1] < 0) return fail(GSL_EINVAL, "offsets[n] must be >= 0");
  const int64_t nnz = s.pin[1];
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when offsets[n] > 0");
  Counters plan = *s.ctr_host;
  // Tier t is the id range [tier_start[t], +tier_count[t]) of s.list; hubs
  // (tier 8) come first, isolated vertices (tier 0) last.
  const int64_t H = plan.tier_count[gsl::kHubTier];
  // the fixed scratch keeps every staging batch within its staging area
  const int64_t staging_bytes = s.fixed ? std::min<int64_t>(hub_lim.staging_bytes, s.hub_staging_cap * 8)
                                        : hub_lim.staging_bytes;
  if ((rc = prepare_hubs(s, offsets, s.list, H, staging_bytes, st))) return rc;
  // Renumbered layout: chosen when vertices of degree > 64 hold most entries
  // (their labels are the usual gather targets).  Batches keep their layout
  // (per-graph vertex ranges).
  int64_t heavy = 0;  // entries of the tiers whose rows all have degree > 64
  for (int t = 1; t < gsl::kNumTiers; ++t)
    if (cfg.bound[t - 1] >= 64) heavy += plan.tier_edges[t];
  const bool renumber = !batch && (o.layout == 1 || (o.layout == 0 && 2 * heavy > nnz));
  const int64_t np = n - plan.tier_count[0];  // non-isolated vertices
  const int64_t *g_off = offsets;
  const int32_t *g_cols = cols;
  const uint32_t *g_w = weights;
  const int32_t *g_list = s.list;
  int32_t *C = labels_out;
  int64_t n_sweep = n;
  unsigned long long *dn_arr = sweep_array(s.ctr, 0, max_iters);
  unsigned long long *pr_arr = sweep_array(s.ctr, 1, max_iters);
  unsigned long long *ed_arr = sweep_array(s.ctr, 2, max_iters);
  unsigned long long *mk_arr = sweep_array(s.ctr, 3, max_iters);
  if (renumber) {
    if ((rc = ensure_copy(s, n, nnz, weights != nullptr))) return rc;
    if (o.timing) {
      if (!s.ev_reorder && hipEventCreate(&s.ev_reorder) != hipSuccess)
        return fail(GSL_EDEVICE, "hipEventCreate failed");
      HIP_TRY(hipEventRecord(s.ev_reorder, st));
    }
    HIP_TRY(gsl::launch_reorder(offsets, cols, weights, n, s.list, plan.tier_count, plan.tier_start,
                                s.hub_chunk_start, s.hub_chunk_owner, H > 0 ? s.h_chunk[(size_t)H] : 0, s.old2new, s.off2,
                                s.cols2, weights ? s.w2 : nullptr, s.lab2, s.blk_counts, s.first_key,
                                s.hub_rowsum, reinterpret_cast<unsigned long long *>(&s.ctr->first_flags),
                                dn_arr, max_iters > 0 ? 1 : 0, cfg, st));
    g_off = s.off2;
    g_cols = s.cols2;
    g_w = weights ? s.w2 : nullptr;
    g_list = nullptr;
    C = s.lab2;
    n_sweep = np;
  } else {
    HIP_TRY(gsl::launch_init_labels(C, s.Cn, n, st));
  }
  const int64_t flag_bytes = (n + 3) / 4 * 4;
  HIP_TRY(gsl::launch_fill_u8(s.chg, 0, flag_bytes, st));
  HIP_TRY(gsl::launch_fill_u8(s.act[0], 0, flag_bytes, st));
  HIP_TRY(gsl::launch_fill_u8(s.act[1], 0, flag_bytes, st));
  // Loop state on the device; the renumbered layout may have run sweep 0.
  gsl::SweepCtrl hc;
  memset(&hc, 0, sizeof(hc));
  hc.max_iters = max_iters;
  hc.graph_max_iters = max_iters;
  hc.prune = o.prune ? 1 : 0;
  hc.limit = gsl_convergence_limit(n, tolerance);
  hc.n = n;
  hc.graphs = batch ? batch->graphs : 0;
  HIP_TRY(hipMemcpyAsync(s.ctrl, &hc, sizeof(hc), hipMemcpyHostToDevice, st));
  HIP_TRY(gsl::launch_loop_init(
      s.ctrl, renumber ? reinterpret_cast<const unsigned long long *>(&s.ctr->first_flags) : nullptr, dn_arr,
      mk_arr, f32 ? 0 : 1, st));
  if (f32 && H > 0) {
    const int64_t slots = gsl::hub_f32_slots(s.h_chunk[(size_t)H]);
    if (slots > s.fslots_cap) {
      hipFree(s.fkeys);
      hipFree(s.fsums);
      s.fkeys = nullptr;
      s.fsums = nullptr;
      s.fslots_cap = -1;
      if (dmalloc(&s.fkeys, slots) != hipSuccess || dmalloc(&s.fsums, slots) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GSL_ENOMEM, "hub table allocation (%lld slots) failed", (long long)slots);
      }
      s.fslots_cap = slots;
    }
    HIP_TRY(gsl::launch_hub_f32_clear(s.fkeys, s.fsums, slots, st));
  }
  if (batch)
    HIP_TRY(gsl::launch_batch_init(batch->vtx_base, batch->graphs, max_iters, tolerance, s.gid, s.glimit,
                                   s.giters, s.gdone, s.gdn, st));
  if (o.timing) HIP_TRY(hipEventRecord(s.ev[1], st));

  gsl::SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.off = g_off;
  a.cols = g_cols;
  a.w = g_w;
  a.C = C;
  a.Cn = s.Cn;
  a.chg = s.chg;
  a.act0 = s.act[0];
  a.act1 = s.act[1];
  a.ctrl = s.ctrl;
  a.dn = dn_arr;
  a.processed = pr_arr;
  a.edges = ed_arr;
  a.marked_sweeps = mk_arr;
  a.overflow = reinterpret_cast<unsigned long long *>(&s.ctr->overflow);
  a.gid = batch ? s.gid : nullptr;
  a.gdone = batch ? s.gdone : nullptr;
  a.inplace = o.async_sweeps ? 1 : 0;
  a.n = n;
  // Sparse sweeps walk a frontier of the active vertices per tier, built at
  // the start of the sweep into the split's parent array (unused until the
  // split) with the counts in the counters block; fp32 weights keep the scan,
  // and so do graphs under kFrontierMinVertices, whose flag scan costs less
  // than the build's launch in every sweep (a loop of 4,096 calls on graphs
  // of ~29K vertices: 2.59 s without, 2.89 s with it).
  const bool frontier = o.prune && !f32 && n_sweep >= kFrontierMinVertices;
  a.flist = frontier ? s.parent : nullptr;
  const gsl::HubLayout L{s.hub_chunk_start, s.hub_part_start, s.hub_hist_start, s.hub_chunk_owner,
                         s.hub_part_owner, s.hub_records};

  // Timing records (timing mode only).
  std::vector<Launch> launches;
  std::vector<size_t> sweep_ev;
  size_t nev = 0;
  auto rec = [&](size_t k) -> int {
    hipEvent_t e = pool_event(s, k);
    if (!e) return fail(GSL_EDEVICE, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(e, st));
    return GSL_OK;
  };
  const bool timed = o.timing != 0;

  // Enqueues one sweep; every kernel checks the device loop state, so a sweep
  // enqueued after convergence costs only empty launches.
  hipStream_t cur = st;  // stream the sweeps are enqueued on
  auto enqueue_sweep = [&](int k) -> int {
    if (timed) {
      sweep_ev.push_back(nev);
      if ((rc = rec(nev++))) return rc;
    }
    gsl::TierGrids grids;
    for (int t = 0; t < gsl::kNumTiers; ++t) grids.g[t] = 0;
    if (frontier)
      HIP_TRY(gsl::launch_frontier(a, n_sweep, cfg, plan.tier_start, s.parent, s.ctr->fcount, cur));
    for (int t = 1; t < gsl::kNumTiers; ++t) {
      const int64_t cnt = plan.tier_count[t];
      if (cnt <= 0) continue;
      a.tier = &s.ctr->tier_stats[t][0];
      a.part = s.tier_part + (size_t)t * gsl::kMaxTierGrid * gsl::kCountFields;
      a.fcount = frontier && t != gsl::kHubTier ? &s.ctr->fcount[t] : nullptr;
      if (timed) {
        launches.push_back({t, k, 0, nev});
        if ((rc = rec(nev++))) return rc;
      }
      if (t == gsl::kHubTier && f32) {
        HIP_TRY(gsl::launch_hub_f32(a, g_list, s.hub_chunk_start, cnt, s.h_chunk[(size_t)cnt], s.fkeys, s.fsums,
                                    cur));
      } else if (t == gsl::kHubTier) {
        for (size_t bi = 0; bi < s.hub_batches.size(); ++bi) {
          const auto &bt = s.hub_batches[bi];
          for (int stage = 0; stage < 2; ++stage) {
            if (timed && (bi > 0 || stage > 0)) {
              launches.push_back({t, k, stage, nev});
              if ((rc = rec(nev++))) return rc;
            }
            HIP_TRY(gsl::launch_hub_sweep(a, g_list, L, s.h_chunk.data(), s.h_part.data(), s.hub_staging,
                                          s.hub_hist, s.hub_best, s.hub_rowsum, bt.first, bt.second,
                                          s.hub_max_parts[bi], hub_lim.merge_cap, stage, cur));
          }
        }
      } else {
        if (f32)
          HIP_TRY(gsl::launch_sweep_tier_f32(t, a, g_list, plan.tier_start[t], cnt, &grids.g[t], cur));
        else
          HIP_TRY(gsl::launch_sweep_tier(cfg.variant[t], a, g_list, plan.tier_start[t], cnt, &grids.g[t], cur));
      }
      if (timed && (rc = rec(nev++))) return rc;
    }
    HIP_TRY(gsl::launch_reduce_counts(s.tier_part, grids, s.ctr->tier_stats, s.ctrl, dn_arr, pr_arr, ed_arr,
                                      a.overflow, cur));
    HIP_TRY(gsl::launch_apply(a, C, n_sweep, batch ? s.gdn : nullptr, cur));
    if (batch)
      HIP_TRY(gsl::launch_graph_end(s.ctrl, s.gdn, s.glimit, s.giters, s.gdone, batch->graphs, cur));
    HIP_TRY(gsl::launch_sweep_end(s.ctrl, dn_arr, mk_arr, a.overflow, cur, frontier ? s.ctr->fcount : nullptr,
                                  s.ctr->ftotal));
    if (timed && (rc = rec(nev++))) return rc;
    return GSL_OK;
  };

  // launches of one sweep, at most: one per tier, four per hub batch, the
  // closing kernels
  const int64_t sweep_launches = gsl::kNumTiers + 4 * (int64_t)s.hub_batches.size() + 8;
  if (timed || max_iters == 0) {
    for (int k = 0; k < max_iters; ++k)
      if ((rc = enqueue_sweep(k))) return rc;
  } else if (s.fixed || sweep_launches > kMaxGraphLaunches) {
    // Without allocation there is no loop graph (instantiating one
    // allocates), nor for a sweep too wide for one: the sweeps are enqueued
    // directly, and the loop state is read back after every kChunkSweeps
    // sweeps to stop early.
    for (int k = 0; k < max_iters; ++k) {
      if ((rc = enqueue_sweep(k))) return rc;
      if ((k + 1) % kChunkSweeps == 0 && k + 1 < max_iters) {
        int32_t done = 0;
        HIP_TRY(hipMemcpyAsync(&done, &s.ctrl->done, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (done) break;
      }
    }
  } else {
    // The loop as a captured graph, reused while every pointer and size it
    // was built from stays the same.  Small graphs: all max_iters sweeps in
    // one graph (a sweep enqueued after convergence costs only empty
    // launches, a few microseconds each).  Large graphs: a graph of
    // kChunkSweeps sweeps (wide sweeps: as many as kMaxGraphLaunches
    // allows) launched repeatedly; the host queues chunk c before
    // it waits for the stop flag after chunk c - 1, so the device never waits
    // for the host and at most one chunk runs after the loop has stopped
    // (every sweep kernel reads the same device loop state, so the chunks
    // are identical).
    int len = nnz >= kChunkMinEntries && max_iters > kChunkSweeps ? kChunkSweeps : max_iters;
    if ((int64_t)len * sweep_launches > kMaxGraphLaunches) len = (int)(kMaxGraphLaunches / sweep_launches);
    const bool chunked = len < max_iters;
    std::vector<uint64_t> key = {(uint64_t)len, (uint64_t)n, (uint64_t)n_sweep, (uint64_t)nnz, (uint64_t)max_iters,
                                 (uint64_t)o.prune, (uint64_t)renumber, (uint64_t)a.inplace, (uint64_t)f32,
                                 (uint64_t)(uintptr_t)s.fkeys, (uint64_t)(uintptr_t)s.fsums,
                                 (uint64_t)(uintptr_t)g_off, (uint64_t)(uintptr_t)g_cols,
                                 (uint64_t)(uintptr_t)g_w, (uint64_t)(uintptr_t)C, (uint64_t)(uintptr_t)g_list,
                                 (uint64_t)(uintptr_t)s.Cn, (uint64_t)(uintptr_t)s.chg,
                                 (uint64_t)(uintptr_t)s.act[0], (uint64_t)(uintptr_t)s.act[1],
                                 (uint64_t)(uintptr_t)s.ctr, (uint64_t)(uintptr_t)s.ctrl,
                                 (uint64_t)(uintptr_t)s.tier_part, (uint64_t)(uintptr_t)s.hub_staging,
                                 (uint64_t)(uintptr_t)s.hub_hist, (uint64_t)(uintptr_t)s.hub_best,
                                 (uint64_t)(uintptr_t)s.hub_rowsum, (uint64_t)(uintptr_t)s.hub_chunk_start,
                                 (uint64_t)(uintptr_t)s.hub_part_start, (uint64_t)(uintptr_t)s.hub_hist_start,
                                 (uint64_t)(uintptr_t)s.hub_chunk_owner, (uint64_t)(uintptr_t)s.hub_part_owner,
                                 (uint64_t)(uintptr_t)s.hub_records,
                                 (uint64_t)(uintptr_t)(batch ? batch->vtx_base : nullptr),
                                 (uint64_t)(batch ? batch->graphs : 0), (uint64_t)(uintptr_t)s.gid,
                                 (uint64_t)(uintptr_t)s.gdn, (uint64_t)(uintptr_t)s.glimit,
                                 (uint64_t)(uintptr_t)s.giters, (uint64_t)(uintptr_t)s.gdone};
    for (int t = 0; t < gsl::kNumTiers; ++t) {
      key.push_back((uint64_t)plan.tier_count[t]);
      key.push_back((uint64_t)plan.tier_start[t]);
      key.push_back((uint64_t)cfg.variant[t]);
    }
    // Hub launches bake in their grid sizes (chunks and partitions of each
    // batch, all chunks for fp32 weights) and dynamic LDS (largest partition
    // count), so those totals belong to the key as well.
    key.push_back((uint64_t)hub_lim.merge_cap);
    key.push_back((uint64_t)(H > 0 ? s.h_chunk[(size_t)H] : 0));
    for (size_t bi = 0; bi < s.hub_batches.size(); ++bi) {
      const auto &bt = s.hub_batches[bi];
      key.push_back((uint64_t)bt.first);
      key.push_back((uint64_t)bt.second);
      key.push_back((uint64_t)s.hub_max_parts[bi]);
      key.push_back((uint64_t)(s.h_chunk[(size_t)bt.second] - s.h_chunk[(size_t)bt.first]));
      key.push_back((uint64_t)(s.h_part[(size_t)bt.second] - s.h_part[(size_t)bt.first]));
    }
    if (!s.loop_exec || key != s.loop_key) {
      // The previous graph's launches have finished: every call ends with a
      // stream synchronisation, except one that failed while launching;
      // synchronise here so that an exec is never destroyed in flight.
      if (s.loop_exec) {
        HIP_TRY(hipStreamSynchronize(st));
        hipGraphExecDestroy(s.loop_exec);
      }
      s.loop_exec = nullptr;
      s.loop_key.clear();
      // Captured on a private stream (the caller's may be the null stream,
      // which cannot be captured); launched on the caller's stream.
      if (!s.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking));
      const hipStream_t user_st = st;
      cur = s.cap_stream;
      HIP_TRY(hipStreamBeginCapture(cur, hipStreamCaptureModeThreadLocal));
      int crc = GSL_OK;
      for (int k = 0; k < len && crc == GSL_OK; ++k) crc = enqueue_sweep(k);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(cur, &graph);
      cur = user_st;
      if (crc != GSL_OK) {
        if (graph) hipGraphDestroy(graph);
        return crc;
      }
      if (ec != hipSuccess) return fail(GSL_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&s.loop_exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        s.loop_exec = nullptr;
        return fail(GSL_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
      }
      s.loop_key = key;
    }
    if (!chunked) {
      HIP_TRY(hipGraphLaunch(s.loop_exec, st));
    } else {
      if (!s.done_host) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&s.done_host), 2 * sizeof(int32_t)));
        for (auto &e : s.chunk_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      }
      const int chunks = (max_iters + len - 1) / len;  // sweeps past max_iters are empty
      for (int c = 0; c < chunks; ++c) {
        HIP_TRY(hipGraphLaunch(s.loop_exec, st));
        HIP_TRY(hipMemcpyAsync(&s.done_host[c & 1], &s.ctrl->done, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(s.chunk_ev[c & 1], st));
        if (c > 0) {
          HIP_TRY(hipEventSynchronize(s.chunk_ev[(c - 1) & 1]));
          if (s.done_host[(c - 1) & 1]) break;
        }
      }
    }
  }
  if (timed) HIP_TRY(hipEventRecord(s.ev[2], st));
  if (renumber) {
    if (o.split)
      HIP_TRY(gsl::launch_split(g_off, g_cols, np, C, s.parent, labels_out, nullptr, plan.tier_count,
                                plan.tier_start, s.list, s.minorig, n, s.rep, s.sigma, cfg, st));
    else
      HIP_TRY(gsl::launch_reorder_scatter(s.list, C, np, n, labels_out, st));
  } else if (o.split) {
    HIP_TRY(gsl::launch_split(offsets, cols, n, C, s.parent, labels_out, s.list, plan.tier_count,
                              plan.tier_start, nullptr, nullptr, n, s.rep, s.sigma, cfg, st));
  }
  if (batch) {
    HIP_TRY(gsl::launch_localize(labels_out, batch->vtx_base, batch->graphs, n, st));
    if (batch->scatter)
      HIP_TRY(gsl::launch_scatter_labels(batch->scatter, labels_out, batch->vtx_base, batch->flags,
                                         batch->graphs, n, st));
    if (batch->flags_host)
      HIP_TRY(hipMemcpyAsync(batch->flags_host, batch->flags, (size_t)batch->graphs * sizeof(uint32_t),
                             hipMemcpyDeviceToHost, st));
    if (batch->iters_dev)
      HIP_TRY(hipMemcpyAsync(batch->iters_dev, s.giters, (size_t)batch->graphs * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, st));
    if (batch->iters_host)
      HIP_TRY(hipMemcpyAsync(batch->iters_host, s.giters, (size_t)batch->graphs * sizeof(int32_t),
                             hipMemcpyDeviceToHost, st));
  }
  if (timed) HIP_TRY(hipEventRecord(s.ev[3], st));
  static_assert(sizeof(gsl::SweepCtrl) <= (kPinSmall - 2) * sizeof(int64_t), "loop state fits the pinned words");
  gsl::SweepCtrl *pfc = reinterpret_cast<gsl::SweepCtrl *>(s.pin + 2);
  HIP_TRY(hipMemcpyAsync(pfc, s.ctrl, sizeof(gsl::SweepCtrl), hipMemcpyDeviceToHost, st));
  if (stats) HIP_TRY(hipMemcpyAsync(s.ctr_host, s.ctr, (size_t)s.ctr_bytes, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const gsl::SweepCtrl fc = *pfc;
  if (fc.error)
    return fail(GSL_EOVERFLOW, "a vertex's summed row weight reaches 2^32; weights are summed in 32 bits");
  const int32_t it = fc.it;
  if (stats) {
    // Sweep 0 ran inside the renumbering copy when the loop started at 1.
    const unsigned long long ff = s.ctr_host->first_flags;
    const bool fused_first = renumber && max_iters > 0 && !(ff & 1ull);
    const int first_kernel_sweep = fused_first ? 1 : 0;
    stats->iterations = it;
    stats->split_rounds = o.split ? 1 : 0;
    stats->nnz = nnz;
    stats->max_degree = (int64_t)plan.max_degree;
    const unsigned long long *hd = sweep_array(s.ctr_host, 0, max_iters);
    const unsigned long long *hp = sweep_array(s.ctr_host, 1, max_iters);
    const unsigned long long *he = sweep_array(s.ctr_host, 2, max_iters);
    const unsigned long long *hm = sweep_array(s.ctr_host, 3, max_iters);
    for (int k = 0; k < it && k < GSL_STATS_MAX_ITERS; ++k) {
      stats->changed[k] = (int64_t)hd[k];
      stats->processed[k] = (int64_t)hp[k];
      stats->edges[k] = (int64_t)he[k];
      stats->marked[k] = (int64_t)hm[k];
    }
    if (fused_first && it > 0) {
      stats->processed[0] = np;
      stats->edges[0] = nnz;
    }
    for (int t = 0; t < gsl::kNumTiers; ++t) {
      stats->tier_vertices[t] = plan.tier_count[t];
      stats->tier_processed[t] = (int64_t)s.ctr_host->tier_stats[t][0];
      stats->tier_edges[t] = (int64_t)s.ctr_host->tier_stats[t][1];
      stats->tier_changed[t] = (int64_t)s.ctr_host->tier_stats[t][2];
      stats->tier_marked[t] = (int64_t)s.ctr_host->tier_stats[t][3];
      if (t == 0 || plan.tier_count[t] <= 0) continue;
      for (int k = first_kernel_sweep; k < it; ++k) {
        stats->tier_launches[t] += 1;
        const bool sparse = k > 0 && o.prune && hm[k - 1];
        // the loop state's rule: after a sweep with at most n/16 changes
        const bool front = sparse && frontier && t != gsl::kHubTier && (int64_t)hd[k - 1] * 16 <= n;
        stats->tier_sparse[t] += sparse && !front ? 1 : 0;
        stats->tier_frontier[t] += front ? 1 : 0;
      }
      stats->tier_frontier_listed[t] = s.ctr_host->ftotal[t];
    }
    stats->renumbered = renumber ? 1 : 0;
    if (timed) {
      if (renumber) stats->ms_reorder = elapsed(s.ev_reorder, s.ev[1]);
      stats->ms_plan = elapsed(s.ev[0], s.ev[1]);
      stats->ms_sweeps = elapsed(s.ev[1], s.ev[2]);
      stats->ms_split = elapsed(s.ev[2], s.ev[3]);
      stats->ms_total = elapsed(s.ev[0], s.ev[3]);
      // Only sweeps that ran count: enqueued sweep e is sweep e +
      // first_kernel_sweep of the loop.  A record spans its event to the next
      // one.  Hub finishing kernels (kind 1) go to ms_hub_finish.
      const int ran = it - first_kernel_sweep;
      for (const Launch &l : launches) {
        if (l.sweep >= ran) continue;
        const float ms = elapsed(s.pool[l.ev], s.pool[l.ev + 1]);
        if (l.kind == 1)
          stats->ms_hub_finish += ms;
        else
          stats->ms_tier[l.tier] += ms;
      }
      for (int k = first_kernel_sweep; k < it && k < GSL_STATS_MAX_ITERS; ++k) {
        const int e = k - first_kernel_sweep;
        if (e >= (int)sweep_ev.size()) break;
        const size_t end = e + 1 < (int)sweep_ev.size() ? sweep_ev[(size_t)e + 1] - 1 : nev - 1;
        stats->ms_sweep[k] = elapsed(s.pool[sweep_ev[(size_t)e]], s.pool[end]);
      }
    }
  }
  return GSL_OK;
}

int check_labels(Scratch &s, const int32_t *labels, int64_t n, hipStream_t st) {
  HIP_TRY(hipMemsetAsync(&s.ctr->bad_label, 0, sizeof(uint64_t), st));
  HIP_TRY(gsl::launch_check_labels(labels, n, reinterpret_cast<unsigned long long *>(&s.ctr->bad_label), st));
  uint64_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, &s.ctr->bad_label, sizeof(bad), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad) return fail(GSL_EINVAL, "a label is outside [0, n)");
  return GSL_OK;
}

// ---- gsl_lpa_noalloc: every buffer carved from the static scratch ----
constexpr int64_t kNoAllocPlanEntries =
    ((GSL_NOALLOC_MAX_VERTICES + 1023) / 1024 + ((GSL_NOALLOC_MAX_VERTICES + 1023) / 1024 + 1023) / 1024) *
    gsl::kNumTiers;
constexpr int64_t kNoAllocStagingPairs = (int64_t)1 << 20;  // 512 chunks: hub rows up to 2^20 entries
constexpr int64_t kNoAllocStagingChunks = kNoAllocStagingPairs / gsl::kHubChunk;
// Partition records of one staging batch: sum over its hubs of chunks * (partitions + 1), partitions == chunks.
constexpr int64_t kNoAllocHistEntries = kNoAllocStagingChunks * (kNoAllocStagingChunks + 1);
constexpr int64_t kNoAllocHubChunks = (int64_t)1 << 16;  // hub rows of up to 2^27 entries in all
constexpr int64_t kNoAllocCtrBytes =
    (int64_t)sizeof(Counters) + 4 * (int64_t)sizeof(uint64_t) * GSL_NOALLOC_MAX_ITERS;

// Bytes of every buffer, each rounded up to 256: the carve order of
// noalloc_setup.
constexpr int64_t al256(int64_t b) { return (b + 255) / 256 * 256; }
constexpr int64_t kNoAllocFlagBytes = (GSL_NOALLOC_MAX_VERTICES + 3) / 4 * 4 + 16;
constexpr int64_t kNoAllocLayoutBytes =
    al256(sizeof(gsl::SweepCtrl)) + al256(kNoAllocCtrBytes) +
    al256((int64_t)gsl::kNumTiers * gsl::kMaxTierGrid * gsl::kCountFields * 8) +
    al256(4LL * GSL_NOALLOC_MAX_VERTICES) + 3 * al256(kNoAllocFlagBytes) +   // Cn, chg, act[2]
    3 * al256(4LL * GSL_NOALLOC_MAX_VERTICES) +                              // list, parent, rep
    al256(8LL * GSL_NOALLOC_MAX_VERTICES) + al256(8 * kNoAllocPlanEntries) +  // sigma, plan counts
    3 * al256(8LL * (GSL_NOALLOC_MAX_HUBS + 1)) + 3 * al256(8LL * GSL_NOALLOC_MAX_HUBS) +
    2 * al256(4 * kNoAllocHubChunks) +
    al256(8 * kNoAllocStagingPairs) + al256(4 * kNoAllocHistEntries);
static_assert(kNoAllocLayoutBytes <= GSL_NOALLOC_SCRATCH_BYTES, "the no-alloc buffers fit the static scratch");

struct NoAlloc {
  bool ready = false;
  Scratch s;
  std::vector<int64_t> pin;      // host words for small reads (pageable: nothing is allocated per call)
  std::vector<uint64_t> ctr_host;  // host mirror of the counters
};
std::map<int, NoAlloc> g_noalloc;

// Once per device, with that device current: the array's device address,
// every buffer carved from it at its largest size, host mirrors sized.
int noalloc_setup(NoAlloc &na) {
  unsigned char *base = nullptr;
  const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&base), HIP_SYMBOL(scratch));
  if (e != hipSuccess || !base)
    return fail(GSL_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  int64_t used = 0;
  auto carve = [&](auto **p, int64_t bytes) {
    *p = reinterpret_cast<std::remove_pointer_t<decltype(p)>>(base + used);
    used += al256(bytes);
  };
  Scratch &s = na.s;
  s.fixed = true;
  carve(&s.ctrl, sizeof(gsl::SweepCtrl));
  carve(&s.ctr, kNoAllocCtrBytes);
  s.ctr_bytes = kNoAllocCtrBytes;
  carve(&s.tier_part, (int64_t)gsl::kNumTiers * gsl::kMaxTierGrid * gsl::kCountFields * 8);
  carve(&s.Cn, 4LL * GSL_NOALLOC_MAX_VERTICES);
  carve(&s.chg, kNoAllocFlagBytes);
  carve(&s.act[0], kNoAllocFlagBytes);
  carve(&s.act[1], kNoAllocFlagBytes);
  carve(&s.list, 4LL * GSL_NOALLOC_MAX_VERTICES);
  carve(&s.parent, 4LL * GSL_NOALLOC_MAX_VERTICES);
  carve(&s.rep, 4LL * GSL_NOALLOC_MAX_VERTICES);
  carve(&s.sigma, 8LL * GSL_NOALLOC_MAX_VERTICES);
  carve(&s.blk_counts, 8 * kNoAllocPlanEntries);
  s.n_cap = GSL_NOALLOC_MAX_VERTICES;
  carve(&s.hub_chunk_start, 8LL * (GSL_NOALLOC_MAX_HUBS + 1));
  carve(&s.hub_part_start, 8LL * (GSL_NOALLOC_MAX_HUBS + 1));
  carve(&s.hub_hist_start, 8LL * (GSL_NOALLOC_MAX_HUBS + 1));
  carve(&s.hub_best, 8LL * GSL_NOALLOC_MAX_HUBS);
  carve(&s.hub_rowsum, 8LL * GSL_NOALLOC_MAX_HUBS);
  carve(&s.hub_records, 8LL * GSL_NOALLOC_MAX_HUBS);
  s.hub_cap = GSL_NOALLOC_MAX_HUBS;
  carve(&s.hub_chunk_owner, 4 * kNoAllocHubChunks);
  carve(&s.hub_part_owner, 4 * kNoAllocHubChunks);
  s.hub_chunk_owner_cap = s.hub_part_owner_cap = kNoAllocHubChunks;
  carve(&s.hub_staging, 8 * kNoAllocStagingPairs);
  s.hub_staging_cap = kNoAllocStagingPairs;
  carve(&s.hub_hist, 4 * kNoAllocHistEntries);
  s.hub_hist_cap = kNoAllocHistEntries;
  if (used != kNoAllocLayoutBytes) return fail(GSL_EDEVICE, "no-alloc layout mismatch");
  // host side: pageable mirrors, and room for the hub layout vectors
  na.pin.assign((size_t)(kPinSmall + 3 * (GSL_NOALLOC_MAX_HUBS + 1)), 0);
  s.pin = na.pin.data();
  s.pin_cap = (int64_t)na.pin.size();
  na.ctr_host.assign((size_t)(kNoAllocCtrBytes / 8), 0);
  s.ctr_host = reinterpret_cast<Counters *>(na.ctr_host.data());
  s.h_chunk.reserve(GSL_NOALLOC_MAX_HUBS + 1);
  s.h_part.reserve(GSL_NOALLOC_MAX_HUBS + 1);
  s.h_hist.reserve(GSL_NOALLOC_MAX_HUBS + 1);
  s.hub_max_parts.reserve(GSL_NOALLOC_MAX_HUBS);
  s.hub_batches.reserve(GSL_NOALLOC_MAX_HUBS);
  na.ready = true;
  return GSL_OK;
}

// Host-only argument checks, run before any HIP call.  Return GSL_OK to go
// on, kNoop when the call has nothing to do, or an error status.
constexpr int kNoop = 1;

int check_lpa(int64_t n, int32_t max_iters, double tolerance, const int64_t *offsets, const int32_t *labels_out) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n = %lld out of range", (long long)n);
  if (max_iters < 0) return fail(GSL_EINVAL, "max_iters must be >= 0");
  if (bad_tolerance(tolerance)) return fail(GSL_EINVAL, "tolerance must be in [0, 1]");
  if (n == 0) return kNoop;
  if (!offsets || !labels_out) return fail(GSL_EINVAL, "offsets and labels_out must not be NULL");
  return GSL_OK;
}

int check_batch(int64_t G, int32_t max_iters, double tolerance) {
  if (G < 0 || G >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "num_graphs out of range");
  if (max_iters < 0) return fail(GSL_EINVAL, "max_iters must be >= 0");
  if (bad_tolerance(tolerance)) return fail(GSL_EINVAL, "tolerance must be in [0, 1]");
  return G == 0 ? kNoop : GSL_OK;
}

// Per-graph arrays of a batch: N vertices, G graphs.
int ensure_batch(Scratch &s, int64_t N, int64_t G) {
  if (N > s.batch_n_cap) {
    hipFree(s.gid);
    s.gid = nullptr;
    s.batch_n_cap = -1;
    if (dmalloc(&s.gid, N) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "batch allocation (%lld vertices) failed", (long long)N);
    }
    s.batch_n_cap = N;
  }
  if (G > s.batch_g_cap) {
    hipFree(s.giters);
    hipFree(s.glimit);
    hipFree(s.gdn);
    hipFree(s.gdone);
    hipFree(s.gvb);
    hipFree(s.geb);
    hipFree(s.gcnt);
    hipFree(s.gdesc);
    hipFree(s.gflag);
    s.giters = nullptr; s.glimit = nullptr; s.gdn = nullptr; s.gdone = nullptr;
    s.gvb = nullptr; s.geb = nullptr; s.gcnt = nullptr; s.gdesc = nullptr; s.gflag = nullptr;
    s.batch_g_cap = -1;
    if (dmalloc(&s.giters, G) != hipSuccess || dmalloc(&s.glimit, G) != hipSuccess ||
        dmalloc(&s.gdn, G) != hipSuccess || dmalloc(&s.gdone, G) != hipSuccess ||
        dmalloc(&s.gvb, G + 1) != hipSuccess || dmalloc(&s.geb, G + 1) != hipSuccess ||
        dmalloc(&s.gcnt, G) != hipSuccess || dmalloc(&s.gdesc, G) != hipSuccess ||
        dmalloc(&s.gflag, G) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSL_ENOMEM, "batch allocation (%lld graphs) failed", (long long)G);
    }
    s.batch_g_cap = G;
  }
  if (!s.gbad && dmalloc(&s.gbad, 1) != hipSuccess) return fail(GSL_ENOMEM, "device allocation failed");
  return GSL_OK;
}

template <class T>
int ensure_array(T **p, int64_t *cap, int64_t count, const char *what) {
  if (count <= *cap) return GSL_OK;
  hipFree(*p);
  *p = nullptr;
  *cap = -1;
  if (dmalloc(p, count) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GSL_ENOMEM, "allocation of %s (%lld elements) failed", what, (long long)count);
  }
  *cap = count;
  return GSL_OK;
}

// Batch as concatenated CSR: offsets index the concatenated cols (global
// entry positions), cols hold local ids.
int batched_concat(Scratch &s, hipStream_t st, int64_t G, const int64_t *vtx_base, const int64_t *edge_base,
                   const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int32_t max_iters,
                   double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *labels_out,
                   int32_t *iters_out) {
  if (stats) memset(stats, 0, sizeof(*stats));
  if (G < 0 || G >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "num_graphs out of range");
  if (max_iters < 0) return fail(GSL_EINVAL, "max_iters must be >= 0");
  if (bad_tolerance(tolerance)) return fail(GSL_EINVAL, "tolerance must be in [0, 1]");
  if (G == 0) return GSL_OK;
  if (!vtx_base || !edge_base || !offsets) return fail(GSL_EINVAL, "NULL argument");
  int64_t ends[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&ends[0], vtx_base + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&ends[1], edge_base + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t N = ends[0], nnz = ends[1];
  if (N < 0 || N >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "total vertex count %lld out of range", (long long)N);
  if (nnz < 0) return fail(GSL_EINVAL, "edge_base[num_graphs] must be >= 0");
  if (N == 0) {
    if (iters_out) HIP_TRY(hipMemsetAsync(iters_out, 0, (size_t)G * sizeof(int32_t), st));
    HIP_TRY(hipStreamSynchronize(st));
    return GSL_OK;
  }
  if (!labels_out) return fail(GSL_EINVAL, "labels_out must not be NULL");
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when entries exist");
  int64_t total = 0;
  int rc = read_nnz(offsets, N, &total, st);
  if (rc) return rc;
  if (total != nnz) return fail(GSL_EINVAL, "offsets[N] (%lld) differs from edge_base[num_graphs] (%lld)",
                                (long long)total, (long long)nnz);
  if ((rc = ensure_batch(s, N, G))) return rc;
  unsigned long long bad = 0;
  HIP_TRY(hipMemsetAsync(s.gbad, 0, sizeof(unsigned long long), st));
  HIP_TRY(gsl::launch_check_bases(vtx_base, edge_base, G, N, nnz, s.gbad, st));
  HIP_TRY(hipMemcpyAsync(&bad, s.gbad, sizeof(bad), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad) return fail(GSL_EINVAL, "vtx_base / edge_base must start at 0, end at the totals and not decrease");
  if ((rc = ensure_array(&s.gcols, &s.gcols_cap, nnz, "global cols"))) return rc;
  HIP_TRY(gsl::launch_globalize_cols(cols, edge_base, vtx_base, G, nnz, s.gcols, st));
  gsl_options o = {1, 1, 0, 0, 0};
  if (opt) o = *opt;
  o.layout = 2;
  const Batch b{G, vtx_base, iters_out, nullptr, nullptr, nullptr, nullptr};
  return lpa_impl(s, st, offsets, s.gcols, weights, N, max_iters, tolerance, &o, stats, labels_out, &b);
}

// Batch of separate graphs (host array of descriptors).  A graph whose
// offsets decrease or whose entries leave [0, n) gets status GSL_EINVAL and
// keeps its output untouched; the others run as usual.
int batched_graphs(Scratch &s, hipStream_t st, int64_t G, const gsl_graph *graphs, int32_t max_iters,
                   double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *iters_out,
                   int32_t *status_out) {
  static_assert(sizeof(gsl_graph) == sizeof(gsl::GraphDesc), "gsl_graph layout");
  int rc = ensure_batch(s, 1, G);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(s.gdesc, graphs, (size_t)G * sizeof(gsl_graph), hipMemcpyHostToDevice, st));
  HIP_TRY(gsl::launch_graph_entries(s.gdesc, G, s.gcnt, st));
  std::vector<int64_t> cnt((size_t)G);
  HIP_TRY(hipMemcpyAsync(cnt.data(), s.gcnt, (size_t)G * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // Graphs with decreasing offsets are left out (no vertices in the batch).
  std::vector<int64_t> vb((size_t)G + 1, 0), eb((size_t)G + 1, 0);
  std::vector<int32_t> status((size_t)G, GSL_OK);
  bool weighted = false;
  for (int64_t g = 0; g < G; ++g) {
    const gsl_graph &x = graphs[g];
    int64_t n = x.n, c = cnt[(size_t)g];
    if (c < 0 || (c > 0 && !x.cols)) {
      status[(size_t)g] = GSL_EINVAL;
      n = 0;
      c = 0;
    }
    vb[(size_t)g + 1] = vb[(size_t)g] + n;
    eb[(size_t)g + 1] = eb[(size_t)g] + c;
    weighted = weighted || (x.weights != nullptr && c > 0);
  }
  const int64_t N = vb[(size_t)G], nnz = eb[(size_t)G];
  std::vector<uint32_t> flags((size_t)G, 0);
  if (iters_out) memset(iters_out, 0, (size_t)G * sizeof(int32_t));
  if (N > 0) {
    if ((rc = ensure_batch(s, N, G))) return rc;
    HIP_TRY(hipMemcpyAsync(s.gvb, vb.data(), (size_t)(G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s.geb, eb.data(), (size_t)(G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(s.gflag, 0, (size_t)G * sizeof(uint32_t), st));
    if ((rc = ensure_array(&s.goff, &s.goff_cap, N + 1, "global offsets"))) return rc;
    if ((rc = ensure_array(&s.gcols, &s.gcols_cap, nnz, "global cols"))) return rc;
    if (weighted && (rc = ensure_array(&s.gw, &s.gw_cap, nnz, "global weights"))) return rc;
    if ((rc = ensure_array(&s.glab, &s.batch_glab_cap, N, "batch labels"))) return rc;
    HIP_TRY(gsl::launch_gather(s.gdesc, s.gvb, s.geb, G, N, nnz, 0, 0, s.goff, s.gcols, weighted ? s.gw : nullptr,
                               s.gflag, st));
    gsl_options o = {1, 1, 0, 0, 0};
    if (opt) o = *opt;
    o.layout = 2;
    const Batch b{G, s.gvb, nullptr, iters_out, s.gdesc, s.gflag, flags.data()};
    rc = lpa_impl(s, st, s.goff, s.gcols, weighted ? s.gw : nullptr, N, max_iters, tolerance, &o, stats, s.glab,
                  &b);
    if (rc) return rc;
  }
  bool any_bad = false;
  for (int64_t g = 0; g < G; ++g) {
    if (flags[(size_t)g]) status[(size_t)g] = GSL_EINVAL;
    if (status[(size_t)g] != GSL_OK) {
      any_bad = true;
      if (iters_out) iters_out[g] = 0;
    }
  }
  if (status_out) {
    memcpy(status_out, status.data(), (size_t)G * sizeof(int32_t));
    return GSL_OK;
  }
  return any_bad ? fail(GSL_EINVAL, "a graph of the batch has decreasing offsets or an entry outside [0, n)")
                 : GSL_OK;
}

// One graph: offsets start at 0 and never decrease, cols in [0, n).
int check_graph_impl(Scratch &s, hipStream_t st, const int64_t *offsets, const int32_t *cols, int64_t n) {
  int64_t nnz = 0;
  int64_t ends[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&ends[1], offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ends[0] != 0) return fail(GSL_EINVAL, "offsets[0] must be 0");
  if (ends[1] < 0) return fail(GSL_EINVAL, "offsets[n] must be >= 0");
  nnz = ends[1];
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when offsets[n] > 0");
  int rc = ensure_batch(s, 1, 1);
  if (rc) return rc;
  unsigned long long bad = 0;
  HIP_TRY(hipMemsetAsync(s.gbad, 0, sizeof(unsigned long long), st));
  HIP_TRY(gsl::launch_check_graph(offsets, cols, n, nnz, s.gbad, st));
  HIP_TRY(hipMemcpyAsync(&bad, s.gbad, sizeof(bad), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad & 1) return fail(GSL_EINVAL, "offsets decrease");
  if (bad & 2) return fail(GSL_EINVAL, "a column index is outside [0, n)");
  return GSL_OK;
}

// Bound of the hub tier's buffers for nnz entries: at most one hub per
// 4,097 entries (H + 1 prefix entries and three records each), at most
// nnz / kHubChunk + H chunks C, partition owners no more than chunks, a
// staging batch of min(C, staging limit) chunks or the largest hub's chunks
// (a batch holds at least one hub), and per chunk of a batch one partition
// histogram of P + 1 counts, P <= min(largest hub's chunks, kHubMaxParts).
int64_t hub_bytes_bound(int64_t nnz) {
  const int64_t hubs = nnz / 4097 + 1, chunks = nnz / gsl::kHubChunk + hubs;
  const int64_t widest = nnz / gsl::kHubChunk + 1;  // chunks of the largest possible hub
  const int64_t limit = current_hub_limits().staging_bytes / ((int64_t)gsl::kHubChunk * 8);
  const int64_t batch = std::min<int64_t>(chunks, std::max<int64_t>(limit, widest));
  const int64_t P = std::min<int64_t>(widest, gsl::kHubMaxParts);
  return hubs * (3 * 8 + 3 * 8) + 2 * chunks * 4 + batch * gsl::kHubChunk * 8 + batch * (P + 1) * 4;
}

// Device scratch a gsl_lpa_graphs call on a batch of `graphs` graphs with n
// vertices and nnz entries in all grows the cache to (an upper bound: the
// per-vertex arrays, the gathered global CSR and labels, the per-graph
// arrays, the counters for max_iters sweeps and the hub-tier bound).
int64_t graphs_bytes(int64_t n, int64_t nnz, int64_t graphs, bool weighted, int32_t max_iters) {
  const int64_t G = graphs + 1;
  const int64_t flag = (n + 3) / 4 * 4 + 16;
  int64_t b = n * (4 + 4 + 4 + 4 + 8) + 3 * flag + gsl::plan_scratch(n) * 8;   // Cn list parent rep sigma, flags, plan
  b += 2 * 4096 * 8 + (int64_t)gsl::kNumTiers * gsl::kMaxTierGrid * gsl::kCountFields * 8;
  b += (int64_t)sizeof(Counters) + 4 * 8 * (int64_t)(max_iters > 0 ? max_iters : 1) + (int64_t)sizeof(gsl::SweepCtrl);
  b += n * 4 + G * (4 + 8 + 8 + 1 + 8 + 8 + 8 + (int64_t)sizeof(gsl::GraphDesc) + 4) + 8;  // batch arrays
  b += (n + 1) * 8 + nnz * 4 * (weighted ? 2 : 1) + n * 4;                          // gathered CSR, labels
  return b + hub_bytes_bound(nnz);
}

// ---- sessions ----
// Device bytes of a session of this capacity: the arena (two buffers), the
// split buffers and per-graph records, the per-vertex and per-graph scratch,
// and a bound on the hub tier's layout and staging (at most one hub per
// 4,097 entries, every entry in a hub row).
int64_t session_bytes(int64_t cap_v, int64_t cap_e, int64_t cap_g, bool weighted) {
  const int64_t G = cap_g + 1;
  const int64_t flag = (cap_v + 3) / 4 * 4 + 16;
  int64_t b = 2 * ((cap_v + 1) * 8 + cap_e * 4 * (weighted ? 2 : 1) + cap_v * 4);  // arena
  b += 2 * cap_v * 4 + G + cap_g * (int64_t)sizeof(gsl::SessionRange);           // split, sel, ranges
  b += cap_v * (4 + 4 + 4 + 4 + 8) + 3 * flag + gsl::plan_scratch(cap_v) * 8;      // Cn list parent rep sigma, flags, plan
  b += 2 * 4096 * 8 + (int64_t)gsl::kNumTiers * gsl::kMaxTierGrid * gsl::kCountFields * 8;  // partials, tier records
  b += (int64_t)sizeof(Counters) + 4 * 8 * (kSessionSweepCap + 2) + (int64_t)sizeof(gsl::SweepCtrl);
  b += cap_v * 4 + G * (4 + 8 + 8 + 1 + 8 + 8 + 8 + (int64_t)sizeof(gsl::GraphDesc) + 4) + 8;  // batch arrays
  return b + hub_bytes_bound(cap_e);
}

void session_free(gsl_session &S) {
  for (int b = 0; b < 2; ++b) {
    hipFree(S.off[b]);
    hipFree(S.cols[b]);
    hipFree(S.w[b]);
    hipFree(S.lab[b]);
  }
  hipFree(S.split_in);
  hipFree(S.split_out);
  hipFree(S.sel);
  hipFree(S.ranges);
  free_scratch(S.s);
}

// One sweep of every live graph of the arena (tiers, hubs, counts, apply,
// per-graph stop decisions, loop state), enqueued on st; every kernel returns
// at once once the loop state says done.
int session_enqueue_sweep(gsl_session &S, const gsl::SweepArgs &a0, const gsl::TierConfig &cfg,
                          const HubLimits &lim, hipStream_t st) {
  Scratch &s = S.s;
  gsl::SweepArgs a = a0;
  const Counters &plan = S.plan;
  const gsl::HubLayout L{s.hub_chunk_start, s.hub_part_start, s.hub_hist_start, s.hub_chunk_owner,
                         s.hub_part_owner, s.hub_records};
  gsl::TierGrids grids;
  for (int t = 0; t < gsl::kNumTiers; ++t) grids.g[t] = 0;
  for (int t = 1; t < gsl::kNumTiers; ++t) {
    const int64_t cnt = plan.tier_count[t];
    if (cnt <= 0) continue;
    a.tier = &s.ctr->tier_stats[t][0];
    a.part = s.tier_part + (size_t)t * gsl::kMaxTierGrid * gsl::kCountFields;
    if (t == gsl::kHubTier) {
      for (size_t bi = 0; bi < s.hub_batches.size(); ++bi)
        for (int stage = 0; stage < 2; ++stage)
          HIP_TRY(gsl::launch_hub_sweep(a, s.list, L, s.h_chunk.data(), s.h_part.data(), s.hub_staging, s.hub_hist,
                                        s.hub_best, s.hub_rowsum, s.hub_batches[bi].first, s.hub_batches[bi].second,
                                        s.hub_max_parts[bi], lim.merge_cap, stage, st));
    } else {
      HIP_TRY(gsl::launch_sweep_tier(cfg.variant[t], a, s.list, plan.tier_start[t], cnt, &grids.g[t], st));
    }
  }
  HIP_TRY(gsl::launch_reduce_counts(s.tier_part, grids, s.ctr->tier_stats, s.ctrl, a.dn, a.processed, a.edges,
                                    a.overflow, st));
  HIP_TRY(gsl::launch_apply(a, S.lab[S.cur], S.vtop, s.gdn, st));
  HIP_TRY(gsl::launch_graph_end(s.ctrl, s.gdn, s.glimit, s.giters, s.gdone, (int64_t)S.cap_g + 1, st));
  HIP_TRY(gsl::launch_sweep_end(s.ctrl, a.dn, a.marked_sweeps, a.overflow, st));
  return GSL_OK;
}

// Moves the live graphs to the front of the other arena buffer, in order.
int session_compact(gsl_session &S) {
  Scratch &s = S.s;
  const hipStream_t st = S.stream;
  std::vector<int32_t> live;
  for (int32_t k = 0; k < S.cap_g; ++k)
    if (S.slot[(size_t)k].live) live.push_back(k);
  std::sort(live.begin(), live.end(), [&](int32_t x, int32_t y) { return S.slot[(size_t)x].vb < S.slot[(size_t)y].vb; });
  std::vector<gsl::SessionRange> r(live.size());
  int64_t v = 0, e = 0;
  for (size_t i = 0; i < live.size(); ++i) {
    SessionSlot &x = S.slot[(size_t)live[i]];
    r[i] = gsl::SessionRange{x.vb, x.n, x.eb, x.nnz, v, e, x.limit, x.labels_out, live[i], 0};
    x.vb = v;
    x.eb = e;
    v += x.n;
    e += x.nnz;
  }
  const int o = 1 - S.cur;
  if (!r.empty()) {
    HIP_TRY(hipMemcpyAsync(S.ranges, r.data(), r.size() * sizeof(gsl::SessionRange), hipMemcpyHostToDevice, st));
    HIP_TRY(gsl::launch_session_move(S.ranges, (int64_t)r.size(), S.off[S.cur], S.cols[S.cur],
                                     S.weighted ? S.w[S.cur] : nullptr, S.lab[S.cur], S.off[o], S.cols[o],
                                     S.weighted ? S.w[o] : nullptr, S.lab[o], s.gid, s.act[0], s.act[1], st));
  }
  HIP_TRY(hipMemcpyAsync(S.off[o] + v, &e, sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));  // r and e are host temporaries
  S.cur = o;
  S.vtop = v;
  S.etop = e;
  S.dirty = true;
  return GSL_OK;
}

int session_add(gsl_session &S, int64_t G, const gsl_graph *graphs, int64_t *tickets, int32_t *status) {
  Scratch &s = S.s;
  const hipStream_t st = S.stream;
  for (int64_t g = 0; g < G; ++g) {
    tickets[g] = -1;
    status[g] = GSL_OK;
  }
  // entry counts (and decreasing offsets) of every graph on the device; a
  // descriptor the host can already reject (negative or oversized n, NULL
  // offsets or output) goes to the device with n = 0, so nothing reads it
  std::vector<gsl_graph> desc(graphs, graphs + G);
  std::vector<uint8_t> rejected((size_t)G, 0);
  for (int64_t g = 0; g < G; ++g) {
    const gsl_graph &x = graphs[g];
    if (x.n < 0 || x.n > S.cap_v || (x.n > 0 && (!x.offsets || !x.labels_out))) {
      rejected[(size_t)g] = 1;
      desc[(size_t)g].n = 0;
    }
  }
  HIP_TRY(hipMemcpyAsync(s.gdesc, desc.data(), (size_t)G * sizeof(gsl_graph), hipMemcpyHostToDevice, st));
  HIP_TRY(gsl::launch_graph_entries(s.gdesc, G, s.gcnt, st));
  std::vector<int64_t> cnt((size_t)G);
  HIP_TRY(hipMemcpyAsync(cnt.data(), s.gcnt, (size_t)G * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));  // also keeps desc alive until the copy is done
  // admit in order while the arena has room (compacting once if that makes room)
  std::vector<int64_t> take;
  int64_t need_v = 0, need_e = 0;
  bool full = false;
  for (int64_t g = 0; g < G; ++g) {
    const gsl_graph &x = graphs[g];
    const int64_t c = cnt[(size_t)g];
    if (rejected[(size_t)g] || c < 0 || (c > 0 && !x.cols) || c > S.cap_e || (x.weights && !S.weighted)) {
      status[g] = GSL_EINVAL;
      continue;
    }
    if (full) {
      status[g] = GSL_EAGAIN;
      continue;
    }
    if (x.n == 0) continue;  // nothing to run: done at once, ticket -1
    const bool slot_ok = (int64_t)S.free_slot.size() > (int64_t)take.size();
    bool room = S.vtop + need_v + x.n <= S.cap_v && S.etop + need_e + c <= S.cap_e;
    if (slot_ok && !room && S.live_v + need_v + x.n <= S.cap_v && S.live_e + need_e + c <= S.cap_e &&
        (S.vtop > S.live_v || S.etop > S.live_e)) {
      // the graphs taken so far are placed after the compaction, from vtop
      int rc = session_compact(S);
      if (rc) return rc;
      room = S.vtop + need_v + x.n <= S.cap_v && S.etop + need_e + c <= S.cap_e;
    }
    if (!slot_ok || !room) {
      full = true;
      status[g] = GSL_EAGAIN;
      continue;
    }
    take.push_back(g);
    need_v += x.n;
    need_e += c;
  }
  if (take.empty()) return GSL_OK;
  // gather the admitted graphs to the top of the arena
  const int64_t T = (int64_t)take.size();
  std::vector<gsl_graph> d((size_t)T);
  std::vector<int64_t> vb((size_t)T + 1, 0), eb((size_t)T + 1, 0);
  for (int64_t i = 0; i < T; ++i) {
    const gsl_graph &x = graphs[take[(size_t)i]];
    d[(size_t)i] = x;
    vb[(size_t)i + 1] = vb[(size_t)i] + x.n;
    eb[(size_t)i + 1] = eb[(size_t)i] + cnt[(size_t)take[(size_t)i]];
  }
  HIP_TRY(hipMemcpyAsync(s.gdesc, d.data(), (size_t)T * sizeof(gsl_graph), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s.gvb, vb.data(), (size_t)(T + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s.geb, eb.data(), (size_t)(T + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(gsl::launch_fill_u8(reinterpret_cast<uint8_t *>(s.gflag), 0, T * (int64_t)sizeof(uint32_t), st));
  HIP_TRY(gsl::launch_gather(s.gdesc, s.gvb, s.geb, T, need_v, need_e, S.vtop, S.etop, S.off[S.cur] + S.vtop,
                             S.cols[S.cur] + S.etop, S.weighted ? S.w[S.cur] + S.etop : nullptr, s.gflag, st));
  std::vector<uint32_t> bad((size_t)T, 0);
  HIP_TRY(hipMemcpyAsync(bad.data(), s.gflag, (size_t)T * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // slots and loop state of the admitted graphs; a graph with an entry
  // outside [0, n) is rejected (its arena space becomes dead space)
  std::vector<gsl::SessionRange> r;
  std::vector<gsl::SessionRange> dead;
  for (int64_t i = 0; i < T; ++i) {
    const int64_t g = take[(size_t)i];
    const int64_t n = vb[(size_t)i + 1] - vb[(size_t)i], c = eb[(size_t)i + 1] - eb[(size_t)i];
    const gsl::SessionRange x{S.vtop + vb[(size_t)i], n, S.etop + eb[(size_t)i], c, 0, 0,
                              gsl_convergence_limit(n, S.tol), graphs[g].labels_out, 0, 0};
    if (bad[(size_t)i]) {
      status[g] = GSL_EINVAL;
      gsl::SessionRange y = x;
      y.slot = S.cap_g;  // the dead slot
      dead.push_back(y);
      continue;
    }
    const int32_t k = S.free_slot.back();
    S.free_slot.pop_back();
    SessionSlot &sl = S.slot[(size_t)k];
    sl = SessionSlot{true, S.next_ticket++, x.vb, n, x.eb, c, x.limit, graphs[g].labels_out};
    tickets[g] = sl.ticket;
    gsl::SessionRange y = x;
    y.slot = k;
    r.push_back(y);
    S.live_v += n;
    S.live_e += c;
  }
  std::vector<gsl::SessionRange> all(r);
  all.insert(all.end(), dead.begin(), dead.end());
  HIP_TRY(hipMemcpyAsync(S.ranges, all.data(), all.size() * sizeof(gsl::SessionRange), hipMemcpyHostToDevice, st));
  HIP_TRY(gsl::launch_session_admit(S.ranges, (int64_t)all.size(), s.gid, S.lab[S.cur], s.act[0], s.act[1], st));
  HIP_TRY(gsl::launch_session_slots(S.ranges, (int64_t)r.size(), S.max_iters, S.tol, s.glimit, s.giters, s.gdone,
                                    s.gdn, st));
  HIP_TRY(hipStreamSynchronize(st));  // the records are host temporaries
  S.vtop += need_v;
  S.etop += need_e;
  S.dirty = true;
  return GSL_OK;
}

int session_step(gsl_session &S, int32_t sweeps, int64_t capacity, int64_t *done_tickets, int32_t *done_iters,
                 int64_t *done_count) {
  Scratch &s = S.s;
  const hipStream_t st = S.stream;
  *done_count = 0;
  int64_t live = 0;
  for (const SessionSlot &x : S.slot) live += x.live ? 1 : 0;
  if (live == 0) return GSL_OK;
  // Dead space (finished or rejected graphs) costs every step its plan, a
  // flag check per listed vertex and split passes; once it outgrows the live
  // graphs, they are moved together first.
  if (S.vtop - S.live_v > std::max<int64_t>(S.live_v, kSessionCompactVertices) ||
      S.etop - S.live_e > std::max<int64_t>(S.live_e, kSessionCompactEntries)) {
    const int crc = session_compact(S);
    if (crc) return crc;
  }
  const gsl::TierConfig cfg = current_tiers();
  const HubLimits lim = current_hub_limits();
  const int64_t N = S.vtop;
  const int64_t *off = S.off[S.cur];
  int rc = GSL_OK;
  if (S.dirty) {
    if ((rc = run_plan(s, off, N, cfg, st))) return rc;
    S.plan = *s.ctr_host;
    if ((rc = prepare_hubs(s, off, s.list, S.plan.tier_count[gsl::kHubTier], lim.staging_bytes, st))) return rc;
    S.dirty = false;
  }
  // loop state: the sweep index keeps the parity of the active-flag arrays
  // from step to step; the per-sweep counters restart
  const int p = S.ctrl.it & 1;
  gsl::SweepCtrl hc = S.ctrl;
  hc.it = p;
  hc.done = 0;
  hc.max_iters = p + sweeps;
  hc.graph_max_iters = S.max_iters;
  hc.prune = 1;
  hc.error = 0;
  hc.limit = 0;
  hc.n = S.live_v;
  hc.graphs = (int64_t)S.cap_g + 1;
  hc.active = 0;
  HIP_TRY(gsl::launch_fill_u64(reinterpret_cast<uint64_t *>(s.ctr), 0, s.ctr_bytes / 8, st));
  HIP_TRY(hipMemcpyAsync(s.ctrl, &hc, sizeof(hc), hipMemcpyHostToDevice, st));
  gsl::SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.off = off;
  a.cols = S.cols[S.cur];
  a.w = S.weighted ? S.w[S.cur] : nullptr;
  a.C = S.lab[S.cur];
  a.Cn = s.Cn;
  a.chg = s.chg;
  a.act0 = s.act[0];
  a.act1 = s.act[1];
  a.ctrl = s.ctrl;
  a.dn = sweep_array(s.ctr, 0, kSessionSweepCap + 2);
  a.processed = sweep_array(s.ctr, 1, kSessionSweepCap + 2);
  a.edges = sweep_array(s.ctr, 2, kSessionSweepCap + 2);
  a.marked_sweeps = sweep_array(s.ctr, 3, kSessionSweepCap + 2);
  a.overflow = reinterpret_cast<unsigned long long *>(&s.ctr->overflow);
  a.gid = s.gid;
  a.gdone = s.gdone;
  a.inplace = 0;
  a.n = N;
  for (int k = 0; k < sweeps; ++k)
    if ((rc = session_enqueue_sweep(S, a, cfg, lim, st))) return rc;
  // which graphs stopped
  std::vector<uint8_t> gdone((size_t)S.cap_g);
  std::vector<int32_t> giters((size_t)S.cap_g);
  HIP_TRY(hipMemcpyAsync(&hc, s.ctrl, sizeof(hc), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(gdone.data(), s.gdone, (size_t)S.cap_g, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(giters.data(), s.giters, (size_t)S.cap_g * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  S.ctrl = hc;
  if (hc.error)
    return fail(GSL_EOVERFLOW, "a vertex's summed row weight reaches 2^32; the session's graphs are lost");
  std::vector<int32_t> fin;
  for (int32_t k = 0; k < S.cap_g; ++k)
    if (S.slot[(size_t)k].live && gdone[(size_t)k] && (int64_t)fin.size() < capacity) fin.push_back(k);
  if (fin.empty()) return GSL_OK;
  // the split of the finishing graphs, their labels out, their space dead
  std::vector<uint8_t> sel((size_t)S.cap_g + 1, 0);
  std::vector<gsl::SessionRange> r;
  for (int32_t k : fin) {
    sel[(size_t)k] = 1;
    const SessionSlot &x = S.slot[(size_t)k];
    r.push_back(gsl::SessionRange{x.vb, x.n, x.eb, x.nnz, 0, 0, x.limit, x.labels_out, k, 0});
  }
  HIP_TRY(hipMemcpyAsync(S.sel, sel.data(), sel.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(S.ranges, r.data(), r.size() * sizeof(gsl::SessionRange), hipMemcpyHostToDevice, st));
  HIP_TRY(gsl::launch_session_split_labels(S.lab[S.cur], s.gid, S.sel, N, S.split_in, st));
  HIP_TRY(gsl::launch_split(off, S.cols[S.cur], N, S.split_in, s.parent, S.split_out, s.list, S.plan.tier_count,
                            S.plan.tier_start, nullptr, nullptr, N, s.rep, s.sigma, cfg, st, s.gid, S.sel));
  HIP_TRY(gsl::launch_session_finish(S.ranges, (int64_t)r.size(), S.split_out, s.gid, S.cap_g, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (size_t i = 0; i < fin.size(); ++i) {
    SessionSlot &x = S.slot[(size_t)fin[i]];
    done_tickets[i] = x.ticket;
    if (done_iters) done_iters[i] = giters[(size_t)fin[i]];
    S.live_v -= x.n;
    S.live_e -= x.nnz;
    x = SessionSlot{};
    S.free_slot.push_back(fin[i]);
  }
  *done_count = (int64_t)fin.size();
  // an empty arena starts again from the bottom
  if (S.live_v == 0 && S.live_e == 0) {
    S.vtop = 0;
    S.etop = 0;
    HIP_TRY(hipMemcpyAsync(S.off[S.cur], &S.etop, sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    S.dirty = true;
  }
  return GSL_OK;
}

}  // namespace

extern "C" {

int gsl_lpa(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
            int32_t max_iters, double tolerance, int32_t *labels_out) {
  return gsl_lpa_ex(offsets, cols, weights, n, max_iters, tolerance, nullptr, nullptr, labels_out);
}

int gsl_lpa_ex(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
               int32_t max_iters, double tolerance, const gsl_options *opt, gsl_stats *stats,
               int32_t *labels_out) {
  if (stats) memset(stats, 0, sizeof(*stats));
  int rc = check_lpa(n, max_iters, tolerance, offsets, labels_out);
  if (rc) return rc == kNoop ? GSL_OK : rc;
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch *sp = nullptr;
  if ((rc = get_scratch(&sp))) return rc;
  return lpa_impl(*sp, g_stream, offsets, cols, weights, n, max_iters, tolerance, opt, stats, labels_out);
}

int gsl_lpa_noalloc(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
                    int32_t max_iters, double tolerance, int32_t *labels_out) {
  int rc = check_lpa(n, max_iters, tolerance, offsets, labels_out);
  if (rc) return rc == kNoop ? GSL_OK : rc;
  if (n > GSL_NOALLOC_MAX_VERTICES)
    return fail(GSL_EINVAL, "n = %lld exceeds the %d vertices of gsl_lpa_noalloc", (long long)n,
                GSL_NOALLOC_MAX_VERTICES);
  if (max_iters > GSL_NOALLOC_MAX_ITERS)
    return fail(GSL_EINVAL, "max_iters = %d exceeds the %d sweeps of gsl_lpa_noalloc", max_iters,
                GSL_NOALLOC_MAX_ITERS);
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  NoAlloc &na = g_noalloc[dev];
  if (!na.ready && (rc = noalloc_setup(na))) return rc;
  const gsl_options o = {1, 1, 0, 2, 0};  // pruning, split, no timing, original layout, synchronous
  return lpa_impl(na.s, g_stream, offsets, cols, weights, n, max_iters, tolerance, &o, nullptr, labels_out);
}

int gsl_lpa_f32(const int64_t *offsets, const int32_t *cols, const float *weights, int64_t n, int32_t max_iters,
                double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *labels_out) {
  if (stats) memset(stats, 0, sizeof(*stats));
  int rc = check_lpa(n, max_iters, tolerance, offsets, labels_out);
  if (rc) return rc == kNoop ? GSL_OK : rc;
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch *sp = nullptr;
  if ((rc = get_scratch(&sp))) return rc;
  Scratch &s = *sp;
  const hipStream_t st = g_stream;
  if (weights) {
    int64_t nnz = 0;
    if ((rc = read_nnz(offsets, n, &nnz, st))) return rc;
    if ((rc = ensure_batch(s, 1, 1))) return rc;
    unsigned long long bad = 0;
    HIP_TRY(hipMemsetAsync(s.gbad, 0, sizeof(unsigned long long), st));
    HIP_TRY(gsl::launch_check_f32(weights, nnz, s.gbad, st));
    HIP_TRY(hipMemcpyAsync(&bad, s.gbad, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(GSL_EINVAL, "weights must be finite and >= 0");
  }
  return lpa_impl(s, st, offsets, cols, reinterpret_cast<const uint32_t *>(weights), n, max_iters, tolerance, opt,
                  stats, labels_out, nullptr, weights != nullptr);
}

int gsl_lpa_batched(int64_t num_graphs, const int64_t *vtx_base, const int64_t *edge_base, const int64_t *offsets,
                    const int32_t *cols, const uint32_t *weights, int32_t max_iters, double tolerance,
                    int32_t *labels_out) {
  return gsl_lpa_batched_ex(num_graphs, vtx_base, edge_base, offsets, cols, weights, max_iters, tolerance,
                            nullptr, nullptr, labels_out, nullptr);
}

int gsl_lpa_batched_ex(int64_t num_graphs, const int64_t *vtx_base, const int64_t *edge_base,
                       const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int32_t max_iters,
                       double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *labels_out,
                       int32_t *iterations_out) {
  if (stats) memset(stats, 0, sizeof(*stats));
  int rc = check_batch(num_graphs, max_iters, tolerance);
  if (rc) return rc == kNoop ? GSL_OK : rc;
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch *sp = nullptr;
  if ((rc = get_scratch(&sp))) return rc;
  return batched_concat(*sp, g_stream, num_graphs, vtx_base, edge_base, offsets, cols, weights, max_iters,
                        tolerance, opt, stats, labels_out, iterations_out);
}

int gsl_check_graph(const int64_t *offsets, const int32_t *cols, int64_t n) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return GSL_OK;
  if (!offsets) return fail(GSL_EINVAL, "offsets must not be NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch *sp = nullptr;
  const int rc = get_scratch(&sp);
  if (rc) return rc;
  return check_graph_impl(*sp, g_stream, offsets, cols, n);
}

int gsl_context_create(gsl_context **out) {
  if (!out) return fail(GSL_EINVAL, "out must not be NULL");
  *out = nullptr;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  gsl_context *c = new (std::nothrow) gsl_context();
  if (!c) return fail(GSL_ENOMEM, "host allocation failed");
  c->device = dev;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(GSL_EDEVICE, "hipStreamCreateWithFlags failed");
  }
  c->own_stream = true;
  *out = c;
  return GSL_OK;
}

void gsl_context_destroy(gsl_context *ctx) {
  if (!ctx) return;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (hipSetDevice(ctx->device) == hipSuccess) {
      if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
      free_scratch(ctx->s);
      if (ctx->own_stream && ctx->stream) hipStreamDestroy(ctx->stream);
    }
    if (have) (void)hipSetDevice(cur);
  }
  delete ctx;
}

int gsl_context_set_stream(gsl_context *ctx, void *hip_stream) {
  if (!ctx) return fail(GSL_EINVAL, "ctx must not be NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->own_stream && ctx->stream) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipStreamDestroy(ctx->stream));
  }
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->own_stream = false;
  return GSL_OK;
}

void *gsl_context_stream(gsl_context *ctx) { return ctx ? reinterpret_cast<void *>(ctx->stream) : nullptr; }

int gsl_lpa_graphs(gsl_context *ctx, int64_t num_graphs, const gsl_graph *graphs, int32_t max_iters,
                   double tolerance, const gsl_options *opt, gsl_stats *stats, int32_t *iterations_out,
                   int32_t *status_out) {
  if (stats) memset(stats, 0, sizeof(*stats));
  int rc = check_batch(num_graphs, max_iters, tolerance);
  if (rc) return rc == kNoop ? GSL_OK : rc;
  if (!graphs) return fail(GSL_EINVAL, "graphs must not be NULL");
  int64_t total = 0;
  for (int64_t g = 0; g < num_graphs; ++g) {
    const gsl_graph &x = graphs[g];
    if (x.n < 0 || x.n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "graph %lld: n out of range", (long long)g);
    if (x.n > 0 && (!x.offsets || !x.labels_out))
      return fail(GSL_EINVAL, "graph %lld: offsets and labels_out must not be NULL", (long long)g);
    total += x.n;
    if (total >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "total vertex count out of range");
  }
  if (total == 0) {
    if (iterations_out) memset(iterations_out, 0, (size_t)num_graphs * sizeof(int32_t));
    if (status_out) memset(status_out, 0, (size_t)num_graphs * sizeof(int32_t));
    return GSL_OK;
  }
  if (!ctx) {
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch *sp = nullptr;
    if ((rc = get_scratch(&sp))) return rc;
    return batched_graphs(*sp, g_stream, num_graphs, graphs, max_iters, tolerance, opt, stats, iterations_out,
                          status_out);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != ctx->device) return fail(GSL_EINVAL, "the context belongs to device %d, current is %d", ctx->device, cur);
  return batched_graphs(ctx->s, ctx->stream, num_graphs, graphs, max_iters, tolerance, opt, stats, iterations_out,
                        status_out);
}

int gsl_split(const int64_t *offsets, const int32_t *cols, int64_t n, const int32_t *labels_in,
              int32_t *labels_out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n out of range");
  if (n == 0) return GSL_OK;
  if (!offsets || !labels_in || !labels_out) return fail(GSL_EINVAL, "NULL argument");
  if (labels_in == labels_out) return fail(GSL_EINVAL, "labels_out must not alias labels_in");
  const hipStream_t st = g_stream;
  Scratch *sp = nullptr;
  int rc = get_scratch(&sp);
  if (rc) return rc;
  Scratch &s = *sp;
  int64_t nnz = 0;
  if ((rc = read_nnz(offsets, n, &nnz, st))) return rc;
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when offsets[n] > 0");
  if ((rc = ensure_scratch(s, n, 1))) return rc;
  if ((rc = check_labels(s, labels_in, n, st))) return rc;
  const gsl::TierConfig cfg = current_tiers();
  if ((rc = run_plan(s, offsets, n, cfg, st))) return rc;
  Counters plan = *s.ctr_host;
  HIP_TRY(gsl::launch_split(offsets, cols, n, labels_in, s.parent, labels_out, s.list,
                            plan.tier_count, plan.tier_start, nullptr, nullptr, n, s.rep, s.sigma, cfg, st));
  HIP_TRY(hipStreamSynchronize(st));
  return GSL_OK;
}

int gsl_split_ex(const int64_t *offsets, const int32_t *cols, int64_t n, const int32_t *labels_in,
                 int32_t *labels_out, int32_t technique, int32_t *rounds_out, float *ms_out) {
  if (rounds_out) *rounds_out = 0;
  if (ms_out) *ms_out = 0.f;
  if (technique < GSL_SPLIT_UNION_FIND || technique > GSL_SPLIT_LPP)
    return fail(GSL_EINVAL, "unknown split technique %d", technique);
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n out of range");
  if (n == 0) return GSL_OK;
  if (!offsets || !labels_in || !labels_out) return fail(GSL_EINVAL, "NULL argument");
  if (labels_in == labels_out) return fail(GSL_EINVAL, "labels_out must not alias labels_in");
  std::lock_guard<std::mutex> lk(g_mu);
  const hipStream_t st = g_stream;
  Scratch *sp = nullptr;
  int rc = get_scratch(&sp);
  if (rc) return rc;
  Scratch &s = *sp;
  int64_t nnz = 0;
  if ((rc = read_nnz(offsets, n, &nnz, st))) return rc;
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when offsets[n] > 0");
  if ((rc = ensure_scratch(s, n, 1))) return rc;
  if ((rc = check_labels(s, labels_in, n, st))) return rc;
  const gsl::TierConfig cfg = current_tiers();
  if ((rc = run_plan(s, offsets, n, cfg, st))) return rc;
  Counters plan = *s.ctr_host;
  if ((rc = ensure_events(s))) return rc;
  HIP_TRY(hipEventRecord(s.ev[0], st));
  int32_t rounds = 0;
  if (technique == GSL_SPLIT_UNION_FIND) {
    HIP_TRY(gsl::launch_split(offsets, cols, n, labels_in, s.parent, labels_out, s.list, plan.tier_count,
                              plan.tier_start, nullptr, nullptr, n, s.rep, s.sigma, cfg, st));
    rounds = 1;
  } else {
    const bool prune = technique == GSL_SPLIT_LPP;
    uint8_t *f[2] = {prune ? s.act[0] : nullptr, prune ? s.act[1] : nullptr};
    unsigned long long *chg = reinterpret_cast<unsigned long long *>(&s.ctr->split_changed);
    HIP_TRY(gsl::launch_split_lp_init(labels_out, f[0], f[1], n, st));
    for (;;) {
      HIP_TRY(hipMemsetAsync(chg, 0, sizeof(*chg), st));
      HIP_TRY(gsl::launch_split_lp_round(offsets, cols, n, labels_in, labels_out, s.list, plan.tier_count,
                                         plan.tier_start, cfg, f[rounds & 1], f[(rounds + 1) & 1], chg, st));
      ++rounds;
      unsigned long long host = 0;
      HIP_TRY(hipMemcpyAsync(&host, chg, sizeof(host), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (!host) break;
      if (rounds > n + 1) return fail(GSL_EDEVICE, "label propagation split did not converge");
    }
  }
  HIP_TRY(hipEventRecord(s.ev[1], st));
  HIP_TRY(hipStreamSynchronize(st));
  if (rounds_out) *rounds_out = rounds;
  if (ms_out) *ms_out = elapsed(s.ev[0], s.ev[1]);
  return GSL_OK;
}

int gsl_disconnected(const int64_t *offsets, const int32_t *cols, int64_t n, const int32_t *labels,
                     uint8_t *flags_out, int64_t *count_out) {
  if (count_out) *count_out = 0;
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n out of range");
  if (n == 0) return GSL_OK;
  if (!offsets || !labels) return fail(GSL_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_mu);
  const hipStream_t st = g_stream;
  Scratch *sp = nullptr;
  int rc = get_scratch(&sp);
  if (rc) return rc;
  Scratch &s = *sp;
  int64_t nnz = 0;
  if ((rc = read_nnz(offsets, n, &nnz, st))) return rc;
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when offsets[n] > 0");
  if ((rc = ensure_scratch(s, n, 1))) return rc;
  if ((rc = check_labels(s, labels, n, st))) return rc;
  const gsl::TierConfig cfg = current_tiers();
  if ((rc = run_plan(s, offsets, n, cfg, st))) return rc;
  Counters plan = *s.ctr_host;
  // split labels into Cn, then piece counts per community in parent
  HIP_TRY(gsl::launch_split(offsets, cols, n, labels, s.parent, s.Cn, s.list, plan.tier_count, plan.tier_start,
                            nullptr, nullptr, n, s.rep, s.sigma, cfg, st));
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(&s.ctr->split_changed);
  HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(*cnt), st));
  HIP_TRY(gsl::launch_disconnected(labels, s.Cn, n, s.parent, flags_out, cnt, st));
  unsigned long long host = 0;
  HIP_TRY(hipMemcpyAsync(&host, cnt, sizeof(host), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (count_out) *count_out = (int64_t)host;
  return GSL_OK;
}

int gsl_modularity(const int64_t *offsets, const int32_t *cols, const uint32_t *weights, int64_t n,
                   const int32_t *labels, double *q_out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!q_out) return fail(GSL_EINVAL, "q_out must not be NULL");
  *q_out = 0.0;
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GSL_EINVAL, "n out of range");
  if (n == 0) return GSL_OK;
  if (!offsets || !labels) return fail(GSL_EINVAL, "NULL argument");
  const hipStream_t st = g_stream;
  Scratch *sp = nullptr;
  int rc = get_scratch(&sp);
  if (rc) return rc;
  Scratch &s = *sp;
  int64_t nnz = 0;
  if ((rc = read_nnz(offsets, n, &nnz, st))) return rc;
  if (nnz > 0 && !cols) return fail(GSL_EINVAL, "cols must not be NULL when offsets[n] > 0");
  if ((rc = ensure_scratch(s, n, 1))) return rc;
  if ((rc = check_labels(s, labels, n, st))) return rc;
  HIP_TRY(hipMemsetAsync(s.ctr, 0, sizeof(Counters), st));
  HIP_TRY(hipMemsetAsync(s.sigma, 0, (size_t)n * sizeof(unsigned long long), st));
  HIP_TRY(gsl::launch_modularity(offsets, cols, weights, n, labels, s.sigma, s.partials,
                                 s.partial_blocks, s.ctr, st));
  HIP_TRY(hipMemcpyAsync(s.ctr_host, s.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *q_out = s.ctr_host->q;
  return GSL_OK;
}

int gsl_set_tiers(const gsl_tier *levels) {
  gsl::TierConfig c = gsl::kDefaultTiers;
  if (levels) {
    int64_t prev = 0;
    for (int l = 0; l < GSL_TIER_LEVELS; ++l) {
      const int t = l + 1;
      const int32_t v = levels[l].variant;
      const int64_t b = levels[l].max_degree;
      if (v < 0 || v >= gsl::kNumVariants) return fail(GSL_EINVAL, "level %d: no variant %d", l, v);
      if (b < prev) return fail(GSL_EINVAL, "level %d: degree bounds must not decrease", l);
      if (b > gsl::variant_capacity(v))
        return fail(GSL_EINVAL, "level %d: bound %lld exceeds variant %d's %lld entries", l, (long long)b, v,
                    (long long)gsl::variant_capacity(v));
      c.bound[t] = b;
      c.variant[t] = v;
      prev = b;
    }
  }
  std::lock_guard<std::mutex> lk(g_tier_mu);
  g_tiers = c;
  return GSL_OK;
}

int gsl_set_hub_limits(int64_t staging_bytes, int32_t merge_claims) {
  if (staging_bytes < 0 || (staging_bytes > 0 && staging_bytes < (int64_t)gsl::kHubChunk * 8))
    return fail(GSL_EINVAL, "staging_bytes must be 0 (default) or at least %lld",
                (long long)gsl::kHubChunk * 8);
  if (merge_claims < 0 || merge_claims > gsl::kHubMergeCapMax)
    return fail(GSL_EINVAL, "merge_claims must be in [0, %d]", gsl::kHubMergeCapMax);
  std::lock_guard<std::mutex> lk(g_tier_mu);
  g_hub_limits.staging_bytes = staging_bytes ? staging_bytes : kDefaultHubStagingBytes;
  g_hub_limits.merge_cap = merge_claims ? merge_claims : gsl::kHubMergeCapMax;
  return GSL_OK;
}

int gsl_get_tiers(gsl_tier *levels_out) {
  if (!levels_out) return fail(GSL_EINVAL, "levels_out must not be NULL");
  const gsl::TierConfig c = current_tiers();
  for (int l = 0; l < GSL_TIER_LEVELS; ++l) {
    levels_out[l].max_degree = (int32_t)c.bound[l + 1];
    levels_out[l].variant = c.variant[l + 1];
  }
  return GSL_OK;
}

int gsl_tier_variant(int32_t variant, gsl_variant_info *info) {
  if (variant < 0 || variant >= gsl::kNumVariants || !info) return fail(GSL_EINVAL, "no such variant");
  const gsl::SweepVariant &x = gsl::kVariants[variant];
  info->group = x.group;
  info->table_log2 = x.log2s;
  info->block = x.block;
  info->per_lane = x.per_lane;
  info->capacity = (int32_t)gsl::variant_capacity(variant);
  return GSL_OK;
}

int64_t gsl_convergence_limit(int64_t n, double tolerance) {
  if (!(tolerance >= 0.0 && tolerance <= 1.0)) return -1;
  if (n <= 0) return 0;
  const double dn = (double)n;
  int64_t k = (int64_t)std::floor(tolerance * dn);
  if (k < 0) k = 0;
  if (k > n) k = n;
  while (k > 0 && !((double)k / dn <= tolerance)) --k;
  while (k < n && (double)(k + 1) / dn <= tolerance) ++k;
  // k == 0 may itself fail only if tolerance < 0, excluded above.
  return k;
}

int gsl_set_stream(void *hip_stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_stream = reinterpret_cast<hipStream_t>(hip_stream);
  return GSL_OK;
}

const char *gsl_last_error(void) { return g_err.c_str(); }

void gsl_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto &kv : g_scratch) {
    if (hipSetDevice(kv.first) == hipSuccess) free_scratch(kv.second);
  }
  g_scratch.clear();
  if (have) (void)hipSetDevice(cur);
}

const char *gsl_version(void) { return "gsl_lpa 0.3 (gfx950)"; }

int64_t gsl_graphs_bytes(int64_t n, int64_t nnz, int64_t graphs, int32_t weighted, int32_t max_iters) {
  if (n < 0 || n >= ((int64_t)1 << 31) || nnz < 0 || graphs < 0 || max_iters < 0) return -1;
  return graphs_bytes(n, nnz, graphs, weighted != 0, max_iters);
}

int64_t gsl_session_bytes(int64_t max_vertices, int64_t max_entries, int32_t max_graphs, int32_t weighted) {
  if (max_vertices < 1 || max_vertices >= ((int64_t)1 << 31) - 1 || max_entries < 0 || max_graphs < 1) return -1;
  return session_bytes(max_vertices, max_entries, max_graphs, weighted != 0);
}

int gsl_session_create(int64_t max_vertices, int64_t max_entries, int32_t max_graphs, int32_t max_iters,
                       double tolerance, int32_t weighted, gsl_session **out) {
  if (!out) return fail(GSL_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (max_vertices < 1 || max_vertices >= ((int64_t)1 << 31) - 1)
    return fail(GSL_EINVAL, "max_vertices must be in [1, 2^31 - 1)");
  if (max_entries < 0) return fail(GSL_EINVAL, "max_entries must be >= 0");
  if (max_graphs < 1 || max_graphs > (1 << 24)) return fail(GSL_EINVAL, "max_graphs must be in [1, 2^24]");
  if (max_iters < 0) return fail(GSL_EINVAL, "max_iters must be >= 0");
  if (bad_tolerance(tolerance)) return fail(GSL_EINVAL, "tolerance must be in [0, 1]");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  gsl_session *S = new (std::nothrow) gsl_session();
  if (!S) return fail(GSL_ENOMEM, "host allocation failed");
  S->device = dev;
  S->cap_v = max_vertices;
  S->cap_e = max_entries;
  S->cap_g = max_graphs;
  S->max_iters = max_iters;
  S->tol = tolerance;
  S->weighted = weighted != 0;
  S->slot.assign((size_t)max_graphs, SessionSlot{});
  for (int32_t k = max_graphs - 1; k >= 0; --k) S->free_slot.push_back(k);
  auto bail = [&](int code) {
    if (S->stream) {
      (void)hipStreamSynchronize(S->stream);
      hipStreamDestroy(S->stream);
    }
    session_free(*S);
    delete S;
    return code;
  };
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    S->stream = nullptr;
    return bail(fail(GSL_EDEVICE, "hipStreamCreateWithFlags failed"));
  }
  Scratch &s = S->s;
  int rc = GSL_OK;
  if ((rc = ensure_pinned(s, kPinSmall)) || (rc = ensure_scratch(s, max_vertices, kSessionSweepCap + 2)) ||
      (rc = ensure_batch(s, max_vertices, (int64_t)max_graphs + 1)))
    return bail(rc);
  for (int b = 0; b < 2; ++b) {
    if (dmalloc(&S->off[b], max_vertices + 1) != hipSuccess || dmalloc(&S->cols[b], max_entries) != hipSuccess ||
        dmalloc(&S->lab[b], max_vertices) != hipSuccess ||
        (S->weighted && dmalloc(&S->w[b], max_entries) != hipSuccess)) {
      (void)hipGetLastError();
      return bail(fail(GSL_ENOMEM, "session arena allocation failed"));
    }
  }
  if (dmalloc(&S->split_in, max_vertices) != hipSuccess || dmalloc(&S->split_out, max_vertices) != hipSuccess ||
      dmalloc(&S->sel, (int64_t)max_graphs + 1) != hipSuccess || dmalloc(&S->ranges, max_graphs) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(GSL_ENOMEM, "session allocation failed"));
  }
  // every slot (and the dead slot, max_graphs) starts stopped; the arena
  // starts empty.  The change flags start clear and stay clear between
  // sweeps (the apply kernel clears what a sweep sets): a stale flag would
  // copy an unwritten Cn entry into the labels and count a change for the
  // graph id of a vertex that may lie past the arena's top.
  const int64_t zero = 0;
  const int64_t flag_bytes = (s.n_cap + 3) / 4 * 4 + 16;
  if (gsl::launch_fill_u8(s.chg, 0, flag_bytes, S->stream) != hipSuccess ||
      gsl::launch_fill_u8(s.act[0], 0, flag_bytes, S->stream) != hipSuccess ||
      gsl::launch_fill_u8(s.act[1], 0, flag_bytes, S->stream) != hipSuccess ||
      gsl::launch_fill_u8(s.gdone, 1, (int64_t)max_graphs + 1, S->stream) != hipSuccess ||
      hipMemcpyAsync(S->off[0], &zero, sizeof(int64_t), hipMemcpyHostToDevice, S->stream) != hipSuccess ||
      hipStreamSynchronize(S->stream) != hipSuccess)
    return bail(fail(GSL_EDEVICE, "session initialisation failed"));
  memset(&S->ctrl, 0, sizeof(S->ctrl));
  S->ctrl.dense = 1;
  S->bytes = session_bytes(max_vertices, max_entries, max_graphs, S->weighted);
  *out = S;
  return GSL_OK;
}

void gsl_session_destroy(gsl_session *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (hipSetDevice(S->device) == hipSuccess) {
      if (S->stream) (void)hipStreamSynchronize(S->stream);
      session_free(*S);
      if (S->stream) hipStreamDestroy(S->stream);
    }
    if (have) (void)hipSetDevice(cur);
  }
  delete S;
}

void *gsl_session_stream(gsl_session *S) { return S ? reinterpret_cast<void *>(S->stream) : nullptr; }

int gsl_session_add(gsl_session *S, int64_t num_graphs, const gsl_graph *graphs, int64_t *tickets_out,
                    int32_t *status_out) {
  if (!S) return fail(GSL_EINVAL, "session must not be NULL");
  if (num_graphs < 0) return fail(GSL_EINVAL, "num_graphs must be >= 0");
  if (num_graphs == 0) return GSL_OK;
  if (!graphs || !tickets_out || !status_out) return fail(GSL_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != S->device) return fail(GSL_EINVAL, "the session belongs to device %d, current is %d", S->device, cur);
  const int64_t G = std::min<int64_t>(num_graphs, S->cap_g);
  const int rc = session_add(*S, G, graphs, tickets_out, status_out);
  for (int64_t g = G; g < num_graphs; ++g) {
    tickets_out[g] = -1;
    status_out[g] = GSL_EAGAIN;
  }
  return rc;
}

int gsl_session_step(gsl_session *S, int32_t sweeps, int64_t capacity, int64_t *done_tickets,
                     int32_t *done_iterations, int64_t *done_count) {
  if (!S || !done_count) return fail(GSL_EINVAL, "NULL argument");
  *done_count = 0;
  if (sweeps < 1 || sweeps > kSessionSweepCap) return fail(GSL_EINVAL, "sweeps must be in [1, %d]", kSessionSweepCap);
  if (capacity < 0 || (capacity > 0 && !done_tickets)) return fail(GSL_EINVAL, "bad done_tickets / capacity");
  std::lock_guard<std::mutex> lk(S->mu);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != S->device) return fail(GSL_EINVAL, "the session belongs to device %d, current is %d", S->device, cur);
  return session_step(*S, sweeps, capacity, done_tickets, done_iterations, done_count);
}

int gsl_session_info(gsl_session *S, int64_t *live_graphs, int64_t *live_vertices, int64_t *live_entries,
                     int64_t *free_vertices, int64_t *free_entries, int64_t *device_bytes) {
  if (!S) return fail(GSL_EINVAL, "session must not be NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t g = 0;
  for (const SessionSlot &x : S->slot) g += x.live ? 1 : 0;
  if (live_graphs) *live_graphs = g;
  if (live_vertices) *live_vertices = S->live_v;
  if (live_entries) *live_entries = S->live_e;
  if (free_vertices) *free_vertices = S->cap_v - S->live_v;
  if (free_entries) *free_entries = S->cap_e - S->live_e;
  if (device_bytes) *device_bytes = S->bytes;
  return GSL_OK;
}

}  // extern "C"
