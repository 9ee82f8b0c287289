// Many independent slit problems of uneven size in one submission.
//
// A batch owns one plan per instance (each with its own box, grid, split
// parameter and workspace) and a few branch streams.  An evaluation of the
// batch forks from an origin stream into the branches, enqueues every
// instance's full GGEM pipeline on the branch it was assigned to (the
// assignment balances an estimate of each instance's work: points times the
// local neighbourhood plus the grid), and joins back.  The same enqueue can
// be captured once into a HIP graph and replayed: one launch then submits
// every kernel of every instance, and the branches run concurrently.
//
// Shared launches (built, switched off; see ggem_batch_create): when every
// instance's targets are its sources (the suspension case) and the
// instances share one precision, the three pair-sum kernels would run as
// shared launches instead: one spread over every instance's tiles, one local sum
// over every instance's target items and one over every instance's wall
// nodes (job lists of per-instance arguments, uploaded when the batch is
// created).  A small instance then no longer leaves most of the GPU idle
// while it runs, and a large one no longer waits for a free stream.  The
// per-instance stages around them (binning, wall transforms, the grid
// stages, interpolation) stay on the branches.  Every block of a shared
// launch does exactly the work of the same block in the instance's own
// launch, so each instance still equals its solo evaluation bit for bit.
//
// Nothing in an evaluation allocates, synchronises with the host or records
// a memset node; domain checks are deferred (ggem_batch_status).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "ggem_internal.h"

using namespace ggem;

// One shared launch: its job list on the device.
struct JobGroup {
  void* jobs = nullptr;
  int* boff = nullptr;
  int n = 0, nblocks = 0;
  bool flag = false;  // spread: tile-relative staging; local sums: the FP32 fast path
};

struct ggem_batch_s {
  int n;
  std::vector<ggem_plan_t> plans;
  std::vector<int> branch_of;      // instance -> branch
  hipStream_t origin;              // fork/join point (owned, non-blocking)
  std::vector<hipStream_t> branches;
  hipEvent_t fork;
  std::vector<hipEvent_t> join;
  hipEvent_t caller_ready, done;
  hipGraph_t graph;
  hipGraphExec_t exec;
  // shared launches (all instances of one precision)
  bool shared = false;
  bool fp64 = false;
  hipStream_t side = nullptr;      // the local sums, beside the spread on origin
  hipEvent_t ev_go = nullptr, ev_spread = nullptr, ev_wall = nullptr, ev_near = nullptr;
  std::vector<JobGroup> spread_g, near_g, wall_g;
  void* job_mem = nullptr;
};

static thread_local char g_batch_err[256];

#define BATCH_TRY(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      snprintf(g_batch_err, sizeof g_batch_err, "%s: %s", #expr, hipGetErrorString(e_));  \
      return ggem_set_error(GGEM_E_DEVICE, g_batch_err);                                  \
    }                                                                                     \
  } while (0)

static void free_batch(ggem_batch_s* b) {
  if (b->job_mem) (void)hipFree(b->job_mem);
  for (hipEvent_t e : {b->ev_go, b->ev_spread, b->ev_wall, b->ev_near})
    if (e) (void)hipEventDestroy(e);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (ggem_plan_t p : b->plans)
    if (p) (void)ggem_plan_destroy(p);
  for (hipStream_t s : b->branches)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->caller_ready) (void)hipEventDestroy(b->caller_ready);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->origin) (void)hipStreamDestroy(b->origin);
}

// Work estimate of an instance: points times the local neighbourhood, plus
// the grid.
static double instance_cost(const ggem_params& q) {
  const double rc = q.rc > 0 ? q.rc : 4.0 / q.alpha;
  const double vol = q.Lx * q.Lz * 2.0 * q.H;
  const double nb = 4.18879 * rc * rc * rc;  // neighbourhood volume
  const double pts = (double)q.max_src;
  const double grid = (double)q.Nx * q.Nz * q.Ny;
  return pts * (1.0 + pts * nb / vol) + 20.0 * grid;
}

// Longest-processing-time assignment of instances to branches.
static void assign_branches(ggem_batch_s* b, const ggem_params* prm, int nbranch) {
  std::vector<double> cost(b->n);
  for (int i = 0; i < b->n; ++i) cost[i] = instance_cost(prm[i]);
  std::vector<int> order(b->n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  std::vector<double> load(nbranch, 0.0);
  b->branch_of.assign(b->n, 0);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->branch_of[i] = k;
    load[k] += cost[i];
  }
}

// Job lists of the shared launches, heaviest instances first (so that the
// long tiles start early), split by the kernel variant each instance takes.
static int setup_shared(ggem_batch_s* b, const ggem_params* prm) {
  const int n = b->n;
  b->fp64 = b->plans[0]->p.fp64;
  for (int i = 1; i < n; ++i)
    if (b->plans[i]->p.fp64 != b->fp64) return GGEM_OK;  // mixed precisions: no shared launches
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return instance_cost(prm[a]) > instance_cost(prm[c]);
  });
  std::vector<std::vector<Plan*>> lists(6);  // spread rel/not, near fast/not, wall fast/not
  for (int i : order) {
    Plan& p = b->plans[i]->p;
    lists[spread_job_rel(p) ? 0 : 1].push_back(&p);
    lists[near_job_fast(p) ? 2 : 3].push_back(&p);
    lists[near_job_fast(p) ? 4 : 5].push_back(&p);
  }
  const size_t nbytes = near_job_bytes(b->fp64);
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t total = 0;
  for (int g = 0; g < 6; ++g) {
    const size_t m = lists[g].size();
    if (m) total += align(m * (g < 2 ? spread_job_bytes() : nbytes)) + align((m + 1) * sizeof(int));
  }
  if (hipMalloc(&b->job_mem, total) != hipSuccess)
    return ggem_set_error(GGEM_E_NOMEM, "device allocation failed");
  char* mem = (char*)b->job_mem;
  for (int g = 0; g < 6; ++g) {
    const int m = (int)lists[g].size();
    if (!m) continue;
    JobGroup jg;
    jg.n = m;
    jg.jobs = mem;
    mem += align(m * (g < 2 ? spread_job_bytes() : nbytes));
    jg.boff = (int*)mem;
    mem += align((m + 1) * sizeof(int));
    jg.flag = (g % 2) == 0;
    jg.nblocks = g < 2 ? spread_jobs_upload(lists[g].data(), m, jg.jobs, jg.boff)
                       : near_jobs_upload(lists[g].data(), m, g >= 4, jg.jobs, jg.boff);
    if (jg.nblocks < 0) return ggem_set_error(GGEM_E_DEVICE, "job list upload failed");
    (g < 2 ? b->spread_g : g < 4 ? b->near_g : b->wall_g).push_back(jg);
  }
  if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_go, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_spread, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_wall, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_near, hipEventDisableTiming) != hipSuccess)
    return ggem_set_error(GGEM_E_DEVICE, "stream or event creation failed");
  b->shared = true;
  return GGEM_OK;
}

extern "C" int ggem_batch_create(int n_inst, const ggem_params* params, int n_branches,
                                 ggem_batch_t* out) {
  if (!out || !params) return ggem_set_error(GGEM_E_ARG, "null argument");
  *out = nullptr;
  if (n_inst < 1 || n_inst > 4096) return ggem_set_error(GGEM_E_ARG, "n_inst must be in 1..4096");
  if (n_branches < 1 || n_branches > 16)
    return ggem_set_error(GGEM_E_ARG, "n_branches must be in 1..16");
  ggem_batch_s* b = new (std::nothrow) ggem_batch_s();
  if (!b) return ggem_set_error(GGEM_E_NOMEM, "host allocation failed");
  b->n = n_inst;
  b->origin = nullptr;
  b->fork = b->caller_ready = b->done = nullptr;
  b->graph = nullptr;
  b->exec = nullptr;
  auto bail = [&](int rc) {
    free_batch(b);
    delete b;
    return rc;
  };
  if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->caller_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess)
    return bail(ggem_set_error(GGEM_E_DEVICE, "stream or event creation failed"));
  b->branches.assign(n_branches, nullptr);
  b->join.assign(n_branches, nullptr);
  for (int k = 0; k < n_branches; ++k)
    if (hipStreamCreateWithFlags(&b->branches[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) != hipSuccess)
      return bail(ggem_set_error(GGEM_E_DEVICE, "stream or event creation failed"));
  b->plans.assign(n_inst, nullptr);
  for (int i = 0; i < n_inst; ++i) {
    ggem_params q = params[i];
    q.sync_checks = 0;
    if (int rc = ggem_plan_create(&q, nullptr, &b->plans[i])) {
      char msg[200];
      snprintf(msg, sizeof msg, "instance %d: %s", i, ggem_last_error());
      return bail(ggem_set_error(rc, msg));
    }
  }
  assign_branches(b, params, n_branches);
  for (int i = 0; i < n_inst; ++i) b->plans[i]->p.stream = b->branches[b->branch_of[i]];
  // The shared launches stay switched off: the one graph capture of them
  // that ran ended in a host-side segmentation fault, whose cause has not
  // been shown.  Every evaluation takes the per-instance path below.
  (void)setup_shared;
  *out = b;
  return GGEM_OK;
}

extern "C" int ggem_batch_destroy(ggem_batch_t b) {
  if (!b) return ggem_set_error(GGEM_E_ARG, "null batch");
  (void)hipStreamSynchronize(b->origin);
  for (hipStream_t s : b->branches) (void)hipStreamSynchronize(s);
  if (b->side) (void)hipStreamSynchronize(b->side);
  free_batch(b);
  delete b;
  return GGEM_OK;
}

static int check_offsets(ggem_batch_s* b, const long long* src_off, const long long* tgt_off) {
  if (!src_off || !tgt_off) return ggem_set_error(GGEM_E_ARG, "null offsets");
  if (src_off[0] != 0 || tgt_off[0] != 0) return ggem_set_error(GGEM_E_ARG, "offsets must start at 0");
  for (int i = 0; i < b->n; ++i) {
    const long long ns = src_off[i + 1] - src_off[i], nt = tgt_off[i + 1] - tgt_off[i];
    if (ns < 0 || nt < 0) return ggem_set_error(GGEM_E_ARG, "offsets must not decrease");
    const ggem_params& q = b->plans[i]->p.p;
    if (ns > q.max_src || nt > q.max_tgt) {
      char msg[160];
      snprintf(msg, sizeof msg, "instance %d: %lld sources / %lld targets exceed its capacity", i,
               ns, nt);
      return ggem_set_error(GGEM_E_CAPACITY, msg);
    }
  }
  return GGEM_OK;
}

#define PHASE_TRY(i, expr)                                                    \
  do {                                                                        \
    if (int rc_ = (expr)) {                                                   \
      char msg_[200];                                                         \
      snprintf(msg_, sizeof msg_, "instance %d: %s", (i), ggem_last_error()); \
      return ggem_set_error(rc_, msg_);                                       \
    }                                                                         \
  } while (0)

// Shared launches (targets = sources for every instance).  origin forks to
// the branches, which bin their instances' sources; after the join, origin
// runs the shared spread while the side stream runs the shared local sums
// at the wall nodes and then at the targets; each branch then finishes its
// instances' wall data (after the wall sums), grid stages (after the
// spread) and interpolation (after the target sums), and joins.
template <typename T>
static int enqueue_shared_t(ggem_batch_s* b, const long long* so, const double* xs, const double* f,
                            double* u) {
  BATCH_TRY(hipEventRecord(b->fork, b->origin));
  for (hipStream_t s : b->branches) BATCH_TRY(hipStreamWaitEvent(s, b->fork, 0));
  for (int i = 0; i < b->n; ++i) {
    const long long ns = so[i + 1] - so[i];
    PHASE_TRY(i, batch_phase_bin<T>(b->plans[i]->p, ns, xs ? xs + 3 * so[i] : nullptr,
                                    f ? f + 3 * so[i] : nullptr));
  }
  for (size_t k = 0; k < b->branches.size(); ++k) {
    BATCH_TRY(hipEventRecord(b->join[k], b->branches[k]));
    BATCH_TRY(hipStreamWaitEvent(b->origin, b->join[k], 0));
  }
  BATCH_TRY(hipEventRecord(b->ev_go, b->origin));
  BATCH_TRY(hipStreamWaitEvent(b->side, b->ev_go, 0));
  for (const JobGroup& g : b->spread_g)
    BATCH_TRY(launch_spread_jobs<T>(b->origin, g.jobs, g.boff, g.n, g.nblocks, g.flag));
  BATCH_TRY(hipEventRecord(b->ev_spread, b->origin));
  for (const JobGroup& g : b->wall_g)
    BATCH_TRY(launch_near_jobs(b->side, b->fp64, g.flag, true, g.jobs, g.boff, g.n, g.nblocks));
  BATCH_TRY(hipEventRecord(b->ev_wall, b->side));
  for (const JobGroup& g : b->near_g)
    BATCH_TRY(launch_near_jobs(b->side, b->fp64, g.flag, false, g.jobs, g.boff, g.n, g.nblocks));
  BATCH_TRY(hipEventRecord(b->ev_near, b->side));
  for (hipStream_t s : b->branches) BATCH_TRY(hipStreamWaitEvent(s, b->ev_wall, 0));
  for (int i = 0; i < b->n; ++i) PHASE_TRY(i, batch_phase_wall<T>(b->plans[i]->p));
  for (hipStream_t s : b->branches) BATCH_TRY(hipStreamWaitEvent(s, b->ev_spread, 0));
  for (int i = 0; i < b->n; ++i) PHASE_TRY(i, batch_phase_grid<T>(b->plans[i]->p));
  for (hipStream_t s : b->branches) BATCH_TRY(hipStreamWaitEvent(s, b->ev_near, 0));
  for (int i = 0; i < b->n; ++i)
    PHASE_TRY(i, batch_phase_interp<T>(b->plans[i]->p, so[i + 1] - so[i], u + 3 * so[i]));
  for (size_t k = 0; k < b->branches.size(); ++k) {
    BATCH_TRY(hipEventRecord(b->join[k], b->branches[k]));
    BATCH_TRY(hipStreamWaitEvent(b->origin, b->join[k], 0));
  }
  BATCH_TRY(hipStreamWaitEvent(b->origin, b->ev_near, 0));
  return GGEM_OK;
}

// fork from the origin stream, every instance on its branch, join
static int enqueue(ggem_batch_s* b, const long long* so, const double* xs, const double* f,
                   const long long* to, const double* xt, double* u) {
  bool coincide = b->shared && xs == xt;
  for (int i = 0; coincide && i <= b->n; ++i) coincide = so[i] == to[i];
  if (coincide)
    return b->fp64 ? enqueue_shared_t<double>(b, so, xs, f, u) : enqueue_shared_t<float>(b, so, xs, f, u);
  BATCH_TRY(hipEventRecord(b->fork, b->origin));
  for (hipStream_t s : b->branches) BATCH_TRY(hipStreamWaitEvent(s, b->fork, 0));
  for (int i = 0; i < b->n; ++i) {
    const long long ns = so[i + 1] - so[i], nt = to[i + 1] - to[i];
    if (nt == 0) continue;
    const double* xsi = xs ? xs + 3 * so[i] : nullptr;
    const double* fi = f ? f + 3 * so[i] : nullptr;
    const double* xti = xt + 3 * to[i];
    // sources that coincide with the targets share their binning
    const double* xt_use = (xs == xt && so[i] == to[i] && ns == nt) ? xsi : xti;
    if (int rc = ggem_single_layer(b->plans[i], ns, xsi, fi, nt, xt_use, u + 3 * to[i],
                                   GGEM_PART_ALL)) {
      char msg[200];
      snprintf(msg, sizeof msg, "instance %d: %s", i, ggem_last_error());
      return ggem_set_error(rc, msg);
    }
  }
  for (size_t k = 0; k < b->branches.size(); ++k) {
    BATCH_TRY(hipEventRecord(b->join[k], b->branches[k]));
    BATCH_TRY(hipStreamWaitEvent(b->origin, b->join[k], 0));
  }
  return GGEM_OK;
}

extern "C" int ggem_batch_single_layer(ggem_batch_t b, void* hip_stream, const long long* src_off,
                                       const double* xs, const double* f, const long long* tgt_off,
                                       const double* xt, double* u) {
  if (!b) return ggem_set_error(GGEM_E_ARG, "null batch");
  if (int rc = check_offsets(b, src_off, tgt_off)) return rc;
  if (tgt_off[b->n] > 0 && (!xt || !u)) return ggem_set_error(GGEM_E_ARG, "null target array");
  if (src_off[b->n] > 0 && (!xs || !f)) return ggem_set_error(GGEM_E_ARG, "null source array");
  hipStream_t caller = (hipStream_t)hip_stream;
  BATCH_TRY(hipEventRecord(b->caller_ready, caller));
  BATCH_TRY(hipStreamWaitEvent(b->origin, b->caller_ready, 0));
  if (int rc = enqueue(b, src_off, xs, f, tgt_off, xt, u)) return rc;
  BATCH_TRY(hipEventRecord(b->done, b->origin));
  BATCH_TRY(hipStreamWaitEvent(caller, b->done, 0));
  return GGEM_OK;
}

extern "C" int ggem_batch_capture_single_layer(ggem_batch_t b, const long long* src_off,
                                               const double* xs, const double* f,
                                               const long long* tgt_off, const double* xt,
                                               double* u) {
  if (!b) return ggem_set_error(GGEM_E_ARG, "null batch");
  if (int rc = check_offsets(b, src_off, tgt_off)) return rc;
  if (tgt_off[b->n] > 0 && (!xt || !u)) return ggem_set_error(GGEM_E_ARG, "null target array");
  if (src_off[b->n] > 0 && (!xs || !f)) return ggem_set_error(GGEM_E_ARG, "null source array");
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  BATCH_TRY(hipStreamSynchronize(b->origin));
  BATCH_TRY(hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal));
  int rc = enqueue(b, src_off, xs, f, tgt_off, xt, u);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->origin, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  BATCH_TRY(e);
  b->graph = g;
  BATCH_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return GGEM_OK;
}

extern "C" int ggem_batch_graph_launch(ggem_batch_t b, void* hip_stream) {
  if (!b) return ggem_set_error(GGEM_E_ARG, "null batch");
  if (!b->exec) return ggem_set_error(GGEM_E_ARG, "nothing captured");
  BATCH_TRY(hipGraphLaunch(b->exec, (hipStream_t)hip_stream));
  return GGEM_OK;
}

extern "C" int ggem_batch_status(ggem_batch_t b, void* hip_stream) {
  if (!b) return ggem_set_error(GGEM_E_ARG, "null batch");
  BATCH_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
  BATCH_TRY(hipStreamSynchronize(b->origin));
  for (int i = 0; i < b->n; ++i) {
    Plan& p = b->plans[i]->p;
    BATCH_TRY(hipMemcpy(p.flags_host, p.flags, sizeof(unsigned), hipMemcpyDeviceToHost));
    const unsigned fl = *p.flags_host;
    if (fl & (kFlagNonFinite | kFlagOutside)) {
      char msg[160];
      snprintf(msg, sizeof msg, "instance %d: %s", i,
               (fl & kFlagNonFinite) ? "non-finite input position" : "point outside the slit");
      return ggem_set_error(GGEM_E_DOMAIN, msg);
    }
  }
  return GGEM_OK;
}

extern "C" int ggem_batch_branch(ggem_batch_t b, int instance) {
  if (!b || instance < 0 || instance >= b->n) return ggem_set_error(GGEM_E_ARG, "bad instance");
  return b->branch_of[instance];
}
