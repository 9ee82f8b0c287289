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

// Longest-processing-time assignment of instances to branches.
static void assign_branches(ggem_batch_s* b, const ggem_params* prm, int nbranch) {
  std::vector<double> cost(b->n);
  for (int i = 0; i < b->n; ++i) {
    const ggem_params& q = prm[i];
    const double rc = q.rc > 0 ? q.rc : 4.0 / q.alpha;
    const double vol = q.Lx * q.Lz * 2.0 * q.H;
    const double nb = 4.18879 * rc * rc * rc;  // neighbourhood volume
    const double pts = (double)q.max_src;
    const double grid = (double)q.Nx * q.Nz * q.Ny;
    cost[i] = pts * (1.0 + pts * nb / vol) + 20.0 * grid;
  }
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
  *out = b;
  return GGEM_OK;
}

extern "C" int ggem_batch_destroy(ggem_batch_t b) {
  if (!b) return ggem_set_error(GGEM_E_ARG, "null batch");
  (void)hipStreamSynchronize(b->origin);
  for (hipStream_t s : b->branches) (void)hipStreamSynchronize(s);
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

// fork from the origin stream, every instance on its branch, join
static int enqueue(ggem_batch_s* b, const long long* so, const double* xs, const double* f,
                   const long long* to, const double* xt, double* u) {
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
