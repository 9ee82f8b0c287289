// Fredholm second-kind equation for the single-layer density (Eq. qa,
// discretised as in Sec. 5): at every element node x_b
//   q_j(x_b) + (kappa_b/4pi) n_k(x_b) sum_n int q_i(x) T_jik(x_b, x) dS(x) = b_j(x_b),
// i.e. (I + kappa/4pi D) q = b, solved by restarted GMRES (Sec. 5) with
// every matrix-vector product evaluated by the GGEM double layer.
//
// Surface integral: q is linear on each flat triangle (Sec. 3.3.1); the
// integral over a triangle uses its three interior Gauss points (barycentric
// (2/3,1/6,1/6) and permutations, weight area/3), so
//   int q_i T_jik n_k dS ~= 8 pi v_j,  v = ggem_double_layer(Gauss points,
//   strengths q(x_g) w_g; targets = nodes, target normals n(x_b)),
// and the operator is y = q + 2 kappa v.  Nodes never coincide with Gauss
// points, so no pair is singular.
//
// GMRES(m) of gmres.h: classical Gram-Schmidt applied twice; Krylov vectors,
// dot products and norms in FP64 with fixed-order reductions; the small
// Hessenberg problem (Givens rotations) on the host.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "ggem_internal.h"
#include "gmres.h"

using namespace ggem;

namespace {

// Gauss points and weights of every triangle.  A triangle whose node index
// lies outside [0, nnode) raises *bad and gets zero weight at the origin, so
// nothing reads outside the node array.
__global__ void gauss_setup(int ntri, int nnode, const int* __restrict__ tri,
                            const double* __restrict__ xn, double* __restrict__ gpos,
                            double* __restrict__ gw, int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  if ((unsigned)a >= (unsigned)nnode || (unsigned)b >= (unsigned)nnode ||
      (unsigned)c >= (unsigned)nnode) {
    atomicOr(bad, 1);
    for (int g = 3 * t; g < 3 * t + 3; ++g) {
      gpos[3 * (size_t)g] = gpos[3 * (size_t)g + 1] = gpos[3 * (size_t)g + 2] = 0.0;
      gw[g] = 0.0;
    }
    return;
  }
  double A[3], B[3], Cc[3];
  for (int d = 0; d < 3; ++d) {
    A[d] = xn[3 * (size_t)a + d];
    B[d] = xn[3 * (size_t)b + d];
    Cc[d] = xn[3 * (size_t)c + d];
  }
  const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  const double e2[3] = {Cc[0] - A[0], Cc[1] - A[1], Cc[2] - A[2]};
  const double cx = e1[1] * e2[2] - e1[2] * e2[1];
  const double cy = e1[2] * e2[0] - e1[0] * e2[2];
  const double cz = e1[0] * e2[1] - e1[1] * e2[0];
  const double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
  const double hi = 2.0 / 3.0, lo = 1.0 / 6.0;
  for (int gp = 0; gp < 3; ++gp) {
    const double la = gp == 0 ? hi : lo, lb = gp == 1 ? hi : lo, lc = gp == 2 ? hi : lo;
    const size_t g = 3 * (size_t)t + gp;
    for (int d = 0; d < 3; ++d) gpos[3 * g + d] = la * A[d] + lb * B[d] + lc * Cc[d];
    gw[g] = area / 3.0;
  }
}

// Gauss-point strengths q(x_g) w_g from nodal q (linear interpolation).
__global__ void gauss_strengths(int ntri, const int* __restrict__ tri, const double* __restrict__ q,
                                const double* __restrict__ gw, double* __restrict__ gs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  const double hi = 2.0 / 3.0, lo = 1.0 / 6.0;
  for (int gp = 0; gp < 3; ++gp) {
    const double la = gp == 0 ? hi : lo, lb = gp == 1 ? hi : lo, lc = gp == 2 ? hi : lo;
    const size_t g = 3 * (size_t)t + gp;
    for (int d = 0; d < 3; ++d)
      gs[3 * g + d] = gw[g] * (la * q[3 * (size_t)a + d] + lb * q[3 * (size_t)b + d] +
                               lc * q[3 * (size_t)c + d]);
  }
}

// y = x + 2 kappa v (per node kappa, or a uniform value)
__global__ void fredholm_combine(int n3, const double* __restrict__ x, const double* __restrict__ v,
                                 const double* __restrict__ kappa, double kappa0,
                                 double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const double k = kappa ? kappa[i / 3] : kappa0;
  y[i] = x[i] + 2.0 * k * v[i];
}

__global__ void fill_ints(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

struct ggem_solver_s {
  ggem_plan_s* plan;
  long long max_nodes, max_tri;
  int restart;
  double *gpos, *gw, *gs;  // Gauss points, weights, strengths
  double* v;               // double-layer output of one product
  gm::Work W;              // GMRES workspace (Krylov basis of 3 max_nodes)
  int *bad, *bad_host;  // triangle index check
  // geometry of the current solve
  int n_nodes, n_tri;
  const double *nodes, *normals, *kappa;
  double kappa0;
  const int* tri;
};

namespace ggem {
hipStream_t solver_stream(ggem_solver_t s) { return s->plan->p.stream; }
long long solver_max_nodes(ggem_solver_t s) { return s->max_nodes; }
long long solver_max_tri(ggem_solver_t s) { return s->max_tri; }
}  // namespace ggem

static thread_local char g_solver_err[256];

#define SOLVER_TRY(expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      snprintf(g_solver_err, sizeof g_solver_err, "%s: %s", #expr, hipGetErrorString(e_)); \
      ggem_set_error(GGEM_E_DEVICE, g_solver_err);                                    \
      return GGEM_E_DEVICE;                                                           \
    }                                                                                 \
  } while (0)

static void free_solver(ggem_solver_s* s) {
  void* ptrs[] = {s->gpos, s->gw, s->gs, s->v, s->bad};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (s->bad_host) (void)hipHostFree(s->bad_host);
  gm::free_work(s->W);
}

extern "C" int ggem_solver_create(ggem_plan_t plan, const ggem_solver_params* prm,
                                  ggem_solver_t* out) {
  if (!plan || !prm || !out) return ggem_set_error(GGEM_E_ARG, "null argument");
  *out = nullptr;
  if (prm->restart < 1 || prm->restart > 200)
    return ggem_set_error(GGEM_E_ARG, "restart must be in 1..200");
  if (prm->max_nodes < 1 || prm->max_tri < 1 || prm->max_nodes > (1LL << 28) ||
      prm->max_tri > (1LL << 28))
    return ggem_set_error(GGEM_E_ARG, "capacities out of range");
  if (3 * prm->max_tri > plan->p.p.max_src || prm->max_nodes > plan->p.p.max_tgt)
    return ggem_set_error(GGEM_E_CAPACITY,
                          "plan capacity must cover 3 Gauss points per triangle and the nodes");
  ggem_solver_s* s = new (std::nothrow) ggem_solver_s();
  if (!s) return ggem_set_error(GGEM_E_NOMEM, "host allocation failed");
  memset(s, 0, sizeof *s);
  s->plan = plan;
  s->max_nodes = prm->max_nodes;
  s->max_tri = prm->max_tri;
  s->restart = prm->restart;
  const size_t n3 = 3 * (size_t)prm->max_nodes, ng = 3 * (size_t)prm->max_tri;
  bool ok = hipMalloc((void**)&s->gpos, 3 * ng * 8) == hipSuccess &&
            hipMalloc((void**)&s->gw, ng * 8) == hipSuccess &&
            hipMalloc((void**)&s->gs, 3 * ng * 8) == hipSuccess &&
            hipMalloc((void**)&s->v, n3 * 8) == hipSuccess &&
            hipMalloc((void**)&s->bad, sizeof(int)) == hipSuccess &&
            hipHostMalloc((void**)&s->bad_host, sizeof(int), 0) == hipSuccess &&
            gm::alloc_work(s->W, n3, prm->restart) == GGEM_OK;
  s->W.st = plan->p.stream;
  if (!ok) {
    free_solver(s);
    delete s;
    return ggem_set_error(GGEM_E_NOMEM, "device allocation failed");
  }
  *out = s;
  return GGEM_OK;
}

extern "C" int ggem_solver_destroy(ggem_solver_t s) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  (void)hipStreamSynchronize(s->plan->p.stream);
  free_solver(s);
  delete s;
  return GGEM_OK;
}

static int set_geometry(ggem_solver_s* s, long long n_nodes, const double* nodes,
                        const double* normals, const double* kappa, double kappa0,
                        long long n_tri, const int* tri) {
  if (n_nodes < 1 || n_tri < 1) return ggem_set_error(GGEM_E_ARG, "empty surface");
  if (n_nodes > s->max_nodes || n_tri > s->max_tri)
    return ggem_set_error(GGEM_E_CAPACITY, "surface exceeds the solver capacity");
  if (!nodes || !normals || !tri) return ggem_set_error(GGEM_E_ARG, "null surface array");
  s->n_nodes = (int)n_nodes;
  s->n_tri = (int)n_tri;
  s->nodes = nodes;
  s->normals = normals;
  s->kappa = kappa;
  s->kappa0 = kappa0;
  s->tri = tri;
  hipStream_t st = s->plan->p.stream;
  fill_ints<<<1, 64, 0, st>>>(s->bad, 1, 0);
  gauss_setup<<<(s->n_tri + 255) / 256, 256, 0, st>>>(s->n_tri, s->n_nodes, tri, nodes, s->gpos,
                                                      s->gw, s->bad);
  SOLVER_TRY(hipGetLastError());
  SOLVER_TRY(hipMemcpyAsync(s->bad_host, s->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  SOLVER_TRY(hipStreamSynchronize(st));
  if (*s->bad_host) return ggem_set_error(GGEM_E_ARG, "triangle node index out of range");
  return GGEM_OK;
}

// y = (I + kappa/4pi D) x
static int apply(ggem_solver_s* s, const double* x, double* y) {
  hipStream_t st = s->plan->p.stream;
  gauss_strengths<<<(s->n_tri + 255) / 256, 256, 0, st>>>(s->n_tri, s->tri, x, s->gw, s->gs);
  SOLVER_TRY(hipGetLastError());
  int rc = ggem_double_layer(s->plan, 3LL * s->n_tri, s->gpos, s->gs, s->n_nodes, s->nodes,
                             s->normals, s->v, GGEM_PART_ALL);
  if (rc) return rc;
  const int n3 = 3 * s->n_nodes;
  fredholm_combine<<<(n3 + 255) / 256, 256, 0, st>>>(n3, x, s->v, s->kappa, s->kappa0, y);
  SOLVER_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_fredholm_apply(ggem_solver_t s, long long n_nodes, const double* nodes,
                                   const double* normals, const double* kappa, double kappa0,
                                   long long n_tri, const int* tri, const double* x, double* y) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (!x || !y) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (int rc = set_geometry(s, n_nodes, nodes, normals, kappa, kappa0, n_tri, tri)) return rc;
  return apply(s, x, y);
}

// GMRES(m) from the guess q; with dq, the first residual is first reduced
// along A dq (see ggem_fredholm_solve_guided).
static int solve_impl(ggem_solver_t s, long long n_nodes, const double* nodes,
                      const double* normals, const double* kappa, double kappa0, long long n_tri,
                      const int* tri, const double* b, double* q, const double* dq, double tol,
                      int max_iter, int* iters, double* rel_res, double* step) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (!b || !q) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (!(tol > 0) || max_iter < 1) return ggem_set_error(GGEM_E_ARG, "bad tolerance or max_iter");
  if (int rc = set_geometry(s, n_nodes, nodes, normals, kappa, kappa0, n_tri, tri)) return rc;
  gm::Work& W = s->W;
  W.st = s->plan->p.stream;
  const int n = 3 * (int)n_nodes;
  if (step) *step = 0.0;
  auto op = [s](const double* x, double* y) { return apply(s, x, y); };
  // guided start: c = argmin |r - c A dq| over c >= 0; q += c dq, r -= c A dq
  auto guide = [&](double* r) -> int {
    if (!dq) return GGEM_OK;
    if (int rc = apply(s, dq, W.w)) return rc;
    double rw, ww;
    if (int rc = gm::dots(W, r, 0, 1, W.w, n, &rw)) return rc;
    if (int rc = gm::dots(W, W.w, 0, 1, W.w, n, &ww)) return rc;
    const double c = (ww > 0.0 && rw > 0.0) ? rw / ww : 0.0;
    if (c > 0.0) {
      if (int rc = gm::axpy_host(W, n, c, dq, q)) return rc;
      if (int rc = gm::axpy_host(W, n, -c, W.w, r)) return rc;
    }
    if (step) *step = c;
    return GGEM_OK;
  };
  return gm::solve(W, n, b, q, tol, max_iter, op, guide, iters, rel_res);
}

extern "C" int ggem_fredholm_solve(ggem_solver_t s, long long n_nodes, const double* nodes,
                                   const double* normals, const double* kappa, double kappa0,
                                   long long n_tri, const int* tri, const double* b, double* q,
                                   double tol, int max_iter, int* iters, double* rel_res) {
  return solve_impl(s, n_nodes, nodes, normals, kappa, kappa0, n_tri, tri, b, q, nullptr, tol,
                    max_iter, iters, rel_res, nullptr);
}

extern "C" int ggem_fredholm_solve_guided(ggem_solver_t s, long long n_nodes, const double* nodes,
                                          const double* normals, const double* kappa,
                                          double kappa0, long long n_tri, const int* tri,
                                          const double* b, double* q, const double* dq,
                                          double tol, int max_iter, int* iters, double* rel_res,
                                          double* step) {
  if (!dq) return ggem_set_error(GGEM_E_ARG, "null correction");
  return solve_impl(s, n_nodes, nodes, normals, kappa, kappa0, n_tri, tri, b, q, dq, tol,
                    max_iter, iters, rel_res, step);
}

// ---- surface quantities of a drop suspension ------------------------------

namespace {

// Per node: area-averaged normal (Sec. 3.5.2), node area (one third of each
// incident triangle, Sec. 4) and the cotangent Laplace-Beltrami of the
// position, (Lap x)_i = 1/(2 A_i) sum (cot a + cot b)(x_j - x_i), gathered
// over the node's incident triangles (fixed order, no atomics).  A node
// whose incidence list names a triangle out of range, or a triangle that
// does not contain the node or has a corner out of range, raises *bad.
__global__ void surface_geometry(int nnode, int ntri, const double* __restrict__ xn,
                                 const int* __restrict__ tri, const int* __restrict__ off,
                                 const int* __restrict__ adj, double* __restrict__ nrm,
                                 double* __restrict__ area, double* __restrict__ lap,
                                 int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnode) return;
  const int b0 = off[i], b1 = off[i + 1];
  if (b0 < 0 || b1 < b0 || b1 > 3 * ntri) {
    atomicOr(bad, 1);
    return;
  }
  const double xi0 = xn[3 * (size_t)i], xi1 = xn[3 * (size_t)i + 1], xi2 = xn[3 * (size_t)i + 2];
  double an0 = 0, an1 = 0, an2 = 0, A = 0, l0 = 0, l1 = 0, l2 = 0;
  for (int e = b0; e < b1; ++e) {
    const int t = adj[e];
    if ((unsigned)t >= (unsigned)ntri) {
      atomicOr(bad, 1);
      return;
    }
    const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    int j, k;
    if (a == i) {
      j = b;
      k = c;
    } else if (b == i) {
      j = c;
      k = a;
    } else if (c == i) {
      j = a;
      k = b;
    } else {
      atomicOr(bad, 1);
      return;
    }
    if ((unsigned)j >= (unsigned)nnode || (unsigned)k >= (unsigned)nnode) {
      atomicOr(bad, 1);
      return;
    }
    const double ej0 = xn[3 * (size_t)j] - xi0, ej1 = xn[3 * (size_t)j + 1] - xi1,
                 ej2 = xn[3 * (size_t)j + 2] - xi2;
    const double ek0 = xn[3 * (size_t)k] - xi0, ek1 = xn[3 * (size_t)k + 1] - xi1,
                 ek2 = xn[3 * (size_t)k + 2] - xi2;
    // twice the area vector (orientation of the triangle as given)
    const double c0 = ej1 * ek2 - ej2 * ek1, c1 = ej2 * ek0 - ej0 * ek2, c2 = ej0 * ek1 - ej1 * ek0;
    const double cn = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    an0 += c0;
    an1 += c1;
    an2 += c2;
    A += cn / 6.0;
    // cot of the angle at k (faces edge i-j) and at j (faces edge i-k)
    const double jk0 = ek0 - ej0, jk1 = ek1 - ej1, jk2 = ek2 - ej2;  // x_k - x_j
    const double cot_k = ((-ek0) * (ej0 - ek0) + (-ek1) * (ej1 - ek1) + (-ek2) * (ej2 - ek2)) / cn;
    const double cot_j = ((-ej0) * jk0 + (-ej1) * jk1 + (-ej2) * jk2) / cn;
    l0 += cot_k * ej0 + cot_j * ek0;
    l1 += cot_k * ej1 + cot_j * ek1;
    l2 += cot_k * ej2 + cot_j * ek2;
  }
  const double inv = 1.0 / sqrt(an0 * an0 + an1 * an1 + an2 * an2);
  nrm[3 * (size_t)i] = an0 * inv;
  nrm[3 * (size_t)i + 1] = an1 * inv;
  nrm[3 * (size_t)i + 2] = an2 * inv;
  area[i] = A;
  const double s = 1.0 / (2.0 * A);
  lap[3 * (size_t)i] = l0 * s;
  lap[3 * (size_t)i + 1] = l1 * s;
  lap[3 * (size_t)i + 2] = l2 * s;
}

// b = -(1/4pi) (dF/(lambda+1) + kappa f_inf), dF = -(1/Ca) Lap x,
// f_inf = shear (n_y, n_x, 0)
__global__ void drop_rhs_kernel(int nnode, const double* __restrict__ nrm,
                                const double* __restrict__ lap, double lam, double inv_ca,
                                double shear, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnode) return;
  const double kappa = (lam - 1.0) / (lam + 1.0);
  const double s = -1.0 / (4.0 * M_PI);
  const double fi[3] = {shear * nrm[3 * (size_t)i + 1], shear * nrm[3 * (size_t)i], 0.0};
  for (int d = 0; d < 3; ++d) {
    const double df = -inv_ca * lap[3 * (size_t)i + d];
    b[3 * (size_t)i + d] = s * (df / (lam + 1.0) + kappa * fi[d]);
  }
}

// b = -(1/4pi) (dF/(lambda+1) + kappa f_inf) for a given traction jump dF
__global__ void traction_rhs_kernel(int nnode, const double* __restrict__ nrm,
                                    const double* __restrict__ df, double lam, double shear,
                                    double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnode) return;
  const double kappa = (lam - 1.0) / (lam + 1.0);
  const double s = -1.0 / (4.0 * M_PI);
  const double fi[3] = {shear * nrm[3 * (size_t)i + 1], shear * nrm[3 * (size_t)i], 0.0};
  for (int d = 0; d < 3; ++d)
    b[3 * (size_t)i + d] = s * (df[3 * (size_t)i + d] / (lam + 1.0) + kappa * fi[d]);
}

// u = (shear y, 0, 0) + 8 pi u_sl
__global__ void velocity_finish(int nnode, const double* __restrict__ xn, double shear,
                                double* __restrict__ u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnode) return;
  const double e = 8.0 * M_PI;
  u[3 * (size_t)i] = fma(e, u[3 * (size_t)i], shear * xn[3 * (size_t)i + 1]);
  u[3 * (size_t)i + 1] *= e;
  u[3 * (size_t)i + 2] *= e;
}

__global__ void axpy_out(long long n, const double* __restrict__ x, const double* __restrict__ u,
                         double dt, double* __restrict__ out) {
  const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (j < n) out[j] = fma(dt, u[j], x[j]);
}

}  // namespace

static int read_flag(ggem_solver_s* s, const char* msg) {
  hipStream_t st = s->plan->p.stream;
  SOLVER_TRY(hipGetLastError());
  SOLVER_TRY(hipMemcpyAsync(s->bad_host, s->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  SOLVER_TRY(hipStreamSynchronize(st));
  if (*s->bad_host) return ggem_set_error(GGEM_E_ARG, msg);
  return GGEM_OK;
}

extern "C" int ggem_surface_geometry(ggem_solver_t s, long long n_nodes, const double* nodes,
                                     long long n_tri, const int* tri, const int* node_tri_off,
                                     const int* node_tri, double* normals, double* area,
                                     double* lap) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (n_nodes < 1 || n_tri < 1) return ggem_set_error(GGEM_E_ARG, "empty surface");
  if (n_nodes > s->max_nodes || n_tri > s->max_tri)
    return ggem_set_error(GGEM_E_CAPACITY, "surface exceeds the solver capacity");
  if (!nodes || !tri || !node_tri_off || !node_tri || !normals || !area || !lap)
    return ggem_set_error(GGEM_E_ARG, "null array");
  hipStream_t st = s->plan->p.stream;
  const int n = (int)n_nodes;
  fill_ints<<<1, 64, 0, st>>>(s->bad, 1, 0);
  surface_geometry<<<(n + 255) / 256, 256, 0, st>>>(n, (int)n_tri, nodes, tri, node_tri_off,
                                                    node_tri, normals, area, lap, s->bad);
  return read_flag(s, "inconsistent triangle incidence lists");
}

extern "C" int ggem_drop_rhs(ggem_solver_t s, long long n_nodes, const double* normals,
                             const double* lap, double lambda, double inv_ca, double shear_rate,
                             double* b) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (n_nodes < 1 || n_nodes > s->max_nodes)
    return ggem_set_error(GGEM_E_CAPACITY, "node count outside 1..capacity");
  if (!normals || !lap || !b) return ggem_set_error(GGEM_E_ARG, "null array");
  if (!(lambda > 0) || !isfinite(inv_ca) || !isfinite(shear_rate))
    return ggem_set_error(GGEM_E_ARG, "lambda must be positive, inv_ca and shear finite");
  const int n = (int)n_nodes;
  drop_rhs_kernel<<<(n + 255) / 256, 256, 0, s->plan->p.stream>>>(n, normals, lap, lambda, inv_ca,
                                                                  shear_rate, b);
  SOLVER_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_traction_rhs(ggem_solver_t s, long long n_nodes, const double* normals,
                                 const double* df, double lambda, double shear_rate, double* b) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (n_nodes < 1 || n_nodes > s->max_nodes)
    return ggem_set_error(GGEM_E_CAPACITY, "node count outside 1..capacity");
  if (!normals || !df || !b) return ggem_set_error(GGEM_E_ARG, "null array");
  if (!(lambda > 0) || !isfinite(lambda) || !isfinite(shear_rate))
    return ggem_set_error(GGEM_E_ARG, "lambda must be positive, shear finite");
  const int n = (int)n_nodes;
  traction_rhs_kernel<<<(n + 255) / 256, 256, 0, s->plan->p.stream>>>(n, normals, df, lambda,
                                                                      shear_rate, b);
  SOLVER_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_surface_velocity(ggem_solver_t s, long long n_nodes, const double* nodes,
                                     long long n_tri, const int* tri, const double* q,
                                     double shear_rate, double* u) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (!q || !u) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (!isfinite(shear_rate)) return ggem_set_error(GGEM_E_ARG, "shear rate must be finite");
  // the normals are not used by the single layer; the node array stands in
  if (int rc = set_geometry(s, n_nodes, nodes, nodes, nullptr, 0.0, n_tri, tri)) return rc;
  hipStream_t st = s->plan->p.stream;
  gauss_strengths<<<(s->n_tri + 255) / 256, 256, 0, st>>>(s->n_tri, s->tri, q, s->gw, s->gs);
  SOLVER_TRY(hipGetLastError());
  int rc = ggem_single_layer(s->plan, 3LL * s->n_tri, s->gpos, s->gs, s->n_nodes, s->nodes, u,
                             GGEM_PART_ALL);
  if (rc) return rc;
  velocity_finish<<<(s->n_nodes + 255) / 256, 256, 0, st>>>(s->n_nodes, nodes, shear_rate, u);
  SOLVER_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_advance(ggem_solver_t s, long long n, const double* x, const double* u,
                            double dt, double* out) {
  if (!s) return ggem_set_error(GGEM_E_ARG, "null solver");
  if (n < 0 || (n > 0 && (!x || !u || !out))) return ggem_set_error(GGEM_E_ARG, "bad arrays");
  if (n == 0) return GGEM_OK;
  axpy_out<<<(unsigned)((n + 255) / 256), 256, 0, s->plan->p.stream>>>(n, x, u, dt, out);
  SOLVER_TRY(hipGetLastError());
  return GGEM_OK;
}
