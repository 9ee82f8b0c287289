// Neo-Hookean capsules: membrane traction jump, volumes, volume and overlap
// corrections and the minimum node separation of the time-step rule.
//
// Membrane (Sec. 4).  Each flat element stores the neo-Hookean energy
// A0 W(C), W = (G/2)(tr C + 1/det C - 3) (Eq. WNH: tr C = l1^2 + l2^2,
// det C = l1^2 l2^2), C = F^T F the right Cauchy-Green tensor of the
// element's uniform deformation.  With the reference edges expressed in the
// reference element's own orthonormal frame, D = [E1 E2] (2 x 2), and the
// deformed edges in space, e = [e1 e2] (3 x 2), the deformation gradient is
// the 3 x 2 matrix F = e D^-1, which needs no rotation of the deformed
// element into a common plane (the energy is invariant under rigid motions,
// and out-of-plane virtual displacements of a flat element change it only
// at second order).  The virtual-work derivatives of the energy are
//   dE/de = A0 P D^-T,  P = F S,  S = 2 dW/dC = G (I - C^-1 / det C),
// so dE/dx_b = dE/de1, dE/dx_c = dE/de2, dE/dx_a = -(both).  The traction
// jump at a node is (1/A_p) sum over its elements of dE/dx_p (Eq. cntr2 with
// the reaction force F_p = -dE/dx_p), A_p one third of the current area of
// its elements.  Every node sums its elements in the order of its incidence
// list: no atomics, results bitwise reproducible.
//
// Capsules are consecutive, equal groups of nodes and triangles; every
// triangle names nodes of its own capsule (checked at creation).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ggem_internal.h"

namespace {

constexpr int kPairsPerCapsule = 64;  // capacity of the close-pair list per capsule

struct Pair {
  int i, j;
  double gap;
};

__device__ inline double3 ld3(const double* x, size_t i) {
  return make_double3(x[3 * i], x[3 * i + 1], x[3 * i + 2]);
}
__device__ inline double3 sub(double3 a, double3 b) { return make_double3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline double dot(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline double3 cross(double3 a, double3 b) {
  return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline double3 axpy(double s, double3 a, double3 b) {
  return make_double3(fma(s, a.x, b.x), fma(s, a.y, b.y), fma(s, a.z, b.z));
}

// Reference data of each element: D^-1 (row-major, 4) and the reference area.
__global__ void membrane_ref(int ntri, int npc, int tpc, const int* __restrict__ tri,
                             const double* __restrict__ x0, double* __restrict__ ref,
                             int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  const int lo = (t / tpc) * npc, hi = lo + npc;
  const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  if (a < lo || a >= hi || b < lo || b >= hi || c < lo || c >= hi) {
    atomicOr(bad, 1);
    return;
  }
  const double3 xa = ld3(x0, a), e1 = sub(ld3(x0, b), xa), e2 = sub(ld3(x0, c), xa);
  const double l1 = sqrt(dot(e1, e1));
  const double3 t1 = make_double3(e1.x / l1, e1.y / l1, e1.z / l1);
  double3 n = cross(e1, e2);
  const double nn = sqrt(dot(n, n));
  n = make_double3(n.x / nn, n.y / nn, n.z / nn);
  const double3 t2 = cross(n, t1);
  // D = [[l1, e2.t1], [0, e2.t2]] (columns: the reference edges in the frame)
  const double d11 = l1, d12 = dot(e2, t1), d22 = dot(e2, t2);
  const double det = d11 * d22;
  double* r = ref + 5 * (size_t)t;
  r[0] = 1.0 / d11;          // D^-1 = [[1/d11, -d12/det], [0, 1/d22]]
  r[1] = -d12 / det;
  r[2] = 0.0;
  r[3] = 1.0 / d22;
  r[4] = 0.5 * det;          // A0
}

// Per element: dE/dx at its three vertices (9), its energy and its current
// area.
__global__ void membrane_elem(int ntri, const int* __restrict__ tri, const double* __restrict__ x,
                              const double* __restrict__ ref, double G, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  const double3 xa = ld3(x, a), e1 = sub(ld3(x, b), xa), e2 = sub(ld3(x, c), xa);
  const double* r = ref + 5 * (size_t)t;
  const double i00 = r[0], i01 = r[1], i10 = r[2], i11 = r[3], A0 = r[4];
  // F = e D^-1: columns f1 = e1 i00 + e2 i10, f2 = e1 i01 + e2 i11
  const double3 f1 = axpy(i00, e1, make_double3(i10 * e2.x, i10 * e2.y, i10 * e2.z));
  const double3 f2 = axpy(i01, e1, make_double3(i11 * e2.x, i11 * e2.y, i11 * e2.z));
  const double c11 = dot(f1, f1), c12 = dot(f1, f2), c22 = dot(f2, f2);
  const double J2 = c11 * c22 - c12 * c12;  // det C = l1^2 l2^2
  const double W = 0.5 * G * (c11 + c22 + 1.0 / J2 - 3.0);
  // S = G (I - adj(C) / J2^2)
  const double q = G / (J2 * J2);
  const double s11 = G - q * c22, s12 = q * c12, s22 = G - q * c11;
  // P = F S (3 x 2)
  const double3 p1 = axpy(s11, f1, make_double3(s12 * f2.x, s12 * f2.y, s12 * f2.z));
  const double3 p2 = axpy(s12, f1, make_double3(s22 * f2.x, s22 * f2.y, s22 * f2.z));
  // dE/de_k = A0 (p1 D^-1_{k0} + p2 D^-1_{k1})
  const double3 g1 = make_double3(A0 * (p1.x * i00 + p2.x * i01), A0 * (p1.y * i00 + p2.y * i01),
                                  A0 * (p1.z * i00 + p2.z * i01));
  const double3 g2 = make_double3(A0 * (p1.x * i10 + p2.x * i11), A0 * (p1.y * i10 + p2.y * i11),
                                  A0 * (p1.z * i10 + p2.z * i11));
  const double3 cr = cross(e1, e2);
  double* o = out + 11 * (size_t)t;
  o[0] = -g1.x - g2.x;
  o[1] = -g1.y - g2.y;
  o[2] = -g1.z - g2.z;
  o[3] = g1.x;
  o[4] = g1.y;
  o[5] = g1.z;
  o[6] = g2.x;
  o[7] = g2.y;
  o[8] = g2.z;
  o[9] = A0 * W;
  o[10] = 0.5 * sqrt(dot(cr, cr));
}

// Per node: df = (1/A_p) sum over its elements of dE/dx_p.  Inconsistent
// incidence lists raise *bad.
__global__ void membrane_node(int nnode, int ntri, const int* __restrict__ tri,
                              const int* __restrict__ off, const int* __restrict__ adj,
                              const double* __restrict__ elem, double* __restrict__ df,
                              int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnode) return;
  const int b0 = off[i], b1 = off[i + 1];
  if (b0 < 0 || b1 <= b0 || b1 > 3 * ntri) {
    atomicOr(bad, 1);
    return;
  }
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, A = 0.0;
  for (int e = b0; e < b1; ++e) {
    const int t = adj[e];
    if ((unsigned)t >= (unsigned)ntri) {
      atomicOr(bad, 1);
      return;
    }
    const int k = tri[3 * t] == i ? 0 : (tri[3 * t + 1] == i ? 1 : (tri[3 * t + 2] == i ? 2 : -1));
    if (k < 0) {
      atomicOr(bad, 1);
      return;
    }
    const double* o = elem + 11 * (size_t)t;
    s0 += o[3 * k];
    s1 += o[3 * k + 1];
    s2 += o[3 * k + 2];
    A += o[10] / 3.0;
  }
  const double inv = 1.0 / A;
  df[3 * (size_t)i] = s0 * inv;
  df[3 * (size_t)i + 1] = s1 * inv;
  df[3 * (size_t)i + 2] = s2 * inv;
}

// Fixed-order block sum / min / max of 256 values.
template <typename Op>
__device__ double block_reduce(double v, double* sh, Op op) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

struct Add {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct Min {
  __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct Max {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

// One block per capsule: volume (1/6 sum x_a . (x_b x x_c)), shortest edge,
// centroid, largest distance of a node from it, lowest and highest y, and
// (when elem is given) the membrane energy.  st: [c][8] = vol, min edge,
// cx, cy, cz, radius, ymin, ymax; energy: [c] or null.
__global__ void __launch_bounds__(256) capsule_stats(int npc, int tpc, const int* __restrict__ tri,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ elem,
                                                     double* __restrict__ st,
                                                     double* __restrict__ energy) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  const int t0 = c * tpc, n0 = c * npc;
  double v = 0.0, me = INFINITY, en = 0.0;
  for (int t = t0 + (int)threadIdx.x; t < t0 + tpc; t += 256) {
    const double3 xa = ld3(x, tri[3 * t]), xb = ld3(x, tri[3 * t + 1]), xc = ld3(x, tri[3 * t + 2]);
    v += dot(xa, cross(xb, xc));
    const double3 ab = sub(xb, xa), bc = sub(xc, xb), ca = sub(xa, xc);
    me = fmin(me, fmin(sqrt(dot(ab, ab)), fmin(sqrt(dot(bc, bc)), sqrt(dot(ca, ca)))));
    if (elem) en += elem[11 * (size_t)t + 9];
  }
  v = block_reduce(v, sh, Add()) / 6.0;
  me = block_reduce(me, sh, Min());
  if (elem) en = block_reduce(en, sh, Add());
  double cx = 0.0, cy = 0.0, cz = 0.0, ylo = INFINITY, yhi = -INFINITY;
  for (int p = n0 + (int)threadIdx.x; p < n0 + npc; p += 256) {
    cx += x[3 * (size_t)p];
    cy += x[3 * (size_t)p + 1];
    cz += x[3 * (size_t)p + 2];
    ylo = fmin(ylo, x[3 * (size_t)p + 1]);
    yhi = fmax(yhi, x[3 * (size_t)p + 1]);
  }
  cx = block_reduce(cx, sh, Add()) / npc;
  cy = block_reduce(cy, sh, Add()) / npc;
  cz = block_reduce(cz, sh, Add()) / npc;
  ylo = block_reduce(ylo, sh, Min());
  yhi = block_reduce(yhi, sh, Max());
  double rad = 0.0;
  for (int p = n0 + (int)threadIdx.x; p < n0 + npc; p += 256) {
    const double dx = x[3 * (size_t)p] - cx, dy = x[3 * (size_t)p + 1] - cy,
                 dz = x[3 * (size_t)p + 2] - cz;
    rad = fmax(rad, sqrt(dx * dx + dy * dy + dz * dz));
  }
  rad = block_reduce(rad, sh, Max());
  if (threadIdx.x == 0) {
    double* o = st + 8 * (size_t)c;
    o[0] = v;
    o[1] = me;
    o[2] = cx;
    o[3] = cy;
    o[4] = cz;
    o[5] = rad;
    o[6] = ylo;
    o[7] = yhi;
    if (energy) energy[c] = en;
  }
}

__device__ inline double min_image(double d, double L) { return d - L * rint(d / L); }

// One block per ordered capsule pair (blockIdx.y = i < blockIdx.x = j):
// pairs whose bounding spheres (minimum image) are more than `reach` apart
// are skipped; otherwise the smallest node-to-node distance over all node
// pairs, and the pair is listed when it is below `reach`.
__global__ void __launch_bounds__(256) pair_gaps(int npc, const double* __restrict__ x,
                                                 const double* __restrict__ st, double Lx, double Lz,
                                                 double reach, Pair* __restrict__ list,
                                                 int* __restrict__ count, int cap) {
  __shared__ double sh[256];
  const int i = blockIdx.y, j = blockIdx.x;
  if (j <= i) return;
  const double* si = st + 8 * (size_t)i;
  const double* sj = st + 8 * (size_t)j;
  const double cx = min_image(sj[2] - si[2], Lx), cy = sj[3] - si[3], cz = min_image(sj[4] - si[4], Lz);
  if (sqrt(cx * cx + cy * cy + cz * cz) > si[5] + sj[5] + reach) return;  // uniform over the block
  const size_t a0 = (size_t)i * npc, b0 = (size_t)j * npc;
  const long long np2 = (long long)npc * npc;
  double best = INFINITY;
  for (long long k = threadIdx.x; k < np2; k += 256) {
    const size_t a = a0 + (size_t)(k / npc), b = b0 + (size_t)(k % npc);
    const double dx = min_image(x[3 * a] - x[3 * b], Lx), dy = x[3 * a + 1] - x[3 * b + 1],
                 dz = min_image(x[3 * a + 2] - x[3 * b + 2], Lz);
    best = fmin(best, dx * dx + dy * dy + dz * dz);
  }
  best = block_reduce(best, sh, Min());
  if (threadIdx.x == 0) {
    const double g = sqrt(best);
    if (g < reach) {
      const int slot = atomicAdd(count, 1);
      if (slot < cap) list[slot] = Pair{i, j, g};
    }
  }
}

// x_p += move[capsule of p]
__global__ void translate(int nnode, int npc, const double* __restrict__ move, double* __restrict__ x) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnode) return;
  const int c = p / npc;
  x[3 * (size_t)p] += move[3 * c];
  x[3 * (size_t)p + 1] += move[3 * c + 1];
  x[3 * (size_t)p + 2] += move[3 * c + 2];
}

// One block per capsule: the volume shift (V0 - V)/A when |V - V0| > tol |V0|
// (A the sum of its node areas), else 0.
__global__ void __launch_bounds__(256) volume_shift(int npc, const double* __restrict__ st,
                                                    const double* __restrict__ area,
                                                    const double* __restrict__ v0, double tol,
                                                    double* __restrict__ shift) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  double A = 0.0;
  for (int p = c * npc + (int)threadIdx.x; p < (c + 1) * npc; p += 256) A += area[p];
  A = block_reduce(A, sh, Add());
  if (threadIdx.x == 0) {
    const double v = st[8 * (size_t)c], w = v0[c];
    shift[c] = fabs(v - w) > tol * fabs(w) ? (w - v) / A : 0.0;
  }
}

__global__ void volume_apply(int nnode, int npc, const double* __restrict__ shift,
                             const double* __restrict__ nrm, double* __restrict__ x) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnode) return;
  const double s = shift[p / npc];
  if (s == 0.0) return;
  x[3 * (size_t)p] = fma(s, nrm[3 * (size_t)p], x[3 * (size_t)p]);
  x[3 * (size_t)p + 1] = fma(s, nrm[3 * (size_t)p + 1], x[3 * (size_t)p + 1]);
  x[3 * (size_t)p + 2] = fma(s, nrm[3 * (size_t)p + 2], x[3 * (size_t)p + 2]);
}

__global__ void zero_int(int* p) { *p = 0; }

}  // namespace

struct ggem_membrane_s {
  ggem_solver_t solver;
  int ncap, npc, tpc, n_nodes, n_tri;
  double G;
  int* tri;          // own copy (n_tri x 3)
  double* ref;       // 5 per element
  double* elem;      // 11 per element
  double* st;        // 8 per capsule
  double* energy;    // per capsule
  double* move;      // 3 per capsule (translations; volume shifts use the first ncap)
  Pair* pairs;
  int* count;
  int* bad;
  int* host_int;     // pinned: [0] bad, [1] count
  int pair_cap;
};

static void free_membrane(ggem_membrane_s* m) {
  void* ptrs[] = {m->tri, m->ref, m->elem, m->st, m->energy, m->move, m->pairs, m->count, m->bad};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (m->host_int) (void)hipHostFree(m->host_int);
}

#define MEM_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) return ggem_set_error(GGEM_E_DEVICE, hipGetErrorString(e_)); \
  } while (0)

static hipStream_t stream_of(ggem_membrane_s* m) { return ggem::solver_stream(m->solver); }

static unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

extern "C" int ggem_membrane_create(ggem_solver_t solver, long long n_capsules,
                                    int nodes_per_capsule, int tri_per_capsule, const int* tri,
                                    const double* ref_nodes, double shear_modulus,
                                    ggem_membrane_t* out) {
  if (!solver || !tri || !ref_nodes || !out) return ggem_set_error(GGEM_E_ARG, "null argument");
  *out = nullptr;
  if (n_capsules < 1 || n_capsules > 65535 || nodes_per_capsule < 4 || tri_per_capsule < 4)
    return ggem_set_error(GGEM_E_ARG, "need 1..65535 capsules of >= 4 nodes and triangles");
  if (!(shear_modulus > 0) || !isfinite(shear_modulus))
    return ggem_set_error(GGEM_E_ARG, "shear modulus must be positive");
  const long long nn = n_capsules * nodes_per_capsule, nt = n_capsules * tri_per_capsule;
  if (nn > ggem::solver_max_nodes(solver) || nt > ggem::solver_max_tri(solver))
    return ggem_set_error(GGEM_E_CAPACITY, "capsules exceed the solver capacity");
  ggem_membrane_s* m = new (std::nothrow) ggem_membrane_s();
  if (!m) return ggem_set_error(GGEM_E_NOMEM, "host allocation failed");
  memset(m, 0, sizeof *m);
  m->solver = solver;
  m->ncap = (int)n_capsules;
  m->npc = nodes_per_capsule;
  m->tpc = tri_per_capsule;
  m->n_nodes = (int)nn;
  m->n_tri = (int)nt;
  m->G = shear_modulus;
  m->pair_cap = kPairsPerCapsule * m->ncap;
  bool ok = hipMalloc((void**)&m->tri, 3 * (size_t)nt * sizeof(int)) == hipSuccess &&
            hipMalloc((void**)&m->ref, 5 * (size_t)nt * 8) == hipSuccess &&
            hipMalloc((void**)&m->elem, 11 * (size_t)nt * 8) == hipSuccess &&
            hipMalloc((void**)&m->st, 8 * (size_t)m->ncap * 8) == hipSuccess &&
            hipMalloc((void**)&m->energy, (size_t)m->ncap * 8) == hipSuccess &&
            hipMalloc((void**)&m->move, 3 * (size_t)m->ncap * 8) == hipSuccess &&
            hipMalloc((void**)&m->pairs, (size_t)m->pair_cap * sizeof(Pair)) == hipSuccess &&
            hipMalloc((void**)&m->count, sizeof(int)) == hipSuccess &&
            hipMalloc((void**)&m->bad, sizeof(int)) == hipSuccess &&
            hipHostMalloc((void**)&m->host_int, 2 * sizeof(int), 0) == hipSuccess;
  if (!ok) {
    free_membrane(m);
    delete m;
    return ggem_set_error(GGEM_E_NOMEM, "device allocation failed");
  }
  hipStream_t st = stream_of(m);
  int rc = GGEM_OK;
  do {
    if (hipMemcpyAsync(m->tri, tri, 3 * (size_t)nt * sizeof(int), hipMemcpyDeviceToDevice, st) !=
        hipSuccess) {
      rc = ggem_set_error(GGEM_E_DEVICE, "copy of the triangles failed");
      break;
    }
    zero_int<<<1, 1, 0, st>>>(m->bad);
    membrane_ref<<<nblk(nt), 256, 0, st>>>(m->n_tri, m->npc, m->tpc, m->tri, ref_nodes, m->ref, m->bad);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(m->host_int, m->bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = ggem_set_error(GGEM_E_DEVICE, "reference elements failed");
      break;
    }
    if (m->host_int[0]) rc = ggem_set_error(GGEM_E_ARG, "a triangle names a node of another capsule");
  } while (false);
  if (rc) {
    free_membrane(m);
    delete m;
    return rc;
  }
  *out = m;
  return GGEM_OK;
}

extern "C" int ggem_membrane_destroy(ggem_membrane_t m) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null membrane");
  (void)hipStreamSynchronize(stream_of(m));
  free_membrane(m);
  delete m;
  return GGEM_OK;
}

extern "C" int ggem_membrane_traction(ggem_membrane_t m, const double* nodes,
                                      const int* node_tri_off, const int* node_tri, double* df,
                                      double* energy) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null membrane");
  if (!nodes || !node_tri_off || !node_tri || !df) return ggem_set_error(GGEM_E_ARG, "null array");
  hipStream_t st = stream_of(m);
  zero_int<<<1, 1, 0, st>>>(m->bad);
  membrane_elem<<<nblk(m->n_tri), 256, 0, st>>>(m->n_tri, m->tri, nodes, m->ref, m->G, m->elem);
  membrane_node<<<nblk(m->n_nodes), 256, 0, st>>>(m->n_nodes, m->n_tri, m->tri, node_tri_off,
                                                  node_tri, m->elem, df, m->bad);
  MEM_TRY(hipGetLastError());
  std::vector<double> e;
  if (energy) {
    capsule_stats<<<m->ncap, 256, 0, st>>>(m->npc, m->tpc, m->tri, nodes, m->elem, m->st, m->energy);
    MEM_TRY(hipGetLastError());
    e.resize(m->ncap);
    MEM_TRY(hipMemcpyAsync(e.data(), m->energy, (size_t)m->ncap * 8, hipMemcpyDeviceToHost, st));
  }
  MEM_TRY(hipMemcpyAsync(m->host_int, m->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  MEM_TRY(hipStreamSynchronize(st));
  if (m->host_int[0]) return ggem_set_error(GGEM_E_ARG, "inconsistent triangle incidence lists");
  if (energy) {
    double s = 0.0;
    for (double v : e) s += v;
    *energy = s;
  }
  return GGEM_OK;
}

extern "C" int ggem_capsule_volumes(ggem_membrane_t m, const double* nodes, double* vol) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null membrane");
  if (!nodes || !vol) return ggem_set_error(GGEM_E_ARG, "null array");
  hipStream_t st = stream_of(m);
  capsule_stats<<<m->ncap, 256, 0, st>>>(m->npc, m->tpc, m->tri, nodes, nullptr, m->st, nullptr);
  MEM_TRY(hipGetLastError());
  MEM_TRY(hipMemcpy2DAsync(vol, sizeof(double), m->st, 8 * sizeof(double), sizeof(double),
                           (size_t)m->ncap, hipMemcpyDeviceToDevice, st));
  return GGEM_OK;
}

extern "C" int ggem_volume_correct(ggem_membrane_t m, double* nodes, const double* normals,
                                   const double* area, const double* v0, double tol,
                                   int* n_corrected) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null membrane");
  if (!nodes || !normals || !area || !v0) return ggem_set_error(GGEM_E_ARG, "null array");
  if (!(tol >= 0)) return ggem_set_error(GGEM_E_ARG, "tolerance must be >= 0");
  hipStream_t st = stream_of(m);
  capsule_stats<<<m->ncap, 256, 0, st>>>(m->npc, m->tpc, m->tri, nodes, nullptr, m->st, nullptr);
  volume_shift<<<m->ncap, 256, 0, st>>>(m->npc, m->st, area, v0, tol, m->move);
  volume_apply<<<nblk(m->n_nodes), 256, 0, st>>>(m->n_nodes, m->npc, m->move, normals, nodes);
  MEM_TRY(hipGetLastError());
  if (n_corrected) {
    std::vector<double> s(m->ncap);
    MEM_TRY(hipMemcpyAsync(s.data(), m->move, (size_t)m->ncap * 8, hipMemcpyDeviceToHost, st));
    MEM_TRY(hipStreamSynchronize(st));
    int k = 0;
    for (double v : s) k += v != 0.0;
    *n_corrected = k;
  }
  return GGEM_OK;
}

// Capsule statistics (host copy) and the close pairs within `reach`, sorted
// by (i, j).
static int close_pairs(ggem_membrane_s* m, const double* nodes, double Lx, double Lz, double reach,
                       std::vector<double>& stats, std::vector<Pair>& pairs) {
  hipStream_t st = stream_of(m);
  capsule_stats<<<m->ncap, 256, 0, st>>>(m->npc, m->tpc, m->tri, nodes, nullptr, m->st, nullptr);
  zero_int<<<1, 1, 0, st>>>(m->count);
  if (m->ncap > 1)
    pair_gaps<<<dim3(m->ncap, m->ncap), 256, 0, st>>>(m->npc, nodes, m->st, Lx, Lz, reach, m->pairs,
                                                      m->count, m->pair_cap);
  MEM_TRY(hipGetLastError());
  stats.resize(8 * (size_t)m->ncap);
  MEM_TRY(hipMemcpyAsync(stats.data(), m->st, stats.size() * 8, hipMemcpyDeviceToHost, st));
  MEM_TRY(hipMemcpyAsync(m->host_int + 1, m->count, sizeof(int), hipMemcpyDeviceToHost, st));
  MEM_TRY(hipStreamSynchronize(st));
  const int n = m->host_int[1];
  if (n > m->pair_cap)
    return ggem_set_error(GGEM_E_CAPACITY, "more than 64 close pairs per capsule");
  pairs.resize(n);
  if (n) {
    MEM_TRY(hipMemcpyAsync(pairs.data(), m->pairs, (size_t)n * sizeof(Pair), hipMemcpyDeviceToHost, st));
    MEM_TRY(hipStreamSynchronize(st));
  }
  std::sort(pairs.begin(), pairs.end(),
            [](const Pair& a, const Pair& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
  return GGEM_OK;
}

static bool finite_box(double Lx, double Lz) { return Lx > 0 && Lz > 0 && isfinite(Lx) && isfinite(Lz); }

extern "C" int ggem_capsule_separation(ggem_membrane_t m, const double* nodes, double Lx,
                                       double Lz, double reach, double* min_edge,
                                       double* min_gap) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null membrane");
  if (!nodes || !min_edge || !min_gap) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (!finite_box(Lx, Lz) || !(reach > 0)) return ggem_set_error(GGEM_E_ARG, "bad box or reach");
  std::vector<double> stats;
  std::vector<Pair> pairs;
  if (int rc = close_pairs(m, nodes, Lx, Lz, reach, stats, pairs)) return rc;
  double me = INFINITY, mg = INFINITY;
  for (int c = 0; c < m->ncap; ++c) me = std::min(me, stats[8 * (size_t)c + 1]);
  for (const Pair& p : pairs) mg = std::min(mg, p.gap);
  *min_edge = me;
  *min_gap = mg;
  return GGEM_OK;
}

extern "C" int ggem_overlap_correct(ggem_membrane_t m, double* nodes, double Lx, double Lz,
                                    double H, double h_min, int max_sweeps, int* sweeps) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null membrane");
  if (!nodes) return ggem_set_error(GGEM_E_ARG, "null array");
  if (!finite_box(Lx, Lz) || !(H > 0) || !(h_min > 0) || max_sweeps < 0)
    return ggem_set_error(GGEM_E_ARG, "bad box, gap or sweep count");
  hipStream_t st = stream_of(m);
  std::vector<double> stats, move(3 * (size_t)m->ncap);
  std::vector<Pair> pairs;
  int done = 0;
  for (int s = 0; s < max_sweeps; ++s) {
    if (int rc = close_pairs(m, nodes, Lx, Lz, h_min, stats, pairs)) return rc;
    std::fill(move.begin(), move.end(), 0.0);
    bool any = false;
    for (const Pair& p : pairs) {
      const double* ci = &stats[8 * (size_t)p.i + 2];
      const double* cj = &stats[8 * (size_t)p.j + 2];
      double e[3] = {cj[0] - ci[0], cj[1] - ci[1], cj[2] - ci[2]};
      e[0] -= Lx * rint(e[0] / Lx);
      e[2] -= Lz * rint(e[2] / Lz);
      const double n = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      const double h = 0.5 * (h_min - p.gap);
      for (int d = 0; d < 3; ++d) {
        move[3 * (size_t)p.i + d] -= h * (e[d] / n);
        move[3 * (size_t)p.j + d] += h * (e[d] / n);
      }
      any = true;
    }
    for (int c = 0; c < m->ncap; ++c) {
      const double lo = stats[8 * (size_t)c + 6], hi = stats[8 * (size_t)c + 7];
      if (hi > H - h_min) {
        move[3 * (size_t)c + 1] -= hi - (H - h_min);
        any = true;
      } else if (lo < -H + h_min) {
        move[3 * (size_t)c + 1] += (-H + h_min) - lo;
        any = true;
      }
    }
    if (!any) break;
    MEM_TRY(hipMemcpyAsync(m->move, move.data(), move.size() * 8, hipMemcpyHostToDevice, st));
    translate<<<nblk(m->n_nodes), 256, 0, st>>>(m->n_nodes, m->npc, m->move, nodes);
    MEM_TRY(hipGetLastError());
    MEM_TRY(hipStreamSynchronize(st));  // `move` is reused by the next sweep
    ++done;
  }
  if (sweeps) *sweeps = done;
  return GGEM_OK;
}
