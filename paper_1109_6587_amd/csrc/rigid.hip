// Boundary-integral single layer on a triangulated surface and the
// rigid-particle problem.
//
// Single layer at the mesh nodes (Sec. 3.4), traction f linear on flat
// triangles (basis of Sec. 3.3.1: phi1 = 1 - xi - eta, phi2 = xi, phi3 = eta):
//
//   w(z) = (1/8pi) [ sum_k int_{S_k} f G^l(z - x) dS  +  sum_b G^g(z, x_b) f_b A_b ]
//
// Local part (Sec. 3.4.1, Eq. int_l): every element within r_c of z (its
// nearest vertex within r_c) is integrated over its parent triangle with the
// product of two 4-point Gauss-Legendre rules (xi in [0, 1 - eta] for each
// eta); when z is a vertex of the element the parent triangle is taken in
// polar coordinates about that vertex, which removes the 1/r singularity.
// Global part (Sec. 3.4.2): nodal trapezoid strengths f_b A_b (A_b one third
// of the areas of the triangles at b) through the GGEM global problem.
//
// Double layer at the nodes (Sec. 3.5), normal n(z) at the target:
//
//   v_j(z) = (1/8pi) [ n_k(z) sum_k int_{S_k} q_i T^l_jik(z - x) dS + n_k(z) sigma^g_jk(z) ],
//
// with the same elements and rules; on an element that has z as a vertex the
// normal is replaced inside the integral by n~(x) = n_D phi_z + n(z)(1 - phi_z)
// (Eq. dbl_l1, Eq. ntilde), n_D the element normal on the side of n(z), and
// the global stress is that of the nodal point forces q_b A_b.
//
// Rigid particle (Sec. 6.1, Eq. sl_r): unknowns f at the nodes, U and Omega;
// at every node U + Omega x (x_b - x_c) + w(x_b) = u_inf(x_b), with
// sum_b A_b f_b = 0 and sum_b A_b (x_b - x_c) x f_b = 0; solved by GMRES (Sec. 5).
#include <math.h>
#include <string.h>

#include <new>

#include "ggem_internal.h"
#include "gmres.h"

using namespace ggem;

namespace {

constexpr double kInv8Pi = 0.039788735772973833942;  // 1/(8 pi)
constexpr double kSqrtPi = 1.7724538509055160273;

// 4-point Gauss-Legendre rule on [0, 1]
__constant__ double kGLt[4] = {0.069431844202973712, 0.33000947820757187, 0.66999052179242813,
                               0.93056815579702629};
__constant__ double kGLw[4] = {0.17392742256872693, 0.32607257743127307, 0.32607257743127307,
                               0.17392742256872693};
// cos and sin of the polar angles (pi/2) t_o at the same nodes
__constant__ double kPolC[4] = {0.994058492765765, 0.8686241377879603, 0.49547160085329073,
                                0.10884720005703206};
__constant__ double kPolS[4] = {0.10884720005703191, 0.49547160085329056, 0.8686241377879602,
                                0.994058492765765};

__device__ inline double min_img(double d, double L, double invL) {
  return fma(-L, rint(d * invL), d);
}

__device__ inline double d2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

struct BiArgs {
  CellGeom g;
  double rc2, alpha;
  int n, ntri;
  const double* x;        // nodes (n, 3), any periodic image
  const int* tri;         // (ntri, 3)
  const int* off;         // node -> incident triangles (CSR, n + 1)
  const int* adj;
  const int* keys;        // bucket of every node (binning of the nodes)
  const int* cell_start;  // sorted ranges per cell
  const int* perm;        // sorted -> original
  const double* f;        // (n, 3) traction (single layer) or density (double layer)
  const double* nrm;      // (n, 3) node normals (double layer)
  double* out;            // (n, 3)
};

// displacement x[q] - z by the minimum image in x and z
__device__ inline void rel(const BiArgs& a, int q, double zx, double zy, double zz, double& dx,
                           double& dy, double& dz) {
  dx = min_img(a.x[3 * (size_t)q] - zx, a.g.Lx, a.g.invLx);
  dy = a.x[3 * (size_t)q + 1] - zy;
  dz = min_img(a.x[3 * (size_t)q + 2] - zz, a.g.Lz, a.g.invLz);
}

__device__ inline bool within(const BiArgs& a, int q, double zx, double zy, double zz) {
  double dx, dy, dz;
  rel(a, q, zx, zy, zz, dx, dy, dz);
  return d2(dx, dy, dz) <= a.rc2;
}

// acc += w * G^l(d) fv,  G^l = (I/r + dd/r^3) erfc(alpha r) - c (I - dd/r^2) e^{-alpha^2 r^2}
__device__ inline void add_stokeslet(double dx, double dy, double dz, double fx, double fy,
                                     double fz, double alpha, double w, double* acc) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double r = sqrt(r2);
  const double ec = erfc(alpha * r), ex = exp(-alpha * alpha * r2);
  const double c = 2.0 * alpha / kSqrtPi * ex;
  const double ir = 1.0 / r;
  const double A = ec * ir - c;                // coefficient of I
  const double B = (ec * ir + c) * (ir * ir);  // coefficient of d d^T
  const double df = dx * fx + dy * fy + dz * fz;
  acc[0] += w * (A * fx + B * df * dx);
  acc[1] += w * (A * fy + B * df * dy);
  acc[2] += w * (A * fz + B * df * dz);
}

// acc += w * T^l_jik(d) q_i m_k = w [C d (d.q)(d.m) + D (d (q.m) + q (d.m) + m (d.q))],
// C = -6 erfc/r^5 - (12 alpha/sqrt(pi)) e/r^4 - (8 alpha^3/sqrt(pi)) e/r^2,
// D = (4 alpha^3/sqrt(pi)) e,  e = exp(-alpha^2 r^2)
__device__ inline void add_stresslet(double dx, double dy, double dz, double qx, double qy,
                                     double qz, double mx, double my, double mz, double alpha,
                                     double w, double* acc) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double r = sqrt(r2);
  const double ec = erfc(alpha * r), ex = exp(-alpha * alpha * r2);
  const double a3 = alpha * alpha * alpha / kSqrtPi;
  const double ir = 1.0 / r, ir2 = ir * ir;
  const double C = -ir2 * (ir2 * (6.0 * ec * ir + 12.0 * alpha / kSqrtPi * ex) + 8.0 * a3 * ex);
  const double D = 4.0 * a3 * ex;
  const double dq = dx * qx + dy * qy + dz * qz, dm = dx * mx + dy * my + dz * mz;
  const double qm = qx * mx + qy * my + qz * mz;
  const double cd = C * dq * dm;
  acc[0] += w * (cd * dx + D * (dx * qm + qx * dm + mx * dq));
  acc[1] += w * (cd * dy + D * (dy * qm + qy * dm + my * dq));
  acc[2] += w * (cd * dz + D * (dz * qm + qz * dm + mz * dq));
}

// One quadrature point (o, i) of the product rule over an element:
// acc += w f G^l(z - x) (DL: w q_i T^l_jik(z - x) m_k, m = n(z), or n~ when
// polar).  e[v]: vertex positions relative to z, fe[v]: nodal values; local
// vertex 0 is z itself when polar.
template <bool DL>
__device__ void element_point(const double (&e)[3][3], const double (&fe)[3][3], bool polar, int o,
                              int i, double alpha, const double* nz, double* acc) {
  const double u1x = e[1][0] - e[0][0], u1y = e[1][1] - e[0][1], u1z = e[1][2] - e[0][2];
  const double u2x = e[2][0] - e[0][0], u2y = e[2][1] - e[0][1], u2z = e[2][2] - e[0][2];
  const double cx = u1y * u2z - u1z * u2y, cy = u1z * u2x - u1x * u2z, cz = u1x * u2y - u1y * u2x;
  const double omega = sqrt(cx * cx + cy * cy + cz * cz);
  double xi, eta, w;
  if (polar) {
    const double c = kPolC[o], s = kPolS[o];
    const double rmax = 1.0 / (c + s);
    const double rho = rmax * kGLt[i];
    xi = rho * c;
    eta = rho * s;
    w = (0.5 * M_PI * kGLw[o]) * rmax * kGLw[i] * rho * omega;
  } else {
    eta = kGLt[o];
    xi = (1.0 - eta) * kGLt[i];
    w = kGLw[o] * kGLw[i] * (1.0 - eta) * omega;
  }
  const double p0 = 1.0 - xi - eta, p1 = xi, p2 = eta;
  // d = z - x(xi, eta)
  const double dx = -(p0 * e[0][0] + p1 * e[1][0] + p2 * e[2][0]);
  const double dy = -(p0 * e[0][1] + p1 * e[1][1] + p2 * e[2][1]);
  const double dz = -(p0 * e[0][2] + p1 * e[1][2] + p2 * e[2][2]);
  const double vx = p0 * fe[0][0] + p1 * fe[1][0] + p2 * fe[2][0];
  const double vy = p0 * fe[0][1] + p1 * fe[1][1] + p2 * fe[2][1];
  const double vz = p0 * fe[0][2] + p1 * fe[1][2] + p2 * fe[2][2];
  if (DL) {
    // element normal on the side of n(z); n~ = n_D phi_z + n(z)(1 - phi_z)
    const double sg = (cx * nz[0] + cy * nz[1] + cz * nz[2]) < 0.0 ? -1.0 / omega : 1.0 / omega;
    const double a0 = polar ? p0 : 0.0, a1 = 1.0 - a0;
    add_stresslet(dx, dy, dz, vx, vy, vz, a0 * (sg * cx) + a1 * nz[0], a0 * (sg * cy) + a1 * nz[1],
                  a0 * (sg * cz) + a1 * nz[2], alpha, w, acc);
  } else {
    add_stokeslet(dx, dy, dz, vx, vy, vz, alpha, w, acc);
  }
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kElemCap = 256;  // element list of a wave (LDS ints)

// The 16 quadrature points of each listed element, one lane per (element,
// point), four elements per round; each lane accumulates its points in list
// order.
template <bool DL>
__device__ void eval_list(const BiArgs& a, const int* list, int cnt, int t, double zx, double zy,
                          double zz, const double* nz, int lane, double* acc) {
  const CellGeom& g = a.g;
  const int o = (lane & 15) >> 2, i = lane & 3;
  for (int base = 0; base < cnt; base += 4) {
    const int idx = base + (lane >> 4);
    if (idx >= cnt) continue;
    const int k = list[idx];
    const int ia = a.tri[3 * (size_t)k], ib = a.tri[3 * (size_t)k + 1], ic = a.tri[3 * (size_t)k + 2];
    const int vv[3] = {ia, ib, ic};
    const bool polar = ia == t || ib == t || ic == t;
    const int rot = ib == t ? 1 : (ic == t ? 2 : 0);
    double e0x, e0y, e0z;
    rel(a, ia, zx, zy, zz, e0x, e0y, e0z);
    double ea[3][3];
    ea[0][0] = e0x;
    ea[0][1] = e0y;
    ea[0][2] = e0z;
    for (int m = 1; m < 3; ++m) {
      const int q2 = vv[m];
      ea[m][0] = e0x + min_img(a.x[3 * (size_t)q2] - a.x[3 * (size_t)ia], g.Lx, g.invLx);
      ea[m][1] = e0y + (a.x[3 * (size_t)q2 + 1] - a.x[3 * (size_t)ia + 1]);
      ea[m][2] = e0z + min_img(a.x[3 * (size_t)q2 + 2] - a.x[3 * (size_t)ia + 2], g.Lz, g.invLz);
    }
    double e[3][3], fe[3][3];
    for (int m = 0; m < 3; ++m) {
      const int src = (rot + m) % 3;
      const int node = vv[src];
      for (int d = 0; d < 3; ++d) {
        e[m][d] = (polar && m == 0) ? 0.0 : ea[src][d];
        fe[m][d] = a.f[3 * (size_t)node + d];
      }
    }
    element_point<DL>(e, fe, polar, o, i, a.alpha, nz, acc);
  }
}

// One wave per target node z.  (1) The nodes of the cells around z are taken
// as one flat range over the (up to 27) cells, 64 at a time; a lane whose
// node v lies within r_c of z lists every triangle at v for which v is the
// first of the triangle's vertices (in their stored order) within r_c of z,
// so that each element within r_c is listed exactly once; one triangle per
// lane and round, compacted by ballot into the wave's list in lane order.
// (2) Whenever the list could overflow, and at the end, its elements are
// integrated with one lane per (element, quadrature point).  Lane sums are
// added in a fixed tree order: the result depends only on the inputs.
template <bool DL>
__global__ void __launch_bounds__(256) bi_local(BiArgs a) {
  __shared__ int elist[4][kElemCap];
  __shared__ int cstart[4][27], cpref[4][28];
  __shared__ double red[4][3][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = blockIdx.x * 4 + wave;
  if (t >= a.n) return;  // uniform over the wave
  const CellGeom& g = a.g;
  const double zx = a.x[3 * (size_t)t], zy = a.x[3 * (size_t)t + 1], zz = a.x[3 * (size_t)t + 2];
  const int c = a.keys[t] / g.nzs;
  const int iz = c % g.ncz, ix = (c / g.ncz) % g.ncx, iy = c / (g.ncz * g.ncx);
  const int nxo = g.ncx >= 3 ? 3 : g.ncx, nzo = g.ncz >= 3 ? 3 : g.ncz;
  const int ncell = 3 * nxo * nzo;
  double nz[3] = {0.0, 0.0, 0.0};
  if (DL)
    for (int d = 0; d < 3; ++d) nz[d] = a.nrm[3 * (size_t)t + d];
  // the neighbour cells' ranges and their running total
  int cnt = 0, s0 = 0;
  if (lane < ncell) {
    const int oy = lane / (nxo * nzo) - 1, oxi = (lane / nzo) % nxo, ozi = lane % nzo;
    const int cy = iy + oy;
    if (cy >= 0 && cy < g.ncy) {
      const int cx = g.ncx >= 3 ? (ix + oxi - 1 + g.ncx) % g.ncx : oxi;
      const int cz = g.ncz >= 3 ? (iz + ozi - 1 + g.ncz) % g.ncz : ozi;
      const int cc = (cy * g.ncx + cx) * g.ncz + cz;
      s0 = a.cell_start[cc];
      cnt = a.cell_start[cc + 1] - s0;
    }
  }
  int pref = cnt;  // inclusive scan over the lanes
  for (int o = 1; o < 32; o <<= 1) {
    const int v = __shfl_up(pref, o);
    if (lane >= o) pref += v;
  }
  if (lane < ncell) {
    cstart[wave][lane] = s0;
    cpref[wave][lane + 1] = pref;
  }
  if (lane == 0) cpref[wave][0] = 0;
  wave_sync();
  const int total = cpref[wave][ncell];
  double acc[3] = {0.0, 0.0, 0.0};
  int listed = 0;
  for (int b = 0; b < total; b += 64) {
    const int ii = b + lane;
    int v = -1, q0 = 0, q1 = 0;
    if (ii < total) {
      int lo = 0, hi = ncell - 1;  // the cell m with cpref[m] <= ii < cpref[m + 1]
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cpref[wave][mid] <= ii) lo = mid;
        else hi = mid - 1;
      }
      const int node = a.perm[cstart[wave][lo] + (ii - cpref[wave][lo])];
      if (within(a, node, zx, zy, zz)) {
        v = node;
        q0 = a.off[v];
        q1 = a.off[v + 1];
      }
    }
    // rounds: the r-th incident triangle of every lane
    int rounds = q1 - q0;
    for (int o = 32; o > 0; o >>= 1) rounds = max(rounds, __shfl_xor(rounds, o));
    for (int r = 0; r < rounds; ++r) {
      bool take = false;
      int k = 0;
      if (v >= 0 && q0 + r < q1) {
        k = a.adj[q0 + r];
        const int ia = a.tri[3 * (size_t)k], ib = a.tri[3 * (size_t)k + 1];
        take = !((ia != v && within(a, ia, zx, zy, zz)) ||
                 (ia != v && ib != v && within(a, ib, zx, zy, zz)));
      }
      const unsigned long long m = __ballot(take);
      const int nnew = __popcll(m);
      if (nnew == 0) continue;
      if (listed + nnew > kElemCap) {
        eval_list<DL>(a, elist[wave], listed, t, zx, zy, zz, nz, lane, acc);
        wave_sync();
        listed = 0;
      }
      if (take) elist[wave][listed + __popcll(m & ((1ull << lane) - 1))] = k;
      listed += nnew;
      wave_sync();
    }
  }
  eval_list<DL>(a, elist[wave], listed, t, zx, zy, zz, nz, lane, acc);
  for (int d = 0; d < 3; ++d) red[wave][d][lane] = acc[d];
  wave_sync();
  for (int o = 32; o > 0; o >>= 1) {
    if (lane < o)
      for (int d = 0; d < 3; ++d) red[wave][d][lane] += red[wave][d][lane + o];
    wave_sync();
  }
  if (lane == 0)
    for (int d = 0; d < 3; ++d) a.out[3 * (size_t)t + d] = kInv8Pi * red[wave][d][0];
}

// Node areas A_b (one third of the areas of the triangles at b, in incidence
// order) and checks of the mesh arrays: an index out of range, or a triangle
// listed at a node it does not contain, raises *bad.
__global__ void bi_node_areas(int n, int ntri, const double* __restrict__ x,
                              const int* __restrict__ tri, const int* __restrict__ off,
                              const int* __restrict__ adj, double* __restrict__ area,
                              int* __restrict__ bad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double s = 0.0;
  const int q0 = off[b], q1 = off[b + 1];
  if (q0 < 0 || q1 < q0) {
    atomicOr(bad, 1);
    area[b] = 0.0;
    return;
  }
  for (int q = q0; q < q1; ++q) {
    const int k = adj[q];
    if ((unsigned)k >= (unsigned)ntri) {
      atomicOr(bad, 1);
      continue;
    }
    const int ia = tri[3 * (size_t)k], ib = tri[3 * (size_t)k + 1], ic = tri[3 * (size_t)k + 2];
    if ((unsigned)ia >= (unsigned)n || (unsigned)ib >= (unsigned)n || (unsigned)ic >= (unsigned)n ||
        (ia != b && ib != b && ic != b)) {
      atomicOr(bad, 1);
      continue;
    }
    double u[3], w[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = x[3 * (size_t)ib + d] - x[3 * (size_t)ia + d];
      w[d] = x[3 * (size_t)ic + d] - x[3 * (size_t)ia + d];
    }
    const double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2],
                 cz = u[0] * w[1] - u[1] * w[0];
    s += sqrt(cx * cx + cy * cy + cz * cz) / 6.0;
  }
  area[b] = s;
}

__global__ void bi_scale(int n, const double* __restrict__ area, const double* __restrict__ f,
                         double* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * n) q[i] = area[i / 3] * f[i];
}

__global__ void bi_add(int n, const double* __restrict__ a, const double* __restrict__ b,
                       double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] + b[i];
}

// velocity rows of the rigid system: y_b = U + Omega x (x_b - x_c) + w_l + w_g
__global__ void bi_rigid_rows(int n, const double* __restrict__ x, double xc0, double xc1,
                              double xc2, const double* __restrict__ motion,
                              const double* __restrict__ wl, const double* __restrict__ wg,
                              double* __restrict__ y) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double r0 = x[3 * (size_t)b] - xc0, r1 = x[3 * (size_t)b + 1] - xc1,
               r2 = x[3 * (size_t)b + 2] - xc2;
  const double U0 = motion[0], U1 = motion[1], U2 = motion[2];
  const double O0 = motion[3], O1 = motion[4], O2 = motion[5];
  y[3 * (size_t)b] = U0 + (O1 * r2 - O2 * r1) + wl[3 * (size_t)b] + wg[3 * (size_t)b];
  y[3 * (size_t)b + 1] = U1 + (O2 * r0 - O0 * r2) + wl[3 * (size_t)b + 1] + wg[3 * (size_t)b + 1];
  y[3 * (size_t)b + 2] = U2 + (O0 * r1 - O1 * r0) + wl[3 * (size_t)b + 2] + wg[3 * (size_t)b + 2];
}

constexpr int kMomBlock = 256, kMomBlocks = 64;

// part[m][blk]: block sums over its node range of the force A f (m = 0..2)
// and the torque A r x f (m = 3..5)
__global__ void __launch_bounds__(kMomBlock) bi_moments_partial(int n, const double* __restrict__ x,
                                                                double xc0, double xc1, double xc2,
                                                                const double* __restrict__ area,
                                                                const double* __restrict__ f,
                                                                double* __restrict__ part) {
  __shared__ double red[6][kMomBlock];
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int b = blockIdx.x * kMomBlock + threadIdx.x; b < n; b += kMomBlocks * kMomBlock) {
    const double A = area[b];
    const double f0 = A * f[3 * (size_t)b], f1 = A * f[3 * (size_t)b + 1],
                 f2 = A * f[3 * (size_t)b + 2];
    const double r0 = x[3 * (size_t)b] - xc0, r1 = x[3 * (size_t)b + 1] - xc1,
                 r2 = x[3 * (size_t)b + 2] - xc2;
    s[0] += f0;
    s[1] += f1;
    s[2] += f2;
    s[3] += r1 * f2 - r2 * f1;
    s[4] += r2 * f0 - r0 * f2;
    s[5] += r0 * f1 - r1 * f0;
  }
  for (int m = 0; m < 6; ++m) red[m][threadIdx.x] = s[m];
  __syncthreads();
  for (int o = kMomBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int m = 0; m < 6; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 6) part[threadIdx.x * kMomBlocks + blockIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(64) bi_moments_final(const double* __restrict__ part,
                                                       double* __restrict__ out) {
  const int m = blockIdx.x;  // one block per moment, 64 lanes over the 64 partials
  __shared__ double red[64];
  red[threadIdx.x] = part[m * kMomBlocks + threadIdx.x];
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = red[0];
}

// part[m][blk] (m = 3 i + j): block sums over its node range of
// A_b [df_i x_j + (lambda - 1)(u_i n_j + u_j n_i)] (fixed order)
__global__ void __launch_bounds__(kMomBlock) particle_stress_partial(
    int n, const double* __restrict__ x, const double* __restrict__ area,
    const double* __restrict__ nrm, const double* __restrict__ df, const double* __restrict__ u,
    double lm1, double* __restrict__ part) {
  __shared__ double red[9][kMomBlock];
  double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = blockIdx.x * kMomBlock + threadIdx.x; b < n; b += kMomBlocks * kMomBlock) {
    const double A = area[b];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        s[3 * i + j] += A * (df[3 * (size_t)b + i] * x[3 * (size_t)b + j] +
                             lm1 * (u[3 * (size_t)b + i] * nrm[3 * (size_t)b + j] +
                                    u[3 * (size_t)b + j] * nrm[3 * (size_t)b + i]));
  }
  for (int m = 0; m < 9; ++m) red[m][threadIdx.x] = s[m];
  __syncthreads();
  for (int o = kMomBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int m = 0; m < 9; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 9) part[threadIdx.x * kMomBlocks + blockIdx.x] = red[threadIdx.x][0];
}

// Poiseuille flow between the walls y = -H and y = +H (Appendix B)
__global__ void poiseuille_kernel(int n, double U0, double H, const double* __restrict__ x,
                                  double* __restrict__ u) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double s = x[3 * (size_t)b + 1] / H;
  u[3 * (size_t)b] = U0 * (1.0 - s * s);
  u[3 * (size_t)b + 1] = 0.0;
  u[3 * (size_t)b + 2] = 0.0;
}

__global__ void fill_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// y = x + k2 (wl + wg): the operator of Eq. qa, k2 = 2 kappa with the 1/8pi
// of the discretised double layer
__global__ void bi_fredholm_combine(int n3, const double* __restrict__ x,
                                    const double* __restrict__ wl, const double* __restrict__ wg,
                                    double k2, double* __restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n3) y[j] = fma(k2, wl[j] + wg[j], x[j]);
}

// u = (shear y, 0, 0) + 8 pi (wl + wg)
__global__ void bi_velocity_finish(int n, const double* __restrict__ x,
                                   const double* __restrict__ wl, const double* __restrict__ wg,
                                   double shear, double* __restrict__ u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double e = 8.0 * M_PI;
  const size_t j = 3 * (size_t)i;
  u[j] = fma(e, wl[j] + wg[j], shear * x[j + 1]);
  u[j + 1] = e * (wl[j + 1] + wg[j + 1]);
  u[j + 2] = e * (wl[j + 2] + wg[j + 2]);
}

}  // namespace

struct ggem_rigid_s {
  ggem_plan_s* plan;
  long long max_nodes, max_tri;
  double *area, *wl, *wg, *q, *part;
  double* stress;       // particle-stress partials (9 x kMomBlocks) and totals (9)
  double *xsys, *bsys;  // solution and right-hand side of the rigid system (3n + 6)
  int *bad, *bad_host;
  gm::Work W;
  // current surface
  int n, ntri;
  const double* x;
  const int *tri, *off, *adj;
  double xc[3];
};

#define RIGID_TRY(expr)                                              \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) return gm::device_error(e_, #expr);        \
  } while (0)

static void free_rigid(ggem_rigid_s* r) {
  void* ptrs[] = {r->area, r->wl, r->wg, r->q, r->part, r->stress, r->xsys, r->bsys, r->bad};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (r->bad_host) (void)hipHostFree(r->bad_host);
  gm::free_work(r->W);
}

extern "C" int ggem_rigid_create(ggem_plan_t plan, long long max_nodes, long long max_tri,
                                 int restart, ggem_rigid_t* out) {
  if (!plan || !out) return ggem_set_error(GGEM_E_ARG, "null argument");
  *out = nullptr;
  if (restart < 1 || restart > 400) return ggem_set_error(GGEM_E_ARG, "restart must be in 1..400");
  if (max_nodes < 1 || max_tri < 1 || max_nodes > (1LL << 26) || max_tri > (1LL << 27))
    return ggem_set_error(GGEM_E_ARG, "capacities out of range");
  if (max_nodes > plan->p.p.max_src || max_nodes > plan->p.p.max_tgt)
    return ggem_set_error(GGEM_E_CAPACITY, "plan capacity must cover the nodes");
  ggem_rigid_s* r = new (std::nothrow) ggem_rigid_s();
  if (!r) return ggem_set_error(GGEM_E_NOMEM, "host allocation failed");
  memset(r, 0, sizeof *r);
  r->plan = plan;
  r->max_nodes = max_nodes;
  r->max_tri = max_tri;
  const size_t n3 = 3 * (size_t)max_nodes, ns = n3 + 6;
  const bool ok = hipMalloc((void**)&r->area, max_nodes * 8) == hipSuccess &&
                  hipMalloc((void**)&r->stress, 9 * kMomBlocks * 8 + 9 * 8) == hipSuccess &&
                  hipMalloc((void**)&r->wl, n3 * 8) == hipSuccess &&
                  hipMalloc((void**)&r->wg, n3 * 8) == hipSuccess &&
                  hipMalloc((void**)&r->q, n3 * 8) == hipSuccess &&
                  hipMalloc((void**)&r->part, 6 * kMomBlocks * 8) == hipSuccess &&
                  hipMalloc((void**)&r->xsys, ns * 8) == hipSuccess &&
                  hipMalloc((void**)&r->bsys, ns * 8) == hipSuccess &&
                  hipMalloc((void**)&r->bad, sizeof(int)) == hipSuccess &&
                  hipHostMalloc((void**)&r->bad_host, sizeof(int), 0) == hipSuccess &&
                  gm::alloc_work(r->W, ns, restart) == GGEM_OK;
  if (!ok) {
    free_rigid(r);
    delete r;
    return ggem_set_error(GGEM_E_NOMEM, "device allocation failed");
  }
  *out = r;
  return GGEM_OK;
}

extern "C" int ggem_rigid_destroy(ggem_rigid_t r) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  (void)hipStreamSynchronize(r->plan->p.stream);
  free_rigid(r);
  delete r;
  return GGEM_OK;
}

// Validate the surface, compute the node areas and keep the arrays.
static int set_surface(ggem_rigid_s* r, long long n, const double* x, long long ntri,
                       const int* tri, const int* off, const int* adj) {
  if (n < 1 || ntri < 1) return ggem_set_error(GGEM_E_ARG, "empty surface");
  if (n > r->max_nodes || ntri > r->max_tri)
    return ggem_set_error(GGEM_E_CAPACITY, "surface exceeds the solver capacity");
  if (!x || !tri || !off || !adj) return ggem_set_error(GGEM_E_ARG, "null surface array");
  r->n = (int)n;
  r->ntri = (int)ntri;
  r->x = x;
  r->tri = tri;
  r->off = off;
  r->adj = adj;
  hipStream_t st = r->plan->p.stream;
  fill_int<<<1, 64, 0, st>>>(r->bad, 0);
  bi_node_areas<<<(r->n + 255) / 256, 256, 0, st>>>(r->n, r->ntri, x, tri, off, adj, r->area,
                                                    r->bad);
  RIGID_TRY(hipGetLastError());
  RIGID_TRY(hipMemcpyAsync(r->bad_host, r->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  RIGID_TRY(hipStreamSynchronize(st));
  if (*r->bad_host) return ggem_set_error(GGEM_E_ARG, "mesh index out of range or inconsistent incidence");
  return GGEM_OK;
}

// w = discretised single layer of f at the nodes, or with normals the double
// layer of f (local part into r->wl, global part into r->wg, their sum into w
// when w is given)
static int layer(ggem_rigid_s* r, const double* f, const double* normals, double* w) {
  Plan& p = r->plan->p;
  hipStream_t st = p.stream;
  const int n = r->n;
  // local part: bin the nodes, then one wave per node
  RIGID_TRY(launch_bin(p, p.src, n, r->x, nullptr, nullptr, true, true));
  BiArgs a;
  a.g = p.cg;
  a.rc2 = p.rc2;
  a.alpha = p.p.alpha;
  a.n = n;
  a.ntri = r->ntri;
  a.x = r->x;
  a.tri = r->tri;
  a.off = r->off;
  a.adj = r->adj;
  a.keys = p.src.keys;
  a.cell_start = p.src.cell_start;
  a.perm = p.src.perm;
  a.f = f;
  a.nrm = normals;
  a.out = r->wl;
  if (normals)
    bi_local<true><<<(n + 3) / 4, 256, 0, st>>>(a);
  else
    bi_local<false><<<(n + 3) / 4, 256, 0, st>>>(a);
  RIGID_TRY(hipGetLastError());
  // global part: nodal trapezoid strengths through the GGEM global problem
  bi_scale<<<(3 * n + 255) / 256, 256, 0, st>>>(n, r->area, f, r->q);
  RIGID_TRY(hipGetLastError());
  const int rc = normals ? ggem_double_layer(r->plan, n, r->x, r->q, n, r->x, normals, r->wg,
                                             GGEM_PART_GLOBAL)
                         : ggem_single_layer(r->plan, n, r->x, r->q, n, r->x, r->wg,
                                             GGEM_PART_GLOBAL);
  if (rc) return rc;
  if (w) {
    bi_add<<<(3 * n + 255) / 256, 256, 0, st>>>(3 * n, r->wl, r->wg, w);
    RIGID_TRY(hipGetLastError());
  }
  return GGEM_OK;
}

extern "C" int ggem_bi_single_layer(ggem_rigid_t r, long long n_nodes, const double* nodes,
                                    long long n_tri, const int* tri, const int* inc_off,
                                    const int* inc_tri, const double* f, double* w) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  if (!f || !w) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (int rc = set_surface(r, n_nodes, nodes, n_tri, tri, inc_off, inc_tri)) return rc;
  return layer(r, f, nullptr, w);
}

extern "C" int ggem_bi_double_layer(ggem_rigid_t r, long long n_nodes, const double* nodes,
                                    long long n_tri, const int* tri, const int* inc_off,
                                    const int* inc_tri, const double* normals, const double* q,
                                    double* v) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  if (!normals || !q || !v) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (int rc = set_surface(r, n_nodes, nodes, n_tri, tri, inc_off, inc_tri)) return rc;
  return layer(r, q, normals, v);
}

extern "C" int ggem_bi_surface_velocity(ggem_rigid_t r, long long n_nodes, const double* nodes,
                                        long long n_tri, const int* tri, const int* inc_off,
                                        const int* inc_tri, const double* q, double shear_rate,
                                        double* u) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  if (!q || !u) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (!isfinite(shear_rate)) return ggem_set_error(GGEM_E_ARG, "shear rate must be finite");
  if (int rc = set_surface(r, n_nodes, nodes, n_tri, tri, inc_off, inc_tri)) return rc;
  if (int rc = layer(r, q, nullptr, nullptr)) return rc;
  bi_velocity_finish<<<(r->n + 255) / 256, 256, 0, r->plan->p.stream>>>(r->n, r->x, r->wl, r->wg,
                                                                      shear_rate, u);
  RIGID_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_bi_fredholm_solve(ggem_rigid_t r, long long n_nodes, const double* nodes,
                                      long long n_tri, const int* tri, const int* inc_off,
                                      const int* inc_tri, const double* normals, double kappa,
                                      const double* b, double* q, double tol, int max_iter,
                                      int* iters, double* rel_res) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  if (!normals || !b || !q) return ggem_set_error(GGEM_E_ARG, "null vector");
  if (!(tol > 0) || max_iter < 1 || !isfinite(kappa))
    return ggem_set_error(GGEM_E_ARG, "bad tolerance, max_iter or kappa");
  if (int rc = set_surface(r, n_nodes, nodes, n_tri, tri, inc_off, inc_tri)) return rc;
  hipStream_t st = r->plan->p.stream;
  const int n3 = 3 * r->n;
  gm::Work& W = r->W;
  W.st = st;
  auto op = [r, normals, kappa, n3, st](const double* x, double* y) {
    if (int rc = layer(r, x, normals, nullptr)) return rc;
    bi_fredholm_combine<<<(n3 + 255) / 256, 256, 0, st>>>(n3, x, r->wl, r->wg, 2.0 * kappa, y);
    RIGID_TRY(hipGetLastError());
    return (int)GGEM_OK;
  };
  auto none = [](double*) { return (int)GGEM_OK; };
  return gm::solve(W, n3, b, q, tol, max_iter, op, none, iters, rel_res);
}

// y = A x for x = (f, U, Omega)
static int rigid_apply(ggem_rigid_s* r, const double* x, double* y) {
  hipStream_t st = r->plan->p.stream;
  const int n = r->n;
  if (int rc = layer(r, x, nullptr, nullptr)) return rc;
  bi_rigid_rows<<<(n + 255) / 256, 256, 0, st>>>(n, r->x, r->xc[0], r->xc[1], r->xc[2],
                                                 x + 3 * (size_t)n, r->wl, r->wg, y);
  bi_moments_partial<<<kMomBlocks, kMomBlock, 0, st>>>(n, r->x, r->xc[0], r->xc[1], r->xc[2],
                                                       r->area, x, r->part);
  bi_moments_final<<<6, 64, 0, st>>>(r->part, y + 3 * (size_t)n);
  RIGID_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_rigid_solve(ggem_rigid_t r, long long n_nodes, const double* nodes,
                                long long n_tri, const int* tri, const int* inc_off,
                                const int* inc_tri, const double* center, const double* uinf,
                                double* f, double* motion, double tol, int max_iter, int* iters,
                                double* rel_res) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  if (!center || !uinf || !f || !motion) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (!(tol > 0) || max_iter < 1) return ggem_set_error(GGEM_E_ARG, "bad tolerance or max_iter");
  if (int rc = set_surface(r, n_nodes, nodes, n_tri, tri, inc_off, inc_tri)) return rc;
  for (int d = 0; d < 3; ++d) r->xc[d] = center[d];
  hipStream_t st = r->plan->p.stream;
  const int n = r->n;
  const size_t n3 = 3 * (size_t)n;
  // system vectors: x = (f, U, Omega), b = (u_inf, 0, 0)
  const double zero[6] = {0, 0, 0, 0, 0, 0};
  RIGID_TRY(hipMemcpyAsync(r->xsys, f, n3 * 8, hipMemcpyDeviceToDevice, st));
  RIGID_TRY(hipMemcpyAsync(r->xsys + n3, motion, 6 * 8, hipMemcpyHostToDevice, st));
  RIGID_TRY(hipMemcpyAsync(r->bsys, uinf, n3 * 8, hipMemcpyDeviceToDevice, st));
  RIGID_TRY(hipMemcpyAsync(r->bsys + n3, zero, 6 * 8, hipMemcpyHostToDevice, st));
  RIGID_TRY(hipStreamSynchronize(st));
  gm::Work& W = r->W;
  W.st = st;
  auto op = [r](const double* x, double* y) { return rigid_apply(r, x, y); };
  auto none = [](double*) { return (int)GGEM_OK; };
  if (int rc = gm::solve(W, (int)n3 + 6, r->bsys, r->xsys, tol, max_iter, op, none, iters,
                         rel_res))
    return rc;
  RIGID_TRY(hipMemcpyAsync(f, r->xsys, n3 * 8, hipMemcpyDeviceToDevice, st));
  RIGID_TRY(hipMemcpyAsync(motion, r->xsys + n3, 6 * 8, hipMemcpyDeviceToHost, st));
  RIGID_TRY(hipStreamSynchronize(st));
  return GGEM_OK;
}

extern "C" int ggem_poiseuille(ggem_plan_t plan, double U0, long long n, const double* x,
                               double* u) {
  if (!plan) return ggem_set_error(GGEM_E_ARG, "null plan");
  if (n < 0) return ggem_set_error(GGEM_E_ARG, "negative point count");
  if (n == 0) return GGEM_OK;
  if (!x || !u) return ggem_set_error(GGEM_E_ARG, "null array");
  Plan& p = plan->p;
  poiseuille_kernel<<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>((int)n, U0, p.p.H, x, u);
  RIGID_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_particle_stress(ggem_rigid_t r, long long n_nodes, const double* nodes,
                                    long long n_tri, const int* tri, const int* inc_off,
                                    const int* inc_tri, const double* normals, const double* df,
                                    const double* u, double lambda, double volume,
                                    double* out) {
  if (!r) return ggem_set_error(GGEM_E_ARG, "null rigid solver");
  if (!normals || !df || !u || !out) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (!(volume > 0)) return ggem_set_error(GGEM_E_ARG, "volume must be positive");
  if (int rc = set_surface(r, n_nodes, nodes, n_tri, tri, inc_off, inc_tri)) return rc;
  hipStream_t st = r->plan->p.stream;
  particle_stress_partial<<<kMomBlocks, kMomBlock, 0, st>>>(r->n, r->x, r->area, normals, df, u,
                                                            lambda - 1.0, r->stress);
  double* tot = r->stress + 9 * kMomBlocks;
  bi_moments_final<<<9, 64, 0, st>>>(r->stress, tot);
  RIGID_TRY(hipGetLastError());
  RIGID_TRY(hipMemcpyAsync(out, tot, 9 * 8, hipMemcpyDeviceToHost, st));
  RIGID_TRY(hipStreamSynchronize(st));
  for (int m = 0; m < 9; ++m) out[m] /= volume;
  return GGEM_OK;
}
