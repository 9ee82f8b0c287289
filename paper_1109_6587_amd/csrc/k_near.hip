// Local (near-field) part of the GGEM sum, Eq. u_loc with the kernels of
// Eq. local, truncated at r_c and periodic in x, z by the minimum image
// (Sec. 3.2.2).  One work item = up to kNearBlock sorted targets of one cell;
// the sources of each neighbour cell are staged through LDS and every thread
// accumulates its own target in registers (no atomics, fixed order).
//
// Displacements and the cutoff test are always formed in FP64 (so the set of
// interacting pairs does not depend on the precision mode); the kernel values
// are evaluated in T (double, or float in mixed mode).
#include "ggem_internal.h"

namespace ggem {

template <typename T>
struct Kc {
  T alpha, a2, c2a, c12a, c8a3, c4a3, selfc;
};

template <typename T>
__host__ Kc<T> make_kc(double alpha) {
  const double sp = 1.7724538509055160273;  // sqrt(pi)
  Kc<T> k;
  k.alpha = (T)alpha;
  k.a2 = (T)(alpha * alpha);
  k.c2a = (T)(2.0 * alpha / sp);
  k.c12a = (T)(12.0 * alpha / sp);
  k.c8a3 = (T)(8.0 * alpha * alpha * alpha / sp);
  k.c4a3 = (T)(4.0 * alpha * alpha * alpha / sp);
  k.selfc = (T)(-4.0 * alpha / sp);
  return k;
}

__device__ inline double t_erfc(double v) { return erfc(v); }
__device__ inline float t_erfc(float v) { return erfcf(v); }
__device__ inline double t_exp(double v) { return exp(v); }
__device__ inline float t_exp(float v) { return expf(v); }
__device__ inline double t_sqrt(double v) { return sqrt(v); }
__device__ inline float t_sqrt(float v) { return sqrtf(v); }

// d - L rint(d/L) using a multiply by 1/L: for every pair within r_c < L/2
// the rounding picks the same image as the division would.
__device__ inline double min_image(double d, double L, double invL) {
  return fma(-L, rint(d * invL), d);
}

__device__ inline double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// G^l(d) f accumulated (without the 1/8pi factor).
template <typename T>
__device__ inline void stokeslet_acc(T dx, T dy, T dz, T r2, T fx, T fy, T fz, const Kc<T>& k,
                                     T& ux, T& uy, T& uz) {
  T r = t_sqrt(r2);
  T ir = (T)1 / r;
  T ec = t_erfc(k.alpha * r);
  T ex = t_exp(-k.a2 * r2);
  T A = ec * ir - k.c2a * ex;
  T B = (ec * ir + k.c2a * ex) * (ir * ir);
  T df = dx * fx + dy * fy + dz * fz;
  T Bdf = B * df;
  ux += A * fx + Bdf * dx;
  uy += A * fy + Bdf * dy;
  uz += A * fz + Bdf * dz;
}

// n . T^l(d) . q accumulated (without 1/8pi): T^l is fully symmetric,
// T_ijk = A d_i d_j d_k + B (delta_jk d_i + delta_ik d_j + delta_ij d_k).
template <typename T>
__device__ inline void stresslet_acc(T dx, T dy, T dz, T r2, T qx, T qy, T qz, T nx, T ny, T nz,
                                     const Kc<T>& k, T& vx, T& vy, T& vz) {
  T r = t_sqrt(r2);
  T ir = (T)1 / r;
  T ir2 = ir * ir;
  T ec = t_erfc(k.alpha * r);
  T ex = t_exp(-k.a2 * r2);
  T ir4 = ir2 * ir2;
  T A = -(T)6 * ec * ir4 * ir - k.c12a * ex * ir4 - k.c8a3 * ex * ir2;
  T B = k.c4a3 * ex;
  T dq = dx * qx + dy * qy + dz * qz;
  T dn = dx * nx + dy * ny + dz * nz;
  T qn = qx * nx + qy * ny + qz * nz;
  T Ad = A * dq * dn;
  T Bqn = B * qn, Bdn = B * dn, Bdq = B * dq;
  vx += Ad * dx + Bdn * qx + Bdq * nx + Bqn * dx;
  vy += Ad * dy + Bdn * qy + Bdq * ny + Bqn * dy;
  vz += Ad * dz + Bdn * qz + Bdq * nz + Bqn * dz;
}

struct NearArgs {
  CellGeom g;
  double rc2;
  const int* item_start;   // target items per cell (prefix)
  const int* tcell;        // target cell_start
  const double *tx, *ty, *tz;
  const void* tn;          // sorted target normals (T, SoA) for the double layer
  size_t tcap;
  const int* scell;        // source cell_start
  const double *sx, *sy, *sz;
  const void* sf;          // sorted strengths (T, SoA)
  size_t scap;
  void* out;               // (3 x tcap, T) at sorted targets
};

__device__ inline int find_cell(const int* __restrict__ start, int ncells, int item) {
  int lo = 0, hi = ncells - 1;
  while (lo < hi) {  // largest c with start[c] <= item
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, bool DL>
__global__ void __launch_bounds__(kNearBlock) near_field(NearArgs a, Kc<T> k) {
  __shared__ double lx[kNearBlock], ly[kNearBlock], lz[kNearBlock];
  __shared__ T lf[3][kNearBlock];
  const CellGeom& g = a.g;
  const int item = blockIdx.x;
  const int nitems = a.item_start[g.ncells];
  if (item >= nitems) return;
  const int c = find_cell(a.item_start, g.ncells, item);
  const int t0 = a.tcell[c] + (item - a.item_start[c]) * kNearBlock;
  const int t1 = min(a.tcell[c + 1], t0 + kNearBlock);
  const int t = t0 + threadIdx.x;
  const bool active = t < t1;
  double px = 0, py = 0, pz = 0;
  T nx = 0, ny = 0, nz = 0;
  if (active) {
    px = a.tx[t];
    py = a.ty[t];
    pz = a.tz[t];
    if (DL) {
      const T* tn = (const T*)a.tn;
      nx = tn[t];
      ny = tn[a.tcap + t];
      nz = tn[2 * a.tcap + t];
    }
  }
  const T* sf = (const T*)a.sf;
  T ux = 0, uy = 0, uz = 0;
  T sfx = 0, sfy = 0, sfz = 0;  // self contributions
  const int iz = c % g.ncz;
  const int ix = (c / g.ncz) % g.ncx;
  const int iy = c / (g.ncz * g.ncx);
  const int xa = g.ncx >= 3 ? -1 : 0, xb = g.ncx >= 3 ? 1 : g.ncx - 1;
  const int za = g.ncz >= 3 ? -1 : 0, zb = g.ncz >= 3 ? 1 : g.ncz - 1;
  for (int oy = -1; oy <= 1; ++oy) {
    const int cy = iy + oy;
    if (cy < 0 || cy >= g.ncy) continue;
    for (int ox = xa; ox <= xb; ++ox) {
      const int cx = g.ncx >= 3 ? (ix + ox + g.ncx) % g.ncx : ox;
      for (int oz = za; oz <= zb; ++oz) {
        const int cz = g.ncz >= 3 ? (iz + oz + g.ncz) % g.ncz : oz;
        const int nc = (cy * g.ncx + cx) * g.ncz + cz;
        const int s0 = a.scell[nc], s1 = a.scell[nc + 1];
        for (int b = s0; b < s1; b += kNearBlock) {
          __syncthreads();
          const int si = b + threadIdx.x;
          if (si < s1) {
            lx[threadIdx.x] = a.sx[si];
            ly[threadIdx.x] = a.sy[si];
            lz[threadIdx.x] = a.sz[si];
            lf[0][threadIdx.x] = sf[si];
            lf[1][threadIdx.x] = sf[a.scap + si];
            lf[2][threadIdx.x] = sf[2 * a.scap + si];
          }
          __syncthreads();
          const int cnt = min(kNearBlock, s1 - b);
          if (active) {
            for (int j = 0; j < cnt; ++j) {
              const double dx = min_image(px - lx[j], g.Lx, g.invLx);
              const double dy = py - ly[j];
              const double dz = min_image(pz - lz[j], g.Lz, g.invLz);
              const double r2 = dist2(dx, dy, dz);
              if (r2 <= a.rc2) {
                if (r2 > 0.0) {
                  if (DL)
                    stresslet_acc<T>((T)dx, (T)dy, (T)dz, (T)r2, lf[0][j], lf[1][j], lf[2][j], nx,
                                     ny, nz, k, ux, uy, uz);
                  else
                    stokeslet_acc<T>((T)dx, (T)dy, (T)dz, (T)r2, lf[0][j], lf[1][j], lf[2][j], k,
                                     ux, uy, uz);
                } else if (!DL) {
                  sfx += lf[0][j];
                  sfy += lf[1][j];
                  sfz += lf[2][j];
                }
              }
            }
          }
        }
      }
    }
  }
  if (active) {
    const T s = (T)0.039788735772973833942;  // 1/(8 pi)
    T* out = (T*)a.out;
    out[t] = s * (ux + k.selfc * sfx);
    out[a.tcap + t] = s * (uy + k.selfc * sfy);
    out[2 * a.tcap + t] = s * (uz + k.selfc * sfz);
  }
}

// Wall data of the global problem: u^g = -u^l at the wall nodes (Sec. 3.2.2).
// One thread per node of the planes y = -H (w = 0) and y = +H (w = 1).  The
// cells have height >= r_c, so only the wall-adjacent cell layer contributes.
template <typename T>
__global__ void wall_velocity(CellGeom g, double rc2, int Nx, int Nz, double dx, double dz,
                              const int* __restrict__ scell, const double* __restrict__ sx,
                              const double* __restrict__ sy, const double* __restrict__ sz,
                              const T* __restrict__ sf, size_t scap, Kc<T> k,
                              T* __restrict__ wall) {
  const int nplane = Nx * Nz;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 2 * nplane) return;
  const int w = gid / nplane;
  const int r = gid - w * nplane;
  const int i = r / Nz, kk = r - (r / Nz) * Nz;
  const double px = i * dx, pz = kk * dz, py = w ? g.H : -g.H;
  const int ix = min((int)floor(px * g.icx), g.ncx - 1);
  const int iz = min((int)floor(pz * g.icz), g.ncz - 1);
  const int cy = w ? g.ncy - 1 : 0;
  const int xa = g.ncx >= 3 ? -1 : 0, xb = g.ncx >= 3 ? 1 : g.ncx - 1;
  const int za = g.ncz >= 3 ? -1 : 0, zb = g.ncz >= 3 ? 1 : g.ncz - 1;
  T ux = 0, uy = 0, uz = 0;
  for (int ox = xa; ox <= xb; ++ox) {
    const int cx = g.ncx >= 3 ? (ix + ox + g.ncx) % g.ncx : ox;
    for (int oz = za; oz <= zb; ++oz) {
      const int cz = g.ncz >= 3 ? (iz + oz + g.ncz) % g.ncz : oz;
      const int nc = (cy * g.ncx + cx) * g.ncz + cz;
      const int s1 = scell[nc + 1];
      for (int s = scell[nc]; s < s1; ++s) {
        const double ddx = min_image(px - sx[s], g.Lx, g.invLx);
        const double ddy = py - sy[s];
        const double ddz = min_image(pz - sz[s], g.Lz, g.invLz);
        const double r2 = dist2(ddx, ddy, ddz);
        if (r2 <= rc2 && r2 > 0.0)
          stokeslet_acc<T>((T)ddx, (T)ddy, (T)ddz, (T)r2, sf[s], sf[scap + s], sf[2 * scap + s],
                           k, ux, uy, uz);
      }
    }
  }
  // -1/(8 pi), times the 1/(Nx Nz) of the forward DFT: the wall planes are
  // transformed in x, z only (the grid fields get that factor through the
  // Chebyshev forward matrix)
  const T s = (T)(-0.039788735772973833942 / ((double)Nx * (double)Nz));
  wall[(size_t)(w * 3 + 0) * nplane + r] = s * ux;
  wall[(size_t)(w * 3 + 1) * nplane + r] = s * uy;
  wall[(size_t)(w * 3 + 2) * nplane + r] = s * uz;
}

// Pressure gauge of the double layer: the k = 0 pressure at y = -H equals
// (1/(Lx Lz)) sum_s q_y,s Phi(-(y_s + H)), Phi(s) = 1/2 (1 + erf(alpha s)) +
// alpha s/(2 sqrt(pi)) exp(-alpha^2 s^2) (the plane-integrated global density
// integrated up to s), so the lateral mean of the total pressure vanishes at
// the lower wall.  Two-pass fixed-order reduction.
template <typename T>
__global__ void __launch_bounds__(256) gauge_partial(int n, double alpha, double H,
                                                     const double* __restrict__ sy,
                                                     const T* __restrict__ sf, size_t scap,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double s = -(sy[i] + H);
    const double as = alpha * s;
    const double phi = 0.5 * (1.0 + erf(as)) + as * 0.28209479177387814347 * exp(-as * as);
    v = (double)sf[scap + i] * phi;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[1 + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) gauge_final(int nblk, double scale, double* part) {
  __shared__ double red[256];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) v += part[1 + b];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[0] = red[0] * scale;
}

static NearArgs near_args(Plan& p) {
  NearArgs a;
  a.g = p.cg;
  a.rc2 = p.rc2;
  a.item_start = p.tgt.item_start;
  a.tcell = p.tgt.cell_start;
  a.tx = p.tgt.x;
  a.ty = p.tgt.y;
  a.tz = p.tgt.z;
  a.tn = p.tgt.s;
  a.tcap = (size_t)p.p.max_tgt;
  a.scell = p.src.cell_start;
  a.sx = p.src.x;
  a.sy = p.src.y;
  a.sz = p.src.z;
  a.sf = p.src.s;
  a.scap = (size_t)p.p.max_src;
  a.out = p.ul;
  return a;
}

static unsigned near_grid(Plan& p, int nt) {
  return (unsigned)((nt + kNearBlock - 1) / kNearBlock + p.cg.ncells);
}

template <typename T>
hipError_t launch_near_sl(Plan& p, int nt) {
  if (nt <= 0) return hipSuccess;
  near_field<T, false><<<near_grid(p, nt), kNearBlock, 0, p.stream>>>(near_args(p),
                                                                      make_kc<T>(p.p.alpha));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_near_dl(Plan& p, int nt) {
  if (nt <= 0) return hipSuccess;
  near_field<T, true><<<near_grid(p, nt), kNearBlock, 0, p.stream>>>(near_args(p),
                                                                     make_kc<T>(p.p.alpha));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wall(Plan& p) {
  const int n = 2 * p.p.Nx * p.p.Nz;
  wall_velocity<T><<<(n + 255) / 256, 256, 0, p.stream>>>(
      p.cg, p.rc2, p.p.Nx, p.p.Nz, p.dx, p.dz, p.src.cell_start, p.src.x, p.src.y, p.src.z,
      (const T*)p.src.s, (size_t)p.p.max_src, make_kc<T>(p.p.alpha), (T*)p.wall_phys);
  return hipGetLastError();
}

hipError_t launch_gauge(Plan& p) {
  const int n = p.src.n;
  const int nblk = (n + 255) / 256;
  if (nblk > 0) {
    if (p.fp64)
      gauge_partial<double><<<nblk, 256, 0, p.stream>>>(n, p.p.alpha, p.p.H, p.src.y,
                                                        (const double*)p.src.s,
                                                        (size_t)p.p.max_src, p.gauge);
    else
      gauge_partial<float><<<nblk, 256, 0, p.stream>>>(n, p.p.alpha, p.p.H, p.src.y,
                                                       (const float*)p.src.s,
                                                       (size_t)p.p.max_src, p.gauge);
  }
  gauge_final<<<1, 256, 0, p.stream>>>(nblk, 1.0 / (p.p.Lx * p.p.Lz), p.gauge);
  return hipGetLastError();
}

template hipError_t launch_near_sl<double>(Plan&, int);
template hipError_t launch_near_sl<float>(Plan&, int);
template hipError_t launch_near_dl<double>(Plan&, int);
template hipError_t launch_near_dl<float>(Plan&, int);
template hipError_t launch_wall<double>(Plan&);
template hipError_t launch_wall<float>(Plan&);

}  // namespace ggem
