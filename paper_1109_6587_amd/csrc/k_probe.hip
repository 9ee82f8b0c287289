// Velocity, pressure and stress at probes, and the traction of the
// undisturbed flows.
//
// Probes: u = u^l + u^g, p = p^l + p^g, sigma = sigma^l + sigma^g for point
// forces g^nu.  The local parts are summed over the sources within r_c of a
// probe (minimum image), with the kernels of Eq. local (a)-(c):
//   u^l = (1/8pi) sum G^l g,  p^l = (1/8pi) sum P^l . g,
//   sigma^l_jk = (1/8pi) sum_i T^l_jik g_i,
// a coincident source adding -(4 alpha/sqrt(pi))/(8pi) g to the velocity only.
// The global parts are the slit solution of Appendix C interpolated with the
// 4th-order Lagrange stencil of Sec. 3.2.2.  The local sums run in FP64, one
// block of four waves per work item of up to 64 probes of one cell of the
// probes' binning (probe_local); the interpolation takes one thread per
// probe and sums in FP64 (the grid fields keep the plan's precision).
//
// Undisturbed flows (Appendix B), walls at y = -H and y = +H:
//   simple shear sigma = rate e;  Poiseuille (centre-line velocity U0)
//   sigma = (2 U0/H^2) x I - (2 U0 y/H^2) e,  e_xy = e_yx = 1;
// the traction is f = sigma . n.
#include "ggem_internal.h"

namespace ggem {

namespace {

constexpr double kInv8Pi = 0.039788735772973833942;
constexpr double kSqrtPi = 1.7724538509055160273;

__device__ inline double wrap_p(double v, double L) {
  double r = fmod(v, L);
  if (r < 0.0) r += L;
  if (r >= L) r = 0.0;
  return r;
}

struct ProbeArgs {
  CellGeom g;
  double rc2, alpha;
  int nt;
  const double* xt;        // probes (nt, 3), any periodic image
  const int* order;        // probes in cell order (their binning's permutation)
  const int* cell_start;   // binned sources
  const int* perm;
  const double *sx, *sy, *sz;
  const double* f;         // (ns, 3) original strengths
  double* u;               // (nt, 3)
  double* p;               // (nt)
  double* s;               // (nt, 6): xx, yy, zz, xy, xz, yz
  unsigned* flags;
};

// One pair within r_c (r2 > 0): its terms of u^l, p^l and sigma^l (without
// the 1/8pi), added to u, pr and s.
__device__ inline void probe_pair(double dx, double dy, double dz, double r2, double fx, double fy,
                                  double fz, double al, double a3, double* u, double& pr,
                                  double* s) {
  const double r = sqrt(r2), ir2 = 1.0 / r2;
  const double ec = erfc(al * r), ex = exp(-al * al * r2);
  const double df = dx * fx + dy * fy + dz * fz;
  // G^l g = A g + B d (d.g)
  const double er = ec / r, ce = 2.0 * al / kSqrtPi * ex;
  const double A = er - ce, B = (er + ce) * ir2;
  u[0] += A * fx + B * df * dx;
  u[1] += A * fy + B * df * dy;
  u[2] += A * fz + B * df * dz;
  // P^l . g = (2 erfc/r^3 + (4 alpha/sqrt(pi)) (1/r^2 - alpha^2) e) (d.g)
  pr += (2.0 * er * ir2 + 4.0 * al / kSqrtPi * (ir2 - al * al) * ex) * df;
  // T^l_jik g_i = C d_j d_k (d.g) + D (d_j g_k + d_k g_j + delta_jk (d.g))
  const double C = -6.0 * er * ir2 * ir2 - 12.0 * al / kSqrtPi * ex * ir2 * ir2 - 8.0 * a3 * ex * ir2;
  const double D = 4.0 * a3 * ex;
  const double d[3] = {dx, dy, dz}, gv[3] = {fx, fy, fz};
  const int ja[6] = {0, 1, 2, 0, 0, 1}, ka[6] = {0, 1, 2, 1, 2, 2};
  for (int m = 0; m < 6; ++m) {
    const int jj = ja[m], kk = ka[m];
    s[m] += C * d[jj] * d[kk] * df + D * (d[jj] * gv[kk] + d[kk] * gv[jj] + (jj == kk ? df : 0.0));
  }
}

// minimum-image displacement and its square, formed as the pair sums decide
// the cutoff (FP64, fixed association)
__device__ inline double probe_disp(const CellGeom& g, double px, double py, double pz, double qx,
                                    double qy, double qz, double& dx, double& dy, double& dz) {
  dx = fma(-g.Lx, rint((px - qx) * g.invLx), px - qx);
  dy = py - qy;
  dz = fma(-g.Lz, rint((pz - qz) * g.invLz), pz - qz);
  double r2;
  {
#pragma clang fp contract(off)
    r2 = (dx * dx + dy * dy) + dz * dz;
  }
  return r2;
}

// One block of four waves per work item: up to 64 probes of one cell of the
// probes' binning, one probe per lane of every wave.  The item's neighbour
// cells are walked in a fixed order (y, then x, then z offsets) and their
// sorted sources numbered in batches of 64; wave w takes batches w, w + 4,
// ..., staged through its own LDS slice.  Every lane first marks its sources
// within r_c in the batch (a coincident source goes to the self term at
// once), then evaluates the marked ones in source order, so the expensive
// pair terms cost a wave only as many steps as its busiest lane has pairs.
// The four partial sums are added in wave order at the end: the result does
// not depend on timing.
constexpr int kProbeWaves = 4;

__global__ void __launch_bounds__(64 * kProbeWaves) probe_local(ProbeArgs a,
                                                                const int* __restrict__ item_start,
                                                                const int* __restrict__ item_cell,
                                                                const int* __restrict__ tcell) {
  __shared__ double lq[kProbeWaves][3][64], lf[kProbeWaves][3][64];
  __shared__ double part[kProbeWaves - 1][13][64];
  const CellGeom& g = a.g;
  const int item = blockIdx.x;
  if (item >= item_start[g.ncells]) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = item_cell[item];
  const int t0 = tcell[c] + (item - item_start[c]) * 64;
  const bool active = t0 + lane < tcell[c + 1];
  const int t = active ? a.order[t0 + lane] : 0;
  double px = 0.0, py = 0.0, pz = 0.0;
  bool ok = false;
  if (active) {
    px = a.xt[3 * (size_t)t];
    py = a.xt[3 * (size_t)t + 1];
    pz = a.xt[3 * (size_t)t + 2];
    const bool finite = isfinite(px) && isfinite(py) && isfinite(pz);
    if (finite && fabs(py) <= g.H) {
      ok = true;
      px = wrap_p(px, g.Lx);
      pz = wrap_p(pz, g.Lz);
    } else if (wave == 0) {
      atomicOr(a.flags, finite ? kFlagOutside : kFlagNonFinite);
    }
  }
  const int iz = c % g.ncz, ix = (c / g.ncz) % g.ncx, iy = c / (g.ncz * g.ncx);
  const int nxo = g.ncx >= 3 ? 3 : g.ncx, nzo = g.ncz >= 3 ? 3 : g.ncz;
  const double al = a.alpha, a3 = al * al * al / kSqrtPi;
  // u (3), p, sigma (6), self (3)
  double acc[13];
  for (int m = 0; m < 13; ++m) acc[m] = 0.0;
  int bc = 0;  // batches numbered in walk order (uniform)
  for (int oy = -1; oy <= 1; ++oy) {
    const int cy = iy + oy;
    if (cy < 0 || cy >= g.ncy) continue;
    for (int oxi = 0; oxi < nxo; ++oxi) {
      const int cx = g.ncx >= 3 ? (ix + oxi - 1 + g.ncx) % g.ncx : oxi;
      for (int ozi = 0; ozi < nzo; ++ozi) {
        const int cz = g.ncz >= 3 ? (iz + ozi - 1 + g.ncz) % g.ncz : ozi;
        const int cc = (cy * g.ncx + cx) * g.ncz + cz;
        const int s0 = a.cell_start[cc], s1 = a.cell_start[cc + 1];
        for (int b = s0; b < s1; b += 64) {
          if (bc++ % kProbeWaves != wave) continue;
          const int j = b + lane;
          __builtin_amdgcn_wave_barrier();
          if (j < s1) {
            lq[wave][0][lane] = a.sx[j];
            lq[wave][1][lane] = a.sy[j];
            lq[wave][2][lane] = a.sz[j];
            const int src = a.perm[j];
            lf[wave][0][lane] = a.f[3 * (size_t)src];
            lf[wave][1][lane] = a.f[3 * (size_t)src + 1];
            lf[wave][2][lane] = a.f[3 * (size_t)src + 2];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const int n = min(64, s1 - b);
          unsigned long long mask = 0;
          if (ok) {
            for (int e = 0; e < n; ++e) {
              double dx, dy, dz;
              const double r2 = probe_disp(g, px, py, pz, lq[wave][0][e], lq[wave][1][e],
                                           lq[wave][2][e], dx, dy, dz);
              if (r2 > a.rc2) continue;
              if (r2 == 0.0) {
                acc[10] += lf[wave][0][e];
                acc[11] += lf[wave][1][e];
                acc[12] += lf[wave][2][e];
                continue;
              }
              mask |= 1ull << e;
            }
          }
          while (mask) {
            const int e = __builtin_ctzll(mask);
            mask &= mask - 1;
            double dx, dy, dz;
            const double r2 = probe_disp(g, px, py, pz, lq[wave][0][e], lq[wave][1][e],
                                         lq[wave][2][e], dx, dy, dz);
            probe_pair(dx, dy, dz, r2, lf[wave][0][e], lf[wave][1][e], lf[wave][2][e], al, a3,
                       acc, acc[3], acc + 4);
          }
        }
      }
    }
  }
  if (wave > 0)
    for (int m = 0; m < 13; ++m) part[wave - 1][m][lane] = acc[m];
  __syncthreads();
  if (wave != 0 || !active) return;
  for (int w = 0; w < kProbeWaves - 1; ++w)
    for (int m = 0; m < 13; ++m) acc[m] += part[w][m][lane];
  if (ok) {
    const double sc = -4.0 * al / kSqrtPi;
    for (int d = 0; d < 3; ++d) a.u[3 * (size_t)t + d] = kInv8Pi * (acc[d] + sc * acc[10 + d]);
    a.p[t] = kInv8Pi * acc[3];
    for (int m = 0; m < 6; ++m) a.s[6 * (size_t)t + m] = kInv8Pi * acc[4 + m];
  } else {
    for (int d = 0; d < 3; ++d) a.u[3 * (size_t)t + d] = 0.0;
    a.p[t] = 0.0;
    for (int m = 0; m < 6; ++m) a.s[6 * (size_t)t + m] = 0.0;
  }
}

struct ProbeInterpArgs {
  int nt, Nx, Nz, Ny, ncomp;
  double dx, dz, H, Lx, Lz;
  const double* y;     // Gauss-Lobatto nodes
  const double* xt;    // probes (nt, 3)
  const int* order;    // probes in the cell order of their binning
  const void* grid;    // [ncomp][Ny][Nx][Nz] T
  double* out[2];      // components [0, split) to out[0], [split, ncomp) to out[1]
  int split;
  int stride[2];
};

// out += the Lagrange interpolant of every grid component at the probe.
// The threads take the probes in cell order, so that a block's stencils
// overlap in the caches.  G lanes per probe (G = 16 for few probes, else 1):
// lane r of a probe's group takes the stencil rows (y, x) = r, r + G, ... of
// the 25 rows of five z nodes, and the group adds its partial sums in a fixed
// tree order.
template <typename T, int G>
__global__ void __launch_bounds__(256) probe_interp(ProbeInterpArgs a) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int ts = gid / G, r = gid % G;
  const bool valid = ts < a.nt;
  const int t = valid ? a.order[ts] : 0;
  double x = 0.0, y = 0.0, z = 0.0;
  if (valid) {
    x = a.xt[3 * (size_t)t];
    y = a.xt[3 * (size_t)t + 1];
    z = a.xt[3 * (size_t)t + 2];
  }
  // probes outside the slit are flagged by probe_local and left alone
  const bool ok = valid && isfinite(x) && isfinite(z) && fabs(y) <= a.H;
  if (G == 1 && !ok) return;
  if (!ok) x = y = z = 0.0;
  x = wrap_p(x, a.Lx);
  z = wrap_p(z, a.Lz);
  const int i0 = (int)floor(x / a.dx + 0.5), k0 = (int)floor(z / a.dz + 0.5);
  double wx[5], wz[5], wy[5], yn[5];
  lagrange5_uniform(x / a.dx - i0, wx);
  lagrange5_uniform(z / a.dz - k0, wz);
  const int N = a.Ny - 1;
  const int j0 = min(a.Ny - 3, max(2, (int)rint(acos(y / a.H) * N / M_PI)));
  for (int q = 0; q < 5; ++q) yn[q] = a.y[j0 - 2 + q];
  lagrange5(y, yn, wy);
  const T* Gr = (const T*)a.grid;
  const size_t plane = (size_t)a.Nx * a.Nz, field = plane * a.Ny;
  for (int c = 0; c < a.ncomp; ++c) {
    double acc = 0.0;
    for (int row = r; row < 25; row += G) {
      const int jy = row / 5, ix = row % 5;
      const int ii = wrap1(i0 - 2 + ix, a.Nx);
      const T* rowp = Gr + c * field + (size_t)(j0 - 2 + jy) * plane + (size_t)ii * a.Nz;
      double rz = 0.0;
      for (int kz = 0; kz < 5; ++kz) rz += wz[kz] * (double)rowp[wrap1(k0 - 2 + kz, a.Nz)];
      acc += wy[jy] * wx[ix] * rz;
    }
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, G);
    if (ok && r == 0) {
      const int o = c < a.split ? 0 : 1;
      const int cc = c < a.split ? c : c - a.split;
      a.out[o][(size_t)t * a.stride[o] + cc] += acc;
    }
  }
}

__global__ void undisturbed_traction_kernel(int n, int kind, double rate, double H,
                                            const double* __restrict__ x,
                                            const double* __restrict__ nrm,
                                            double* __restrict__ f) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double nx = nrm[3 * (size_t)b], ny = nrm[3 * (size_t)b + 1], nz = nrm[3 * (size_t)b + 2];
  double iso = 0.0, off = rate;  // sigma = iso I + off e
  if (kind == GGEM_FLOW_POISEUILLE) {
    const double c = 2.0 * rate / (H * H);
    iso = c * x[3 * (size_t)b];
    off = -c * x[3 * (size_t)b + 1];
  }
  f[3 * (size_t)b] = iso * nx + off * ny;
  f[3 * (size_t)b + 1] = iso * ny + off * nx;
  f[3 * (size_t)b + 2] = iso * nz;
}

}  // namespace

hipError_t launch_probe_local(Plan& p, int nt, const double* xt, const double* f, double* u,
                              double* pr, double* sigma) {
  if (nt <= 0) return hipSuccess;
  // cell order of the probes (p.tgt.perm); non-finite or outside probes are
  // flagged here as in an evaluation and again by the kernel
  if (hipError_t e = launch_bin(p, p.tgt, nt, xt, nullptr, nullptr, false, false)) return e;
  ProbeArgs a;
  a.g = p.cg;
  a.rc2 = p.rc2;
  a.alpha = p.p.alpha;
  a.nt = nt;
  a.xt = xt;
  a.order = p.tgt.perm;
  a.cell_start = p.src.cell_start;
  a.perm = p.src.perm;
  a.sx = p.src.x;
  a.sy = p.src.y;
  a.sz = p.src.z;
  a.f = f;
  a.u = u;
  a.p = pr;
  a.s = sigma;
  a.flags = p.flags;
  // an upper bound of the work items: one per 64 probes of a cell
  const unsigned nitems = (unsigned)((nt + 63) / 64 + p.cg.ncells);
  probe_local<<<nitems, 64 * kProbeWaves, 0, p.stream>>>(a, p.tgt.item_start, p.tgt.item_cell,
                                                         p.tgt.cell_start);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_probe_interp(Plan& p, int nt, const double* xt, int ncomp, int split,
                               double* out0, int stride0, double* out1, int stride1) {
  if (nt <= 0) return hipSuccess;
  ProbeInterpArgs a;
  a.nt = nt;
  a.Nx = p.p.Nx;
  a.Nz = p.p.Nz;
  a.Ny = p.p.Ny;
  a.ncomp = ncomp;
  a.dx = p.dx;
  a.dz = p.dz;
  a.H = p.p.H;
  a.Lx = p.p.Lx;
  a.Lz = p.p.Lz;
  a.y = p.y;
  a.xt = xt;
  a.order = p.tgt.perm;  // binned by launch_probe_local
  a.grid = p.phys;
  a.out[0] = out0;
  a.out[1] = out1;
  a.split = split;
  a.stride[0] = stride0;
  a.stride[1] = stride1;
  if (nt < 65536)
    probe_interp<T, 16><<<(unsigned)(((size_t)nt * 16 + 255) / 256), 256, 0, p.stream>>>(a);
  else
    probe_interp<T, 1><<<(nt + 255) / 256, 256, 0, p.stream>>>(a);
  return hipGetLastError();
}

template hipError_t launch_probe_interp<double>(Plan&, int, const double*, int, int, double*, int,
                                                double*, int);
template hipError_t launch_probe_interp<float>(Plan&, int, const double*, int, int, double*, int,
                                               double*, int);

hipError_t launch_undisturbed_traction(Plan& p, int kind, double rate, int n, const double* x,
                                       const double* nrm, double* f) {
  if (n <= 0) return hipSuccess;
  undisturbed_traction_kernel<<<(n + 255) / 256, 256, 0, p.stream>>>(n, kind, rate, p.p.H, x, nrm,
                                                                     f);
  return hipGetLastError();
}

}  // namespace ggem
