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
// 4th-order Lagrange stencil of Sec. 3.2.2.  One thread per probe, FP64 sums
// (the grid fields keep the plan's precision).  The local sums take the
// probes in the cell order of their binning, so that neighbouring lanes walk
// the same cells; each probe's own sum is unchanged by that order.
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

__global__ void __launch_bounds__(256) probe_local(ProbeArgs a) {
  const int ts = blockIdx.x * blockDim.x + threadIdx.x;
  if (ts >= a.nt) return;
  const int t = a.order[ts];
  const CellGeom& g = a.g;
  double px = a.xt[3 * (size_t)t], py = a.xt[3 * (size_t)t + 1], pz = a.xt[3 * (size_t)t + 2];
  double u[3] = {0, 0, 0}, pr = 0.0, s[6] = {0, 0, 0, 0, 0, 0};
  const bool finite = isfinite(px) && isfinite(py) && isfinite(pz);
  if (!finite || !(fabs(py) <= g.H)) {
    atomicOr(a.flags, finite ? kFlagOutside : kFlagNonFinite);
  } else {
    px = wrap_p(px, g.Lx);
    pz = wrap_p(pz, g.Lz);
    const int ix = min(g.ncx - 1, max(0, (int)floor(px * g.icx)));
    const int iy = min(g.ncy - 1, max(0, (int)floor((py + g.H) * g.icy)));
    const int iz = min(g.ncz - 1, max(0, (int)floor(pz * g.icz)));
    const int nxo = g.ncx >= 3 ? 3 : g.ncx, nzo = g.ncz >= 3 ? 3 : g.ncz;
    const double al = a.alpha, a3 = al * al * al / kSqrtPi;
    double selfx = 0, selfy = 0, selfz = 0;
    for (int oy = -1; oy <= 1; ++oy) {
      const int cy = iy + oy;
      if (cy < 0 || cy >= g.ncy) continue;
      for (int oxi = 0; oxi < nxo; ++oxi) {
        const int cx = g.ncx >= 3 ? (ix + oxi - 1 + g.ncx) % g.ncx : oxi;
        for (int ozi = 0; ozi < nzo; ++ozi) {
          const int cz = g.ncz >= 3 ? (iz + ozi - 1 + g.ncz) % g.ncz : ozi;
          const int c = (cy * g.ncx + cx) * g.ncz + cz;
          for (int j = a.cell_start[c]; j < a.cell_start[c + 1]; ++j) {
            const double dx = fma(-g.Lx, rint((px - a.sx[j]) * g.invLx), px - a.sx[j]);
            const double dy = py - a.sy[j];
            const double dz = fma(-g.Lz, rint((pz - a.sz[j]) * g.invLz), pz - a.sz[j]);
            double r2;
            {
#pragma clang fp contract(off)
              r2 = (dx * dx + dy * dy) + dz * dz;
            }
            if (r2 > a.rc2) continue;
            const int src = a.perm[j];
            const double fx = a.f[3 * (size_t)src], fy = a.f[3 * (size_t)src + 1],
                         fz = a.f[3 * (size_t)src + 2];
            if (r2 == 0.0) {
              selfx += fx;
              selfy += fy;
              selfz += fz;
              continue;
            }
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
            const double C = -6.0 * er * ir2 * ir2 - 12.0 * al / kSqrtPi * ex * ir2 * ir2 -
                             8.0 * a3 * ex * ir2;
            const double D = 4.0 * a3 * ex;
            const double d[3] = {dx, dy, dz}, gv[3] = {fx, fy, fz};
            const int ja[6] = {0, 1, 2, 0, 0, 1}, ka[6] = {0, 1, 2, 1, 2, 2};
            for (int m = 0; m < 6; ++m) {
              const int jj = ja[m], kk = ka[m];
              s[m] += C * d[jj] * d[kk] * df +
                      D * (d[jj] * gv[kk] + d[kk] * gv[jj] + (jj == kk ? df : 0.0));
            }
          }
        }
      }
    }
    const double sc = -4.0 * al / kSqrtPi;
    u[0] = kInv8Pi * (u[0] + sc * selfx);
    u[1] = kInv8Pi * (u[1] + sc * selfy);
    u[2] = kInv8Pi * (u[2] + sc * selfz);
    pr *= kInv8Pi;
    for (int m = 0; m < 6; ++m) s[m] *= kInv8Pi;
  }
  for (int d = 0; d < 3; ++d) a.u[3 * (size_t)t + d] = u[d];
  a.p[t] = pr;
  for (int m = 0; m < 6; ++m) a.s[6 * (size_t)t + m] = s[m];
}

struct ProbeInterpArgs {
  int nt, Nx, Nz, Ny, ncomp;
  double dx, dz, H, Lx, Lz;
  const double* y;     // Gauss-Lobatto nodes
  const double* xt;    // probes (nt, 3)
  const void* grid;    // [ncomp][Ny][Nx][Nz] T
  double* out[2];      // components [0, split) to out[0], [split, ncomp) to out[1]
  int split;
  int stride[2];
};

// out += the Lagrange interpolant of every grid component at the probe
template <typename T>
__global__ void __launch_bounds__(256) probe_interp(ProbeInterpArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nt) return;
  double x = a.xt[3 * (size_t)t], y = a.xt[3 * (size_t)t + 1], z = a.xt[3 * (size_t)t + 2];
  if (!(isfinite(x) && isfinite(z) && fabs(y) <= a.H)) return;  // flagged by probe_local
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
  const T* G = (const T*)a.grid;
  const size_t plane = (size_t)a.Nx * a.Nz, field = plane * a.Ny;
  for (int c = 0; c < a.ncomp; ++c) {
    double acc = 0.0;
    for (int jy = 0; jy < 5; ++jy)
      for (int ix = 0; ix < 5; ++ix) {
        const int ii = wrap1(i0 - 2 + ix, a.Nx);
        const T* row = G + c * field + (size_t)(j0 - 2 + jy) * plane + (size_t)ii * a.Nz;
        double rz = 0.0;
        for (int kz = 0; kz < 5; ++kz) rz += wz[kz] * (double)row[wrap1(k0 - 2 + kz, a.Nz)];
        acc += wy[jy] * wx[ix] * rz;
      }
    const int o = c < a.split ? 0 : 1;
    const int cc = c < a.split ? c : c - a.split;
    a.out[o][(size_t)t * a.stride[o] + cc] += acc;
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
  probe_local<<<(nt + 255) / 256, 256, 0, p.stream>>>(a);
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
  a.grid = p.phys;
  a.out[0] = out0;
  a.out[1] = out1;
  a.split = split;
  a.stride[0] = stride0;
  a.stride[1] = stride1;
  probe_interp<T><<<(nt + 255) / 256, 256, 0, p.stream>>>(a);
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
