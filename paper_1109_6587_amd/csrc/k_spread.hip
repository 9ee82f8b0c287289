// Global density on the grid (Sec. 3.2.2, assignment of the global density):
//   F(node) = sum_s f_s rho_g(node - x_s),  |node - x_s| <= r_c (minimum image),
//   rho_g(r) = alpha^3 pi^{-3/2} exp(-alpha^2 r^2) (5/2 - alpha^2 r^2)   (Eq. rho_l_g a).
//
// Each thread owns one grid node and sums over the sources in the cells that
// can reach its tile, in sorted order: no atomics, bitwise reproducible.  A
// workgroup covers a tile of 4 (y) x 8 (x) x 8 (z) nodes; sources of every
// overlapping cell are staged through LDS, and sources whose distance to the
// tile's bounding box exceeds r_c are compacted away before the pair loop.
#include "ggem_internal.h"

namespace ggem {

__device__ inline double min_image_s(double d, double L, double invL) {
  return fma(-L, rint(d * invL), d);
}

__device__ inline double dist2_s(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ inline double t_exp_s(double v) { return exp(v); }
__device__ inline float t_exp_s(float v) { return __builtin_amdgcn_exp2f(1.44269504088896341f * v); }

// distance from v to the interval [lo, hi] along a periodic axis
__device__ inline double box_gap_periodic(double v, double lo, double hi, double L, double invL) {
  double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  double d = fabs(min_image_s(v - c, L, invL)) - h;
  return d > 0.0 ? d : 0.0;
}

struct SpreadArgs {
  CellGeom g;
  int Nx, Nz, Ny;
  double dx, dz, rc, rc2, alpha;
  const double* y;     // Gauss-Lobatto nodes
  const int* scell;
  const double *sx, *sy, *sz;
  const void* sf;
  size_t scap;
  void* out;           // (3, Ny, Nx, Nz) T
  unsigned long long* work;  // update counter
};

// Tile of TJ (y) x TI (x) x TK (z) nodes, one node per thread.
constexpr int TJ = 4, TI = 8, TK = 8, TB = TJ * TI * TK;

template <typename T>
struct V4;
template <>
struct V4<double> {
  using t = double4;
};
template <>
struct V4<float> {
  using t = float4;
};

// REL: sources staged relative to the tile corner in T (mixed mode: the
// displacement is formed once per source in FP64, the pair test in FP32);
// otherwise every pair displacement is formed in FP64 with the minimum image.
//
// Sources are visited row by row: for each (y, x) cell pair the cells of the
// z range are contiguous in the sorted order (two segments where the range
// wraps), so one staged batch spans several cells.
template <typename T, bool REL>
__global__ void __launch_bounds__(TB) spread_tile(SpreadArgs a) {
  using Q = typename V4<T>::t;
  __shared__ double lx[REL ? 1 : TB], ly[REL ? 1 : TB], lz[REL ? 1 : TB];
  __shared__ Q lr[REL ? TB : 1];
  __shared__ Q lf[TB];
  __shared__ int wave_cnt[TB / 64];
  const CellGeom& g = a.g;
  const int tid = threadIdx.x;
  const int k = blockIdx.x * TK + (tid % TK);
  const int i = blockIdx.y * TI + ((tid / TK) % TI);
  const int j = blockIdx.z * TJ + tid / (TK * TI);
  const bool valid = (k < a.Nz) && (i < a.Nx) && (j < a.Ny);
  // tile bounds
  const int i_lo = blockIdx.y * TI, i_hi = min(a.Nx - 1, i_lo + TI - 1);
  const int k_lo = blockIdx.x * TK, k_hi = min(a.Nz - 1, k_lo + TK - 1);
  const int j_lo = blockIdx.z * TJ, j_hi = min(a.Ny - 1, j_lo + TJ - 1);
  const double bx0 = i_lo * a.dx, bx1 = i_hi * a.dx;
  const double bz0 = k_lo * a.dz, bz1 = k_hi * a.dz;
  const double by1 = a.y[j_lo], by0 = a.y[j_hi];  // y decreases with j
  const double px = valid ? i * a.dx : 0.0;
  const double pz = valid ? k * a.dz : 0.0;
  const double py = valid ? a.y[j] : 0.0;
  // node relative to the tile corner
  const T nrx = (T)(px - bx0), nry = (T)(py - by0), nrz = (T)(pz - bz0);
  const T rc2t = (T)a.rc2;
  const double eps = 1e-9 * (g.Lx + g.Lz);
  // cell ranges (unwrapped in x, z; clamped in y)
  int cx0 = (int)floor((bx0 - a.rc - eps) * g.icx), cx1 = (int)floor((bx1 + a.rc + eps) * g.icx);
  int cz0 = (int)floor((bz0 - a.rc - eps) * g.icz), cz1 = (int)floor((bz1 + a.rc + eps) * g.icz);
  if (cx1 - cx0 + 1 >= g.ncx) { cx0 = 0; cx1 = g.ncx - 1; }
  if (cz1 - cz0 + 1 >= g.ncz) { cz0 = 0; cz1 = g.ncz - 1; }
  const int cy0 = max(0, (int)floor((by0 - a.rc - eps + g.H) * g.icy));
  const int cy1 = min(g.ncy - 1, (int)floor((by1 + a.rc + eps + g.H) * g.icy));
  // z segments of a row (wrapped cell indices)
  const int zl0 = ((cz0 % g.ncz) + g.ncz) % g.ncz;
  const int zlen = cz1 - cz0 + 1;
  const int nseg = zl0 + zlen > g.ncz ? 2 : 1;
  const int seg_hi0 = nseg == 2 ? g.ncz - 1 : zl0 + zlen - 1, seg_hi1 = zl0 + zlen - 1 - g.ncz;
  const T* sf = (const T*)a.sf;
  const T a2 = (T)(a.alpha * a.alpha);
  const int lane = tid & 63, wave = tid >> 6;
  T fx = 0, fy = 0, fz = 0;
  unsigned nupd = 0;
  for (int cy = cy0; cy <= cy1; ++cy)
    for (int cxu = cx0; cxu <= cx1; ++cxu) {
      const int cx = ((cxu % g.ncx) + g.ncx) % g.ncx;
      const int row = (cy * g.ncx + cx) * g.ncz;
      for (int sg = 0; sg < nseg; ++sg) {
        const int lo = sg == 0 ? zl0 : 0, hi = sg == 0 ? seg_hi0 : seg_hi1;
        const int s0 = a.scell[row + lo], s1 = a.scell[row + hi + 1];
        for (int b = s0; b < s1; b += TB) {
          // stage sources that can reach the tile, compacted per wave
          const int si = b + tid;
          bool keep = false;
          double qx = 0, qy = 0, qz = 0;
          if (si < s1) {
            qx = a.sx[si];
            qy = a.sy[si];
            qz = a.sz[si];
            const double gx = box_gap_periodic(qx, bx0, bx1, g.Lx, g.invLx);
            const double gz = box_gap_periodic(qz, bz0, bz1, g.Lz, g.invLz);
            const double gy = qy < by0 ? by0 - qy : (qy > by1 ? qy - by1 : 0.0);
            keep = dist2_s(gx, gy, gz) <= a.rc2 * (1.0 + 1e-12);
          }
          const unsigned long long m = __ballot(keep);
          const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
          __syncthreads();
          if (lane == 0) wave_cnt[wave] = __popcll(m);
          __syncthreads();
          int off = 0;
          for (int w = 0; w < wave; ++w) off += wave_cnt[w];
          int total = 0;
          for (int w = 0; w < TB / 64; ++w) total += wave_cnt[w];
          if (keep) {
            const int slot = off + __popcll(m & lt);
            if (REL) {
              Q r;
              r.x = (T)min_image_s(qx - bx0, g.Lx, g.invLx);
              r.y = (T)(qy - by0);
              r.z = (T)min_image_s(qz - bz0, g.Lz, g.invLz);
              r.w = (T)0;
              lr[slot] = r;
            } else {
              lx[slot] = qx;
              ly[slot] = qy;
              lz[slot] = qz;
            }
            Q f;
            f.x = sf[si];
            f.y = sf[a.scap + si];
            f.z = sf[2 * a.scap + si];
            f.w = (T)0;
            lf[slot] = f;
          }
          __syncthreads();
          if (valid) {
            for (int s = 0; s < total; ++s) {
              T r2;
              if (REL) {
                const Q q = lr[s];
                const T dx = nrx - q.x, dy = nry - q.y, dz = nrz - q.z;
                r2 = dx * dx + dy * dy + dz * dz;
                if (!(r2 <= rc2t)) continue;
              } else {
                const double dx = min_image_s(px - lx[s], g.Lx, g.invLx);
                const double dy = py - ly[s];
                const double dz = min_image_s(pz - lz[s], g.Lz, g.invLz);
                const double d2 = dist2_s(dx, dy, dz);
                if (!(d2 <= a.rc2)) continue;
                r2 = (T)d2;
              }
              ++nupd;
              const T ar = a2 * r2;
              const T w = t_exp_s(-ar) * ((T)2.5 - ar);
              const Q f = lf[s];
              fx += w * f.x;
              fy += w * f.y;
              fz += w * f.z;
            }
          }
        }
      }
    }
  wave_count_add(a.work, nupd);
  if (valid) {
    const T c = (T)(a.alpha * a.alpha * a.alpha * 0.17958712212516656);  // alpha^3 pi^{-3/2}
    T* out = (T*)a.out;
    const size_t plane = (size_t)a.Ny * a.Nx * a.Nz;
    const size_t idx = ((size_t)j * a.Nx + i) * a.Nz + k;
    out[idx] = c * fx;
    out[plane + idx] = c * fy;
    out[2 * plane + idx] = c * fz;
  }
}

template <typename T>
hipError_t launch_spread(Plan& p, int /*unused*/) {
  SpreadArgs a;
  a.g = p.cg;
  a.Nx = p.p.Nx;
  a.Nz = p.p.Nz;
  a.Ny = p.p.Ny;
  a.dx = p.dx;
  a.dz = p.dz;
  a.rc = p.rc;
  a.rc2 = p.rc2;
  a.alpha = p.p.alpha;
  a.y = p.y;
  a.scell = p.src.cell_start;
  a.sx = p.src.x;
  a.sy = p.src.y;
  a.sz = p.src.z;
  a.sf = p.src.s;
  a.scap = (size_t)p.p.max_src;
  a.out = p.phys;
  a.work = p.work + 1;
  dim3 grid((p.p.Nz + TK - 1) / TK, (p.p.Nx + TI - 1) / TI, (p.p.Ny + TJ - 1) / TJ);
  // tile-relative staging needs one periodic image per (tile, source) pair
  const bool rel = sizeof(T) == 4 && TI * p.dx + p.rc < 0.5 * p.p.Lx && TK * p.dz + p.rc < 0.5 * p.p.Lz;
  if (rel) spread_tile<T, true><<<grid, TB, 0, p.stream>>>(a);
  else spread_tile<T, false><<<grid, TB, 0, p.stream>>>(a);
  return hipGetLastError();
}

template hipError_t launch_spread<double>(Plan&, int);
template hipError_t launch_spread<float>(Plan&, int);

}  // namespace ggem
