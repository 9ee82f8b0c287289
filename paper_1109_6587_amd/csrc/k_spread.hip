// Global density on the grid (Sec. 3.2.2, assignment of the global density):
//   F(node) = sum_s f_s rho_g(node - x_s),  |node - x_s| <= r_c (minimum image),
//   rho_g(r) = alpha^3 pi^{-3/2} exp(-alpha^2 r^2) (5/2 - alpha^2 r^2)   (Eq. rho_l_g a).
//
// Each lane owns two grid nodes and sums over the sources in the cells that
// can reach its tile, in a fixed order: no atomics, bitwise reproducible.
#include <vector>

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
__device__ inline double t_exp2_s(double v) { return exp2(v); }
__device__ inline float t_exp2_s(float v) { return __builtin_amdgcn_exp2f(v); }

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
  const int* scell;    // source bucket starts (cell, z slab)
  const double *sx, *sy, *sz;
  const void* sf;
  size_t scap;
  void* out;           // (3, Ny, Nx, Nz) T
  unsigned long long* work;  // update counter
};

// A block owns one tile of 8 (z) x 4 (x) x 4 (y) nodes; each lane owns two
// nodes, k and k + 4 along z, so every staged source serves two nodes per LDS
// read and the x, y part of the distance is shared by them.  The tile's
// source batches are dealt to the block's four waves in turn, so a heavy
// tile (mid-slab, many sources in reach) is shared by four waves instead of
// setting the kernel's length alone.
constexpr int TZ = 8, TX = 4, TY = 4, TB = 256, WT = 4, WZ = 8, NW = TB / 64;
// single-half list capacity: at most 3 carried over plus one batch
constexpr int kHalf = 68, kSlot = 64 + 2 * kHalf;

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

// a staged source far outside the slit: every pair with it is out of range
template <typename Q>
__device__ inline Q far_q() {
  Q r;
  r.x = 0;
  r.y = 1e30;
  r.z = 0;
  r.w = 0;
  return r;
}

// the wave's LDS writes visible to all its lanes
__device__ inline void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Every wave walks the cell rows that can reach the tile and numbers the
// 64-source batches in sorted order; wave w takes batches w, w + 4, ...  It
// keeps the batch's sources within r_c of the tile's box (compacted in sorted
// order into its own LDS slice) and every lane adds the kept sources to its
// two nodes.  Out-of-range terms add exactly zero, so the loop is branch-free
// and unrolled.  The four partial sums are added in wave order at the end
// (one block barrier), so the result does not depend on timing.
//
// REL: sources staged relative to the tile corner in T (mixed mode: the
// displacement is formed once per source in FP64, the pair test in FP32);
// otherwise every pair displacement is formed in FP64 with the minimum image.
// REL also sorts the kept sources by the z half of the tile they can reach:
// those within r_c of both halves are added at both of a lane's nodes, the
// others go to a per-half list that carries over between batches and is
// added at the lane's node of that half in complete groups of four.
//
// CNT: count the (source, node) pairs within r_c into a.work.
//
// The tile is (z tile bx, x tile by, y tile bz) of the grid of a.
template <typename T, bool REL, bool CNT>
__device__ __forceinline__ void spread_body(const SpreadArgs& a, int bx, int by, int bz) {
  using Q = typename V4<T>::t;
  __shared__ double lx[REL ? 1 : 4][64], ly[REL ? 1 : 4][64], lz[REL ? 1 : 4][64];
  // REL: per wave the both-halves list [0, 64) and the low-only and
  // high-only lists [64, 64 + kHalf) and [64 + kHalf, 64 + 2 kHalf)
  __shared__ Q lr[REL ? 4 : 1][REL ? kSlot : 64];
  __shared__ Q lf[4][REL ? kSlot : 64];
  __shared__ T red[NW - 1][6][64];
  __shared__ int desc0[5 * 64];
  __shared__ unsigned cnt_w[NW];
  const CellGeom& g = a.g;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k_lo = bx * TZ;
  const int i_lo = by * TX;
  const int j_lo = bz * TY;
  const int k = k_lo + (lane & 3), i = i_lo + ((lane >> 2) & 3), j = j_lo + (lane >> 4);
  const int k1 = k + 4;  // the lane's second node
  const bool valid = (k < a.Nz) && (i < a.Nx) && (j < a.Ny);
  const bool valid1 = valid && k1 < a.Nz;
  // tile bounds
  const int i_hi = min(a.Nx - 1, i_lo + WT - 1);
  const int k_hi = min(a.Nz - 1, k_lo + WZ - 1);
  const int j_hi = min(a.Ny - 1, j_lo + TY - 1);
  const double bx0 = i_lo * a.dx, bx1 = i_hi * a.dx;
  const double bz0 = k_lo * a.dz, bz1 = k_hi * a.dz;
  const double by1 = a.y[j_lo], by0 = a.y[j_hi];  // y decreases with j
  const double px = valid ? i * a.dx : 0.0;
  const double pz = valid ? k * a.dz : 0.0;
  const double pz1 = valid1 ? k1 * a.dz : 0.0;
  const double py = valid ? a.y[j] : 0.0;
  // node relative to the tile corner
  // REL: coordinates scaled by alpha sqrt(log2 e), so the squared scaled
  // distance u gives exp(-alpha^2 r^2) = 2^-u and alpha^2 r^2 = u ln 2.
  // A second node past the grid sits far away, so its terms are all zero.
  const double sc = REL ? a.alpha * 1.2011224087864498 : 1.0;  // sqrt(log2 e)
  const T nrx = (T)((px - bx0) * sc), nry = (T)((py - by0) * sc), nrz = (T)((pz - bz0) * sc);
  const T nrz1 = valid1 ? (T)((pz1 - bz0) * sc) : (T)1e30;
  const T rc2t = (T)(a.rc2 * sc * sc);
  const double eps = 1e-9 * (g.Lx + g.Lz);
  // cell ranges (unwrapped in x; clamped in y)
  int cx0 = (int)floor((bx0 - a.rc - eps) * g.icx), cx1 = (int)floor((bx1 + a.rc + eps) * g.icx);
  if (cx1 - cx0 + 1 >= g.ncx) { cx0 = 0; cx1 = g.ncx - 1; }
  const int cy0 = max(0, (int)floor((by0 - a.rc - eps + g.H) * g.icy));
  const int cy1 = min(g.ncy - 1, (int)floor((by1 + a.rc + eps + g.H) * g.icy));
  // Rows of cells along z, culled by the gap between the row's (x, y) cell
  // box and the tile; in each row only the z slabs within the remaining
  // reach sqrt(r_c^2 - gap^2) of the tile are read (two runs where the window
  // wraps).  Every window is conservative: the per-source test below decides.
  const double rc2m = a.rc2 * (1.0 + 1e-12);
  const double szs = g.icz * g.nzs;  // slabs per unit z
  const int nzf = g.ncz * g.nzs;     // slabs per row
  const double hbx = 0.5 * (bx1 - bx0), cbx = 0.5 * (bx0 + bx1);
  const T* sf = (const T*)a.sf;
  const T a2 = (T)(a.alpha * a.alpha);
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  T fx = 0, fy = 0, fz = 0, gx1 = 0, gy1 = 0, gz1 = 0;
  unsigned nupd = 0;
  int bc = 0;  // batches numbered in walk order (uniform)
  // REL: the z halves of the tile and the single-half lists' lengths
  const int k_mid = min(k_hi, k_lo + 3);
  const bool has_hi = k_lo + 4 <= k_hi;
  const double bzm0 = k_mid * a.dz, bzm1 = (k_lo + 4) * a.dz;
  int cl = 0, ch = 0;
  // A single-half list: its complete groups of four evaluated at the lane's
  // node of that half (nz, one exponential per pair), the 0-3 left over moved
  // to the list's front for the next batch; with flush the last group is
  // padded with far-away sources and evaluated too.
  auto half_pass = [&](int base, int& n, T nz, T& ax, T& ay, T& az, bool flush) {
    const int ng = flush ? (n + 3) / 4 : n / 4;
    if (ng == 0) return;
    if (flush && (n & 3)) {
      if (lane >= n && lane < 4 * ng) {
        lr[wave][base + lane] = far_q<Q>();
        Q f;
        f.x = f.y = f.z = f.w = (T)0;
        lf[wave][base + lane] = f;
      }
      lds_wave_sync();
    }
    if (valid) {
      for (int e0 = 0; e0 < 4 * ng; e0 += 4) {
        Q qg[4], fg[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          qg[u] = lr[wave][base + e0 + u];
          fg[u] = lf[wave][base + e0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const T dx = nrx - qg[u].x, dy = nry - qg[u].y, dz = nz - qg[u].z;
          const T r2 = dx * dx + dy * dy + dz * dz;
          const bool in = r2 <= rc2t;
          if (CNT) nupd += (unsigned)__popcll(__ballot(in));
          const T w = in ? t_exp2_s(-r2) * fma((T)-0.69314718055994531, r2, (T)2.5) : (T)0;
          ax += w * fg[u].x;
          ay += w * fg[u].y;
          az += w * fg[u].z;
        }
      }
    }
    if (flush) {
      n = 0;
      return;
    }
    const int rem = n - 4 * ng;
    if (rem > 0) {
      Q r, f;
      if (lane < rem) {
        r = lr[wave][base + 4 * ng + lane];
        f = lf[wave][base + 4 * ng + lane];
      }
      lds_wave_sync();
      if (lane < rem) {
        lr[wave][base + lane] = r;
        lf[wave][base + lane] = f;
      }
      lds_wave_sync();
    }
    n = rem;
  };
  // The rows are described in parallel, one lane per row (64 at a time):
  // its one or two runs of z slabs and their batch counts; an inclusive scan
  // of the counts numbers the batches in walk order, and the wave then takes
  // its own batches (walk number mod 4) without visiting the rows one by one.
  // A sparse tile thus pays one round of bucket loads, not one per row.  The
  // descriptors go to LDS (registers would cost occupancy): wave 0's to its
  // own slice, the others' to their reduction slot, which they write only
  // after their last batch.
  int* const rd = wave == 0 ? desc0 : reinterpret_cast<int*>(&red[wave - 1][0][0]);
  const int ncxr = cx1 - cx0 + 1;
  const int nrows = (cy1 - cy0 + 1) * ncxr;
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    int sa0 = 0, sa1 = 0, sb0 = 0, sb1 = 0;
    if (r0 + lane < nrows) {
      const int cy = cy0 + (r0 + lane) / ncxr, cxu = cx0 + (r0 + lane) % ncxr;
      const double ylo = cy / g.icy - g.H, yhi = (cy + 1) / g.icy - g.H;
      const double gyc = fmax(0.0, fmax(ylo - by1, by0 - yhi) - eps);
      const int cx = ((cxu % g.ncx) + g.ncx) % g.ncx;
      const double xlo = cx / g.icx, xhi = (cx + 1) / g.icx;
      const double gxc = fmax(
          0.0, fabs(min_image_s(0.5 * (xlo + xhi) - cbx, g.Lx, g.invLx)) - 0.5 * (xhi - xlo) - hbx - eps);
      const double h2 = rc2m - (gxc * gxc + gyc * gyc);
      if (h2 >= 0.0) {
        const double hz = sqrt(h2) + eps;
        int fa = (int)floor((bz0 - hz) * szs), fb = (int)floor((bz1 + hz) * szs);
        if (fb - fa + 1 >= nzf) {
          fa = 0;
          fb = nzf - 1;
        }
        const int fl0 = ((fa % nzf) + nzf) % nzf, flen = fb - fa + 1;
        const int row = (cy * g.ncx + cx) * nzf;
        if (fl0 + flen > nzf) {  // the window wraps: slabs fl0..nzf-1, then 0..
          sa0 = a.scell[row + fl0];
          sa1 = a.scell[row + nzf];
          sb0 = a.scell[row];
          sb1 = a.scell[row + fl0 + flen - nzf];
        } else {
          sa0 = a.scell[row + fl0];
          sa1 = a.scell[row + fl0 + flen];
        }
      }
    }
    int bend = ((sa1 - sa0 + 63) >> 6) + ((sb1 - sb0 + 63) >> 6);
    for (int o = 1; o < 64; o <<= 1) {  // inclusive prefix of the batch counts
      const int v = __shfl_up(bend, o);
      if (lane >= o) bend += v;
    }
    const int nun = __builtin_amdgcn_readlane(bend, 63);
    rd[lane] = bend;
    rd[64 + lane] = sa0;
    rd[128 + lane] = sa1;
    rd[192 + lane] = sb0;
    rd[256 + lane] = sb1;
    lds_wave_sync();
    int cc = 0;  // the row of the current batch (uniform, advances monotonically)
    int rend = __builtin_amdgcn_readfirstlane(rd[0]), rbeg = 0;
    for (int u = ((wave - bc) % NW + NW) % NW; u < nun; u += NW) {
      while (u >= rend) {
        rbeg = rend;
        rend = __builtin_amdgcn_readfirstlane(rd[++cc]);
      }
      const int ra0 = __builtin_amdgcn_readfirstlane(rd[64 + cc]);
      const int ra1 = __builtin_amdgcn_readfirstlane(rd[128 + cc]);
      const int na = (ra1 - ra0 + 63) >> 6;
      const int lb = u - rbeg;
      const int b = lb < na ? ra0 + 64 * lb : __builtin_amdgcn_readfirstlane(rd[192 + cc]) + 64 * (lb - na);
      const int s1 = lb < na ? ra1 : __builtin_amdgcn_readfirstlane(rd[256 + cc]);
      {
        {
          // the batch's sources within r_c of the tile's box, compacted; REL
          // sorts them by the z half (nodes k_lo..k_lo+3, k_lo+4..k_lo+7)
          // they can reach
          const int si = b + lane;
          bool keep = false, inlo = false, inhi = false;
          double qx = 0, qy = 0, qz = 0;
          if (si < s1) {
            qx = a.sx[si];
            qy = a.sy[si];
            qz = a.sz[si];
            const double gx = box_gap_periodic(qx, bx0, bx1, g.Lx, g.invLx);
            const double gy = qy < by0 ? by0 - qy : (qy > by1 ? qy - by1 : 0.0);
            if (REL) {
              const double gzl = box_gap_periodic(qz, bz0, bzm0, g.Lz, g.invLz);
              inlo = dist2_s(gx, gy, gzl) <= rc2m;
              if (has_hi) {
                const double gzh = box_gap_periodic(qz, bzm1, bz1, g.Lz, g.invLz);
                inhi = dist2_s(gx, gy, gzh) <= rc2m;
              }
              keep = inlo || inhi;
            } else {
              const double gz = box_gap_periodic(qz, bz0, bz1, g.Lz, g.invLz);
              keep = dist2_s(gx, gy, gz) <= rc2m;
              inlo = inhi = keep;
            }
          }
          const unsigned long long mb = __ballot(inlo && inhi);
          const unsigned long long ml = REL ? __ballot(inlo && !inhi) : 0ull;
          const unsigned long long mh = REL ? __ballot(inhi && !inlo) : 0ull;
          const int nb = __popcll(mb), nl = __popcll(ml), nh = __popcll(mh);
          if (nb + nl + nh == 0) continue;
          const int nb4 = (nb + 3) & ~3;
          __builtin_amdgcn_wave_barrier();
          if (keep) {
            int slot;
            if (inlo && inhi) slot = __popcll(mb & lt);
            else if (inlo) slot = 64 + cl + __popcll(ml & lt);
            else slot = 64 + kHalf + ch + __popcll(mh & lt);
            if (REL) {
              Q r;
              r.x = (T)(min_image_s(qx - bx0, g.Lx, g.invLx) * sc);
              r.y = (T)((qy - by0) * sc);
              r.z = (T)(min_image_s(qz - bz0, g.Lz, g.invLz) * sc);
              r.w = (T)0;
              lr[wave][slot] = r;
            } else {
              lx[wave][slot] = qx;
              ly[wave][slot] = qy;
              lz[wave][slot] = qz;
            }
            Q f;
            f.x = sf[si];
            f.y = sf[a.scap + si];
            f.z = sf[2 * a.scap + si];
            f.w = (T)0;
            lf[wave][slot] = f;
          }
          if (lane >= nb && lane < nb4) {
            // padding of the both-halves list up to a multiple of 4: a
            // source far outside the slit
            if (REL) {
              lr[wave][lane] = far_q<Q>();
            } else {
              lx[wave][lane] = 0.0;
              ly[wave][lane] = 1e30;
              lz[wave][lane] = 0.0;
            }
            Q f;
            f.x = f.y = f.z = f.w = (T)0;
            lf[wave][lane] = f;
          }
          lds_wave_sync();
          if (valid) {
            for (int e0 = 0; e0 < nb4; e0 += 4) {
              // the group's four positions and strengths are read before any
              // is used, so one LDS latency covers four candidates
              Q qg[4], fg[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                if (REL) qg[u] = lr[wave][e0 + u];
                fg[u] = lf[wave][e0 + u];
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int e = e0 + u;
                T r2, r21;
                bool in, in1;
                if (REL) {
                  const Q q = qg[u];
                  const T dx = nrx - q.x, dy = nry - q.y;
                  const T dz = nrz - q.z, dz1 = nrz1 - q.z;
                  const T dxy = dx * dx + dy * dy;
                  r2 = dxy + dz * dz;
                  r21 = dxy + dz1 * dz1;
                  in = r2 <= rc2t;
                  in1 = r21 <= rc2t;
                } else {
                  const double dx = min_image_s(px - lx[wave][e], g.Lx, g.invLx);
                  const double dy = py - ly[wave][e];
                  const double dz = min_image_s(pz - lz[wave][e], g.Lz, g.invLz);
                  const double dz1 = min_image_s(pz1 - lz[wave][e], g.Lz, g.invLz);
                  const double d2 = dist2_s(dx, dy, dz);
                  const double d21 = dist2_s(dx, dy, dz1);
                  in = d2 <= a.rc2;
                  in1 = valid1 && d21 <= a.rc2;
                  r2 = (T)d2;
                  r21 = (T)d21;
                }
                // the wave's counts, scalar
                if (CNT) nupd += (unsigned)__popcll(__ballot(in)) + (unsigned)__popcll(__ballot(in1));
                T w, w1;
                if (REL) {  // r2 is the scaled u
                  w = in ? t_exp2_s(-r2) * fma((T)-0.69314718055994531, r2, (T)2.5) : (T)0;
                  w1 = in1 ? t_exp2_s(-r21) * fma((T)-0.69314718055994531, r21, (T)2.5) : (T)0;
                } else {
                  w = in ? t_exp_s(-a2 * r2) * fma(-a2, r2, (T)2.5) : (T)0;
                  w1 = in1 ? t_exp_s(-a2 * r21) * fma(-a2, r21, (T)2.5) : (T)0;
                }
                const Q f = fg[u];
                fx += w * f.x;
                fy += w * f.y;
                fz += w * f.z;
                gx1 += w1 * f.x;
                gy1 += w1 * f.y;
                gz1 += w1 * f.z;
              }
            }
          }
          if constexpr (REL) {
            cl += nl;
            ch += nh;
            half_pass(64, cl, nrz, fx, fy, fz, false);
            half_pass(64 + kHalf, ch, nrz1, gx1, gy1, gz1, false);
          }
        }
      }
    }
    bc += nun;
    lds_wave_sync();  // the descriptors are read before the next chunk's
  }
  if constexpr (REL) {
    half_pass(64, cl, nrz, fx, fy, fz, true);
    half_pass(64 + kHalf, ch, nrz1, gx1, gy1, gz1, true);
  }
  // partial sums of waves 1..3 through LDS, added by wave 0 in wave order;
  // nupd is the wave's count in every lane (lanes of valid nodes only)
  if (wave > 0) {
    T* r = &red[wave - 1][0][0];
    r[0 * 64 + lane] = fx;
    r[1 * 64 + lane] = fy;
    r[2 * 64 + lane] = fz;
    r[3 * 64 + lane] = gx1;
    r[4 * 64 + lane] = gy1;
    r[5 * 64 + lane] = gz1;
  }
  if (CNT && lane == 0) cnt_w[wave] = nupd;
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < NW - 1; ++w) {
    fx += red[w][0][lane];
    fy += red[w][1][lane];
    fz += red[w][2][lane];
    gx1 += red[w][3][lane];
    gy1 += red[w][4][lane];
    gz1 += red[w][5][lane];
  }
  if (CNT && lane == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < NW; ++w) tot += cnt_w[w];
    if (tot) atomicAdd(a.work, tot);
  }
  if (valid) {
    const T c = (T)(a.alpha * a.alpha * a.alpha * 0.17958712212516656);  // alpha^3 pi^{-3/2}
    T* out = (T*)a.out;
    const size_t plane = (size_t)a.Ny * a.Nx * a.Nz;
    const size_t idx = ((size_t)j * a.Nx + i) * a.Nz + k;
    out[idx] = c * fx;
    out[plane + idx] = c * fy;
    out[2 * plane + idx] = c * fz;
    if (valid1) {
      out[idx + 4] = c * gx1;
      out[plane + idx + 4] = c * gy1;
      out[2 * plane + idx + 4] = c * gz1;
    }
  }
}

// XCD-aware: blocks are dealt round-robin to the 8 XCDs, so block b runs on
// XCD b % 8; each XCD gets a contiguous run of the z tiles of a row
__device__ inline int xcd_z_tile(int b, int nbx) {
  if ((nbx & 7) != 0) return b;
  const int per = nbx >> 3;
  return (b & 7) * per + (b >> 3);
}

template <typename T, bool REL, bool CNT>
__global__ void __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1)))
spread_tile(SpreadArgs a) {
  spread_body<T, REL, CNT>(a, xcd_z_tile(blockIdx.x, gridDim.x), blockIdx.y, blockIdx.z);
}

// Many grids in one launch: job j owns blocks [boff[j], boff[j + 1]) (its
// tiles, z fastest, padded to a multiple of 8 so that every job's rows start
// on XCD 0 as in the single launch).  A block finds its job by bisection and
// does exactly the work of the same tile in the job's own launch.
template <typename T, bool REL>
__global__ void __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1)))
spread_tile_jobs(const SpreadArgs* __restrict__ jobs, const int* __restrict__ boff, int njobs) {
  const int b = blockIdx.x;
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid;
  }
  const SpreadArgs& a = jobs[lo];
  const int nbx = (a.Nz + TZ - 1) / TZ, nby = (a.Nx + TX - 1) / TX, nbz = (a.Ny + TY - 1) / TY;
  const int t = b - boff[lo];
  if (t >= nbx * nby * nbz) return;  // padding
  const int row = t / nbx;
  spread_body<T, REL, false>(a, xcd_z_tile(t - row * nbx, nbx), row % nby, row / nby);
}

static SpreadArgs spread_args(const Plan& p) {
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
  a.scell = p.src.sub_start;
  a.sx = p.src.x;
  a.sy = p.src.y;
  a.sz = p.src.z;
  a.sf = p.src.s;
  a.scap = (size_t)p.p.max_src;
  a.out = p.phys;
  a.work = nullptr;
  return a;
}

// tile-relative staging (FP32 only) needs one periodic image per (tile,
// source) pair
static bool spread_rel(const Plan& p) {
  return !p.fp64 && WT * p.dx + p.rc < 0.5 * p.p.Lx && WZ * p.dz + p.rc < 0.5 * p.p.Lz;
}

template <typename T>
hipError_t launch_spread(Plan& p, int /*unused*/) {
  SpreadArgs a = spread_args(p);
  a.work = p.count_work ? p.work + 1 : nullptr;
  dim3 grid((p.p.Nz + TZ - 1) / TZ, (p.p.Nx + TX - 1) / TX, (p.p.Ny + TY - 1) / TY);
  const bool rel = sizeof(T) == 4 && spread_rel(p);
  const bool cnt = a.work != nullptr;
  if (rel && cnt) spread_tile<T, true, true><<<grid, TB, 0, p.stream>>>(a);
  else if (rel) spread_tile<T, true, false><<<grid, TB, 0, p.stream>>>(a);
  else if (cnt) spread_tile<T, false, true><<<grid, TB, 0, p.stream>>>(a);
  else spread_tile<T, false, false><<<grid, TB, 0, p.stream>>>(a);
  return hipGetLastError();
}

int spread_job_blocks(const Plan& p) {
  const int n = ((p.p.Nz + TZ - 1) / TZ) * ((p.p.Nx + TX - 1) / TX) * ((p.p.Ny + TY - 1) / TY);
  return (n + 7) & ~7;
}

bool spread_job_rel(const Plan& p) { return spread_rel(p); }

int spread_jobs_upload(const Plan* const* plans, int n, void* dev_args, int* dev_boff) {
  std::vector<SpreadArgs> a(n);
  std::vector<int> off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    a[i] = spread_args(*plans[i]);
    off[i + 1] = off[i] + spread_job_blocks(*plans[i]);
  }
  if (n > 0 && (hipMemcpy(dev_args, a.data(), n * sizeof(SpreadArgs), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dev_boff, off.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess))
    return -1;
  return off[n];
}

size_t spread_job_bytes() { return sizeof(SpreadArgs); }

template <typename T>
hipError_t launch_spread_jobs(hipStream_t s, const void* dev_args, const int* dev_boff, int n,
                              int nblocks, bool rel) {
  if (n <= 0 || nblocks <= 0) return hipSuccess;
  const SpreadArgs* a = (const SpreadArgs*)dev_args;
  if (sizeof(T) == 4 && rel) spread_tile_jobs<T, true><<<nblocks, TB, 0, s>>>(a, dev_boff, n);
  else spread_tile_jobs<T, false><<<nblocks, TB, 0, s>>>(a, dev_boff, n);
  return hipGetLastError();
}

template hipError_t launch_spread<double>(Plan&, int);
template hipError_t launch_spread<float>(Plan&, int);
template hipError_t launch_spread_jobs<double>(hipStream_t, const void*, const int*, int, int, bool);
template hipError_t launch_spread_jobs<float>(hipStream_t, const void*, const int*, int, int, bool);

}  // namespace ggem
