// Local (near-field) part of the GGEM sum, Eq. u_loc with the kernels of
// Eq. local, truncated at r_c and periodic in x, z by the minimum image
// (Sec. 3.2.2).  One work item = up to 64 sorted targets of one cell; the
// neighbour cells are shared out among the waves of the block, their sources
// staged through LDS, and every lane accumulates its own target in registers
// (no atomics, fixed order of summation).
//
// FP64 mode forms every displacement and decides every cutoff and coincidence
// in FP64, as the oracle does.  Mixed mode (FAST below) decides the cutoff on
// the FP32 square of the FP64 displacement rounded per component, so pairs
// within an FP32 rounding of r_c may be kept or dropped (their kernel is below
// 1e-7 of its peak).  Pairs with alpha r < 1e-2 are decided and evaluated in
// FP64 in mixed mode, so only exactly coincident points take the self rule and
// no FP32 intermediate overflows.  Other kernel values are evaluated in T
// (double, or float in mixed mode) from the displacement formed in FP64.
#include <vector>

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


// d - L rint(d/L) using a multiply by 1/L: for every pair within r_c < L/2
// the rounding picks the same image as the division would.
__device__ inline double min_image(double d, double L, double invL) {
  return fma(-L, rint(d * invL), d);
}

__device__ inline double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// erfc and exp(-x^2) for the pair kernels.  FP64: the device library.  FP32:
// exp(-x^2) once, shared with the Gaussian terms, and erfc(x) =
// t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2), t = 1/(1 + p x), the
// approximation 7.1.26 of Abramowitz & Stegun (absolute error <= 1.5e-7).
__device__ inline void erfc_exp(double x, double x2, double& ec, double& ex) {
  ec = erfc(x);
  ex = exp(-x2);
}
__device__ inline void erfc_exp(float x, float x2, float& ec, float& ex) {
  ex = __builtin_amdgcn_exp2f(-1.44269504088896341f * x2);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  float p = fmaf(1.061405429f, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  ec = p * t * ex;
}
__device__ inline double t_rsqrt(double v) { return 1.0 / sqrt(v); }
__device__ inline float t_rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }

// G^l(d) f accumulated (without the 1/8pi factor):
// G^l f = f (erfc/r - c e) + d (d.f) (erfc/r + c e)/r^2,  c = 2 alpha/sqrt(pi).
template <typename T>
__device__ inline void stokeslet_acc(T dx, T dy, T dz, T r2, T fx, T fy, T fz, const Kc<T>& k,
                                     T& ux, T& uy, T& uz) {
  const T ir = t_rsqrt(r2);
  const T r = r2 * ir;
  T ec, ex;
  erfc_exp(k.alpha * r, k.a2 * r2, ec, ex);
  const T er = ec * ir;
  const T A = er - k.c2a * ex;
  const T B = (er + k.c2a * ex) * (ir * ir);
  const T df = dx * fx + dy * fy + dz * fz;
  const T Bdf = B * df;
  ux += A * fx + Bdf * dx;
  uy += A * fy + Bdf * dy;
  uz += A * fz + Bdf * dz;
}

// n . T^l(d) . q accumulated (without 1/8pi): T^l is fully symmetric,
// T_ijk = A d_i d_j d_k + B (delta_jk d_i + delta_ik d_j + delta_ij d_k).
template <typename T>
__device__ inline void stresslet_acc(T dx, T dy, T dz, T r2, T qx, T qy, T qz, T nx, T ny, T nz,
                                     const Kc<T>& k, T& vx, T& vy, T& vz) {
  const T ir = t_rsqrt(r2);
  const T r = r2 * ir;
  const T ir2 = ir * ir;
  T ec, ex;
  erfc_exp(k.alpha * r, k.a2 * r2, ec, ex);
  // A = -6 erfc/r^5 - c12 e/r^4 - c8 e/r^2, nested as -(1/r^2)((1/r^2)(6 erfc/r
  // + c12 e) + c8 e); the B (q.n) d term is folded into the A term
  const T A = -(ir2 * fma(ir2, fma((T)6 * ec, ir, k.c12a * ex), k.c8a3 * ex));
  const T B = k.c4a3 * ex;
  const T dq = dx * qx + dy * qy + dz * qz;
  const T dn = dx * nx + dy * ny + dz * nz;
  const T qn = qx * nx + qy * ny + qz * nz;
  const T Ad = fma(A * dq, dn, B * qn);
  const T Bdn = B * dn, Bdq = B * dq;
  vx += Ad * dx + Bdn * qx + Bdq * nx;
  vy += Ad * dy + Bdn * qy + Bdq * ny;
  vz += Ad * dz + Bdn * qz + Bdq * nz;
}

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using t = float4;
};
template <>
struct Vec4<double> {
  using t = double4;
};

// Pairs with alpha r below 1e-2 (alpha^2 r^2 < kNear2 in the FP32 test) are
// decided and evaluated in FP64: a coincident point takes the self rule, and
// a distinct one cannot overflow the FP32 intermediates of the kernels (1/r^3,
// 1/r^5).  There erfc and exp are their Taylor series (the first omitted term
// is below 1e-17 of the sum), so this rare path needs no library call.
constexpr double kNear2 = 1e-4;

template <typename T, bool DL, typename V>
__device__ void near_pair_fp64(double dx, double dy, double dz, const V& fv, T nx, T ny, T nz,
                               double alpha, T& ux, T& uy, T& uz, T& sfx, T& sfy, T& sfz) {
  const double r2 = dist2(dx, dy, dz);
  if (r2 == 0.0) {
    if (!DL) {
      sfx += fv.x;
      sfy += fv.y;
      sfz += fv.z;
    }
    return;
  }
  const double sp = 1.7724538509055160273;  // sqrt(pi)
  const double ir = 1.0 / sqrt(r2), r = r2 * ir, x = alpha * r, x2 = x * x;
  // exp(-x^2) and erfc(x) = 1 - (2/sqrt(pi)) (x - x^3/3 + x^5/10 - x^7/42)
  const double ex = 1.0 + x2 * (-1.0 + x2 * (0.5 + x2 * (-1.0 / 6.0)));
  const double ec = 1.0 - (2.0 / sp) * x * (1.0 + x2 * (-1.0 / 3.0 + x2 * (0.1 + x2 * (-1.0 / 42.0))));
  double vx, vy, vz;
  if (DL) {
    const double a3 = alpha * alpha * alpha;
    const double A = -(6.0 * ec * ir * ir * ir * ir * ir + 12.0 * alpha / sp * ex * ir * ir * ir * ir +
                       8.0 * a3 / sp * ex * ir * ir);
    const double B = 4.0 * a3 / sp * ex;
    const double qx = fv.x, qy = fv.y, qz = fv.z;
    const double dq = dx * qx + dy * qy + dz * qz;
    const double dn = dx * nx + dy * ny + dz * nz;
    const double qn = qx * nx + qy * ny + qz * nz;
    vx = A * dq * dn * dx + B * (dn * qx + dq * nx + qn * dx);
    vy = A * dq * dn * dy + B * (dn * qy + dq * ny + qn * dy);
    vz = A * dq * dn * dz + B * (dn * qz + dq * nz + qn * dz);
  } else {
    const double ce = 2.0 * alpha / sp * ex;
    const double A = ec * ir - ce, B = (ec * ir + ce) * ir * ir;
    const double df = dx * fv.x + dy * fv.y + dz * fv.z;
    vx = A * fv.x + B * df * dx;
    vy = A * fv.y + B * df * dy;
    vz = A * fv.z + B * df * dz;
  }
  ux += (T)vx;
  uy += (T)vy;
  uz += (T)vz;
}

// Constants of the branch-free FP32 kernels: the exponent and the erfc
// argument pre-multiplied.
struct KcF {
  double alpha;           // (FP64, for the near-coincident pairs)
  float nl2a2;            // -alpha^2 log2(e): exp(-alpha^2 r^2) = 2^(nl2a2 r^2)
  float pa;               // 0.3275911 alpha: t = 1/(1 + pa r)
  float c2a, c12a, c8a3, c4a3;
};

__host__ inline KcF make_kcf(double alpha) {
  const double sp = 1.7724538509055160273;
  KcF k;
  k.alpha = alpha;
  k.nl2a2 = (float)(-alpha * alpha * 1.4426950408889634074);
  k.pa = (float)(0.3275911 * alpha);
  k.c2a = (float)(2.0 * alpha / sp);
  k.c12a = (float)(12.0 * alpha / sp);
  k.c8a3 = (float)(8.0 * alpha * alpha * alpha / sp);
  k.c4a3 = (float)(4.0 * alpha * alpha * alpha / sp);
  return k;
}

// (S erfc(alpha r), exp(-alpha^2 r^2)) in FP32, erfc by Abramowitz & Stegun
// 7.1.26 with its coefficients scaled by S at compile time.
template <int S>
__device__ inline void erfc_exp_f(float r, float r2, const KcF& k, float& ec, float& ex) {
  ex = __builtin_amdgcn_exp2f(k.nl2a2 * r2);
  const float t = __builtin_amdgcn_rcpf(fmaf(k.pa, r, 1.0f));
  float p = fmaf((float)(S * 1.061405429), t, (float)(S * -1.453152027));
  p = fmaf(p, t, (float)(S * 1.421413741));
  p = fmaf(p, t, (float)(S * -0.284496736));
  p = fmaf(p, t, (float)(S * 0.254829592));
  ec = p * t * ex;
}

// G^l(d) f for one pair, both coefficients zeroed unless ok (0 < r <= r_c),
// so a lane can take every staged source: an excluded pair adds exact zeros.
__device__ inline void stokeslet_masked(float dx, float dy, float dz, float r2, bool ok, float fx,
                                        float fy, float fz, const KcF& k, float& ux, float& uy,
                                        float& uz) {
  const float ir = __builtin_amdgcn_rsqf(r2);
  float ec, ex;
  erfc_exp_f<1>(r2 * ir, r2, k, ec, ex);
  const float er = ec * ir, ce = k.c2a * ex;
  const float A = ok ? er - ce : 0.0f;
  const float B = ok ? (er + ce) * (ir * ir) : 0.0f;
  const float Bdf = B * (dx * fx + dy * fy + dz * fz);
  ux = fmaf(Bdf, dx, fmaf(A, fx, ux));
  uy = fmaf(Bdf, dy, fmaf(A, fy, uy));
  uz = fmaf(Bdf, dz, fmaf(A, fz, uz));
}

// n . T^l(d) . q for one pair with the same mask; the (B q.d) n term is
// summed into sn and multiplied by the target's normal once at the end.
__device__ inline void stresslet_masked(float dx, float dy, float dz, float r2, bool ok, float qx,
                                        float qy, float qz, float nx, float ny, float nz,
                                        const KcF& k, float& vx, float& vy, float& vz, float& sn) {
  const float ir = __builtin_amdgcn_rsqf(r2);
  const float ir2 = ir * ir;
  float ec6, ex;
  erfc_exp_f<6>(r2 * ir, r2, k, ec6, ex);
  // A = -6 erfc/r^5 - c12 e/r^4 - c8 e/r^2 (ec6 = 6 erfc), B = c4 e
  const float Af = ir2 * fmaf(ir2, fmaf(ec6, ir, k.c12a * ex), k.c8a3 * ex);
  const float Am = ok ? Af : 0.0f;  // -A
  const float B = ok ? k.c4a3 * ex : 0.0f;
  const float dq = dx * qx + dy * qy + dz * qz;
  const float dn = dx * nx + dy * ny + dz * nz;
  const float qn = qx * nx + qy * ny + qz * nz;
  const float Ad = fmaf(-(Am * dq), dn, B * qn);
  const float Bdn = B * dn;
  sn = fmaf(B, dq, sn);
  vx = fmaf(Bdn, qx, fmaf(Ad, dx, vx));
  vy = fmaf(Bdn, qy, fmaf(Ad, dy, vy));
  vz = fmaf(Bdn, qz, fmaf(Ad, dz, vz));
}

struct NearArgs {
  CellGeom g;
  double rc2;
  const int* item_start;   // target items per cell (prefix)
  const int* item_cell;    // cell of each target item
  const int* tcell;        // target cell_start
  const double *tx, *ty, *tz;
  const void* tn;          // sorted target normals (T, SoA) for the double layer
  size_t tcap;
  const int* scell;        // source cell_start
  const double *sx, *sy, *sz;
  const void* sf;          // sorted strengths (T, SoA)
  size_t scap;
  void* out;               // (3 x ostride, T)
  size_t ostride;
  const int* tperm;        // wall mode: sorted target -> wall node index
  int nplane;              // wall mode: nodes per wall plane (0 = ordinary targets)
  int nslice;              // blocks per work item, each over its share of the neighbour cells
  size_t sstride;          // elements between the slices' partial outputs
  double scale;            // output factor
  unsigned long long* work;  // pair counter (null: not counted)
  const int* order;        // targets of each cell in the order items take them (null: sorted)
};

// Work item: up to 64 sorted targets of one cell (one per lane).  Its
// neighbour cells are split into nslice consecutive runs, one block per
// (item, run), each writing its own partial sums (added in run order by the
// consumer), so a crowded neighbourhood is shared by several blocks and the
// dispatcher balances the load.  Within a block the run's source batches
// (64 sources of one cell) are numbered in cell order and batch u goes to
// wave u mod W; each wave stages its batches through its own LDS slice, and
// the W partial sums are added in wave order at the end.
//
// A wave stages only the batch's sources within r_c of the bounding box of
// the item's targets.  FAST (mixed precision, >= 3 cells per periodic
// direction): the sources are staged shifted into the target cell's periodic
// image, and every lane evaluates every staged source without branches: the
// displacement is formed in FP64 and rounded per component, the cutoff is
// decided on the FP32 square, and pairs outside alpha r >= 1e-2, r <= r_c get
// zero coefficients (closer pairs are evaluated in FP64 after the batch).
// Otherwise pass 1 keeps a bit mask of the pairs within r_c, decided on the
// FP64 minimum-image displacement, and pass 2 evaluates the kernel for those
// only.
//
// CNT (FAST only): count the in-range pairs into a.work; the exact path
// counts per batch whenever a.work is set.
//
// item: the work item (after the XCD order); slice: the run of neighbour cells.
template <typename T, bool DL, bool FAST, int W, bool CNT>
__device__ __forceinline__ void near_body(const NearArgs& a, const Kc<T>& k, const KcF& kf, int item,
                                          int slice) {
  // staged sources: FP64 position (x, y, z, unused) and strength (x, y, z,
  // unused), one vector read each
  __shared__ double4 lp[W][64];
  __shared__ typename Vec4<T>::t lf[W][64];
  __shared__ T part[W][3][64];
  const CellGeom& g = a.g;
  const int nitems = a.item_start[g.ncells];
  if (item >= nitems) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = a.item_cell[item];
  const int t0 = a.tcell[c] + (item - a.item_start[c]) * 64;
  const int t1 = min(a.tcell[c + 1], t0 + 64);
  const bool active = t0 + lane < t1;
  // the lane's target (sorted index): items take a cell's targets in the
  // cell's Morton order when one is given, so that they are compact
  const int t = active && a.order ? a.order[t0 + lane] : t0 + lane;
  const int iz = c % g.ncz;
  const int ix = (c / g.ncz) % g.ncx;
  const int iy = c / (g.ncz * g.ncx);
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
  const float rc2f = (float)a.rc2;
  const double alpha = kf.alpha;
  const float near2f = (float)(kNear2 / (alpha * alpha));
  const double near2 = kNear2 / (alpha * alpha);
  // bounding box of the item's targets (they share one cell, so no wrap)
  double bx0 = active ? px : 1e300, bx1 = active ? px : -1e300;
  double by0 = active ? py : 1e300, by1 = active ? py : -1e300;
  double bz0 = active ? pz : 1e300, bz1 = active ? pz : -1e300;
  for (int o = 32; o > 0; o >>= 1) {
    bx0 = fmin(bx0, __shfl_xor(bx0, o));
    bx1 = fmax(bx1, __shfl_xor(bx1, o));
    by0 = fmin(by0, __shfl_xor(by0, o));
    by1 = fmax(by1, __shfl_xor(by1, o));
    bz0 = fmin(bz0, __shfl_xor(bz0, o));
    bz1 = fmax(bz1, __shfl_xor(bz1, o));
  }
  const double bcx = 0.5 * (bx0 + bx1), bhx = 0.5 * (bx1 - bx0);
  const double bcz = 0.5 * (bz0 + bz1), bhz = 0.5 * (bz1 - bz0);
  const double keep_r2 = a.rc2 * (1.0 + 1e-6);
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const T* sf = (const T*)a.sf;
  T ux = 0, uy = 0, uz = 0;
  T sfx = 0, sfy = 0, sfz = 0;  // self contributions
  float sn = 0.0f;              // FAST double layer: sum of B (q.d), times n at the end
  unsigned npairs = 0;          // exact path: per lane
  unsigned long long npairs_w = 0;  // FAST: per wave
  const unsigned long long amask = __ballot(active);
  const int nxo = g.ncx >= 3 ? 3 : g.ncx, nzo = g.ncz >= 3 ? 3 : g.ncz;
  // wall targets only see the wall cell layer (cells are at least r_c high)
  const int oy0 = a.nplane ? 1 : 0, noy = a.nplane ? 1 : 3;
  const int ncand = noy * nxo * nzo;
  const int kc0 = slice * ncand / a.nslice, nk = (slice + 1) * ncand / a.nslice - kc0;
  // lane l < nk describes neighbour cell kc0 + l: source range, periodic
  // shift and number of batches
  int cs0 = 0, cs1 = 0, nbat = 0;
  double cshx = 0.0, cshz = 0.0;
  if (lane < nk) {
    const int kc = kc0 + lane;
    const int oyi = kc / (nxo * nzo) + oy0 - 1;
    const int oxi = (kc / nzo) % nxo, ozi = kc % nzo;
    const int cy = iy + oyi;
    if (cy >= 0 && cy < g.ncy) {
      int cx, cz;
      if (g.ncx >= 3) {
        const int u = ix + oxi - 1;
        cx = u < 0 ? u + g.ncx : (u >= g.ncx ? u - g.ncx : u);
        cshx = u < 0 ? -g.Lx : (u >= g.ncx ? g.Lx : 0.0);
      } else {
        cx = oxi;
      }
      if (g.ncz >= 3) {
        const int u = iz + ozi - 1;
        cz = u < 0 ? u + g.ncz : (u >= g.ncz ? u - g.ncz : u);
        cshz = u < 0 ? -g.Lz : (u >= g.ncz ? g.Lz : 0.0);
      } else {
        cz = ozi;
      }
      const int nc = (cy * g.ncx + cx) * g.ncz + cz;
      cs0 = a.scell[nc];
      cs1 = a.scell[nc + 1];
      nbat = (cs1 - cs0 + 63) >> 6;
    }
  }
  int bend = nbat;  // inclusive prefix of the batch counts over the cells
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(bend, o);
    if (lane >= o) bend += v;
  }
  const int nunits = __shfl(bend, 63);
  int cc = 0;  // the cell of the wave's current batch (advances monotonically)
  for (int u = wave; u < nunits; u += W) {
    while (u >= __shfl(bend, cc)) ++cc;
    const int first = __shfl(bend, cc) - __shfl(nbat, cc);
    const int s1 = __shfl(cs1, cc);
    const double shx = __shfl(cshx, cc), shz = __shfl(cshz, cc);
    {
      const int b = __shfl(cs0, cc) + (u - first) * 64;
      // the batch's sources within r_c of the targets' box, compacted in order
      // (the others are out of range of every target of the item)
      const int si = b + lane;
      bool keep = false;
      double qx = 0, qy = 0, qz = 0;
      if (si < s1) {
        qx = a.sx[si];
        qy = a.sy[si];
        qz = a.sz[si];
        if (FAST) {
          qx += shx;
          qz += shz;
        }
        double gx = fabs(FAST ? qx - bcx : min_image(qx - bcx, g.Lx, g.invLx)) - bhx;
        double gz = fabs(FAST ? qz - bcz : min_image(qz - bcz, g.Lz, g.invLz)) - bhz;
        const double gy = qy < by0 ? by0 - qy : (qy > by1 ? qy - by1 : 0.0);
        gx = gx > 0.0 ? gx : 0.0;
        gz = gz > 0.0 ? gz : 0.0;
        keep = dist2(gx, gy, gz) <= keep_r2;
      }
      const unsigned long long km = __ballot(keep);
      const int cnt = __popcll(km);
      if (cnt == 0) continue;
      const int cnt2 = (cnt + 1) & ~1;
      __builtin_amdgcn_wave_barrier();
      if (FAST && lane >= cnt && lane < cnt2) {
        // padding to a multiple of two: a far-away point of zero strength
        lp[wave][lane] = make_double4(1e30, 1e30, 1e30, 0.0);
        typename Vec4<T>::t z;
        z.x = z.y = z.z = z.w = (T)0;
        lf[wave][lane] = z;
      }
      if (keep) {
        const int slot = __popcll(km & lt);
        lp[wave][slot] = make_double4(qx, qy, qz, 0.0);
        typename Vec4<T>::t fv;
        fv.x = sf[si];
        fv.y = sf[a.scap + si];
        fv.z = sf[2 * a.scap + si];
        fv.w = (T)0;
        lf[wave][slot] = fv;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if constexpr (FAST) {
        // every lane takes every staged source, two per LDS round trip, in
        // staged (sorted) order; pairs outside 0 < r <= r_c add exact zeros.
        // The displacement is formed in FP64 and rounded per component;
        // separations with alpha r < 1e-2 are left to the FP64 pass after the loop.
        unsigned long long tiny_w = 0;
        for (int j0 = 0; j0 < cnt2; j0 += 2) {
          double4 qg[2];
          float4 fg[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            qg[u] = lp[wave][j0 + u];
            fg[u] = lf[wave][j0 + u];
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const float dx = (float)(px - qg[u].x), dy = (float)(py - qg[u].y),
                        dz = (float)(pz - qg[u].z);
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const bool ge = r2 >= near2f;
            const bool ok = ge && r2 <= rc2f;
            // lane masks stay scalar: every lane runs this loop
            tiny_w |= ~__builtin_amdgcn_ballot_w64(ge);
            if (CNT) npairs_w += __popcll(__builtin_amdgcn_ballot_w64(ok) & amask);
            if (DL)
              stresslet_masked(dx, dy, dz, r2, ok, fg[u].x, fg[u].y, fg[u].z, nx, ny, nz, kf, ux,
                               uy, uz, sn);
            else
              stokeslet_masked(dx, dy, dz, r2, ok, fg[u].x, fg[u].y, fg[u].z, kf, ux, uy, uz);
          }
        }
        if (tiny_w & amask) {
          for (int j = 0; j < cnt; ++j) {
            const double4 qp = lp[wave][j];
            const double ddx = px - qp.x, ddy = py - qp.y, ddz = pz - qp.z;
            const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (active && r2 < near2f)
              near_pair_fp64<T, DL>(ddx, ddy, ddz, lf[wave][j], nx, ny, nz, alpha, ux, uy, uz, sfx,
                                    sfy, sfz);
          }
        }
      } else {
        // exact path: the lane's in-range sources as a bit mask, decided on
        // the FP64 minimum-image displacement, then kernel evaluations for
        // those only, in source order
        unsigned long long mask = 0;
        if (active) {
          for (int j = 0; j < cnt; ++j) {
            const double4 q = lp[wave][j];
            const double dx = min_image(px - q.x, g.Lx, g.invLx);
            const double dy = py - q.y;
            const double dz = min_image(pz - q.z, g.Lz, g.invLz);
            const double r2 = dist2(dx, dy, dz);
            if (r2 <= a.rc2) {
              if (sizeof(T) == 4 && r2 < near2) {
                near_pair_fp64<T, DL>(dx, dy, dz, lf[wave][j], nx, ny, nz, alpha, ux, uy, uz, sfx,
                                      sfy, sfz);
              } else if (r2 != 0.0) {
                mask |= 1ull << j;
              } else if (!DL) {
                sfx += lf[wave][j].x;
                sfy += lf[wave][j].y;
                sfz += lf[wave][j].z;
              }
            }
          }
        }
        npairs += __popcll(mask);
        while (mask) {
          const int j = __builtin_ctzll(mask);
          mask &= mask - 1;
          const double4 q = lp[wave][j];
          const double dx = min_image(px - q.x, g.Lx, g.invLx);
          const double dy = py - q.y;
          const double dz = min_image(pz - q.z, g.Lz, g.invLz);
          const typename Vec4<T>::t fv = lf[wave][j];
          // the displacement is formed in FP64; in FP32 its square is taken
          // from the rounded components
          const T tdx = (T)dx, tdy = (T)dy, tdz = (T)dz;
          const T r2 = sizeof(T) == 4 ? tdx * tdx + tdy * tdy + tdz * tdz : (T)dist2(dx, dy, dz);
          if (DL)
            stresslet_acc<T>(tdx, tdy, tdz, r2, fv.x, fv.y, fv.z, nx, ny, nz, k, ux, uy, uz);
          else
            stokeslet_acc<T>(tdx, tdy, tdz, r2, fv.x, fv.y, fv.z, k, ux, uy, uz);
        }
      }
    }
  }
  if (FAST && DL) {
    ux = fmaf(sn, nx, ux);
    uy = fmaf(sn, ny, uy);
    uz = fmaf(sn, nz, uz);
  }
  if (CNT && FAST && lane == 0 && npairs_w) atomicAdd(a.work, npairs_w);
  if (!FAST && a.work) wave_count_add(a.work, npairs);
  part[wave][0][lane] = ux + k.selfc * sfx;
  part[wave][1][lane] = uy + k.selfc * sfy;
  part[wave][2][lane] = uz + k.selfc * sfz;
  __syncthreads();
  if (wave == 0 && active) {
    T v[3];
    for (int d = 0; d < 3; ++d) {
      T acc = part[0][d][lane];
      for (int w = 1; w < W; ++w) acc += part[w][d][lane];
      v[d] = (T)a.scale * acc;
    }
    T* out = (T*)a.out + (size_t)slice * a.sstride;
    size_t o = (size_t)t;
    if (a.nplane) {
      const int r = a.tperm[t];
      const int wall = r / a.nplane;
      o = (size_t)wall * 3 * a.nplane + (r - wall * a.nplane);
    }
    out[o] = v[0];
    out[a.ostride + o] = v[1];
    out[2 * a.ostride + o] = v[2];
  }
}

// XCD-aware: block b runs on XCD b % 8; each XCD takes chunks of 16
// consecutive work items in turn (when the grid is a multiple of 128)
__device__ inline int xcd_item(int b, int nb) {
  if ((nb & 127) != 0) return b;
  const int q = b >> 3;
  return (q >> 4) * 128 + (b & 7) * 16 + (q & 15);
}

template <typename T, bool DL, bool FAST, int W, bool CNT>
__global__ void __launch_bounds__(64 * W) near_field(NearArgs a, Kc<T> k, KcF kf) {
  near_body<T, DL, FAST, W, CNT>(a, k, kf, xcd_item(blockIdx.x, gridDim.x), blockIdx.y);
}

// Many target sets in one launch: job j owns blocks [boff[j], boff[j + 1])
// in x (a multiple of 128 each, so that every job's items are dealt to the
// XCDs as in its own launch) and the slices in y.  A block finds its job by
// bisection and does exactly the work of the same block of the job's own
// launch.
template <typename T>
struct NearJob {
  NearArgs a;
  Kc<T> k;
  KcF kf;
};

template <typename T, bool FAST, int W>
__global__ void __launch_bounds__(64 * W) near_field_jobs(const NearJob<T>* __restrict__ jobs,
                                                          const int* __restrict__ boff, int njobs) {
  const int b = blockIdx.x;
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid;
  }
  const NearJob<T>& j = jobs[lo];
  const int t = b - boff[lo];
  near_body<T, false, FAST, W, false>(j.a, j.k, j.kf, xcd_item(t, boff[lo + 1] - boff[lo]),
                                      blockIdx.y);
}

template <typename T, bool DL, int W>
static void launch_near_w(Plan& p, const NearArgs& a, unsigned grid) {
  const bool fast = sizeof(T) == 4 && p.cg.ncx >= 3 && p.cg.ncz >= 3;
  const dim3 g(grid, (unsigned)a.nslice);
  const KcF kf = make_kcf(p.p.alpha);
  if constexpr (sizeof(T) == 4) {
    if (fast) {
      if (a.work)
        near_field<T, DL, true, W, true><<<g, 64 * W, 0, p.stream>>>(a, make_kc<T>(p.p.alpha), kf);
      else
        near_field<T, DL, true, W, false><<<g, 64 * W, 0, p.stream>>>(a, make_kc<T>(p.p.alpha), kf);
      return;
    }
  }
  near_field<T, DL, false, W, false><<<g, 64 * W, 0, p.stream>>>(a, make_kc<T>(p.p.alpha), kf);
}

// grid = an upper bound of the work items (targets/64 + cells)
template <typename T, bool DL>
static void launch_near_kernel(Plan& p, const NearArgs& a, unsigned grid) {
  launch_near_w<T, DL, 4>(p, a, grid);
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

static NearArgs near_args(Plan& p, const Binned& tg, void* out, size_t ostride) {
  NearArgs a;
  a.g = p.cg;
  a.rc2 = p.rc2;
  a.item_start = tg.item_start;
  a.item_cell = tg.item_cell;
  a.tcell = tg.cell_start;
  a.tx = tg.x;
  a.ty = tg.y;
  a.tz = tg.z;
  a.tn = tg.s;
  a.tcap = ostride;
  a.scell = p.src.cell_start;
  a.sx = p.src.x;
  a.sy = p.src.y;
  a.sz = p.src.z;
  a.sf = p.src.s;
  a.scap = (size_t)p.p.max_src;
  a.out = out;
  a.ostride = ostride;
  a.tperm = tg.perm;
  a.nplane = 0;
  a.nslice = kNearSlices;
  a.sstride = 3 * ostride;
  a.scale = 0.039788735772973833942;  // 1/(8 pi)
  a.work = nullptr;
  a.order = nullptr;
  return a;
}

static unsigned near_grid(Plan& p, int nt) {
  const unsigned n = (unsigned)((nt + 63) / 64 + p.cg.ncells);
  return (n + 127) & ~127u;
}

// Order of the targets inside each cell for the near-field work items: by
// the Morton code of their position on an 8 x 8 x 8 lattice over the cell
// (bits of x, y and z interleaved), stable, so that 64 consecutive targets
// are close together and their bounding box admits fewer candidate sources.
// One wave per cell: a histogram of the 512 codes, its exclusive scan, then
// a scatter in input order with equal codes ranked by wave ballots.
__global__ void __launch_bounds__(64) near_order(CellGeom g, const int* __restrict__ tcell,
                                                 const double* __restrict__ tx,
                                                 const double* __restrict__ ty,
                                                 const double* __restrict__ tz,
                                                 int* __restrict__ order) {
  __shared__ int hist[512];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int s0 = tcell[c], s1 = tcell[c + 1], n = s1 - s0;
  if (n <= 0) return;
  if (n <= 64) {  // one work item: any order
    if (lane < n) order[s0 + lane] = s0 + lane;
    return;
  }
  const int iz = c % g.ncz, ix = (c / g.ncz) % g.ncx, iy = c / (g.ncz * g.ncx);
  auto code = [&](int i) {
    const int a = min(7, max(0, (int)((tx[i] * g.icx - ix) * 8.0)));
    const int b = min(7, max(0, (int)(((ty[i] + g.H) * g.icy - iy) * 8.0)));
    const int d = min(7, max(0, (int)((tz[i] * g.icz - iz) * 8.0)));
    int m = 0;
    for (int k = 0; k < 3; ++k)
      m |= (((a >> k) & 1) << (3 * k)) | (((b >> k) & 1) << (3 * k + 1)) | (((d >> k) & 1) << (3 * k + 2));
    return m;
  };
  for (int k = lane; k < 512; k += 64) hist[k] = 0;
  __syncthreads();
  for (int i = s0 + lane; i < s1; i += 64) atomicAdd(&hist[code(i)], 1);
  __syncthreads();
  if (lane == 0) {
    int run = 0;
    for (int k = 0; k < 512; ++k) {
      const int v = hist[k];
      hist[k] = run;
      run += v;
    }
  }
  __syncthreads();
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int base = s0; base < s1; base += 64) {
    const int i = base + lane;
    const bool valid = i < s1;
    const int key = valid ? code(i) : 0;
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < 9; ++b) {
      const bool bit = (key >> b) & 1;
      const unsigned long long bm = __ballot(bit);
      m &= bit ? bm : ~bm;
    }
    const int rank = __popcll(m & lt);
    const int before = valid ? hist[key] : 0;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) hist[key] = before + __popcll(m);
    __builtin_amdgcn_wave_barrier();
    if (valid) order[s0 + before + rank] = i;
  }
}

static const int* launch_near_order(Plan& p, const Binned& tg) {
  near_order<<<(unsigned)p.cg.ncells, 64, 0, p.stream>>>(p.cg, tg.cell_start, tg.x, tg.y, tg.z,
                                                        p.norder);
  return p.norder;
}

template <typename T>
hipError_t launch_near_sl(Plan& p, int nt) {
  if (nt <= 0) return hipSuccess;
  NearArgs a = near_args(p, *p.tview, p.ul, (size_t)p.p.max_tgt);
  a.tcap = (size_t)p.p.max_tgt;
  a.work = p.count_work ? p.work : nullptr;
  a.order = launch_near_order(p, *p.tview);
  launch_near_kernel<T, false>(p, a, near_grid(p, nt));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_near_dl(Plan& p, int nt) {
  if (nt <= 0) return hipSuccess;
  NearArgs a = near_args(p, *p.tview, p.ul, (size_t)p.p.max_tgt);
  a.tn = p.tnrm;
  a.tcap = (size_t)p.p.max_tgt;
  a.work = p.count_work ? p.work : nullptr;
  a.order = launch_near_order(p, *p.tview);
  launch_near_kernel<T, true>(p, a, near_grid(p, nt));
  return hipGetLastError();
}

// Wall data of the global problem: u^g = -u^l at the wall nodes (Sec. 3.2.2),
// the local sum evaluated at the nodes of y = -H and y = +H (a target set
// binned once per plan), written as -u^l/(Nx Nz) into [wall][component][x][z]:
// the wall planes are transformed in x, z only, while the grid fields get the
// 1/(Nx Nz) of the forward DFT through the Chebyshev forward matrix.
template <typename T>
__global__ void __launch_bounds__(256) sum_slices(const T* __restrict__ part, T* __restrict__ out,
                                                  size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  T v = part[i];
  for (int s = 1; s < kWallSlices; ++s) v += part[(size_t)s * n + i];
  out[i] = v;
}

static NearArgs wall_args(Plan& p) {
  const int nplane = p.p.Nx * p.p.Nz;
  NearArgs a = near_args(p, p.wall, p.wall_part, (size_t)nplane);
  a.nplane = nplane;
  a.nslice = kWallSlices;
  a.sstride = 6 * (size_t)nplane;
  a.scale = -0.039788735772973833942 / ((double)p.p.Nx * (double)p.p.Nz);
  return a;
}

// the wall slices' partial sums added in slice order
template <typename T>
hipError_t launch_wall_sum(Plan& p) {
  const size_t n = 6 * (size_t)p.p.Nx * p.p.Nz;
  sum_slices<T><<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>((const T*)p.wall_part,
                                                                   (T*)p.wall_phys, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wall(Plan& p) {
  launch_near_kernel<T, false>(p, wall_args(p), near_grid(p, 2 * p.p.Nx * p.p.Nz));
  return launch_wall_sum<T>(p);
}

// Job lists of the single-layer local sums of many plans in one launch: at
// the plans' sources as targets (after their binning and target order of
// the current call), or at their wall nodes.
bool near_job_fast(const Plan& p) { return !p.fp64 && p.cg.ncx >= 3 && p.cg.ncz >= 3; }

size_t near_job_bytes(bool fp64) {
  return fp64 ? sizeof(NearJob<double>) : sizeof(NearJob<float>);
}

int near_job_blocks(const Plan& p, bool wall) {
  return (int)near_grid(const_cast<Plan&>(p), wall ? 2 * p.p.Nx * p.p.Nz : (int)p.p.max_tgt);
}

template <typename T>
static int near_jobs_upload_t(Plan* const* plans, int n, bool wall, void* dev_jobs, int* dev_boff) {
  std::vector<NearJob<T>> j(n);
  std::vector<int> off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    Plan& p = *plans[i];
    if (wall) {
      j[i].a = wall_args(p);
    } else {
      j[i].a = near_args(p, p.src, p.ul, (size_t)p.p.max_tgt);
      j[i].a.tcap = (size_t)p.p.max_tgt;
      j[i].a.order = p.norder;
    }
    j[i].k = make_kc<T>(p.p.alpha);
    j[i].kf = make_kcf(p.p.alpha);
    off[i + 1] = off[i] + near_job_blocks(p, wall);
  }
  if (n > 0 && (hipMemcpy(dev_jobs, j.data(), n * sizeof(NearJob<T>), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dev_boff, off.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess))
    return -1;
  return off[n];
}

int near_jobs_upload(Plan* const* plans, int n, bool wall, void* dev_jobs, int* dev_boff) {
  if (n <= 0) return 0;
  return plans[0]->fp64 ? near_jobs_upload_t<double>(plans, n, wall, dev_jobs, dev_boff)
                        : near_jobs_upload_t<float>(plans, n, wall, dev_jobs, dev_boff);
}

hipError_t launch_near_jobs(hipStream_t s, bool fp64, bool fast, bool wall, const void* dev_jobs,
                            const int* dev_boff, int n, int nblocks) {
  if (n <= 0 || nblocks <= 0) return hipSuccess;
  const dim3 g((unsigned)nblocks, (unsigned)(wall ? kWallSlices : kNearSlices));
  if (fp64)
    near_field_jobs<double, false, 4><<<g, 256, 0, s>>>((const NearJob<double>*)dev_jobs, dev_boff, n);
  else if (fast)
    near_field_jobs<float, true, 4><<<g, 256, 0, s>>>((const NearJob<float>*)dev_jobs, dev_boff, n);
  else
    near_field_jobs<float, false, 4><<<g, 256, 0, s>>>((const NearJob<float>*)dev_jobs, dev_boff, n);
  return hipGetLastError();
}

const int* launch_near_order_sources(Plan& p) { return launch_near_order(p, p.src); }

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
template hipError_t launch_wall_sum<double>(Plan&);
template hipError_t launch_wall_sum<float>(Plan&);

}  // namespace ggem
