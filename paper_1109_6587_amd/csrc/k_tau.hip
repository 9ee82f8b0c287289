// Global Stokes problem per Fourier mode (Appendix C), always in FP64.
//
// For mode (k_x, k_z), lam = k_x^2 + k_z^2, with F the Chebyshev
// coefficients of the global force density (momentum: -grad p + lap u + F = 0)
// and g-, g+ the wall velocities (u^g = -u^l at y = -H, +H), the influence
// matrix method solves
//   (a) p_a'' - lam p_a = i k_x F_x + F_y' + i k_z F_z,  p_a(+-H) = 0,
//       u_a'' - lam u_a = i k_x p_a - F_x, u_a(+-H) = g_x+-  (v_a: p_a' - F_y,
//       w_a: i k_z p_a - F_z),
//   (b), (c) the same with no forcing, no-slip, and p = 1 at y = -H resp. +H,
// and superposes u = u_a + p1 u_b + p2 u_c (Eq. cheb_sol) with p1, p2 chosen
// so that the velocity is divergence-free at both walls (Eq. inf_mat).
// (b) and (c) depend only on lam and are solved once per plan; (c) is the
// mirror image of (b) (coefficients times (-1)^n, v also changes sign).  u_b
// and w_b are i k_x and i k_z times one real profile; u and w meet their wall
// values exactly, so the wall divergence needs only v'.
//
// Each Helmholtz problem is the tau system: rows 0..N-2 of
// (D^2/H^2 - lam) a = r plus the two wall rows.  The Chebyshev recurrence
// that expresses a_n (n >= 2) through the coefficients of a'' splits it into
// two independent tridiagonal systems (even and odd n), each bordered by one
// full row (the wall value of that parity).  Writing a_n = P_n + Q_n a_{0|1},
// a backward sweep gives P and the full row gives a_{0|1}; the lam-only
// factors (1/pivot, multiplier, Q and its sum) are computed once per plan.
//
// Kernels of one evaluation:
//   A  one thread per (mode, parity): p_a
//   B  one thread per (mode, parity, component): u_a, v_a, w_a and the
//      parity's share of the wall slopes of v_a
//   D  one thread per (mode, n): p1, p2, superposition, output (and, for the
//      double layer, the stress components that need no y-derivative)
//   E  double layer: one thread per (mode, component) for the stress
//      components with a y-derivative.
// Vectors are stored [n][mode] so a wave's accesses are coalesced.  With few
// modes per compute unit each thread's chain of dependent steps is the time,
// so for Chebyshev order N <= 64 (N <= 128 with FP32 inputs) A, B and E keep
// a parity's column in registers, recompute the sweep factors inline and
// issue their loads ahead of the sweeps; larger orders use the LDS-column
// kernels with the plan-time factor tables.
#include "ggem_internal.h"

namespace ggem {

__device__ inline double2 z2(double a, double b) { return make_double2(a, b); }
__device__ inline double2 zadd(double2 a, double2 b) { return z2(a.x + b.x, a.y + b.y); }
__device__ inline double2 zsub(double2 a, double2 b) { return z2(a.x - b.x, a.y - b.y); }
__device__ inline double2 zscale(double s, double2 a) { return z2(s * a.x, s * a.y); }
__device__ inline double2 zfma(double s, double2 a, double2 b) {
  return z2(fma(s, a.x, b.x), fma(s, a.y, b.y));
}
__device__ inline double2 zi(double k, double2 a) { return z2(-k * a.y, k * a.x); }  // i k a

struct TauArgs {
  int N, Nx, Nz, Nzh, nmodes;
  double H, Lx, Lz;
  const double* nconst;  // per n: 1/(4n(n-1)), 1/(2(n^2-1)), 1/(4n(n+1))  [3][Ny]
  double* pre;           // per mode: [1/pivot, multiplier, Q][Ny], sum Q [2], [p_b, u_b, v_b][Ny]
  double* infl;          // per mode: 2x2 inverse influence matrix (4 doubles)
  const void* in;        // [3][Ny][nmodes] complex T
  const void* wall;      // [2][3][nmodes] complex T
  void* out;             // [3|6][Ny][nmodes] complex T
  double2* scr;          // [8][Ny][nmodes] complex + wall slopes [2][2][nmodes]
  const double* gauge;
};

// scratch slots
enum { kPA = 0, kUA = 1, kVA = 2, kWA = 3, kU = 4, kV = 5, kW = 6, kP = 7, kSlope = 8 };

template <typename T>
struct CT;
template <>
struct CT<double> {
  using t = double2;
};
template <>
struct CT<float> {
  using t = float2;
};
template <typename C>
__device__ inline double2 to_z(C v) {
  return z2((double)v.x, (double)v.y);
}
template <typename T>
__device__ inline typename CT<T>::t from_z(double2 v) {
  typename CT<T>::t r;
  r.x = (T)v.x;
  r.y = (T)v.y;
  return r;
}

struct Mode {
  int q, l, m;
  double kx, kz, lam;
  bool nyquist;
};

__device__ inline Mode mode_of(const TauArgs& a, int q) {
  Mode md;
  md.q = q;
  md.l = q / a.Nzh;
  md.m = q - md.l * a.Nzh;
  const int ls = md.l < a.Nx / 2 ? md.l : md.l - a.Nx;
  md.kx = 6.283185307179586477 * ls / a.Lx;
  md.kz = 6.283185307179586477 * md.m / a.Lz;
  md.lam = md.kx * md.kx + md.kz * md.kz;
  md.nyquist = md.l == a.Nx / 2 || md.m == a.Nz / 2;
  return md;
}

struct Sweep {
  int N;
  double h2, h2l;
  const double* nc;
  const double* pre;  // this mode's factor column (stride S)
  size_t S, NyS;
};

__device__ inline Sweep make_sweep(const TauArgs& a, int q, double lam) {
  Sweep w;
  w.N = a.N;
  w.h2 = a.H * a.H;
  w.h2l = w.h2 * lam;
  w.nc = a.nconst;
  w.S = (size_t)a.nmodes;
  w.NyS = (size_t)(a.N + 1) * w.S;
  w.pre = a.pre + q;
  return w;
}

// Tau Helmholtz solve restricted to the coefficients n = par, par+2, ...:
// on entry lds[i] (stride 64) holds r(par + 2i) for par + 2i <= N-2; g is the
// parity's share of the wall values ((g+ + g-)/2 even, (g+ - g-)/2 odd);
// dst(n, a_n) receives the solution.
template <class DST>
__device__ inline void hel_par(const Sweep& w, int par, double2* lds, double2 g, DST dst) {
  const int N = w.N;
  const int M = (N - par) / 2;
  const int Nc = N + 1;
  // row right-hand sides s_i = h2 (c_{n-2} q1 r_{n-2} - q2 r_n + q3 r_{n+2}), in place
  double2 rprev = lds[0];
#pragma unroll 8
  for (int i = 1; i <= M; ++i) {
    const int n = par + 2 * i;
    const double2 ri = (n <= N - 2) ? lds[i * 64] : z2(0, 0);
    const double2 rn = (n + 2 <= N - 2) ? lds[(i + 1) * 64] : z2(0, 0);
    double2 s = zscale((n == 2 ? 2.0 : 1.0) * w.nc[n], rprev);
    s = zfma(-w.nc[Nc + n], ri, s);
    s = zfma(w.nc[2 * Nc + n], rn, s);
    lds[i * 64] = zscale(w.h2, s);
    rprev = ri;
  }
  // backward: alpha_i = (s_i - u_i alpha_{i+1}) / pivot_i
  double2 an = z2(0, 0);
#pragma unroll 8
  for (int i = M; i >= 1; --i) {
    const int n = par + 2 * i;
    const double u = (n + 2 <= N - 2) ? -w.h2l * w.nc[2 * Nc + n] : 0.0;
    an = zscale(w.pre[(size_t)n * w.S], zfma(-u, an, lds[i * 64]));
    lds[i * 64] = an;
  }
  // forward: P_i = alpha_i + beta_i P_{i-1}
  double2 P = z2(0, 0), SP = z2(0, 0);
#pragma unroll 8
  for (int i = 1; i <= M; ++i) {
    const int n = par + 2 * i;
    P = zfma(w.pre[w.NyS + (size_t)n * w.S], P, lds[i * 64]);
    lds[i * 64] = P;
    SP = zadd(SP, P);
  }
  const double2 x0 = zscale(1.0 / w.pre[3 * w.NyS + par * w.S], zsub(g, SP));
  dst(par, x0);
#pragma unroll 8
  for (int i = 1; i <= M; ++i) {
    const int n = par + 2 * i;
    dst(n, zfma(w.pre[2 * w.NyS + (size_t)n * w.S], x0, lds[i * 64]));
  }
}

// Fill lds[i] = rhs(m, D_m) for m = par + 2i <= N-2, descending, where D_m is
// the y-derivative coefficient (d/dybar) of the vector `a` at index m:
// c_m D_m = 2 sum_{p > m, p + m odd} p a_p.
template <class SRC, class RHS>
__device__ inline void fill_rhs_deriv(int N, int par, double2* lds, SRC a, RHS rhs) {
  int mt = N - 2;
  if ((mt & 1) != par) --mt;
  double2 S = z2(0, 0);
  // contributions of p > mt + 1 of the opposite parity
  for (int p = N - ((N & 1) == par ? 1 : 0); p > mt + 1; p -= 2) S = zfma((double)p, a(p), S);
#pragma unroll 8
  for (int m = mt; m >= par; m -= 2) {
    S = zfma((double)(m + 1), a(m + 1), S);
    const double2 D = zscale(m == 0 ? 1.0 : 2.0, S);
    lds[((m - par) / 2) * 64] = rhs(m, D);
  }
}

template <class RHS>
__device__ inline void fill_rhs(int N, int par, double2* lds, RHS rhs) {
#pragma unroll 8
  for (int m = par; m <= N - 2; m += 2) lds[((m - par) / 2) * 64] = rhs(m);
}

// ---- register-resident sweeps for N <= MAXN -------------------------------
// The same solves with the parity's column held in registers.  Every loop is
// unrolled over the compile-time bound MAXN/2 with the parity a template
// argument, so each row's Chebyshev constants are literals; the sweep
// factors (1/pivot, multiplier, Q and its sum, as in sweep_factors) are
// recomputed in the sweep rather than loaded, and the only global loads left
// are the right-hand-side reads, which carry no control dependence (indices
// beyond N are clamped and their terms masked) and so issue in bulk.
// A wave-uniform int copied into a vector register.  Clamps and masks on the
// Chebyshev order then use per-lane compares; on the scalar unit they would
// all share the one condition bit, whose def-use chain pins every unrolled
// iteration's address arithmetic, and with it its loads, behind the previous
// iteration.
__device__ __forceinline__ int lane_copy(int s) {
  int v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

__device__ constexpr double cheb_c1(int n) { return 1.0 / (4.0 * n * (n - 1)); }
__device__ constexpr double cheb_c2(int n) { return 1.0 / (2.0 * ((double)n * n - 1.0)); }
__device__ constexpr double cheb_c3(int n) { return 1.0 / (4.0 * n * (n + 1)); }

// r[i] holds r(PAR + 2i) for PAR + 2i <= N-2 and zero elsewhere (r[MAXN/2]
// is always zero); dst(n, a_n) receives the solution for n <= N.
template <int MAXN, int PAR, class DST>
__device__ __forceinline__ void hel_reg(int N, double h2, double lam, const double2 (&r)[MAXN / 2 + 1],
                                        double2 g, DST dst) {
  constexpr int MM = MAXN / 2;
  const int M = (N - PAR) / 2;
  const double h2l = h2 * lam;
  // row right-hand sides s_i; zero for i > M since r vanishes there
  double2 s[MM + 1];
#pragma unroll
  for (int i = 1; i <= MM; ++i) {
    const int n = PAR + 2 * i;
    const double2 rn = i < MM ? r[i + 1] : z2(0, 0);
    double2 t = zscale((n == 2 ? 2.0 : 1.0) * cheb_c1(n), r[i - 1]);
    t = zfma(-cheb_c2(n), r[i], t);
    t = zfma(cheb_c3(n), rn, t);
    s[i] = zscale(h2, t);
  }
  // backward: pivots and multipliers b_i, alpha_i = (s_i - u_i alpha_{i+1}) / pivot_i
  double mq[MM + 1];
  double bn = 0.0;
  double2 an = z2(0, 0);
#pragma unroll
  for (int i = MM; i >= 1; --i) {
    const int n = PAR + 2 * i;
    mq[i] = 0.0;
    if (i <= M) {
      const double lo = -h2l * (n == 2 ? 2.0 : 1.0) * cheb_c1(n);
      const double d = 1.0 + ((n <= N - 2) ? h2l * cheb_c2(n) : 0.0);
      const double u = (n + 2 <= N - 2) ? -h2l * cheb_c3(n) : 0.0;
      const double iv = 1.0 / (d + u * bn);
      bn = -lo * iv;
      mq[i] = bn;
      an = zscale(iv, zfma(-u, an, s[i]));
      s[i] = an;
    }
  }
  // forward: P_i = alpha_i + b_i P_{i-1}, Q_i = b_i Q_{i-1}
  double2 P = z2(0, 0), SP = z2(0, 0);
  double Q = 1.0, sq = 1.0;
#pragma unroll
  for (int i = 1; i <= MM; ++i) {
    if (i <= M) {
      P = zfma(mq[i], P, s[i]);
      s[i] = P;
      SP = zadd(SP, P);
      Q *= mq[i];
      mq[i] = Q;
      sq += Q;
    }
  }
  const double2 x0 = zscale(1.0 / sq, zsub(g, SP));
  dst(PAR, x0);
#pragma unroll
  for (int i = 1; i <= MM; ++i)
    if (i <= M) dst(PAR + 2 * i, zfma(mq[i], x0, s[i]));
}

// r[i] = rhs(m, D_m) for rows m = PAR + 2i <= N-2, where D_m is the
// y-derivative coefficient of the vector `a` (c_m D_m = 2 sum over p > m,
// p + m odd, of p a_p); a(p) and rhs(m, .) are called with indices <= N.
template <int MAXN, int PAR, class SRC, class RHS>
__device__ __forceinline__ void fill_reg_deriv(int N, double2 (&r)[MAXN / 2 + 1], SRC a, RHS rhs) {
  constexpr int MM = MAXN / 2;
  double2 S = z2(0, 0);
#pragma unroll
  for (int i = MM - 1; i >= 0; --i) {
    const int m = PAR + 2 * i, p = m + 1;
    const double2 ap = a(p < N ? p : N);
    S = zfma(p <= N ? (double)p : 0.0, ap, S);
    const double2 v = rhs(m < N ? m : N, zscale(m == 0 ? 1.0 : 2.0, S));
    r[i] = m <= N - 2 ? v : z2(0, 0);
  }
  r[MM] = z2(0, 0);
}

template <int MAXN, int PAR, class RHS>
__device__ __forceinline__ void fill_reg(int N, double2 (&r)[MAXN / 2 + 1], RHS rhs) {
  constexpr int MM = MAXN / 2;
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    const int m = PAR + 2 * i;
    const double2 v = rhs(m < N ? m : N);
    r[i] = m <= N - 2 ? v : z2(0, 0);
  }
  r[MM] = z2(0, 0);
}

// ---- A: p_a, one thread per (mode, parity) ---------------------------------
template <typename T>
__global__ void __launch_bounds__(64) tau_pressure(TauArgs a) {
  using C = typename CT<T>::t;
  extern __shared__ double2 tau_lds[];
  const int q = blockIdx.x * 64 + threadIdx.x;
  const int par = blockIdx.y;
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  if (md.nyquist) return;
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const C* in = (const C*)a.in;
  auto F = [&](int c, int n) { return to_z(in[((size_t)c * Ny + n) * S + q]); };
  double2* PA = a.scr + (size_t)kPA * Ny * S + q;
  if (q == 0) {
    // k = 0: p' = F_y (rows 0..N-1) with p(-H) = gauge; integrate b = H F_y:
    // 2n p_n = c_{n-1} b_{n-1} - b_{n+1}.  Written by the even-parity thread.
    if (par) return;
    double2 s = z2(0, 0);
    for (int n = 1; n <= N; ++n) {
      const double2 bm = zscale(a.H * (n == 1 ? 2.0 : 1.0), F(1, n - 1));
      const double2 bp = (n + 1 <= N - 1) ? zscale(a.H, F(1, n + 1)) : z2(0, 0);
      const double2 pn = zscale(1.0 / (2.0 * n), zsub(bm, bp));
      PA[(size_t)n * S] = pn;
      s = (n & 1) ? zsub(s, pn) : zadd(s, pn);
    }
    PA[0] = zsub(z2(a.gauge[0], 0.0), s);
    return;
  }
  double2* lds = tau_lds + threadIdx.x;
  const double iH = 1.0 / a.H;
  fill_rhs_deriv(N, par, lds, [&](int p) { return F(1, p); }, [&](int m, double2 dfy) {
    return zadd(zadd(zi(md.kx, F(0, m)), zscale(iH, dfy)), zi(md.kz, F(2, m)));
  });
  hel_par(make_sweep(a, q, md.lam), par, lds, z2(0, 0),
          [&](int n, double2 v) { PA[(size_t)n * S] = v; });
}

// ---- B: u_a, v_a, w_a, one thread per (mode, parity, component) -----------
template <typename T>
__global__ void __launch_bounds__(64) tau_velocity(TauArgs a) {
  using C = typename CT<T>::t;
  extern __shared__ double2 tau_lds[];
  const int q = blockIdx.x * 64 + threadIdx.x;
  const int par = blockIdx.y, comp = blockIdx.z;
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  if (md.nyquist) return;
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const C* in = (const C*)a.in;
  const C* wall = (const C*)a.wall;
  auto F = [&](int c, int n) { return to_z(in[((size_t)c * Ny + n) * S + q]); };
  const double2* PA = a.scr + (size_t)kPA * Ny * S + q;
  double2* dst = a.scr + (size_t)(kUA + comp) * Ny * S + q;
  const double2 gm = to_z(wall[(size_t)comp * S + q]);
  const double2 gp = to_z(wall[(size_t)(3 + comp) * S + q]);
  const double2 g = par == 0 ? zscale(0.5, zadd(gp, gm)) : zscale(0.5, zsub(gp, gm));
  double2* lds = tau_lds + threadIdx.x;
  const double iH = 1.0 / a.H;
  const bool zero = q == 0;  // k = 0: no pressure coupling, v'' = 0
  if (comp == 1) {
    if (zero) fill_rhs(N, par, lds, [](int) { return z2(0, 0); });
    else
      fill_rhs_deriv(N, par, lds, [&](int p) { return PA[(size_t)p * S]; },
                     [&](int m, double2 dp) { return zsub(zscale(iH, dp), F(1, m)); });
    double2 dm = z2(0, 0), dpl = z2(0, 0);
    hel_par(make_sweep(a, q, md.lam), par, lds, g, [&](int n, double2 v) {
      dst[(size_t)n * S] = v;
      const double2 t = zscale((double)n * n, v);
      dpl = zadd(dpl, t);
      dm = (n & 1) ? zadd(dm, t) : zsub(dm, t);
    });
    double2* sl = a.scr + (size_t)kSlope * Ny * S + q;
    sl[(size_t)(2 * par) * S] = dm;
    sl[(size_t)(2 * par + 1) * S] = dpl;
  } else {
    const double k = comp == 0 ? md.kx : md.kz;
    if (zero) fill_rhs(N, par, lds, [&](int m) { return zscale(-1.0, F(comp, m)); });
    else
      fill_rhs(N, par, lds,
               [&](int m) { return zsub(zi(k, PA[(size_t)m * S]), F(comp, m)); });
    hel_par(make_sweep(a, q, md.lam), par, lds, g,
            [&](int n, double2 v) { dst[(size_t)n * S] = v; });
  }
}

// ---- A and B with register-resident columns (N <= MAXN) -------------------
template <typename T, int MAXN, int PAR>
__device__ __forceinline__ void pressure_par(const TauArgs& a, const Mode& md, int q) {
  using C = typename CT<T>::t;
  const int N = lane_copy(a.N), Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const C* in = (const C*)a.in;
  auto F = [&](int c, int n) { return to_z(in[((size_t)c * Ny + n) * S + q]); };
  double2* PA = a.scr + (size_t)kPA * Ny * S + q;
  const double iH = 1.0 / a.H;
  double2 r[MAXN / 2 + 1];
  fill_reg_deriv<MAXN, PAR>(N, r, [&](int p) { return F(1, p); }, [&](int m, double2 dfy) {
    return zadd(zadd(zi(md.kx, F(0, m)), zscale(iH, dfy)), zi(md.kz, F(2, m)));
  });
  hel_reg<MAXN, PAR>(N, a.H * a.H, md.lam, r, z2(0, 0),
                     [&](int n, double2 v) { PA[(size_t)n * S] = v; });
}

// k = 0: 2n p_n = c_{n-1} b_{n-1} - b_{n+1} with b = H F_y and p(-H) =
// gauge; lane l takes the coefficients n = l + 1, l + 65, ... (one each for
// N <= 64), and the wall condition's alternating sum is each lane's running
// sum, then a fixed-order wave reduction.
template <typename T>
__device__ __forceinline__ void pressure_zero(const TauArgs& a) {
  using C = typename CT<T>::t;
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const C* Fy = (const C*)a.in + (size_t)Ny * S;
  double2* PA = a.scr + (size_t)kPA * Ny * S;
  double2 t = z2(0, 0);
  for (int n = threadIdx.x + 1; n <= N; n += 64) {
    const double2 bm = zscale(a.H * (n == 1 ? 2.0 : 1.0), to_z(Fy[(size_t)(n - 1) * S]));
    const double2 bp = (n + 1 <= N - 1) ? zscale(a.H, to_z(Fy[(size_t)(n + 1) * S])) : z2(0, 0);
    const double2 pn = zscale(1.0 / (2.0 * n), zsub(bm, bp));
    PA[(size_t)n * S] = pn;
    if (n <= 64) t = (n & 1) ? zscale(-1.0, pn) : pn;
    else t = (n & 1) ? zsub(t, pn) : zadd(t, pn);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    t.x += __shfl_xor(t.x, o);
    t.y += __shfl_xor(t.y, o);
  }
  if (threadIdx.x == 0) PA[0] = zsub(z2(a.gauge[0], 0.0), t);
}

template <typename T, int MAXN>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) tau_pressure_r(TauArgs a) {
  const int par = blockIdx.y;
  if (blockIdx.x == gridDim.x - 1) {  // the extra block: mode 0
    if (par == 0) pressure_zero<T>(a);
    return;
  }
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q == 0 || q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  if (md.nyquist) return;
  if (par == 0) pressure_par<T, MAXN, 0>(a, md, q);
  else pressure_par<T, MAXN, 1>(a, md, q);
}

template <typename T, int MAXN, int PAR, bool VCOMP>
__device__ __forceinline__ void velocity_par(const TauArgs& a, const Mode& md, int q, int comp) {
  using C = typename CT<T>::t;
  const int N = lane_copy(a.N), Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const C* in = (const C*)a.in;
  const C* wall = (const C*)a.wall;
  auto F = [&](int c, int n) { return to_z(in[((size_t)c * Ny + n) * S + q]); };
  const double2* PA = a.scr + (size_t)kPA * Ny * S + q;
  double2* dst = a.scr + (size_t)(kUA + comp) * Ny * S + q;
  const double2 gm = to_z(wall[(size_t)comp * S + q]);
  const double2 gp = to_z(wall[(size_t)(3 + comp) * S + q]);
  const double2 g = PAR == 0 ? zscale(0.5, zadd(gp, gm)) : zscale(0.5, zsub(gp, gm));
  const double iH = 1.0 / a.H, h2 = a.H * a.H;
  const bool zero = q == 0;  // k = 0: no pressure coupling, v'' = 0
  double2 r[MAXN / 2 + 1];
  if (VCOMP) {
    if (zero) fill_reg<MAXN, PAR>(N, r, [](int) { return z2(0, 0); });
    else
      fill_reg_deriv<MAXN, PAR>(N, r, [&](int p) { return PA[(size_t)p * S]; },
                                [&](int m, double2 dp) { return zsub(zscale(iH, dp), F(1, m)); });
    double2 dm = z2(0, 0), dpl = z2(0, 0);
    hel_reg<MAXN, PAR>(N, h2, md.lam, r, g, [&](int n, double2 v) {
      dst[(size_t)n * S] = v;
      const double2 t = zscale((double)n * n, v);
      dpl = zadd(dpl, t);
      dm = (n & 1) ? zadd(dm, t) : zsub(dm, t);
    });
    double2* sl = a.scr + (size_t)kSlope * Ny * S + q;
    sl[(size_t)(2 * PAR) * S] = dm;
    sl[(size_t)(2 * PAR + 1) * S] = dpl;
  } else {
    const double k = comp == 0 ? md.kx : md.kz;
    if (zero) fill_reg<MAXN, PAR>(N, r, [&](int m) { return zscale(-1.0, F(comp, m)); });
    else
      fill_reg<MAXN, PAR>(N, r, [&](int m) { return zsub(zi(k, PA[(size_t)m * S]), F(comp, m)); });
    hel_reg<MAXN, PAR>(N, h2, md.lam, r, g, [&](int n, double2 v) { dst[(size_t)n * S] = v; });
  }
}

// Grid z = 3: slice 0 is the v component (the wall slopes), slices 1 and 2
// are u and w.
template <typename T, int MAXN>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) tau_velocity_r(TauArgs a) {
  const int q = blockIdx.x * 64 + threadIdx.x;
  const int par = blockIdx.y, z = blockIdx.z;
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  if (md.nyquist) return;
  if (z == 0) {
    if (par == 0) velocity_par<T, MAXN, 0, true>(a, md, q, 1);
    else velocity_par<T, MAXN, 1, true>(a, md, q, 1);
  } else {
    const int comp = 2 * (z - 1);
    if (par == 0) velocity_par<T, MAXN, 0, false>(a, md, q, comp);
    else velocity_par<T, MAXN, 1, false>(a, md, q, comp);
  }
}

// ---- D: wall pressures and superposition, one thread per (mode, n) --------
template <typename T, bool STRESS>
__global__ void __launch_bounds__(256) tau_combine(TauArgs a) {
  using C = typename CT<T>::t;
  const size_t S = (size_t)a.nmodes;
  const int Ny = a.N + 1;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)Ny * S) return;
  const int n = (int)(idx / S);
  const int q = (int)(idx - (size_t)n * S);
  const Mode md = mode_of(a, q);
  C* out = (C*)a.out;
  auto put = [&](int f, double2 v) { out[((size_t)f * Ny + n) * S + q] = from_z<T>(v); };
  if (md.nyquist) {
    for (int f = 0; f < (STRESS ? 6 : 3); ++f) put(f, z2(0, 0));
    return;
  }
  const double2* scr = a.scr + q;
  auto at = [&](int slot) { return scr[((size_t)slot * Ny + n) * S]; };
  double2 u = at(kUA), v = at(kVA), w = at(kWA), p = at(kPA);
  if (q != 0) {
    const C* wall = (const C*)a.wall;
    const double2* sl = scr + (size_t)kSlope * Ny * S;
    const double iH = 1.0 / a.H;
    const double2 dm = zadd(sl[0], sl[2 * S]), dp = zadd(sl[S], sl[3 * S]);
    const double2 cam = zadd(zadd(zi(md.kx, to_z(wall[q])), zscale(iH, dm)),
                             zi(md.kz, to_z(wall[2 * S + q])));
    const double2 cap = zadd(zadd(zi(md.kx, to_z(wall[3 * S + q])), zscale(iH, dp)),
                             zi(md.kz, to_z(wall[5 * S + q])));
    const double* mi = a.infl + 4 * (size_t)q;
    const double2 p1 = zscale(-1.0, zadd(zscale(mi[0], cam), zscale(mi[1], cap)));
    const double2 p2 = zscale(-1.0, zadd(zscale(mi[2], cam), zscale(mi[3], cap)));
    // (c) mirrors (b): coefficient n times (-1)^n, v also changes sign
    const double sg = (n & 1) ? -1.0 : 1.0;
    const double2 ps = zfma(sg, p2, p1), pd = zfma(-sg, p2, p1);
    const size_t NyS = (size_t)Ny * S;
    const double pb = a.pre[3 * NyS + 2 * S + (size_t)n * S + q];
    const double ub = a.pre[4 * NyS + 2 * S + (size_t)n * S + q];
    const double vb = a.pre[5 * NyS + 2 * S + (size_t)n * S + q];
    u = zadd(u, zi(md.kx, zscale(ub, ps)));
    w = zadd(w, zi(md.kz, zscale(ub, ps)));
    v = zfma(vb, pd, v);
    p = zfma(pb, ps, p);
  }
  if (!STRESS) {
    put(0, u);
    put(1, v);
    put(2, w);
    return;
  }
  double2* o = a.scr + q;
  o[((size_t)kU * Ny + n) * S] = u;
  o[((size_t)kV * Ny + n) * S] = v;
  o[((size_t)kW * Ny + n) * S] = w;
  o[((size_t)kP * Ny + n) * S] = p;
  // sigma = -p I + grad u + grad u^T: xx, yy, zz, xy, xz, yz
  const double2 mp = zscale(-1.0, p);
  put(0, zadd(mp, zscale(2.0, zi(md.kx, u))));
  put(2, zadd(mp, zscale(2.0, zi(md.kz, w))));
  put(4, zadd(zi(md.kz, u), zi(md.kx, w)));
}

// ---- E: stress components with a y-derivative, per (mode, component) -------
template <typename T>
__global__ void __launch_bounds__(64) tau_stress_dy(TauArgs a) {
  using C = typename CT<T>::t;
  const int q = blockIdx.x * 64 + threadIdx.x;
  const int comp = blockIdx.y;  // 0: sigma_yy (v'), 1: sigma_xy (u'), 2: sigma_yz (w')
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  if (md.nyquist) return;
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const double2* scr = a.scr + q;
  const int src = comp == 0 ? kV : (comp == 1 ? kU : kW);
  auto A = [&](int slot, int n) { return scr[((size_t)slot * Ny + n) * S]; };
  C* out = (C*)a.out;
  const int f = comp == 0 ? 1 : (comp == 1 ? 3 : 5);
  const double iH = 1.0 / a.H;
  // c_n b_n = b_{n+2} + 2 (n+1) a_{n+1}, from the top
  double2 b2 = z2(0, 0), b1 = z2(0, 0);
  for (int n = N; n >= 0; --n) {
    double2 b = z2(0, 0);
    if (n < N) {
      b = zfma(2.0 * (n + 1), A(src, n + 1), b2);
      if (n == 0) b = zscale(0.5, b);
    }
    double2 val;
    if (comp == 0) val = zadd(zscale(-1.0, A(kP, n)), zscale(2.0 * iH, b));
    else if (comp == 1) val = zadd(zscale(iH, b), zi(md.kx, A(kV, n)));
    else val = zadd(zi(md.kz, A(kV, n)), zscale(iH, b));
    out[((size_t)f * Ny + n) * S + q] = from_z<T>(val);
    b2 = b1;
    b1 = b;
  }
}

// Branch-free over the unrolled rows: loads use clamped indices, and the
// rows past N (iterated first, descending) store to row N, which its own
// iteration overwrites last.
// (restrict holds as parameters: the output never overlaps the scratch)
template <typename T, int MAXN, int COMP>
__device__ __forceinline__ void stress_dy_comp(const TauArgs& a, const Mode& md,
                                               const double2* __restrict__ scr,
                                               typename CT<T>::t* __restrict__ out) {
  const int N = lane_copy(a.N), Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  constexpr int src = COMP == 0 ? kV : (COMP == 1 ? kU : kW);
  auto A = [&](int slot, int n) { return scr[((size_t)slot * Ny + n) * S]; };
  const double iH = 1.0 / a.H;
  double2 b2 = z2(0, 0), b1 = z2(0, 0);
#pragma unroll
  for (int n = MAXN; n >= 0; --n) {
    const int nn = n < N ? n : N;
    const double2 an1 = A(src, n + 1 < N ? n + 1 : N);
    double2 b = zfma(2.0 * (n + 1), an1, b2);
    if (n == 0) b = zscale(0.5, b);
    b = n < N ? b : z2(0, 0);
    double2 val;
    if (COMP == 0) val = zadd(zscale(-1.0, A(kP, nn)), zscale(2.0 * iH, b));
    else if (COMP == 1) val = zadd(zscale(iH, b), zi(md.kx, A(kV, nn)));
    else val = zadd(zi(md.kz, A(kV, nn)), zscale(iH, b));
    out[(size_t)nn * S] = from_z<T>(val);
    b2 = b1;
    b1 = b;
  }
}

template <typename T, int MAXN>
__global__ void __launch_bounds__(64) tau_stress_dy_r(TauArgs a) {
  const int q = blockIdx.x * 64 + threadIdx.x;
  const int comp = blockIdx.y;  // 0: sigma_yy (v'), 1: sigma_xy (u'), 2: sigma_yz (w')
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  if (md.nyquist) return;
  using C = typename CT<T>::t;
  const size_t NyS = (size_t)(a.N + 1) * a.nmodes;
  const double2* scr = a.scr + q;
  C* out = (C*)a.out + q;
  if (comp == 0) stress_dy_comp<T, MAXN, 0>(a, md, scr, out + 1 * NyS);
  else if (comp == 1) stress_dy_comp<T, MAXN, 1>(a, md, scr, out + 3 * NyS);
  else stress_dy_comp<T, MAXN, 2>(a, md, scr, out + 5 * NyS);
}

// ---- plan time ------------------------------------------------------------
// Step 1: the lam-only factors of the even/odd sweeps per mode.
__global__ void __launch_bounds__(64) sweep_factors(TauArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  const int N = a.N, Nc = N + 1;
  const size_t S = (size_t)a.nmodes, NyS = (size_t)Nc * S;
  const double h2l = a.H * a.H * md.lam;
  const double* nc = a.nconst;
  double* inv = a.pre + q;
  double* mul = a.pre + NyS + q;
  double* Qa = a.pre + 2 * NyS + q;
  double* sq = a.pre + 3 * NyS + q;
  for (int par = 0; par < 2; ++par) {
    const int M = (N - par) / 2;
    double bn = 0.0;
    for (int i = M; i >= 1; --i) {
      const int n = par + 2 * i;
      const double cm2 = (n == 2) ? 2.0 : 1.0;
      const double lo = -h2l * cm2 * nc[n];
      const double d = 1.0 + ((n <= N - 2) ? h2l * nc[Nc + n] : 0.0);
      const double u = (n + 2 <= N - 2) ? -h2l * nc[2 * Nc + n] : 0.0;
      const double iv = 1.0 / (d + u * bn);
      bn = -lo * iv;
      inv[(size_t)n * S] = iv;
      mul[(size_t)n * S] = bn;
    }
    double Q = 1.0, s = 1.0;
    for (int i = 1; i <= M; ++i) {
      const int n = par + 2 * i;
      Q *= mul[(size_t)n * S];
      Qa[(size_t)n * S] = Q;
      s += Q;
    }
    sq[par * S] = s;
  }
}

// Step 2: problem (b) (p = 1 at y = -H): profiles p_b, u_b (u_b = i k_x u_b,
// w_b = i k_z u_b), v_b, and the 2x2 influence matrix of Eq. inf_mat with its
// inverse; (c) follows by reflection.
__global__ void __launch_bounds__(64) influence_modes(TauArgs a) {
  extern __shared__ double2 tau_lds[];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nmodes) return;
  const Mode md = mode_of(a, q);
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes, NyS = (size_t)Ny * S;
  double* pb = a.pre + 3 * NyS + 2 * S + q;
  double* ub = a.pre + 4 * NyS + 2 * S + q;
  double* vb = a.pre + 5 * NyS + 2 * S + q;
  double* o = a.infl + 4 * (size_t)q;
  if (q == 0 || md.nyquist) {
    for (int n = 0; n < Ny; ++n) pb[(size_t)n * S] = ub[(size_t)n * S] = vb[(size_t)n * S] = 0.0;
    o[0] = o[1] = o[2] = o[3] = 0.0;
    return;
  }
  double2* lds = tau_lds + threadIdx.x;
  const Sweep w = make_sweep(a, q, md.lam);
  const double iH = 1.0 / a.H;
  // p_b: zero forcing, p(-H) = 1, p(+H) = 0
  for (int par = 0; par < 2; ++par) {
    fill_rhs(N, par, lds, [](int) { return z2(0, 0); });
    hel_par(w, par, lds, z2(par == 0 ? 0.5 : -0.5, 0), [&](int n, double2 v) { pb[(size_t)n * S] = v.x; });
  }
  double vm = 0.0, vp = 0.0;
  for (int par = 0; par < 2; ++par) {
    // u_b profile: u'' - lam u = p_b, no-slip
    fill_rhs(N, par, lds, [&](int m) { return z2(pb[(size_t)m * S], 0); });
    hel_par(w, par, lds, z2(0, 0), [&](int n, double2 v) { ub[(size_t)n * S] = v.x; });
    // v_b: v'' - lam v = p_b', no-slip
    fill_rhs_deriv(N, par, lds, [&](int p) { return z2(pb[(size_t)p * S], 0); },
                   [&](int, double2 d) { return zscale(iH, d); });
    hel_par(w, par, lds, z2(0, 0), [&](int n, double2 v) {
      vb[(size_t)n * S] = v.x;
      const double t = (double)n * n * v.x;
      vp += t;
      vm += (n & 1) ? t : -t;
    });
  }
  // continuity at the walls: C(y) = v'(y)/H; (c) mirrors (b)
  const double cbm = vm * iH, cbp = vp * iH;
  const double ccm = cbp, ccp = cbm;
  const double det = cbm * ccp - ccm * cbp;
  const double id = 1.0 / det;
  o[0] = ccp * id;
  o[1] = -ccm * id;
  o[2] = -cbp * id;
  o[3] = cbm * id;
}

static TauArgs tau_args(Plan& p) {
  TauArgs a;
  a.N = p.p.Ny - 1;
  a.Nx = p.p.Nx;
  a.Nz = p.p.Nz;
  a.Nzh = p.Nzh;
  a.nmodes = p.nmodes;
  a.H = p.p.H;
  a.Lx = p.p.Lx;
  a.Lz = p.p.Lz;
  a.nconst = p.nconst;
  a.pre = p.sweep;
  a.infl = p.infl;
  a.in = p.specB;
  a.wall = p.wall_spec;
  a.out = p.specA;
  a.scr = (double2*)p.tau_scr;
  a.gauge = p.gauge;
  return a;
}

static size_t tau_lds_bytes(Plan& p) { return (size_t)((p.p.Ny - 1) / 2 + 2) * 64 * sizeof(double2); }

// Chebyshev orders up to 64 keep each parity's column in registers; larger
// orders stage it in LDS.
template <typename T, int MAXN>
static void launch_tau_reg(Plan& p, const TauArgs& a, unsigned nb, unsigned nc, bool stress) {
  tau_pressure_r<T, MAXN><<<dim3(nb + 1, 2), 64, 0, p.stream>>>(a);
  tau_velocity_r<T, MAXN><<<dim3(nb, 2, 3), 64, 0, p.stream>>>(a);
  if (stress) {
    tau_combine<T, true><<<nc, 256, 0, p.stream>>>(a);
    tau_stress_dy_r<T, MAXN><<<dim3(nb, 3), 64, 0, p.stream>>>(a);
  } else {
    tau_combine<T, false><<<nc, 256, 0, p.stream>>>(a);
  }
}

// The global velocity and pressure coefficients that the stress pass of
// tau_combine keeps in its work array (slots kU, kV, kW, kP), as four
// coefficient fields [field][n][mode] of the grid's type (Nyquist modes zero).
template <typename T>
__global__ void __launch_bounds__(256) tau_export(TauArgs a) {
  const size_t S = (size_t)a.nmodes;
  const int Ny = a.N + 1;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)Ny * S) return;
  const int n = (int)(idx / S);
  const int q = (int)(idx - (size_t)n * S);
  const Mode md = mode_of(a, q);
  typename CT<T>::t* out = (typename CT<T>::t*)a.out;
  const int slots[4] = {kU, kV, kW, kP};
  for (int f = 0; f < 4; ++f) {
    const double2 v = md.nyquist ? z2(0, 0) : a.scr[((size_t)slots[f] * Ny + n) * S + q];
    out[((size_t)f * Ny + n) * S + q] = from_z<T>(v);
  }
}

template <typename T>
hipError_t launch_tau_export(Plan& p) {
  TauArgs a = tau_args(p);
  const size_t tot = (size_t)p.p.Ny * p.nmodes;
  tau_export<T><<<(unsigned)((tot + 255) / 256), 256, 0, p.stream>>>(a);
  return hipGetLastError();
}

template hipError_t launch_tau_export<double>(Plan&);
template hipError_t launch_tau_export<float>(Plan&);

template <typename T>
hipError_t launch_tau(Plan& p, bool stress) {
  TauArgs a = tau_args(p);
  const unsigned nb = (unsigned)((p.nmodes + 63) / 64);
  const size_t tot = (size_t)p.p.Ny * p.nmodes;
  const unsigned nc = (unsigned)((tot + 255) / 256);
  if (a.N <= 32) {
    launch_tau_reg<T, 32>(p, a, nb, nc, stress);
    return hipGetLastError();
  }
  if (a.N <= 64) {
    launch_tau_reg<T, 64>(p, a, nb, nc, stress);
    return hipGetLastError();
  }
  // FP32 inputs up to order 96 still fit the register form without spills
  // (about 410 registers for the pressure sweep); up to 128 the pressure
  // sweep spills some 200 registers and is still 2.5x faster than the LDS
  // form; FP64 (whose sweeps spill far more) and higher orders use the LDS
  // columns
  if constexpr (sizeof(T) == 4) {
    if (a.N <= 96) {
      launch_tau_reg<T, 96>(p, a, nb, nc, stress);
      return hipGetLastError();
    }
    if (a.N <= 128) {
      launch_tau_reg<T, 128>(p, a, nb, nc, stress);
      return hipGetLastError();
    }
  }
  const size_t lds = tau_lds_bytes(p);
  tau_pressure<T><<<dim3(nb, 2), 64, lds, p.stream>>>(a);
  tau_velocity<T><<<dim3(nb, 2, 3), 64, lds, p.stream>>>(a);
  if (stress) {
    tau_combine<T, true><<<nc, 256, 0, p.stream>>>(a);
    tau_stress_dy<T><<<dim3(nb, 3), 64, 0, p.stream>>>(a);
  } else {
    tau_combine<T, false><<<nc, 256, 0, p.stream>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_influence(Plan& p) {
  TauArgs a = tau_args(p);
  const unsigned nb = (unsigned)((p.nmodes + 63) / 64);
  sweep_factors<<<nb, 64, 0, p.stream>>>(a);
  influence_modes<<<nb, 64, tau_lds_bytes(p), p.stream>>>(a);
  return hipGetLastError();
}

template hipError_t launch_tau<double>(Plan&, bool);
template hipError_t launch_tau<float>(Plan&, bool);

}  // namespace ggem
