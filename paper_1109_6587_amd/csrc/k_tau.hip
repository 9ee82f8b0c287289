// Global Stokes problem per Fourier mode (Appendix C), always in FP64.
//
// For mode (k_x, k_z), lam = k_x^2 + k_z^2, with F the Chebyshev
// coefficients of the global force density (momentum: -grad p + lap u + F = 0)
// and g-, g+ the wall velocities (u^g = -u^l at y = -H, +H):
//   p'' - lam p = i k_x F_x + F_y' + i k_z F_z,   p(-H) = p1, p(+H) = p2
//   u'' - lam u = i k_x p - F_x   (v: p' - F_y,  w: i k_z p - F_z)
// and p1, p2 make the velocity divergence-free at both walls (the influence
// matrix of Eq. inf_mat).  The 2x2 influence matrix depends only on lam and
// is inverted once per plan; u, w meet their wall values exactly, so the
// wall divergence of problem (a) needs only the v solve.  The final fields
// are obtained by solving again with the wall pressures p1, p2 (the same
// superposition as Eq. cheb_sol).
//
// Each Helmholtz problem is the tau system: rows 0..N-2 of
// (D^2/H^2 - lam) a = r plus the two wall rows.  Substituting the Chebyshev
// recurrence that expresses a_n (n >= 2) through the coefficients of a''
// turns it into two tridiagonal systems (even and odd n) bordered by one full
// row each (the wall conditions); each is solved by a backward sweep that
// writes a_n = P_n + Q_n a_{0|1} and one full-row solve, O(N) per problem.
//
// One thread per mode; per-mode work arrays live in a strided scratch buffer
// so that a wave's accesses are coalesced.
#include "ggem_internal.h"

namespace ggem {

struct Col {
  double2* p;
  size_t s;
  __device__ double2& operator[](int n) const { return p[(size_t)n * s]; }
};

struct RCol {
  double* p;
  size_t s;
  __device__ double& operator[](int n) const { return p[(size_t)n * s]; }
};

__device__ inline double2 z2(double a, double b) { return make_double2(a, b); }
__device__ inline double2 zadd(double2 a, double2 b) { return z2(a.x + b.x, a.y + b.y); }
__device__ inline double2 zsub(double2 a, double2 b) { return z2(a.x - b.x, a.y - b.y); }
__device__ inline double2 zscale(double s, double2 a) { return z2(s * a.x, s * a.y); }
__device__ inline double2 zi(double k, double2 a) { return z2(-k * a.y, k * a.x); }  // i k a

// Tau solution of a'' - lam a = r on [-H, H] with a(-H) = gm, a(+H) = gp.
// r and out must not alias; beta is real scratch.
__device__ void hel_tau(int N, double lam, double H, Col r, double2 gm, double2 gp, Col out,
                        RCol beta) {
  const double h2 = H * H;
  const double h2l = h2 * lam;
  for (int par = 0; par < 2; ++par) {
    const int M = (N - par) / 2;
    double2 an = z2(0, 0);
    double bn = 0.0;
    for (int i = M; i >= 1; --i) {
      const int n = par + 2 * i;
      const double cm2 = (n == 2) ? 2.0 : 1.0;
      const double q1 = 1.0 / (4.0 * n * (n - 1));
      const double q2 = 1.0 / (2.0 * ((double)n * n - 1.0));
      const double q3 = 1.0 / (4.0 * n * (n + 1));
      const bool en = n <= N - 2, ep = n + 2 <= N - 2;
      const double l = -h2l * cm2 * q1;
      const double d = 1.0 + (en ? h2l * q2 : 0.0);
      const double u = ep ? -h2l * q3 : 0.0;
      double2 s = zscale(cm2 * q1, r[n - 2]);
      if (en) s = zsub(s, zscale(q2, r[n]));
      if (ep) s = zadd(s, zscale(q3, r[n + 2]));
      s = zscale(h2, s);
      const double den = d + u * bn;
      const double inv = 1.0 / den;
      const double bi = -l * inv;
      const double2 ai = zscale(inv, zsub(s, zscale(u, an)));
      out[n] = ai;
      beta[n] = bi;
      an = ai;
      bn = bi;
    }
    double2 P = z2(0, 0), SP = z2(0, 0);
    double Q = 1.0, SQ = 1.0;
    for (int i = 1; i <= M; ++i) {
      const int n = par + 2 * i;
      const double b = beta[n];
      P = zadd(out[n], zscale(b, P));
      Q = b * Q;
      out[n] = P;
      beta[n] = Q;
      SP = zadd(SP, P);
      SQ += Q;
    }
    const double2 g = par == 0 ? zscale(0.5, zadd(gp, gm)) : zscale(0.5, zsub(gp, gm));
    const double2 x0 = zscale(1.0 / SQ, zsub(g, SP));
    out[par] = x0;
    for (int i = 1; i <= M; ++i) {
      const int n = par + 2 * i;
      out[n] = zadd(out[n], zscale(beta[n], x0));
    }
  }
}

// b = d/d(ybar) a on coefficients: c_n b_n = b_{n+2} + 2 (n+1) a_{n+1}.
__device__ void cheb_deriv(int N, Col a, Col b) {
  double2 b2 = z2(0, 0), b1 = z2(0, 0);
  b[N] = b1;
  for (int n = N - 1; n >= 0; --n) {
    double2 v = zadd(b2, zscale(2.0 * (n + 1), a[n + 1]));
    if (n == 0) v = zscale(0.5, v);
    b[n] = v;
    b2 = b1;
    b1 = v;
  }
}

// wall slopes: a'(-1) = sum (-1)^(n+1) n^2 a_n, a'(+1) = sum n^2 a_n
__device__ inline void wall_slopes(int N, Col a, double2& dm, double2& dp) {
  dm = z2(0, 0);
  dp = z2(0, 0);
  for (int n = 1; n <= N; ++n) {
    const double w = (double)n * n;
    const double2 v = zscale(w, a[n]);
    dp = zadd(dp, v);
    dm = (n & 1) ? zadd(dm, v) : zsub(dm, v);
  }
}

struct TauArgs {
  int N, Nx, Nz, Nzh, nmodes;
  double H, Lx, Lz;
  const double* infl;
  const void* in;      // [3][Ny][nmodes] complex T
  const void* wall;    // [2][3][nmodes] complex T
  void* out;           // [3|6][Ny][nmodes] complex T
  double2* scr;        // [6][Ny][nmodes] complex + [Ny][nmodes] real
  const double* gauge;
};

template <typename C>
__device__ inline double2 to_z(C v) {
  return z2((double)v.x, (double)v.y);
}

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

template <typename T>
__device__ inline typename CT<T>::t from_z(double2 v) {
  typename CT<T>::t r;
  r.x = (T)v.x;
  r.y = (T)v.y;
  return r;
}

__device__ inline void mode_k(const TauArgs& a, int q, int& l, int& m, double& kx, double& kz) {
  l = q / a.Nzh;
  m = q - l * a.Nzh;
  const int ls = l < a.Nx / 2 ? l : l - a.Nx;
  kx = 6.283185307179586477 * ls / a.Lx;
  kz = 6.283185307179586477 * m / a.Lz;
}

template <typename T, bool STRESS>
__global__ void __launch_bounds__(64) tau_modes(TauArgs a) {
  using C = typename CT<T>::t;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nmodes) return;
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  int l, m;
  double kx, kz;
  mode_k(a, q, l, m, kx, kz);
  const int nout = STRESS ? 6 : 3;
  C* out = (C*)a.out;
  if (l == a.Nx / 2 || m == a.Nz / 2) {
    C zero;
    zero.x = (T)0;
    zero.y = (T)0;
    for (int f = 0; f < nout; ++f)
      for (int n = 0; n < Ny; ++n) out[((size_t)f * Ny + n) * S + q] = zero;
    return;
  }
  const double lam = kx * kx + kz * kz;
  const double H = a.H;
  const C* in = (const C*)a.in;
  const C* wall = (const C*)a.wall;
  const size_t FS = (size_t)Ny * S;
  Col R{a.scr + 0 * FS + q, S}, P{a.scr + 1 * FS + q, S}, U{a.scr + 2 * FS + q, S},
      V{a.scr + 3 * FS + q, S}, W{a.scr + 4 * FS + q, S}, X{a.scr + 5 * FS + q, S};
  RCol B{(double*)(a.scr + 6 * FS) + q, S};
  for (int n = 0; n < Ny; ++n) {
    U[n] = to_z(in[(0 * (size_t)Ny + n) * S + q]);
    V[n] = to_z(in[(1 * (size_t)Ny + n) * S + q]);
    W[n] = to_z(in[(2 * (size_t)Ny + n) * S + q]);
  }
  const double2 gxm = to_z(wall[0 * S + q]), gym = to_z(wall[1 * S + q]),
                gzm = to_z(wall[2 * S + q]);
  const double2 gxp = to_z(wall[3 * S + q]), gyp = to_z(wall[4 * S + q]),
                gzp = to_z(wall[5 * S + q]);
  const double iH = 1.0 / H;
  if (q == 0) {
    // k = 0: u'' = -F_x, w'' = -F_z, v'' = 0 between the wall values;
    // p' = F_y (rows 0..N-1), p(-H) = gauge.
    for (int n = 0; n < Ny; ++n) R[n] = zscale(-1.0, U[n]);
    hel_tau(N, 0.0, H, R, gxm, gxp, X, B);
    for (int n = 0; n < Ny; ++n) U[n] = X[n];
    for (int n = 0; n < Ny; ++n) R[n] = zscale(-1.0, W[n]);
    hel_tau(N, 0.0, H, R, gzm, gzp, X, B);
    for (int n = 0; n < Ny; ++n) W[n] = X[n];
    if (STRESS) {
      // integrate b = H F_y: 2n p_n = c_{n-1} b_{n-1} - b_{n+1}
      for (int n = 1; n <= N; ++n) {
        const double2 bm = zscale(H * (n - 1 == 0 ? 2.0 : 1.0), V[n - 1]);
        const double2 bp = (n + 1 <= N - 1) ? zscale(H, V[n + 1]) : z2(0, 0);
        P[n] = zscale(1.0 / (2.0 * n), zsub(bm, bp));
      }
      double2 s = z2(0, 0);
      for (int n = 1; n <= N; ++n) s = (n & 1) ? zsub(s, P[n]) : zadd(s, P[n]);
      P[0] = zsub(z2(a.gauge[0], 0.0), s);
    }
    for (int n = 0; n < Ny; ++n) R[n] = z2(0, 0);
    hel_tau(N, 0.0, H, R, gym, gyp, V, B);
  } else {
    // (a): pressure with zero wall values, then v for the wall divergence
    cheb_deriv(N, V, X);
    for (int n = 0; n < Ny; ++n) R[n] = zadd(zadd(zi(kx, U[n]), zscale(iH, X[n])), zi(kz, W[n]));
    hel_tau(N, lam, H, R, z2(0, 0), z2(0, 0), P, B);
    cheb_deriv(N, P, X);
    for (int n = 0; n < Ny; ++n) R[n] = zsub(zscale(iH, X[n]), V[n]);
    hel_tau(N, lam, H, R, gym, gyp, X, B);
    double2 dm, dp;
    wall_slopes(N, X, dm, dp);
    const double2 cam = zadd(zadd(zi(kx, gxm), zscale(iH, dm)), zi(kz, gzm));
    const double2 cap = zadd(zadd(zi(kx, gxp), zscale(iH, dp)), zi(kz, gzp));
    const double* mi = a.infl + 4 * (size_t)q;
    const double2 p1 = zscale(-1.0, zadd(zscale(mi[0], cam), zscale(mi[1], cap)));
    const double2 p2 = zscale(-1.0, zadd(zscale(mi[2], cam), zscale(mi[3], cap)));
    // final pressure with wall values p1 (y = -H), p2 (y = +H)
    cheb_deriv(N, V, X);
    for (int n = 0; n < Ny; ++n) R[n] = zadd(zadd(zi(kx, U[n]), zscale(iH, X[n])), zi(kz, W[n]));
    hel_tau(N, lam, H, R, p1, p2, P, B);
    // velocities
    for (int n = 0; n < Ny; ++n) R[n] = zsub(zi(kx, P[n]), U[n]);
    hel_tau(N, lam, H, R, gxm, gxp, U, B);
    for (int n = 0; n < Ny; ++n) R[n] = zsub(zi(kz, P[n]), W[n]);
    hel_tau(N, lam, H, R, gzm, gzp, W, B);
    cheb_deriv(N, P, X);
    for (int n = 0; n < Ny; ++n) R[n] = zsub(zscale(iH, X[n]), V[n]);
    hel_tau(N, lam, H, R, gym, gyp, V, B);
  }
  if (!STRESS) {
    for (int n = 0; n < Ny; ++n) {
      out[((size_t)0 * Ny + n) * S + q] = from_z<T>(U[n]);
      out[((size_t)1 * Ny + n) * S + q] = from_z<T>(V[n]);
      out[((size_t)2 * Ny + n) * S + q] = from_z<T>(W[n]);
    }
  } else {
    // sigma = -p I + grad u + grad u^T: xx, yy, zz, xy, xz, yz
    for (int n = 0; n < Ny; ++n) {
      const double2 mp = zscale(-1.0, P[n]);
      out[((size_t)0 * Ny + n) * S + q] = from_z<T>(zadd(mp, zscale(2.0, zi(kx, U[n]))));
      out[((size_t)2 * Ny + n) * S + q] = from_z<T>(zadd(mp, zscale(2.0, zi(kz, W[n]))));
      out[((size_t)4 * Ny + n) * S + q] = from_z<T>(zadd(zi(kz, U[n]), zi(kx, W[n])));
    }
    cheb_deriv(N, V, X);
    for (int n = 0; n < Ny; ++n)
      out[((size_t)1 * Ny + n) * S + q] =
          from_z<T>(zadd(zscale(-1.0, P[n]), zscale(2.0 * iH, X[n])));
    cheb_deriv(N, U, X);
    for (int n = 0; n < Ny; ++n)
      out[((size_t)3 * Ny + n) * S + q] = from_z<T>(zadd(zscale(iH, X[n]), zi(kx, V[n])));
    cheb_deriv(N, W, X);
    for (int n = 0; n < Ny; ++n)
      out[((size_t)5 * Ny + n) * S + q] = from_z<T>(zadd(zi(kz, V[n]), zscale(iH, X[n])));
  }
}

// Plan time: 2x2 influence matrix of Eq. inf_mat per mode and its inverse.
// (b): p = 1 at y = -H, (c): p = 1 at y = +H, no forcing, no-slip.  The
// continuity expression at the walls reduces to v'/H there because u and w
// vanish at both walls.
__global__ void __launch_bounds__(64) influence_modes(TauArgs a, double* infl) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nmodes) return;
  int l, m;
  double kx, kz;
  mode_k(a, q, l, m, kx, kz);
  double* o = infl + 4 * (size_t)q;
  if (q == 0 || l == a.Nx / 2 || m == a.Nz / 2) {
    o[0] = o[1] = o[2] = o[3] = 0.0;
    return;
  }
  const int N = a.N, Ny = N + 1;
  const size_t S = (size_t)a.nmodes;
  const size_t FS = (size_t)Ny * S;
  const double lam = kx * kx + kz * kz, H = a.H, iH = 1.0 / H;
  Col R{a.scr + 0 * FS + q, S}, P{a.scr + 1 * FS + q, S}, V{a.scr + 3 * FS + q, S},
      X{a.scr + 5 * FS + q, S};
  RCol B{(double*)(a.scr + 6 * FS) + q, S};
  double c[2][2];  // c[wall][problem]
  for (int prob = 0; prob < 2; ++prob) {
    for (int n = 0; n < Ny; ++n) R[n] = z2(0, 0);
    hel_tau(N, lam, H, R, z2(prob == 0 ? 1.0 : 0.0, 0), z2(prob == 1 ? 1.0 : 0.0, 0), P, B);
    cheb_deriv(N, P, X);
    for (int n = 0; n < Ny; ++n) R[n] = zscale(iH, X[n]);
    hel_tau(N, lam, H, R, z2(0, 0), z2(0, 0), V, B);
    double2 dm, dp;
    wall_slopes(N, V, dm, dp);
    c[0][prob] = dm.x * iH;
    c[1][prob] = dp.x * iH;
  }
  const double det = c[0][0] * c[1][1] - c[0][1] * c[1][0];
  const double id = 1.0 / det;
  o[0] = c[1][1] * id;
  o[1] = -c[0][1] * id;
  o[2] = -c[1][0] * id;
  o[3] = c[0][0] * id;
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
  a.infl = p.infl;
  a.in = p.specB;
  a.wall = p.wall_spec;
  a.out = p.specA;
  a.scr = (double2*)p.tau_scr;
  a.gauge = p.gauge;
  return a;
}

template <typename T>
hipError_t launch_tau(Plan& p, bool stress) {
  TauArgs a = tau_args(p);
  const unsigned nb = (unsigned)((p.nmodes + 63) / 64);
  if (stress) tau_modes<T, true><<<nb, 64, 0, p.stream>>>(a);
  else tau_modes<T, false><<<nb, 64, 0, p.stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_influence(Plan& p) {
  TauArgs a = tau_args(p);
  influence_modes<<<(unsigned)((p.nmodes + 63) / 64), 64, 0, p.stream>>>(a, p.infl);
  return hipGetLastError();
}

template hipError_t launch_tau<double>(Plan&, bool);
template hipError_t launch_tau<float>(Plan&, bool);

}  // namespace ggem
