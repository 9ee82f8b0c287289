// Spectrally accurate evaluation of the global part off the mesh, in place
// of the 4th-order Lagrange stencil (whose error is O(h^5), Sec. 3.2.2).
//
// The global field is a Fourier series in x, z times a Chebyshev series in y:
//   u(x, y, z) = sum_n T_n(y/H) sum_{l, m} u_hat[n, l, m] exp(i (k_l x + k_m z)).
// With theta = arccos(y/H), T_n(y/H) = cos(n theta): the field is a Fourier
// series in (x, theta, z), even and 2 pi-periodic in theta with |n| <= N =
// Ny - 1.  It is summed at the targets as a type-2 non-uniform FFT by
// Gaussian gridding (Dutt-Rokhlin, Greengard-Lee) in all three variables:
// with s = 2 pi x/Lx and g_tau(s) the periodised exp(-s^2/(4 tau)), whose
// Fourier coefficients are G_k = sqrt(tau/pi) exp(-k^2 tau),
//   1. deconvolve and zero-pad in x and z: h_hat[k] = u_hat[k] / G_k on the
//      2Nx x 2Nz grid (nufft_pad), inverse FFT of every (field, order) plane;
//   2. in theta, h(theta_j) = sum_n (a_n / G_n) cos(n theta_j) on the
//      M = 2 (2N + 1) nodes theta_j = 2 pi j / M, a GEMM with the plan's
//      (j, n) matrix; the planes j <= M/2 are kept, the others are their
//      mirror images (the series is even);
//   3. at each target, (1/(Mx Mz M)) times the sum over the 2 msp nearest
//      oversampled nodes in each variable of h times the three Gaussians;
// with tau = pi msp / (3 K^2) for a band of K modes (K = Nx, Nz, 2N + 1), for
// which aliasing and window truncation errors are both about exp(-0.75 pi
// msp) (msp = 12: 5e-13; 6: 7e-7).  The local part and the double layer's
// normal are combined as in the Lagrange path.  The cost per target is
// (2 msp)^3 per field, independent of the grid.
#include "ggem_internal.h"

namespace ggem {

namespace {

template <typename T>
struct CxS;
template <>
struct CxS<double> {
  using t = double2;
};
template <>
struct CxS<float> {
  using t = float2;
};

struct PadArgs {
  int Nx, Nzh, Mx, Mzh, Ny, nf;
  size_t nm, mm;            // modes per plane: Nx Nzh and Mx Mzh
  double tx, tz, scale;     // tau_x, tau_z, pi / (sqrt(tau_x tau_z) Mx Mz)
  const void* in;           // [f][n][l][m] complex T (Nx x Nzh)
  void* out;                // [f][n][L][m] complex T (Mx x Mzh)
};

// every oversampled mode: the deconvolved coefficient, or zero outside the
// mesh's band (the Nyquist row and column included)
template <typename T>
__global__ void __launch_bounds__(256) nufft_pad(PadArgs a) {
  using C = typename CxS<T>::t;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = (size_t)a.nf * a.Ny * a.mm;
  if (idx >= tot) return;
  const size_t plane = idx / a.mm;
  const int q = (int)(idx - plane * a.mm);
  const int L = q / a.Mzh, m = q - L * a.Mzh;
  const int ls = L < a.Mx / 2 ? L : L - a.Mx;
  C v;
  v.x = (T)0;
  v.y = (T)0;
  if (ls > -a.Nx / 2 && ls < a.Nx / 2 && m < a.Nzh - 1) {
    const int l = ls >= 0 ? ls : ls + a.Nx;
    const C u = ((const C*)a.in)[plane * a.nm + (size_t)l * a.Nzh + m];
    const double d = a.scale * exp((double)ls * ls * a.tx + (double)m * m * a.tz);
    v.x = (T)(d * (double)u.x);
    v.y = (T)(d * (double)u.y);
  }
  ((C*)a.out)[idx] = v;
}

struct EvalArgs {
  int nt, Mx, Mz, msp, thm, thp;
  int per;                        // 4-target tiles per XCD
  double Lx, Lz, H, tx, tz, tth;
  const int* perm;
  const double *tx_, *ty, *tz_;   // sorted wrapped targets
  const void* tn;                 // sorted normals (T, SoA) for the double layer
  size_t tcap;
  const void* ul;                 // local part (kNearSlices x 3, T, SoA)
  const void* grid;               // [f][j][X][Z] T, the theta planes
  double* out;                    // (nt, 3) in input order
};

// One wave per target.  The W x W window in (x, z) (W = 2 msp) is flattened
// over the 64 lanes, E entries per lane (W^2 <= 64 E): consecutive lanes read
// consecutive z nodes of a row, so each load of a plane is a few contiguous
// runs.  Each lane keeps its entries' products wx_i wz_k and offsets in
// registers and sums its part of the window of each of the W theta planes,
// weighted by that plane's Gaussian; a wave reduction per field ends it.
// Block b serves 4-target tile (b mod 8) per + b/8, so that each XCD walks a
// contiguous run of the cell-sorted targets and their windows overlap in its
// L2.
template <typename T, bool STRESS, int E>
__global__ void __launch_bounds__(256) spectral_eval(EvalArgs a) {
  const int tile = (int)(blockIdx.x & 7) * a.per + (int)(blockIdx.x >> 3);
  const int t = tile * 4 + (int)(threadIdx.x >> 6);
  if (t >= a.nt) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  constexpr int NC = STRESS ? 6 : 3;
  constexpr double kTwoPi = 6.283185307179586477;
  const double sx = kTwoPi * a.tx_[t] / a.Lx, sz = kTwoPi * a.tz_[t] / a.Lz;
  const double th = acos(fmin(1.0, fmax(-1.0, a.ty[t] / a.H)));
  const double hx = kTwoPi / a.Mx, hz = kTwoPi / a.Mz, ht = kTwoPi / a.thm;
  const int W = 2 * a.msp;
  // lane j < W: weight and node of the j-th window point in x, z and theta
  double wxl = 0.0, wzl = 0.0, wtl = 0.0;
  int ixl = 0, izl = 0, jtl = 0;
  if (lane < W) {
    const int ix = (int)floor(sx / hx) - a.msp + 1 + lane;
    const int iz = (int)floor(sz / hz) - a.msp + 1 + lane;
    const int jt = (int)floor(th / ht) - a.msp + 1 + lane;
    const double dx = sx - ix * hx, dz = sz - iz * hz, dt = th - jt * ht;
    wxl = exp(-dx * dx / (4.0 * a.tx));
    wzl = exp(-dz * dz / (4.0 * a.tz));
    wtl = exp(-dt * dt / (4.0 * a.tth));
    ixl = ix < 0 ? ix + a.Mx : (ix >= a.Mx ? ix - a.Mx : ix);
    izl = iz < 0 ? iz + a.Mz : (iz >= a.Mz ? iz - a.Mz : iz);
    // theta node jt mod M, folded onto the stored planes 0 .. M/2
    int jm = jt % a.thm;
    jm = jm < 0 ? jm + a.thm : jm;
    jtl = jm > a.thm / 2 ? a.thm - jm : jm;
  }
  double w[E];
  int off[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int q = lane + 64 * e;
    const int i = q / W, k = q - i * W;  // i < 64 for every bucket
    const double wi = __shfl(wxl, i), wk = __shfl(wzl, k);
    const int xi = __shfl(ixl, i), zk = __shfl(izl, k);
    const bool act = q < W * W;
    w[e] = act ? wi * wk : 0.0;
    off[e] = act ? xi * a.Mz + zk : 0;
  }
  const T* G = (const T*)a.grid;
  const size_t plane = (size_t)a.Mx * a.Mz;
  double val[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double acc = 0.0;
    for (int j = 0; j < W; ++j) {
      const T* g = G + ((size_t)c * a.thp + __shfl(jtl, j)) * plane;
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) s = fma(w[e], (double)g[off[e]], s);
      acc = fma(__shfl(wtl, j), s, acc);
    }
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    val[c] = acc;
  }
  if (lane != 0) return;
  const T* ul = (const T*)a.ul;
  double res[3];
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    for (int s = 0; s < kNearSlices; ++s) v += (double)ul[(size_t)(3 * s + c) * a.tcap + t];
    res[c] = v;
  }
  if (!STRESS) {
    for (int c = 0; c < 3; ++c) res[c] += val[c];
  } else {
    const T* tnr = (const T*)a.tn;
    const double nx = tnr[t], ny = tnr[a.tcap + t], nz = tnr[2 * a.tcap + t];
    res[0] += val[0] * nx + val[3] * ny + val[4] * nz;
    res[1] += val[3] * nx + val[1] * ny + val[5] * nz;
    res[2] += val[4] * nx + val[5] * ny + val[2] * nz;
  }
  const size_t o = 3 * (size_t)a.perm[t];
  a.out[o] = res[0];
  a.out[o + 1] = res[1];
  a.out[o + 2] = res[2];
}

template <typename T, int E>
void launch_eval_e(const EvalArgs& a, unsigned nb, bool stress, hipStream_t st) {
  if (stress) spectral_eval<T, true, E><<<nb, 256, 0, st>>>(a);
  else spectral_eval<T, false, E><<<nb, 256, 0, st>>>(a);
}

}  // namespace

template <typename T>
hipError_t launch_nufft_pad(Plan& p, int nf) {
  PadArgs a;
  a.Nx = p.p.Nx;
  a.Nzh = p.Nzh;
  a.Mx = 2 * p.p.Nx;
  a.Mzh = p.p.Nz + 1;
  a.Ny = p.p.Ny;
  a.nf = nf;
  a.nm = (size_t)a.Nx * a.Nzh;
  a.mm = (size_t)a.Mx * a.Mzh;
  a.tx = p.tau_x;
  a.tz = p.tau_z;
  a.scale = 3.141592653589793238 / (sqrt(p.tau_x * p.tau_z) * (double)a.Mx * (2.0 * p.p.Nz));
  a.in = p.specA;
  a.out = p.over_spec;
  const size_t tot = (size_t)nf * a.Ny * a.mm;
  nufft_pad<T><<<(unsigned)((tot + 255) / 256), 256, 0, p.stream>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spectral_eval(Plan& p, int nt, double* out, bool stress) {
  if (nt <= 0) return hipSuccess;
  EvalArgs a;
  a.nt = nt;
  a.Mx = 2 * p.p.Nx;
  a.Mz = 2 * p.p.Nz;
  a.msp = p.msp;
  a.thm = p.th_m;
  a.thp = p.th_planes;
  const int tiles = (nt + 3) / 4;
  a.per = (tiles + 7) / 8;
  a.Lx = p.p.Lx;
  a.Lz = p.p.Lz;
  a.H = p.p.H;
  a.tx = p.tau_x;
  a.tz = p.tau_z;
  a.tth = p.tau_th;
  a.perm = p.tview->perm;
  a.tx_ = p.tview->x;
  a.ty = p.tview->y;
  a.tz_ = p.tview->z;
  a.tn = p.tnrm;
  a.tcap = (size_t)p.p.max_tgt;
  a.ul = p.ul;
  a.grid = p.over_theta;
  a.out = out;
  const unsigned nb = 8u * (unsigned)a.per;
  // entries per lane: the smallest bucket with 64 E >= W^2
  const int W2 = 4 * p.msp * p.msp;
  if (W2 <= 64) launch_eval_e<T, 1>(a, nb, stress, p.stream);
  else if (W2 <= 128) launch_eval_e<T, 2>(a, nb, stress, p.stream);
  else if (W2 <= 256) launch_eval_e<T, 4>(a, nb, stress, p.stream);
  else if (W2 <= 576) launch_eval_e<T, 9>(a, nb, stress, p.stream);
  else launch_eval_e<T, 16>(a, nb, stress, p.stream);
  return hipGetLastError();
}

template hipError_t launch_nufft_pad<double>(Plan&, int);
template hipError_t launch_nufft_pad<float>(Plan&, int);
template hipError_t launch_spectral_eval<double>(Plan&, int, double*, bool);
template hipError_t launch_spectral_eval<float>(Plan&, int, double*, bool);

}  // namespace ggem
