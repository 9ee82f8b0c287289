// Spectrally accurate evaluation of the global part off the mesh, in place
// of the 4th-order Lagrange stencil (whose error is O(h^5), Sec. 3.2.2).
//
// The global field is a Fourier series in x, z times a Chebyshev series in y:
//   u(x, y, z) = sum_n T_n(y/H) sum_{l, m} u_hat[n, l, m] exp(i (k_l x + k_m z)).
// For each Chebyshev order n the Fourier sum at the targets is a type-2
// non-uniform FFT by Gaussian gridding (Dutt-Rokhlin, Greengard-Lee): with
// s = 2 pi x/Lx and g_tau(s) the periodised exp(-s^2/(4 tau)), whose Fourier
// coefficients are G_k = sqrt(tau/pi) exp(-k^2 tau),
//   1. deconvolve and zero-pad: h_hat[k] = u_hat[k] / G_k on the 2N-point grid;
//   2. inverse FFT of the padded spectrum (one plane per field and order);
//   3. at each target, (1/M) sum over the 2 msp nearest oversampled nodes S_j
//      of h(S_j) g_tau(s - S_j), in x and z,
// with tau = pi msp / (3 N^2), for which aliasing and window truncation
// errors are both about exp(-0.75 pi msp) (msp = 12: 5e-13; 6: 7e-7).  Then
// the Chebyshev sum in y (Clenshaw) gives the field, and the local part and
// the double layer's normal are combined as in the Lagrange path.
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
  int nt, Mx, Mz, Ny, msp;
  double Lx, Lz, H, tx, tz;
  const int* perm;
  const double *tx_, *ty, *tz_;   // sorted wrapped targets
  const void* tn;                 // sorted normals (T, SoA) for the double layer
  size_t tcap;
  const void* ul;                 // local part (kNearSlices x 3, T, SoA)
  const void* grid;               // [f][n][X][Z] T, the oversampled h
  double* out;                    // (nt, 3) in input order
};

// one thread per target: Gaussian window sums per field and order, then the
// Chebyshev sum in y by Clenshaw's recurrence, then the combination
template <typename T, bool STRESS>
__global__ void __launch_bounds__(256) spectral_eval(EvalArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nt) return;
  constexpr int NC = STRESS ? 6 : 3;
  constexpr double kTwoPi = 6.283185307179586477;
  const double x = a.tx_[t], y = a.ty[t], z = a.tz_[t];
  // window weights: the 2 msp oversampled nodes nearest to s in x and z
  const double sx = kTwoPi * x / a.Lx, sz = kTwoPi * z / a.Lz;
  const double hx = kTwoPi / a.Mx, hz = kTwoPi / a.Mz;
  const int ix0 = (int)floor(sx / hx) - a.msp + 1, iz0 = (int)floor(sz / hz) - a.msp + 1;
  double wx[2 * kMaxMsp], wz[2 * kMaxMsp];
  int ixs[2 * kMaxMsp], izs[2 * kMaxMsp];
  const int W = 2 * a.msp;
  for (int j = 0; j < W; ++j) {
    const double ddx = sx - (ix0 + j) * hx, ddz = sz - (iz0 + j) * hz;
    wx[j] = exp(-ddx * ddx / (4.0 * a.tx));
    wz[j] = exp(-ddz * ddz / (4.0 * a.tz));
    ixs[j] = ((ix0 + j) % a.Mx + a.Mx) % a.Mx;
    izs[j] = ((iz0 + j) % a.Mz + a.Mz) % a.Mz;
  }
  const T* G = (const T*)a.grid;
  const size_t plane = (size_t)a.Mx * a.Mz;
  const double yy = y / a.H;
  double val[NC];
  for (int c = 0; c < NC; ++c) {
    // Clenshaw: b_n = a_n + 2 yy b_{n+1} - b_{n+2} down to n = 1, then
    // sum_n a_n T_n(yy) = a_0 + yy b_1 - b_2
    double b1 = 0.0, b2 = 0.0, a0 = 0.0;
    for (int n = a.Ny - 1; n >= 0; --n) {
      const T* g = G + ((size_t)c * a.Ny + n) * plane;
      double an = 0.0;
      for (int i = 0; i < W; ++i) {
        const T* row = g + (size_t)ixs[i] * a.Mz;
        double r = 0.0;
        for (int k = 0; k < W; ++k) r = fma(wz[k], (double)row[izs[k]], r);
        an = fma(wx[i], r, an);
      }
      if (n > 0) {
        const double b0 = fma(2.0 * yy, b1, an - b2);
        b2 = b1;
        b1 = b0;
      } else {
        a0 = an;
      }
    }
    val[c] = a0 + yy * b1 - b2;
  }
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
    const T* tn = (const T*)a.tn;
    const double nx = tn[t], ny = tn[a.tcap + t], nz = tn[2 * a.tcap + t];
    res[0] += val[0] * nx + val[3] * ny + val[4] * nz;
    res[1] += val[3] * nx + val[1] * ny + val[5] * nz;
    res[2] += val[4] * nx + val[5] * ny + val[2] * nz;
  }
  const size_t o = 3 * (size_t)a.perm[t];
  a.out[o] = res[0];
  a.out[o + 1] = res[1];
  a.out[o + 2] = res[2];
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
  a.Ny = p.p.Ny;
  a.msp = p.msp;
  a.Lx = p.p.Lx;
  a.Lz = p.p.Lz;
  a.H = p.p.H;
  a.tx = p.tau_x;
  a.tz = p.tau_z;
  a.perm = p.tview->perm;
  a.tx_ = p.tview->x;
  a.ty = p.tview->y;
  a.tz_ = p.tview->z;
  a.tn = p.tnrm;
  a.tcap = (size_t)p.p.max_tgt;
  a.ul = p.ul;
  a.grid = p.over_phys;
  a.out = out;
  const unsigned nb = (unsigned)((nt + 255) / 256);
  if (stress) spectral_eval<T, true><<<nb, 256, 0, p.stream>>>(a);
  else spectral_eval<T, false><<<nb, 256, 0, p.stream>>>(a);
  return hipGetLastError();
}

template hipError_t launch_nufft_pad<double>(Plan&, int);
template hipError_t launch_nufft_pad<float>(Plan&, int);
template hipError_t launch_spectral_eval<double>(Plan&, int, double*, bool);
template hipError_t launch_spectral_eval<float>(Plan&, int, double*, bool);

}  // namespace ggem
