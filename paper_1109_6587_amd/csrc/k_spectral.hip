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
// errors are both about exp(-0.75 pi msp) (msp = 12: 5e-13; 6: 7e-7).  The
// window sums of every Chebyshev order, weighted by T_n(y/H), give the field;
// the local part and the double layer's normal are combined as in the
// Lagrange path.  An FP32 grid is first transposed to [field][X][Z][n] with a
// periodic halo in Z, so that each window row is one contiguous run read in
// 16-byte vectors (spectral_eval_t); an FP64 grid is gathered plane by plane
// (spectral_eval).
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
  int per;                        // 4-target tiles per XCD
  double Lx, Lz, H, tx, tz;
  const int* perm;
  const double *tx_, *ty, *tz_;   // sorted wrapped targets
  const void* tn;                 // sorted normals (T, SoA) for the double layer
  size_t tcap;
  const void* ul;                 // local part (kNearSlices x 3, T, SoA)
  const void* grid;               // [f][n][X][Z] T, the oversampled h
  double* out;                    // (nt, 3) in input order
};

// One wave per target.  The W x W window (W = 2 msp) is flattened over the
// 64 lanes, E entries per lane (W^2 <= 64 E): consecutive lanes read
// consecutive z nodes of a row, so each load of a plane is a few contiguous
// runs.  Each lane keeps its entries' weights wx_i wz_k and offsets, sums
// its part of the window sum of every plane, and accumulates those against
// T_n(y/H) (the three-term recurrence); a wave reduction per field ends it.
// Block b serves 4-target tile (b mod 8) per + b/8, so that each XCD walks
// a contiguous run of the cell-sorted targets and their windows overlap in
// its L2.
template <typename T, bool STRESS, int E>
__global__ void __launch_bounds__(256) spectral_eval(EvalArgs a) {
  const int tile = (int)(blockIdx.x & 7) * a.per + (int)(blockIdx.x >> 3);
  const int t = tile * 4 + (int)(threadIdx.x >> 6);
  if (t >= a.nt) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  constexpr int NC = STRESS ? 6 : 3;
  constexpr double kTwoPi = 6.283185307179586477;
  const double sx = kTwoPi * a.tx_[t] / a.Lx, sz = kTwoPi * a.tz_[t] / a.Lz;
  const double yy = a.ty[t] / a.H;
  const double hx = kTwoPi / a.Mx, hz = kTwoPi / a.Mz;
  const int W = 2 * a.msp;
  // lane j < W: weight and node of the j-th window point in x and in z
  double wxl = 0.0, wzl = 0.0;
  int ixl = 0, izl = 0;
  if (lane < W) {
    const int ix = (int)floor(sx / hx) - a.msp + 1 + lane;
    const int iz = (int)floor(sz / hz) - a.msp + 1 + lane;
    const double dx = sx - ix * hx, dz = sz - iz * hz;
    wxl = exp(-dx * dx / (4.0 * a.tx));
    wzl = exp(-dz * dz / (4.0 * a.tz));
    ixl = ix < 0 ? ix + a.Mx : (ix >= a.Mx ? ix - a.Mx : ix);
    izl = iz < 0 ? iz + a.Mz : (iz >= a.Mz ? iz - a.Mz : iz);
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
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  double tm1 = 0.0, tn = 1.0;  // T_{n-1}, T_n
  for (int n = 0; n < a.Ny; ++n) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T* g = G + ((size_t)c * a.Ny + n) * plane;
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) s = fma(w[e], (double)g[off[e]], s);
      acc[c] = fma(tn, s, acc[c]);
    }
    const double tp = n == 0 ? yy : 2.0 * yy * tn - tm1;
    tm1 = tn;
    tn = tp;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
    for (int m = 32; m >= 1; m >>= 1) acc[c] += __shfl_xor(acc[c], m);
  if (lane != 0) return;
  const T* ul = (const T*)a.ul;
  double res[3];
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    for (int s = 0; s < kNearSlices; ++s) v += (double)ul[(size_t)(3 * s + c) * a.tcap + t];
    res[c] = v;
  }
  if (!STRESS) {
    for (int c = 0; c < 3; ++c) res[c] += acc[c];
  } else {
    const T* tnr = (const T*)a.tn;
    const double nx = tnr[t], ny = tnr[a.tcap + t], nz = tnr[2 * a.tcap + t];
    res[0] += acc[0] * nx + acc[3] * ny + acc[4] * nz;
    res[1] += acc[3] * nx + acc[1] * ny + acc[5] * nz;
    res[2] += acc[4] * nx + acc[5] * ny + acc[2] * nz;
  }
  const size_t o = 3 * (size_t)a.perm[t];
  a.out[o] = res[0];
  a.out[o + 1] = res[1];
  a.out[o + 2] = res[2];
}

// [f][n][X][Z] -> [f][X][Z + halo][n]: the n (Chebyshev) values of a grid
// node become contiguous, padded with zeros to nyp, and Z runs on past the
// period by the window width (periodic copy), so that a target's window row
// is one contiguous run.  A block moves 32 Z nodes of one (field, X) through
// LDS (reads contiguous in Z, writes contiguous in n).
struct TransArgs {
  int Mx, Mz, Ny, nyp, zp;
  const void* in;
  void* out;
};

template <typename T>
__global__ void __launch_bounds__(256) nufft_transpose(TransArgs a) {
  __shared__ T tile[kMaxNy][33];
  const int z0 = blockIdx.x * 32, X = blockIdx.y, f = blockIdx.z;
  const T* in = (const T*)a.in;
  for (int q = threadIdx.x; q < a.Ny * 32; q += 256) {
    const int n = q >> 5, zl = q & 31;
    int z = z0 + zl;
    if (z < a.zp) {
      z = z >= a.Mz ? z - a.Mz : z;
      tile[n][zl] = in[(((size_t)f * a.Ny + n) * a.Mx + X) * a.Mz + z];
    }
  }
  __syncthreads();
  T* out = (T*)a.out + (((size_t)f * a.Mx + X) * a.zp + z0) * a.nyp;
  const int nz = min(32, a.zp - z0);
  for (int q = threadIdx.x; q < nz * a.nyp; q += 256) {
    const int zl = q / a.nyp, n = q - zl * a.nyp;
    out[q] = n < a.Ny ? tile[n][zl] : (T)0;
  }
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using t = double2;
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  using t = float4;
  static constexpr int n = 4;
};

__device__ inline double vget(const double2& v, int i) { return i == 0 ? v.x : v.y; }
__device__ inline double vget(const float4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

struct EvalTArgs {
  int nt, Mx, Mz, Ny, msp, nyp, zp, per;
  double Lx, Lz, H, tx, tz;
  const int* perm;
  const double *tx_, *ty, *tz_;
  const void* tn;
  size_t tcap;
  const void* ul;
  const void* grid;   // [f][X][zp][nyp] T
  double* out;
};

// One wave per target over the transposed grid.  A window row (fixed X) is
// the contiguous run of W z nodes times nyp orders; lanes read it in 16-byte
// vectors, S per lane, and each lane keeps the weight wz_k T_n(y/H) of its
// S V run positions (k, n).  Per field: sum over the W rows of wx_i times the
// lane's weighted run sum, then one wave reduction.
template <typename T, bool STRESS, int S>
__global__ void __launch_bounds__(256) spectral_eval_t(EvalTArgs a) {
  using VT = typename Vec16<T>::t;
  constexpr int V = Vec16<T>::n;
  const int tile = (int)(blockIdx.x & 7) * a.per + (int)(blockIdx.x >> 3);
  const int t = tile * 4 + (int)(threadIdx.x >> 6);
  if (t >= a.nt) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  constexpr int NC = STRESS ? 6 : 3;
  constexpr double kTwoPi = 6.283185307179586477;
  const double sx = kTwoPi * a.tx_[t] / a.Lx, sz = kTwoPi * a.tz_[t] / a.Lz;
  const double yy = fmin(1.0, fmax(-1.0, a.ty[t] / a.H));
  const double hx = kTwoPi / a.Mx, hz = kTwoPi / a.Mz;
  const int W = 2 * a.msp;
  const int iz0 = (int)floor(sz / hz) - a.msp + 1;
  const int izw = iz0 < 0 ? iz0 + a.Mz : (iz0 >= a.Mz ? iz0 - a.Mz : iz0);
  double wxl = 0.0, wzl = 0.0;
  int ixl = 0;
  if (lane < W) {
    const int ix = (int)floor(sx / hx) - a.msp + 1 + lane;
    const double dx = sx - ix * hx, dz = sz - (iz0 + lane) * hz;
    wxl = exp(-dx * dx / (4.0 * a.tx));
    wzl = exp(-dz * dz / (4.0 * a.tz));
    ixl = ix < 0 ? ix + a.Mx : (ix >= a.Mx ? ix - a.Mx : ix);
  }
  // T_n(y/H) = cos(n arccos(y/H)) for n = lane and lane + 64
  const double th = acos(yy);
  const double tlo = cos(lane * th), thi = cos((lane + 64) * th);
  T w[S][V];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = (lane + 64 * s) * V + v;
      const int k = p / a.nyp, n = p - k * a.nyp;
      const double wk = __shfl(wzl, min(k, 63));
      const double t0 = __shfl(tlo, n & 63), t1 = __shfl(thi, n & 63);
      w[s][v] = (T)((k < W && n < a.Ny) ? wk * (n < 64 ? t0 : t1) : 0.0);
    }
  const T* G = (const T*)a.grid;
  double val[NC];
  for (int c = 0; c < NC; ++c) {
    double acc = 0.0;
    for (int i = 0; i < W; ++i) {
      const int xi = __shfl(ixl, i);
      const double wxi = __shfl(wxl, i);
      const VT* row = (const VT*)(G + (((size_t)c * a.Mx + xi) * a.zp + izw) * a.nyp);
      double r = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const VT g = row[lane + 64 * s];
#pragma unroll
        for (int v = 0; v < V; ++v) r = fma((double)w[s][v], (double)vget(g, v), r);
      }
      acc = fma(wxi, r, acc);
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

template <typename T, int S>
void launch_eval_t(const EvalTArgs& a, unsigned nb, bool stress, hipStream_t st) {
  if (stress) spectral_eval_t<T, true, S><<<nb, 256, 0, st>>>(a);
  else spectral_eval_t<T, false, S><<<nb, 256, 0, st>>>(a);
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
hipError_t launch_nufft_transpose(Plan& p, int nf) {
  if constexpr (sizeof(T) != 4) return hipErrorInvalidValue;  // FP32 grids only
  TransArgs a;
  a.Mx = 2 * p.p.Nx;
  a.Mz = 2 * p.p.Nz;
  a.Ny = p.p.Ny;
  a.nyp = p.over_nyp;
  a.zp = p.over_zp;
  a.in = p.over_phys;
  a.out = p.over_t;
  nufft_transpose<T><<<dim3((unsigned)((a.zp + 31) / 32), (unsigned)a.Mx, (unsigned)nf), 256, 0,
                       p.stream>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spectral_eval(Plan& p, int nt, double* out, bool stress) {
  if (nt <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (p.over_s) {
      EvalTArgs a;
      a.nt = nt;
      a.Mx = 2 * p.p.Nx;
      a.Mz = 2 * p.p.Nz;
      a.Ny = p.p.Ny;
      a.msp = p.msp;
      a.nyp = p.over_nyp;
      a.zp = p.over_zp;
      const int tiles = (nt + 3) / 4;
      a.per = (tiles + 7) / 8;
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
      a.grid = p.over_t;
      a.out = out;
      const unsigned nb = 8u * (unsigned)a.per;
      switch (p.over_s) {
        case 2: launch_eval_t<T, 2>(a, nb, stress, p.stream); break;
        case 4: launch_eval_t<T, 4>(a, nb, stress, p.stream); break;
        case 8: launch_eval_t<T, 8>(a, nb, stress, p.stream); break;
        default: launch_eval_t<T, 16>(a, nb, stress, p.stream); break;
      }
      return hipGetLastError();
    }
  }
  EvalArgs a;
  a.nt = nt;
  a.Mx = 2 * p.p.Nx;
  a.Mz = 2 * p.p.Nz;
  a.Ny = p.p.Ny;
  a.msp = p.msp;
  const int tiles = (nt + 3) / 4;
  a.per = (tiles + 7) / 8;
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
template hipError_t launch_nufft_transpose<double>(Plan&, int);
template hipError_t launch_nufft_transpose<float>(Plan&, int);
template hipError_t launch_spectral_eval<double>(Plan&, int, double*, bool);
template hipError_t launch_spectral_eval<float>(Plan&, int, double*, bool);

}  // namespace ggem
