// Fourier transforms in the periodic directions (Eq. fourier, Appendix C).
// Physical fields are stored [plane][x][z] (z contiguous); spectra are
// [plane][l][m] with the half spectrum m = 0..Nz/2 contiguous.
//
//   forward:  real z-lines -> complex (R2C), then complex x-columns (C2C)
//   inverse:  complex x-columns (C2C), then Hermitian z-lines -> real (C2R)
//
// Each 1-D transform is a mixed-radix (2, 3, 4, 5, 8) Stockham autosort FFT
// in LDS with twiddles from a table computed once per plan in FP64 and staged
// in LDS.  The z transforms carry two real lines per complex line (one as the
// real part, one as the imaginary part) and separate the two spectra by their
// Hermitian symmetry.  The 1/(Nx Nz) normalisation of the forward transform
// is folded into the Chebyshev forward matrix.
#include "ggem_internal.h"

namespace ggem {

template <typename T>
struct Cx;
template <>
struct Cx<double> {
  using t = double2;
};
template <>
struct Cx<float> {
  using t = float2;
};

template <typename C>
__device__ inline C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ inline C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ inline C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}

// The passes of one transform length N: radix R, the product Ns of the
// earlier radices, the twiddle stride N / (Ns R), and multipliers for the
// index divisions by Ns and by N / R: q = (x m) >> 20 equals x / d exactly
// for m = ceil(2^20 / d) whenever x d < 2^20 (here x < 2N, d <= N <= 512).
struct Radices {
  int n;
  int r[12], ns[12], tstep[12], mns[12], mnr[12];
  unsigned long long mnr32[12];  // ceil(2^32 / (N/R)): exact for x < 2^17
};

__device__ inline int fdiv(int x, int m) { return (int)(((unsigned)x * (unsigned)m) >> 20); }
// x / d for 0 <= x < 2^17, d <= 1024, with m = ceil(2^32 / d)
__device__ inline int udiv32(int x, unsigned long long m) {
  return (int)(((unsigned long long)(unsigned)x * m) >> 32);
}

// In-register DFT of length R (2..5), sign -1 forward, +1 inverse.
template <typename T, int SIGN, int R>
__device__ inline void small_dft(typename Cx<T>::t* v) {
  using C = typename Cx<T>::t;
  if constexpr (R == 2) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    // multiply d13 by SIGN * i
    C jd;
    jd.x = -(T)SIGN * d13.y;
    jd.y = (T)SIGN * d13.x;
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, jd);
    v[3] = csub(d02, jd);
  } else if constexpr (R == 3) {
    const T c1 = (T)-0.5, s1 = (T)SIGN * (T)0.86602540378443864676;
    C y0 = cadd(v[0], cadd(v[1], v[2]));
    C t;
    t.x = v[0].x + c1 * (v[1].x + v[2].x);
    t.y = v[0].y + c1 * (v[1].y + v[2].y);
    C d = csub(v[1], v[2]);
    C y1, y2;
    y1.x = t.x - s1 * d.y;
    y1.y = t.y + s1 * d.x;
    y2.x = t.x + s1 * d.y;
    y2.y = t.y - s1 * d.x;
    v[0] = y0;
    v[1] = y1;
    v[2] = y2;
  } else if constexpr (R == 8) {
    // two 4-point DFTs (even, odd samples) joined by the twiddles w8^k
    C e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    small_dft<T, SIGN, 4>(e);
    small_dft<T, SIGN, 4>(o);
    const T h = (T)0.70710678118654752440;
    C t[4];
    t[0] = o[0];
    // w8^1 = h (1 + SIGN i)
    t[1].x = h * (o[1].x - (T)SIGN * o[1].y);
    t[1].y = h * (o[1].y + (T)SIGN * o[1].x);
    // w8^2 = SIGN i
    t[2].x = -(T)SIGN * o[2].y;
    t[2].y = (T)SIGN * o[2].x;
    // w8^3 = h (-1 + SIGN i)
    t[3].x = h * (-o[3].x - (T)SIGN * o[3].y);
    t[3].y = h * (-o[3].y + (T)SIGN * o[3].x);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], t[k]);
      v[k + 4] = csub(e[k], t[k]);
    }
  } else {  // R == 5
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)SIGN * (T)0.95105651629515357212, s2 = (T)SIGN * (T)0.58778525229247312917;
    C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    C y0 = cadd(v[0], cadd(a1, a2));
    C t1, t2;
    t1.x = v[0].x + c1 * a1.x + c2 * a2.x;
    t1.y = v[0].y + c1 * a1.y + c2 * a2.y;
    t2.x = v[0].x + c2 * a1.x + c1 * a2.x;
    t2.y = v[0].y + c2 * a1.y + c1 * a2.y;
    // i * (s1 b1 + s2 b2) and i * (s2 b1 - s1 b2)
    C u1, u2;
    u1.x = -(s1 * b1.y + s2 * b2.y);
    u1.y = s1 * b1.x + s2 * b2.x;
    u2.x = -(s2 * b1.y - s1 * b2.y);
    u2.y = s2 * b1.x - s1 * b2.x;
    v[0] = y0;
    v[1] = cadd(t1, u1);
    v[4] = csub(t1, u1);
    v[2] = cadd(t2, u2);
    v[3] = csub(t2, u2);
  }
}

// One butterfly of a Stockham pass over a line of length N with radix R
// (tw: exp(-2 pi i t/N), conjugated for the inverse).
template <typename T, int SIGN, int R>
__device__ inline void stockham_bfly(const typename Cx<T>::t* __restrict__ src,
                                     typename Cx<T>::t* __restrict__ dst, int NR, int Ns, int tstep,
                                     int mns, int j, const typename Cx<T>::t* __restrict__ tw) {
  using C = typename Cx<T>::t;
  const int q = fdiv(j, mns);
  const int k = j - q * Ns;
  C v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    C a = src[j + r * NR];
    if (r > 0 && k > 0) {
      C w = tw[k * r * tstep];
      if (SIGN > 0) w.y = -w.y;
      a = cmul(a, w);
    }
    v[r] = a;
  }
  small_dft<T, SIGN, R>(v);
  const int base = q * Ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
}

// Butterfly j (< N/R) of pass s of a line.
template <typename T, int SIGN>
__device__ inline void stockham_pass(const typename Cx<T>::t* __restrict__ src,
                                     typename Cx<T>::t* __restrict__ dst, int N,
                                     const Radices& rad, int s,
                                     const typename Cx<T>::t* __restrict__ tw, int j) {
  const int R = rad.r[s], NR = N / R, Ns = rad.ns[s], ts = rad.tstep[s], m = rad.mns[s];
  switch (R) {
    case 2: stockham_bfly<T, SIGN, 2>(src, dst, NR, Ns, ts, m, j, tw); break;
    case 3: stockham_bfly<T, SIGN, 3>(src, dst, NR, Ns, ts, m, j, tw); break;
    case 4: stockham_bfly<T, SIGN, 4>(src, dst, NR, Ns, ts, m, j, tw); break;
    case 8: stockham_bfly<T, SIGN, 8>(src, dst, NR, Ns, ts, m, j, tw); break;
    default: stockham_bfly<T, SIGN, 5>(src, dst, NR, Ns, ts, m, j, tw); break;
  }
}

// Wave-local LDS hand-off: the wave's own writes are visible to all its
// lanes after this (the z transforms keep each line within one wave).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The block's copy of a twiddle table (n entries) in LDS: every pass then
// reads its twiddles at LDS latency.
template <typename C>
__device__ inline void stage_twiddles(C* __restrict__ dst, const C* __restrict__ tw, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) dst[t] = tw[t];
  __syncthreads();
}

// The LPW lines of a wave: the butterflies of all of them are shared out
// over its 64 lanes, so short lines keep every lane busy.
template <typename T, int SIGN>
__device__ inline void wave_lines_fft(typename Cx<T>::t*& b0, typename Cx<T>::t*& b1, int N,
                                      int lpw, const Radices& rad,
                                      const typename Cx<T>::t* __restrict__ tw, int lane) {
  using C = typename Cx<T>::t;
  for (int s = 0; s < rad.n; ++s) {
    const int NR = N / rad.r[s];
    for (int w = lane; w < lpw * NR; w += 64) {
      const int l = fdiv(w, rad.mnr[s]), j = w - l * NR;
      stockham_pass<T, SIGN>(b0 + l * N, b1 + l * N, N, rad, s, tw, j);
    }
    wave_sync();
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
}

// Forward R2C along z: each wave owns LPW complex lines, each carrying two
// consecutive real lines a (real part) and b (imaginary part), 4 waves per
// block; LDS: the twiddles, then per wave two buffers of LPW lines.  With
// Z = FFT(a + i b): A_m = (Z_m + conj Z_{N-m}) / 2, B_m = (Z_m - conj Z_{N-m}) / 2i.
template <typename T>
__global__ void __launch_bounds__(256) fft_z_r2c(const T* __restrict__ in,
                                                 typename Cx<T>::t* __restrict__ out, int nlines,
                                                 int Nz, int lpw, Radices rz,
                                                 const typename Cx<T>::t* __restrict__ tw) {
  using C = typename Cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* twl = (C*)smem_raw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int line0 = (blockIdx.x * 4 + wave) * lpw * 2;  // first real line
  C* b0 = twl + Nz + wave * 2 * lpw * Nz;
  C* b1 = b0 + lpw * Nz;
  for (int l = 0; l < lpw; ++l) {
    const int ra = line0 + 2 * l, rb = ra + 1;
    for (int n = lane; n < Nz; n += 64) {
      C v;
      v.x = ra < nlines ? in[(size_t)ra * Nz + n] : (T)0;
      v.y = rb < nlines ? in[(size_t)rb * Nz + n] : (T)0;
      b0[l * Nz + n] = v;
    }
  }
  stage_twiddles(twl, tw, Nz);  // its barrier also publishes the lines
  wave_lines_fft<T, -1>(b0, b1, Nz, lpw, rz, twl, lane);
  const int Nzh = Nz / 2 + 1;
  for (int l = 0; l < lpw; ++l) {
    const int ra = line0 + 2 * l, rb = ra + 1;
    const C* z = b0 + l * Nz;
    for (int m = lane; m < Nzh; m += 64) {
      const C P = z[m], Qn = z[m == 0 ? 0 : Nz - m];
      // Q = conj(Z_{N-m})
      C A, B;
      A.x = (T)0.5 * (P.x + Qn.x);
      A.y = (T)0.5 * (P.y - Qn.y);
      B.x = (T)0.5 * (P.y + Qn.y);
      B.y = (T)0.5 * (Qn.x - P.x);
      if (ra < nlines) out[(size_t)ra * Nzh + m] = A;
      if (rb < nlines) out[(size_t)rb * Nzh + m] = B;
    }
  }
}

// Inverse C2R along z: two Hermitian lines A, B packed as Z = A + i B (the
// imaginary parts at m = 0 and m = N/2 dropped, as a real line's own C2R
// would), inverse FFT, real part -> line a, imaginary part -> line b.
template <typename T>
__global__ void __launch_bounds__(256) fft_z_c2r(const typename Cx<T>::t* __restrict__ in,
                                                 T* __restrict__ out, int nlines, int Nz, int lpw,
                                                 Radices rz,
                                                 const typename Cx<T>::t* __restrict__ tw) {
  using C = typename Cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* twl = (C*)smem_raw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int line0 = (blockIdx.x * 4 + wave) * lpw * 2;
  C* b0 = twl + Nz + wave * 2 * lpw * Nz;
  C* b1 = b0 + lpw * Nz;
  const int Nzh = Nz / 2 + 1;
  for (int l = 0; l < lpw; ++l) {
    const int ra = line0 + 2 * l, rb = ra + 1;
    for (int m = lane; m < Nz; m += 64) {
      const int mm = m < Nzh ? m : Nz - m;
      C A, B;
      A.x = A.y = B.x = B.y = (T)0;
      if (ra < nlines) A = in[(size_t)ra * Nzh + mm];
      if (rb < nlines) B = in[(size_t)rb * Nzh + mm];
      if (m == 0 || 2 * m == Nz) A.y = B.y = (T)0;
      if (m >= Nzh) {
        A.y = -A.y;
        B.y = -B.y;
      }
      C z;
      z.x = A.x - B.y;
      z.y = A.y + B.x;
      b0[l * Nz + m] = z;
    }
  }
  stage_twiddles(twl, tw, Nz);
  wave_lines_fft<T, 1>(b0, b1, Nz, lpw, rz, twl, lane);
  for (int l = 0; l < lpw; ++l) {
    const int ra = line0 + 2 * l, rb = ra + 1;
    for (int n = lane; n < Nz; n += 64) {
      const C z = b0[l * Nz + n];
      if (ra < nlines) out[(size_t)ra * Nz + n] = z.x;
      if (rb < nlines) out[(size_t)rb * Nz + n] = z.y;
    }
  }
}

// C2C along x on [plane][l][m] data, in place: CB columns per block, each
// column at stride Nx + 1 in LDS so the transposing loads and stores of
// consecutive columns fall in different banks.
template <typename T, int SIGN>
__global__ void __launch_bounds__(256) fft_x(typename Cx<T>::t* __restrict__ data, int Nx,
                                             int Nzh, int CB, Radices rx,
                                             const typename Cx<T>::t* __restrict__ tw) {
  using C = typename Cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* smem = (C*)smem_raw;
  const int plane = blockIdx.y;
  const int m0 = blockIdx.x * CB;
  const int NxP = Nx + 1;
  C* twl = smem;
  C* b0 = smem + Nx;
  C* b1 = b0 + CB * NxP;
  C* base = data + (size_t)plane * Nx * Nzh;
  for (int idx = threadIdx.x; idx < CB * Nx; idx += 256) {
    const int i = idx / CB, c = idx - (idx / CB) * CB;
    const int m = m0 + c;
    C v;
    v.x = (T)0;
    v.y = (T)0;
    if (m < Nzh) v = base[(size_t)i * Nzh + m];
    b0[c * NxP + i] = v;
  }
  stage_twiddles(twl, tw, Nx);
  for (int s = 0; s < rx.n; ++s) {
    const int NR = Nx / rx.r[s];
    // spread the CB lines' butterflies over the block
    for (int w = threadIdx.x; w < CB * NR; w += 256) {
      const int c = fdiv(w, rx.mnr[s]), j = w - c * NR;
      stockham_pass<T, SIGN>(b0 + c * NxP, b1 + c * NxP, Nx, rx, s, twl, j);
    }
    __syncthreads();
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  for (int idx = threadIdx.x; idx < CB * Nx; idx += 256) {
    const int i = idx / CB, c = idx - (idx / CB) * CB;
    const int m = m0 + c;
    if (m < Nzh) base[(size_t)i * Nzh + m] = b0[c * NxP + i];
  }
}

// Whole-plane transforms (planes whose two Nx x (Nz/2 + 1) complex buffers
// fit in LDS): one block of 1024 threads per plane does the z transforms and
// the x transforms with one read and one write of the plane.  Forward: the
// real rows 2l and 2l+1 form complex line l (real, imaginary part), the z
// FFTs run on the Nx/2 lines, the two spectra of each line are separated
// into the columns m = 0..Nz/2 (stored as lines of length Nx, stride Nx + 1),
// then the x FFTs run on those columns.  Inverse: the reverse order, with
// the two Hermitian rows recombined into one complex line before the z FFT.
struct Plane2 {
  int Nx, Nz, Nzh;
  unsigned long long mNz, mNzh;  // ceil(2^32 / Nz), ceil(2^32 / Nzh)
};

template <typename T>
__global__ void __launch_bounds__(1024) fft2_fwd(const T* __restrict__ in,
                                                 typename Cx<T>::t* __restrict__ out, Plane2 pl,
                                                 Radices rx, Radices rz,
                                                 const typename Cx<T>::t* __restrict__ twx,
                                                 const typename Cx<T>::t* __restrict__ twz) {
  using C = typename Cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  const int Nx = pl.Nx, Nz = pl.Nz, Nzh = pl.Nzh, NxP = Nx + 1, nl = Nx / 2;
  C* twxl = (C*)smem_raw;
  C* twzl = twxl + Nx;
  C* b0 = twzl + Nz;
  C* b1 = b0 + (size_t)Nzh * NxP;
  const int tid = threadIdx.x;
  const T* src = in + (size_t)blockIdx.x * Nx * Nz;
  for (int e = tid; e < Nx * Nz; e += 1024) {
    const int x = udiv32(e, pl.mNz), z = e - x * Nz;
    T* line = (T*)(b0 + (x >> 1) * Nz + z);
    line[x & 1] = src[e];
  }
  for (int t = tid; t < Nx; t += 1024) twxl[t] = twx[t];
  for (int t = tid; t < Nz; t += 1024) twzl[t] = twz[t];
  __syncthreads();
  for (int s = 0; s < rz.n; ++s) {
    const int NR = Nz / rz.r[s];
    for (int w = tid; w < nl * NR; w += 1024) {
      const int l = udiv32(w, rz.mnr32[s]), j = w - l * NR;
      stockham_pass<T, -1>(b0 + l * Nz, b1 + l * Nz, Nz, rz, s, twzl, j);
    }
    __syncthreads();
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  // separate the two rows of each line: A_m = (Z_m + conj Z_{N-m}) / 2,
  // B_m = (Z_m - conj Z_{N-m}) / 2i, into column m (stride NxP)
  for (int e = tid; e < nl * Nzh; e += 1024) {
    const int l = udiv32(e, pl.mNzh), m = e - l * Nzh;
    const C P = b0[l * Nz + m], Qn = b0[l * Nz + (m == 0 ? 0 : Nz - m)];
    C A, B;
    A.x = (T)0.5 * (P.x + Qn.x);
    A.y = (T)0.5 * (P.y - Qn.y);
    B.x = (T)0.5 * (P.y + Qn.y);
    B.y = (T)0.5 * (Qn.x - P.x);
    b1[m * NxP + 2 * l] = A;
    b1[m * NxP + 2 * l + 1] = B;
  }
  __syncthreads();
  {
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  for (int s = 0; s < rx.n; ++s) {
    const int NR = Nx / rx.r[s];
    for (int w = tid; w < Nzh * NR; w += 1024) {
      const int c = udiv32(w, rx.mnr32[s]), j = w - c * NR;
      stockham_pass<T, -1>(b0 + c * NxP, b1 + c * NxP, Nx, rx, s, twxl, j);
    }
    __syncthreads();
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  C* dst = out + (size_t)blockIdx.x * Nx * Nzh;
  for (int e = tid; e < Nx * Nzh; e += 1024) {
    const int l = udiv32(e, pl.mNzh), m = e - l * Nzh;
    dst[e] = b0[m * NxP + l];
  }
}

template <typename T>
__global__ void __launch_bounds__(1024) fft2_inv(const typename Cx<T>::t* __restrict__ in,
                                                 T* __restrict__ out, Plane2 pl, Radices rx,
                                                 Radices rz,
                                                 const typename Cx<T>::t* __restrict__ twx,
                                                 const typename Cx<T>::t* __restrict__ twz) {
  using C = typename Cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  const int Nx = pl.Nx, Nz = pl.Nz, Nzh = pl.Nzh, NxP = Nx + 1, nl = Nx / 2;
  C* twxl = (C*)smem_raw;
  C* twzl = twxl + Nx;
  C* b0 = twzl + Nz;
  C* b1 = b0 + (size_t)Nzh * NxP;
  const int tid = threadIdx.x;
  const C* src = in + (size_t)blockIdx.x * Nx * Nzh;
  for (int e = tid; e < Nx * Nzh; e += 1024) {
    const int l = udiv32(e, pl.mNzh), m = e - l * Nzh;
    b0[m * NxP + l] = src[e];
  }
  for (int t = tid; t < Nx; t += 1024) twxl[t] = twx[t];
  for (int t = tid; t < Nz; t += 1024) twzl[t] = twz[t];
  __syncthreads();
  for (int s = 0; s < rx.n; ++s) {
    const int NR = Nx / rx.r[s];
    for (int w = tid; w < Nzh * NR; w += 1024) {
      const int c = udiv32(w, rx.mnr32[s]), j = w - c * NR;
      stockham_pass<T, 1>(b0 + c * NxP, b1 + c * NxP, Nx, rx, s, twxl, j);
    }
    __syncthreads();
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  // rows 2l, 2l+1 as one complex line Z = A + i B over the full length,
  // A and B completed by Hermitian symmetry (imaginary parts dropped at
  // m = 0 and m = N/2)
  for (int e = tid; e < nl * Nz; e += 1024) {
    const int l = udiv32(e, pl.mNz), m = e - l * Nz;
    const int mm = m < Nzh ? m : Nz - m;
    C A = b0[mm * NxP + 2 * l], B = b0[mm * NxP + 2 * l + 1];
    if (m == 0 || 2 * m == Nz) A.y = B.y = (T)0;
    if (m >= Nzh) {
      A.y = -A.y;
      B.y = -B.y;
    }
    C z;
    z.x = A.x - B.y;
    z.y = A.y + B.x;
    b1[l * Nz + m] = z;
  }
  __syncthreads();
  {
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  for (int s = 0; s < rz.n; ++s) {
    const int NR = Nz / rz.r[s];
    for (int w = tid; w < nl * NR; w += 1024) {
      const int l = udiv32(w, rz.mnr32[s]), j = w - l * NR;
      stockham_pass<T, 1>(b0 + l * Nz, b1 + l * Nz, Nz, rz, s, twzl, j);
    }
    __syncthreads();
    C* t = b0;
    b0 = b1;
    b1 = t;
  }
  T* dst = out + (size_t)blockIdx.x * Nx * Nz;
  for (int e = tid; e < Nx * Nz; e += 1024) {
    const int x = udiv32(e, pl.mNz), z = e - x * Nz;
    const T* line = (const T*)(b0 + (x >> 1) * Nz + z);
    dst[e] = line[x & 1];
  }
}

static unsigned long long div_mult32(int d) {
  return (((unsigned long long)1 << 32) + (unsigned long long)d - 1) / (unsigned long long)d;
}

static size_t fft2_lds(int Nx, int Nz, size_t celt) {
  return ((size_t)Nx + Nz + 2 * (size_t)(Nz / 2 + 1) * (Nx + 1)) * celt;
}
constexpr size_t kFft2Lds = 150 * 1024;
// one block per plane pays a chain of passes per block: worth it only with
// enough planes to fill the device (the six wall planes use the line kernels)
constexpr int kFft2MinPlanes = 64;

static int div_mult(int d) { return (int)(((1u << 20) + (unsigned)d - 1) / (unsigned)d); }

static Radices radices(const int* r, int n, int N) {
  Radices R;
  R.n = n;
  int ns = 1;
  for (int i = 0; i < 12; ++i) {
    R.r[i] = i < n ? r[i] : 1;
    R.ns[i] = ns;
    R.tstep[i] = N / (ns * R.r[i]);
    R.mns[i] = div_mult(ns);
    R.mnr[i] = div_mult(N / R.r[i]);
    R.mnr32[i] = div_mult32(N / R.r[i]);
    if (i < n) ns *= r[i];
  }
  return R;
}

// columns per block of the x transform: ping-pong buffers of <= 64 KB, and
// the butterfly index CB N/R below 2048 (exact multiply-shift division)
static int cols_per_block(int Nx, size_t elt, const Radices& rx) {
  int cb = (int)(32768 / ((size_t)(Nx + 1) * elt));
  if (cb < 1) cb = 1;
  if (cb > 16) cb = 16;
  int nrmax = 1;
  for (int s = 0; s < rx.n; ++s) nrmax = Nx / rx.r[s] > nrmax ? Nx / rx.r[s] : nrmax;
  while (cb > 1 && cb * nrmax >= 2048) --cb;
  return cb;
}

// lines per wave of the z transforms (LDS of a block stays within 80 KB)
static int lines_per_wave(int Nz, size_t celt) { return (Nz + 8 * 2 * Nz) * celt <= 81920 ? 2 : 1; }

static size_t fft_z_lds(int Nz, int lpw, size_t celt) { return (size_t)(Nz + 8 * lpw * Nz) * celt; }
static size_t fft_x_lds(int Nx, int CB, size_t celt) { return (size_t)(Nx + 2 * CB * (Nx + 1)) * celt; }

template <typename T>
hipError_t launch_fft_forward(Plan& p, void* phys, void* spec, int nplanes) {
  using C = typename Cx<T>::t;
  const int Nx = p.p.Nx, Nz = p.p.Nz, Nzh = p.Nzh;
  const int nlines = nplanes * Nx;
  Radices rz = radices(p.radz, p.nradz, Nz), rx = radices(p.radx, p.nradx, Nx);
  if (nplanes >= kFft2MinPlanes && fft2_lds(Nx, Nz, sizeof(C)) <= kFft2Lds) {
    const Plane2 pl{Nx, Nz, Nzh, div_mult32(Nz), div_mult32(Nzh)};
    fft2_fwd<T><<<nplanes, 1024, fft2_lds(Nx, Nz, sizeof(C)), p.stream>>>(
        (const T*)phys, (C*)spec, pl, rx, rz, (const C*)p.twx, (const C*)p.twz);
    return hipGetLastError();
  }
  const int lpw = lines_per_wave(Nz, sizeof(C));
  const int lpb = 8 * lpw;  // real lines per block
  fft_z_r2c<T><<<(nlines + lpb - 1) / lpb, 256, fft_z_lds(Nz, lpw, sizeof(C)), p.stream>>>(
      (const T*)phys, (C*)spec, nlines, Nz, lpw, rz, (const C*)p.twz);
  const int CB = cols_per_block(Nx, sizeof(C), rx);
  dim3 g((Nzh + CB - 1) / CB, nplanes);
  fft_x<T, -1><<<g, 256, fft_x_lds(Nx, CB, sizeof(C)), p.stream>>>((C*)spec, Nx, Nzh, CB, rx,
                                                                   (const C*)p.twx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_inverse(Plan& p, void* spec, void* phys, int nplanes) {
  using C = typename Cx<T>::t;
  const int Nx = p.p.Nx, Nz = p.p.Nz, Nzh = p.Nzh;
  const int nlines = nplanes * Nx;
  Radices rz = radices(p.radz, p.nradz, Nz), rx = radices(p.radx, p.nradx, Nx);
  if (nplanes >= kFft2MinPlanes && fft2_lds(Nx, Nz, sizeof(C)) <= kFft2Lds) {
    const Plane2 pl{Nx, Nz, Nzh, div_mult32(Nz), div_mult32(Nzh)};
    fft2_inv<T><<<nplanes, 1024, fft2_lds(Nx, Nz, sizeof(C)), p.stream>>>(
        (const C*)spec, (T*)phys, pl, rx, rz, (const C*)p.twx, (const C*)p.twz);
    return hipGetLastError();
  }
  const int CB = cols_per_block(Nx, sizeof(C), rx);
  dim3 g((Nzh + CB - 1) / CB, nplanes);
  fft_x<T, 1><<<g, 256, fft_x_lds(Nx, CB, sizeof(C)), p.stream>>>((C*)spec, Nx, Nzh, CB, rx,
                                                                  (const C*)p.twx);
  const int lpw = lines_per_wave(Nz, sizeof(C));
  const int lpb = 8 * lpw;  // real lines per block
  fft_z_c2r<T><<<(nlines + lpb - 1) / lpb, 256, fft_z_lds(Nz, lpw, sizeof(C)), p.stream>>>(
      (const C*)spec, (T*)phys, nlines, Nz, lpw, rz, (const C*)p.twz);
  return hipGetLastError();
}

template hipError_t launch_fft_forward<double>(Plan&, void*, void*, int);
template hipError_t launch_fft_forward<float>(Plan&, void*, void*, int);
template hipError_t launch_fft_inverse<double>(Plan&, void*, void*, int);
template hipError_t launch_fft_inverse<float>(Plan&, void*, void*, int);

}  // namespace ggem
