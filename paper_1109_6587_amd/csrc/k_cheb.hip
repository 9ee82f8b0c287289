// Chebyshev transforms in y as dense GEMMs on the matrix cores.
//
// Forward (Gauss-Lobatto values -> coefficients, Sec. 3.2.2):
//   a_n = 2/(N cbar_n) sum_j u_j cos(pi n j/N)/cbar_j,  cbar_0 = cbar_N = 2,
// scaled here by 1/(Nx Nz) (the DFT normalisation).  Inverse:
//   u_j = sum_n a_n cos(pi n j/N).
// The paper evaluates these with FFTs; at N_y <= 129 a dense (Ny x Ny) times
// (Ny x columns) product is cheap on MFMA and keeps the data in one pass.
//
// Data: [field][row][col] with col over the real view of the half spectrum
// (2 * Nx * Nzh reals per row).  Block: 4 waves, each wave two 16-column
// tiles and every 16-row tile of the (padded) output; A fragments come from a
// zero-padded copy of the matrix (MP x KP), B fragments straight from HBM.
#include "ggem_internal.h"

namespace ggem {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMaxRowTiles = 9;   // Ny <= 129 -> 144 padded rows
constexpr int kColTiles = 2;      // column tiles per wave

__device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  using t = d4;
};
template <>
struct Acc<float> {
  using t = f4;
};

// out[f][r][c] = sum_k A[r][k] in[f][k][c] for k < Kin, r < Mout; A is
// zero padded to KP columns and to whole 16-row tiles; blockIdx.z takes the
// rows from 16 RT blockIdx.z on (one z block when Mout <= 16 RT).
template <typename T, int RT>
__global__ void __launch_bounds__(256) cheb_gemm(const T* __restrict__ A, int KP, int Kin, int Mout,
                                                 const T* __restrict__ in, T* __restrict__ out,
                                                 long ncols) {
  using V = typename Acc<T>::t;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = blockIdx.z * 16 * RT;
  const T* src = in + blockIdx.y * (size_t)Kin * ncols;
  T* dst = out + blockIdx.y * (size_t)Mout * ncols;
  A += (size_t)r0 * KP;
  const long col0 = (long)blockIdx.x * (4 * 16 * kColTiles) + wave * 16 * kColTiles;
  const int li = lane & 15, lk = lane >> 4;
  V acc[RT][kColTiles];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) acc[t][c] = (V)0;
  for (int kk = 0; kk < KP; kk += 4) {
    const int k = kk + lk;
    T b[kColTiles];
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) {
      const long col = col0 + c * 16 + li;
      b[c] = (k < Kin && col < ncols) ? src[(size_t)k * ncols + col] : (T)0;
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const T a = A[(size_t)(t * 16 + li) * KP + k];
#pragma unroll
      for (int c = 0; c < kColTiles; ++c) acc[t][c] = mfma16x16x4(a, b[c], acc[t][c]);
    }
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) {
      const long col = col0 + c * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // accumulator layout: FP32 16x16x4 holds rows 4*(lane/16)+v of column
        // lane%16; FP64 16x16x4 holds rows lane/16 + 4*v.
        const int row = r0 + t * 16 + (sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v);
        if (row < Mout && col < ncols) dst[(size_t)row * ncols + col] = acc[t][c][v];
      }
    }
}

// ---- BF16 hi + lo split products (precision GGEM_MIXED_BF16) --------------
//
// out = A in with A = A_hi + A_lo and in = B_hi + B_lo split into bfloat16
// pairs (hi = round-to-nearest-even of the value, lo = that of the
// remainder), evaluated as A_hi B_hi + A_hi B_lo + A_lo B_hi on the
// 16x16x32 BF16 matrix cores with FP32 accumulation (the A_lo B_lo term and
// the split remainders are below 2^-16 of each product).  The matrix halves
// are plan constants ([MP][KP32] row-major, zero padded); the data is split
// as it is loaded.  Lane l of a 16x16x32 product supplies row (A) or column
// (B) l % 16 at k = 8 (l / 16) .. 8 (l / 16) + 7 and receives rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - __uint_as_float((unsigned)hi << 16));
}

template <int RT>
__global__ void __launch_bounds__(256) cheb_gemm_bf16(const unsigned short* __restrict__ Ahi,
                                                      const unsigned short* __restrict__ Alo,
                                                      int KP32, int Ny,
                                                      const float* __restrict__ in,
                                                      float* __restrict__ out, long ncols) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t fstride = (size_t)Ny * ncols;
  const float* src = in + blockIdx.y * fstride;
  float* dst = out + blockIdx.y * fstride;
  const long col0 = (long)blockIdx.x * (4 * 16 * kColTiles) + wave * 16 * kColTiles;
  const int li = lane & 15, lk = lane >> 4;
  f4 acc[RT][kColTiles];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) acc[t][c] = (f4)0;
  for (int k0 = 0; k0 < KP32; k0 += 32) {
    // this lane's eight rows k0 + 8 lk .. + 7 of its columns, split
    u16x8 bh[kColTiles], bl[kColTiles];
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) {
      const long col = col0 + c * 16 + li;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + 8 * lk + i;
        const float v = (k < Ny && col < ncols) ? src[(size_t)k * ncols + col] : 0.0f;
        unsigned short h, l;
        split_bf16(v, h, l);
        bh[c][i] = h;
        bl[c][i] = l;
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const size_t ai = (size_t)(t * 16 + li) * KP32 + k0 + 8 * lk;
      const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const u16x8*)(Ahi + ai));
      const bf16x8 al = __builtin_bit_cast(bf16x8, *(const u16x8*)(Alo + ai));
#pragma unroll
      for (int c = 0; c < kColTiles; ++c) {
        const bf16x8 b_h = __builtin_bit_cast(bf16x8, bh[c]);
        const bf16x8 b_l = __builtin_bit_cast(bf16x8, bl[c]);
        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b_h, acc[t][c], 0, 0, 0);
        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b_l, acc[t][c], 0, 0, 0);
        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b_h, acc[t][c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) {
      const long col = col0 + c * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = t * 16 + 4 * lk + v;
        if (row < Ny && col < ncols) dst[(size_t)row * ncols + col] = acc[t][c][v];
      }
    }
}

static hipError_t launch_cheb_bf16(Plan& p, const void* in, void* out, int nfields,
                                   bool forward) {
  const int Ny = p.p.Ny;
  const int MP = ((Ny + 15) / 16) * 16;
  const int KP32 = ((Ny + 31) / 32) * 32;
  const long ncols = 2L * p.p.Nx * p.Nzh;
  const unsigned short* Ahi = forward ? p.cf_hi : p.ci_hi;
  const unsigned short* Alo = forward ? p.cf_lo : p.ci_lo;
  dim3 grid((unsigned)((ncols + 4 * 16 * kColTiles - 1) / (4 * 16 * kColTiles)), nfields);
  switch (MP / 16) {
#define GGEM_CASE(R)                                                                    \
  case R:                                                                               \
    cheb_gemm_bf16<R><<<grid, 256, 0, p.stream>>>(Ahi, Alo, KP32, Ny, (const float*)in, \
                                                  (float*)out, ncols);                  \
    break;
    GGEM_CASE(1)
    GGEM_CASE(2)
    GGEM_CASE(3)
    GGEM_CASE(4)
    GGEM_CASE(5)
    GGEM_CASE(6)
    GGEM_CASE(7)
    GGEM_CASE(8)
    GGEM_CASE(9)
#undef GGEM_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cheb(Plan& p, const void* in, void* out, int nfields, bool forward) {
  if (sizeof(T) == 4 && p.bf16) return launch_cheb_bf16(p, in, out, nfields, forward);
  const int Ny = p.p.Ny;
  const int MP = ((Ny + 15) / 16) * 16;
  const int KP = ((Ny + 3) / 4) * 4;
  const long ncols = 2L * p.p.Nx * p.Nzh;
  const T* A;
  if (sizeof(T) == 8) A = (const T*)(forward ? (const void*)p.cf64 : (const void*)p.ci64);
  else A = (const T*)(forward ? (const void*)p.cf32 : (const void*)p.ci32);
  dim3 grid((unsigned)((ncols + 4 * 16 * kColTiles - 1) / (4 * 16 * kColTiles)), nfields);
  const int rt = MP / 16;
  switch (rt) {
#define GGEM_CASE(R)                                                                            \
  case R:                                                                                       \
    cheb_gemm<T, R><<<grid, 256, 0, p.stream>>>(A, KP, Ny, Ny, (const T*)in, (T*)out, ncols); \
    break;
    GGEM_CASE(1)
    GGEM_CASE(2)
    GGEM_CASE(3)
    GGEM_CASE(4)
    GGEM_CASE(5)
    GGEM_CASE(6)
    GGEM_CASE(7)
    GGEM_CASE(8)
    GGEM_CASE(9)
#undef GGEM_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// out[f][r][c] = sum_k A[r][k] in[f][k][c], r < Mout, k < Kin, c < ncols
// real columns; A row-major with KP columns and rows padded to a multiple
// of 144 (nine 16-row tiles per block row).
template <typename T>
hipError_t launch_row_gemm(Plan& p, const T* A, int KP, int Kin, int Mout, const void* in,
                           void* out, long ncols, int nfields) {
  const unsigned zb = (unsigned)((Mout + 16 * kMaxRowTiles - 1) / (16 * kMaxRowTiles));
  const int rt = Mout <= 16 * kMaxRowTiles ? (Mout + 15) / 16 : kMaxRowTiles;
  dim3 grid((unsigned)((ncols + 4 * 16 * kColTiles - 1) / (4 * 16 * kColTiles)), nfields, zb);
  switch (rt) {
#define GGEM_CASE(R)                                                                      \
  case R:                                                                                 \
    cheb_gemm<T, R><<<grid, 256, 0, p.stream>>>(A, KP, Kin, Mout, (const T*)in, (T*)out, \
                                                ncols);                                   \
    break;
    GGEM_CASE(1)
    GGEM_CASE(2)
    GGEM_CASE(3)
    GGEM_CASE(4)
    GGEM_CASE(5)
    GGEM_CASE(6)
    GGEM_CASE(7)
    GGEM_CASE(8)
    GGEM_CASE(9)
#undef GGEM_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_row_gemm<double>(Plan&, const double*, int, int, int, const void*,
                                            void*, long, int);
template hipError_t launch_row_gemm<float>(Plan&, const float*, int, int, int, const void*, void*,
                                           long, int);
template hipError_t launch_cheb<double>(Plan&, const void*, void*, int, bool);
template hipError_t launch_cheb<float>(Plan&, const void*, void*, int, bool);

}  // namespace ggem
