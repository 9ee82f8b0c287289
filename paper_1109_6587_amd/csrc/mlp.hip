// Learned warm start of the Fredholm solve: a per-node network
//   13 -> 128 -> 128 -> 128 -> 3, SiLU on the hidden layers,
// trained by mean squared error with Adam.  Not in the paper (its warm start
// is the previous stage's density, Sec. 5); the plain warm start stays the
// fallback (ggem_fredholm_solve_guided).
//
// Every product runs on the matrix cores as v_mfma_f32_16x16x16_bf16:
// bfloat16 operands (input, weights, pre-activations, activations and the
// back-propagated gradients), FP32 accumulation, FP32 biases, FP32 master
// weights and Adam moments.  Samples are stored sample-major ([sample][unit]),
// weights row-major ([out][in]), all in one packed FP32 vector
// (W1, b1, W2, b2, W3, b3, W4, b4).  Sums over samples (weight and bias
// gradients, the loss) are split into fixed chunks whose partial results are
// added in a fixed order: results do not depend on scheduling.
#include <math.h>
#include <string.h>

#include <new>

#include "ggem_internal.h"

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kL = 4;
constexpr int kDim[kL + 1] = {GGEM_MLP_IN, GGEM_MLP_HIDDEN, GGEM_MLP_HIDDEN, GGEM_MLP_HIDDEN,
                              GGEM_MLP_OUT};
constexpr int kChunk = 1024;  // samples per split of a sum over samples

__host__ __device__ constexpr int w_off(int l) {
  return l == 0 ? 0 : w_off(l - 1) + kDim[l - 1] * kDim[l] + kDim[l];
}
__host__ __device__ constexpr int b_off(int l) { return w_off(l) + kDim[l] * kDim[l + 1]; }
static_assert(w_off(kL) == GGEM_MLP_PARAMS, "packed parameter count");

__device__ inline unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

enum Epi { kF32 = 0, kHidden = 1, kBack = 2 };

// C (M x N) = A (M x K) B (K x N) over k in [z kchunk, (z+1) kchunk), with
// element (m, k) of A at A[m am + k ak] and (k, n) of B at B[k bk + n bn].
struct GemmArgs {
  int M, N, K, kchunk;
  const unsigned short* A;
  long am, ak;
  const unsigned short* B;
  long bk, bn;
  const float* bias;          // [M] (kF32, kHidden) or null
  float* C;                   // kF32: C[z cz + m cm + n cn]
  long cm, cn, cz;
  unsigned short* Zo;         // kHidden: bf16(z); kBack: bf16(dz)
  unsigned short* Ho;         // kHidden: bf16(silu(z))
  const unsigned short* Zin;  // kBack: the pre-activation whose silu' scales
  long om, on;                // layout of Zo, Ho, Zin
};

// Block: 4 waves, a 64 x 64 output tile, each wave 32 x 32 (2 x 2 MFMA tiles).
// Fragments (16 x 16 x 16): lane l holds A[m0 + l%16][k0 + 4(l/16) + i] and
// B[k0 + 4(l/16) + i][n0 + l%16] (i = 0..3); the accumulator holds
// D[4(l/16) + v][l%16] (v = 0..3).  Out-of-range rows, columns and k are
// zero-filled.
template <int EPI>
__global__ void __launch_bounds__(256) gemm_bf16(GemmArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int kb = blockIdx.z * a.kchunk;
  const int ke = min(a.K, kb + a.kchunk);
  const int li = lane & 15, lk = (lane >> 4) * 4;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f4)0.0f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    s4 fa[2], fb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int m = m0 + 16 * t + li;
      const int n = n0 + 16 * t + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + lk + i;
        fa[t][i] = (m < a.M && k < ke) ? (short)a.A[m * a.am + k * a.ak] : (short)0;
        fb[t][i] = (n < a.N && k < ke) ? (short)a.B[k * a.bk + n * a.bn] : (short)0;
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[i], fb[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + 16 * i + (lane >> 4) * 4 + v;
        const int n = n0 + 16 * j + li;
        if (m >= a.M || n >= a.N) continue;
        const float s = acc[i][j][v];
        if (EPI == kF32) {
          a.C[blockIdx.z * a.cz + m * a.cm + n * a.cn] = a.bias ? s + a.bias[m] : s;
        } else if (EPI == kHidden) {
          const float z = s + a.bias[m];
          const long o = m * a.om + n * a.on;
          a.Zo[o] = f2bf(z);
          a.Ho[o] = f2bf(z * sigmoid(z));
        } else {
          const long o = m * a.om + n * a.on;
          const float z = bf2f(a.Zin[o]);
          const float sg = sigmoid(z);
          a.Zo[o] = f2bf(s * sg * (1.0f + z * (1.0f - sg)));
        }
      }
}

__global__ void to_bf16(long n, const float* __restrict__ x, unsigned short* __restrict__ y) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// dY = bf16(2 (Y - T) / (3 n)); per-block partial sums of (Y - T)^2
__global__ void __launch_bounds__(256) loss_grad(int n, const float* __restrict__ Y,
                                                 const float* __restrict__ T, float inv,
                                                 unsigned short* __restrict__ dY,
                                                 float* __restrict__ part) {
  __shared__ float red[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float s = 0.0f;
  if (i < 3 * n) {
    const float d = Y[i] - T[i];
    dY[i] = f2bf(2.0f * d * inv);
    s = d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = inv * sum of part[0..np) (one block, fixed order)
__global__ void __launch_bounds__(256) sum_final(int np, const float* __restrict__ part,
                                                 float inv, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * inv;
}

// part[z][o] = sum over the samples of chunk z of dZ[s][o].  A block takes
// 64 columns of one chunk: each of its waves sums 64 consecutive samples
// with 16 loads in flight per lane, and the wave sums are added in wave
// order through LDS, so the result does not depend on timing.
constexpr int kColWaves = kChunk / 64;
static_assert(kChunk % 64 == 0 && kColWaves <= 16, "one block of at most 1024 threads per chunk");

__global__ void __launch_bounds__(64 * kColWaves) colsum_partial(int n, int m,
                                                                 const unsigned short* __restrict__ dZ,
                                                                 float* __restrict__ part) {
  __shared__ float red[kColWaves][64];
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + c;
  const long r0 = (long)blockIdx.y * kChunk + (long)w * 64;
  const long r1 = min((long)n, r0 + 64);
  float acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0f;
  if (o < m) {
    for (long i = r0; i < r1; i += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (i + u < r1) acc[u] += bf2f(dZ[(i + u) * m + o]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += acc[u];
  red[w][c] = s;
  __syncthreads();
  if (w == 0 && o < m) {
    float t = 0.0f;
    for (int k = 0; k < kColWaves; ++k) t += red[k][c];
    part[(long)blockIdx.y * m + o] = t;
  }
}

// dst[i] = sum_z part[z stride + i], z ascending
__global__ void reduce_splits(int count, int splits, const float* __restrict__ part, long stride,
                              float* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += part[z * stride + i];
  dst[i] = s;
}

__global__ void adam_update(int np, float* __restrict__ P, const float* __restrict__ G,
                            float* __restrict__ Mm, float* __restrict__ Vv,
                            unsigned short* __restrict__ Pb, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float g = G[i];
  const float m = b1 * Mm[i] + (1.0f - b1) * g;
  const float v = b2 * Vv[i] + (1.0f - b2) * g * g;
  Mm[i] = m;
  Vv[i] = v;
  const float w = P[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
  P[i] = w;
  Pb[i] = f2bf(w);
}

// per-drop centroid of its nodes (consecutive groups of npd nodes)
__global__ void __launch_bounds__(256) drop_centroid(int npd, const double* __restrict__ x,
                                                     double* __restrict__ cen) {
  __shared__ double red[3][256];
  const long base = (long)blockIdx.x * npd;
  double s[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < npd; i += 256)
    for (int d = 0; d < 3; ++d) s[d] += x[3 * (base + i) + d];
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = s[d];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) cen[3 * blockIdx.x + d] = red[d][0] / npd;
}

struct Scales {
  float s[GGEM_MLP_IN];
};

// X[i] = scaled (x - centroid, n, -(Lap x . n), q_prev, dq_prev)
__global__ void node_features(int n, int npd, const double* __restrict__ x,
                              const double* __restrict__ nrm, const double* __restrict__ lap,
                              const double* __restrict__ qp, const double* __restrict__ dqp,
                              const double* __restrict__ cen, Scales sc, float* __restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d0 = i / npd;
  double f[GGEM_MLP_IN];
  double c = 0.0;
  for (int d = 0; d < 3; ++d) {
    f[d] = x[3 * (long)i + d] - cen[3 * d0 + d];
    f[3 + d] = nrm[3 * (long)i + d];
    c -= lap[3 * (long)i + d] * nrm[3 * (long)i + d];
    f[7 + d] = qp[3 * (long)i + d];
    f[10 + d] = dqp[3 * (long)i + d];
  }
  f[6] = c;
  for (int k = 0; k < GGEM_MLP_IN; ++k) X[(long)i * GGEM_MLP_IN + k] = (float)(sc.s[k] * f[k]);
}

__global__ void scale_out(long n3, const float* __restrict__ Y, double s, double* __restrict__ dq) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n3) dq[i] = s * (double)Y[i];
}

__global__ void copy_f32(int n, const float* __restrict__ a, float* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void zero_f32(int n, float* __restrict__ a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

}  // namespace

struct ggem_mlp_s {
  hipStream_t stream;
  int max_batch;
  int steps;
  float *P, *G, *Mm, *Vv;
  unsigned short* Pb;
  unsigned short* H0;
  unsigned short *Z[3], *H[3], *dZ[3];
  unsigned short* dY;
  float *Y, *part, *lpart, *loss;
  float* loss_host;
  double* cen;
};

static thread_local char g_mlp_err[256];

#define MLP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      snprintf(g_mlp_err, sizeof g_mlp_err, "%s: %s", #expr, hipGetErrorString(e_));    \
      return ggem_set_error(GGEM_E_DEVICE, g_mlp_err);                                  \
    }                                                                                   \
  } while (0)

static unsigned nblk(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static int splits_of(int n) { return (n + kChunk - 1) / kChunk; }

static void free_mlp(ggem_mlp_s* m) {
  void* ptrs[] = {m->P,    m->G,     m->Mm,    m->Vv,    m->Pb,   m->H0,    m->Z[0],
                  m->Z[1], m->Z[2],  m->H[0],  m->H[1],  m->H[2], m->dZ[0], m->dZ[1],
                  m->dZ[2], m->dY,   m->Y,     m->part,  m->lpart, m->loss, m->cen};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (m->loss_host) (void)hipHostFree(m->loss_host);
}

extern "C" int ggem_mlp_create(int max_batch, void* hip_stream, ggem_mlp_t* out) {
  if (!out) return ggem_set_error(GGEM_E_ARG, "null output");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 24))
    return ggem_set_error(GGEM_E_ARG, "max_batch must be in 1..2^24");
  ggem_mlp_s* m = new (std::nothrow) ggem_mlp_s();
  if (!m) return ggem_set_error(GGEM_E_NOMEM, "host allocation failed");
  memset(m, 0, sizeof *m);
  m->stream = (hipStream_t)hip_stream;
  m->max_batch = max_batch;
  const size_t P = GGEM_MLP_PARAMS, nb = (size_t)max_batch, Hd = GGEM_MLP_HIDDEN;
  const size_t sp = (size_t)splits_of(max_batch);
  bool ok = hipMalloc((void**)&m->P, P * 4) == hipSuccess &&
            hipMalloc((void**)&m->G, P * 4) == hipSuccess &&
            hipMalloc((void**)&m->Mm, P * 4) == hipSuccess &&
            hipMalloc((void**)&m->Vv, P * 4) == hipSuccess &&
            hipMalloc((void**)&m->Pb, P * 2) == hipSuccess &&
            hipMalloc((void**)&m->H0, nb * GGEM_MLP_IN * 2) == hipSuccess &&
            hipMalloc((void**)&m->dY, nb * GGEM_MLP_OUT * 2) == hipSuccess &&
            hipMalloc((void**)&m->Y, nb * GGEM_MLP_OUT * 4) == hipSuccess &&
            hipMalloc((void**)&m->part, sp * Hd * Hd * 4) == hipSuccess &&
            hipMalloc((void**)&m->lpart, nblk(3 * nb) * 4) == hipSuccess &&
            hipMalloc((void**)&m->loss, 4) == hipSuccess &&
            hipMalloc((void**)&m->cen, nb * 3 * 8) == hipSuccess &&
            hipHostMalloc((void**)&m->loss_host, 4, 0) == hipSuccess;
  for (int l = 0; l < 3 && ok; ++l)
    ok = hipMalloc((void**)&m->Z[l], nb * Hd * 2) == hipSuccess &&
         hipMalloc((void**)&m->H[l], nb * Hd * 2) == hipSuccess &&
         hipMalloc((void**)&m->dZ[l], nb * Hd * 2) == hipSuccess;
  if (!ok) {
    free_mlp(m);
    delete m;
    return ggem_set_error(GGEM_E_NOMEM, "device allocation failed");
  }
  *out = m;
  return GGEM_OK;
}

extern "C" int ggem_mlp_destroy(ggem_mlp_t m) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null network");
  (void)hipStreamSynchronize(m->stream);
  free_mlp(m);
  delete m;
  return GGEM_OK;
}

extern "C" int ggem_mlp_set_params(ggem_mlp_t m, const float* params) {
  if (!m || !params) return ggem_set_error(GGEM_E_ARG, "null argument");
  const int P = GGEM_MLP_PARAMS;
  copy_f32<<<nblk(P), 256, 0, m->stream>>>(P, params, m->P);
  to_bf16<<<nblk(P), 256, 0, m->stream>>>(P, m->P, m->Pb);
  zero_f32<<<nblk(P), 256, 0, m->stream>>>(P, m->Mm);
  zero_f32<<<nblk(P), 256, 0, m->stream>>>(P, m->Vv);
  m->steps = 0;
  MLP_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_mlp_get_params(ggem_mlp_t m, float* params) {
  if (!m || !params) return ggem_set_error(GGEM_E_ARG, "null argument");
  copy_f32<<<nblk(GGEM_MLP_PARAMS), 256, 0, m->stream>>>(GGEM_MLP_PARAMS, m->P, params);
  MLP_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_mlp_features(ggem_mlp_t m, long long n_nodes, const double* nodes,
                                 const double* normals, const double* lap, const double* q_prev,
                                 const double* dq_prev, int nodes_per_drop, const float* scales,
                                 float* X) {
  if (!m) return ggem_set_error(GGEM_E_ARG, "null network");
  if (n_nodes < 1 || n_nodes > m->max_batch)
    return ggem_set_error(GGEM_E_CAPACITY, "node count outside 1..max_batch");
  if (nodes_per_drop < 1 || n_nodes % nodes_per_drop)
    return ggem_set_error(GGEM_E_ARG, "nodes_per_drop must divide the node count");
  if (!nodes || !normals || !lap || !q_prev || !dq_prev || !scales || !X)
    return ggem_set_error(GGEM_E_ARG, "null array");
  Scales sc;
  for (int k = 0; k < GGEM_MLP_IN; ++k) sc.s[k] = scales[k];
  const int n = (int)n_nodes;
  drop_centroid<<<n / nodes_per_drop, 256, 0, m->stream>>>(nodes_per_drop, nodes, m->cen);
  node_features<<<nblk(n), 256, 0, m->stream>>>(n, nodes_per_drop, nodes, normals, lap, q_prev,
                                                dq_prev, m->cen, sc, X);
  MLP_TRY(hipGetLastError());
  return GGEM_OK;
}

static void launch_gemm(int epi, const GemmArgs& a, hipStream_t st) {
  const int splits = (a.K + a.kchunk - 1) / a.kchunk;
  dim3 grid(nblk(a.N, 64), nblk(a.M, 64), splits < 1 ? 1 : splits);
  if (epi == kF32) gemm_bf16<kF32><<<grid, 256, 0, st>>>(a);
  else if (epi == kHidden) gemm_bf16<kHidden><<<grid, 256, 0, st>>>(a);
  else gemm_bf16<kBack><<<grid, 256, 0, st>>>(a);
}

// z_l = W_l h_{l-1} + b_l for the n samples; Y (FP32) = the output layer
static void forward(ggem_mlp_s* m, int n, const float* X) {
  hipStream_t st = m->stream;
  to_bf16<<<nblk((long)n * GGEM_MLP_IN), 256, 0, st>>>((long)n * GGEM_MLP_IN, X, m->H0);
  const unsigned short* h = m->H0;
  for (int l = 0; l < kL; ++l) {
    GemmArgs a;
    memset(&a, 0, sizeof a);
    a.M = kDim[l + 1];
    a.N = n;
    a.K = kDim[l];
    a.kchunk = a.K;
    a.A = m->Pb + w_off(l);   // W_l (out x in), row-major
    a.am = kDim[l];
    a.ak = 1;
    a.B = h;                  // h (in x n) from [n][in]
    a.bk = 1;
    a.bn = kDim[l];
    a.bias = m->P + b_off(l);
    if (l < kL - 1) {
      a.Zo = m->Z[l];
      a.Ho = m->H[l];
      a.om = 1;
      a.on = kDim[l + 1];
      launch_gemm(kHidden, a, st);
      h = m->H[l];
    } else {
      a.C = m->Y;
      a.cm = 1;
      a.cn = kDim[l + 1];
      launch_gemm(kF32, a, st);
    }
  }
}

// gradients of the mean squared error into m->G, the loss into m->loss
static void backward(ggem_mlp_s* m, int n, const float* T) {
  hipStream_t st = m->stream;
  const int n3 = 3 * n;
  const unsigned nb3 = nblk(n3);
  loss_grad<<<nb3, 256, 0, st>>>(n, m->Y, T, 1.0f / (float)n3, m->dY, m->lpart);
  sum_final<<<1, 256, 0, st>>>((int)nb3, m->lpart, 1.0f / (float)n3, m->loss);
  const int splits = splits_of(n);
  const unsigned short* dz = m->dY;
  for (int l = kL - 1; l >= 0; --l) {
    const int out = kDim[l + 1], in = kDim[l];
    const unsigned short* h = l == 0 ? m->H0 : m->H[l - 1];
    // dW_l = dz (out x n) h^T (n x in), split over samples
    GemmArgs a;
    memset(&a, 0, sizeof a);
    a.M = out;
    a.N = in;
    a.K = n;
    a.kchunk = kChunk;
    a.A = dz;
    a.am = 1;
    a.ak = out;
    a.B = h;
    a.bk = in;
    a.bn = 1;
    a.C = m->part;
    a.cm = in;
    a.cn = 1;
    a.cz = (long)out * in;
    launch_gemm(kF32, a, st);
    reduce_splits<<<nblk(out * in), 256, 0, st>>>(out * in, splits, m->part, (long)out * in,
                                                  m->G + w_off(l));
    colsum_partial<<<dim3(nblk(out, 64), splits), 64 * kColWaves, 0, st>>>(n, out, dz, m->part);
    reduce_splits<<<nblk(out), 256, 0, st>>>(out, splits, m->part, out, m->G + b_off(l));
    if (l == 0) break;
    // dz_{l-1} = (W_l^T dz) * silu'(z_{l-1})
    GemmArgs b;
    memset(&b, 0, sizeof b);
    b.M = in;
    b.N = n;
    b.K = out;
    b.kchunk = out;
    b.A = m->Pb + w_off(l);   // W^T: element (i, o) at W[o in + i]
    b.am = 1;
    b.ak = in;
    b.B = dz;                 // (o, s) at dz[s out + o]
    b.bk = 1;
    b.bn = out;
    b.Zo = m->dZ[l - 1];
    b.Zin = m->Z[l - 1];
    b.om = 1;
    b.on = in;
    launch_gemm(kBack, b, st);
    dz = m->dZ[l - 1];
  }
}

static int check_batch(ggem_mlp_s* m, long long n) {
  if (n < 1 || n > m->max_batch)
    return ggem_set_error(GGEM_E_CAPACITY, "batch size outside 1..max_batch");
  return GGEM_OK;
}

static int read_loss(ggem_mlp_s* m, float* loss) {
  if (!loss) return GGEM_OK;
  MLP_TRY(hipMemcpyAsync(m->loss_host, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
  MLP_TRY(hipStreamSynchronize(m->stream));
  *loss = *m->loss_host;
  return GGEM_OK;
}

extern "C" int ggem_mlp_forward(ggem_mlp_t m, long long n, const float* X, float* Y) {
  if (!m || !X || !Y) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (int rc = check_batch(m, n)) return rc;
  forward(m, (int)n, X);
  copy_f32<<<nblk(3 * n), 256, 0, m->stream>>>((int)(3 * n), m->Y, Y);
  MLP_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_mlp_predict(ggem_mlp_t m, long long n, const float* X, double scale,
                                double* dq) {
  if (!m || !X || !dq) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (int rc = check_batch(m, n)) return rc;
  forward(m, (int)n, X);
  scale_out<<<nblk(3 * n), 256, 0, m->stream>>>(3 * n, m->Y, scale, dq);
  MLP_TRY(hipGetLastError());
  return GGEM_OK;
}

extern "C" int ggem_mlp_gradients(ggem_mlp_t m, long long n, const float* X, const float* T,
                                  float* grads, float* loss) {
  if (!m || !X || !T) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (int rc = check_batch(m, n)) return rc;
  forward(m, (int)n, X);
  backward(m, (int)n, T);
  if (grads) copy_f32<<<nblk(GGEM_MLP_PARAMS), 256, 0, m->stream>>>(GGEM_MLP_PARAMS, m->G, grads);
  MLP_TRY(hipGetLastError());
  return read_loss(m, loss);
}

extern "C" int ggem_mlp_train_step(ggem_mlp_t m, long long n, const float* X, const float* T,
                                   float lr, float* loss) {
  if (!m || !X || !T) return ggem_set_error(GGEM_E_ARG, "null argument");
  if (int rc = check_batch(m, n)) return rc;
  if (!(lr > 0) || !isfinite(lr)) return ggem_set_error(GGEM_E_ARG, "lr must be positive");
  forward(m, (int)n, X);
  backward(m, (int)n, T);
  const double b1 = 0.9, b2 = 0.999;
  m->steps += 1;
  const float c1 = (float)(1.0 / (1.0 - pow(b1, m->steps)));
  const float c2 = (float)(1.0 / (1.0 - pow(b2, m->steps)));
  adam_update<<<nblk(GGEM_MLP_PARAMS), 256, 0, m->stream>>>(GGEM_MLP_PARAMS, m->P, m->G, m->Mm,
                                                            m->Vv, m->Pb, lr, (float)b1,
                                                            (float)b2, 1e-8f, c1, c2);
  MLP_TRY(hipGetLastError());
  return read_loss(m, loss);
}
