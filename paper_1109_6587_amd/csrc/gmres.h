// Restarted GMRES(m) on the device (Sec. 5: the paper solves its boundary
// integral systems iteratively with GMRES).  Krylov vectors, dot products and
// norms in FP64 with fixed-order reductions; classical Gram-Schmidt applied
// twice; the small Hessenberg problem (Givens rotations) on the host.  Every
// cycle starts from, and the solve stops on, the true residual b - A x (the
// Arnoldi estimate can be optimistic when the products carry FP32 rounding).
//
// Shared by the Fredholm solver and the rigid-particle solver; each supplies
// the product A x as a callable and owns the workspace.
#pragma once

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ggem_internal.h"

namespace ggem {
namespace gm {

constexpr int kDotBlock = 256;
constexpr int kDotBlocks = 256;

// part[i][b] = sum over block b's range of V_i . w  (fixed order)
static __global__ void __launch_bounds__(kDotBlock) dots_partial(int n, const double* __restrict__ V,
                                                                 size_t ldv,
                                                                 const double* __restrict__ w,
                                                                 double* __restrict__ part) {
  __shared__ double red[kDotBlock];
  const int i = blockIdx.y;
  const double* vi = V + (size_t)i * ldv;
  double s = 0.0;
  for (int j = blockIdx.x * kDotBlock + threadIdx.x; j < n; j += kDotBlocks * kDotBlock)
    s = fma(vi[j], w[j], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kDotBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)i * kDotBlocks + blockIdx.x] = red[0];
}

static __global__ void __launch_bounds__(kDotBlock) dots_final(const double* __restrict__ part,
                                                               double* __restrict__ out) {
  __shared__ double red[kDotBlock];
  const int i = blockIdx.x;
  red[threadIdx.x] = part[(size_t)i * kDotBlocks + threadIdx.x];
  __syncthreads();
  for (int o = kDotBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// w += sign * sum_i c_i V_i
static __global__ void multi_axpy(int n, int k, const double* __restrict__ V, size_t ldv,
                                  const double* __restrict__ c, double sign,
                                  double* __restrict__ w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s = fma(c[i], V[(size_t)i * ldv + j], s);
  w[j] = fma(sign, s, w[j]);
}

static __global__ void scale_copy(int n, double a, const double* __restrict__ x,
                                  double* __restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) y[j] = a * x[j];
}

static __global__ void sub_into(int n, const double* __restrict__ b, const double* __restrict__ ax,
                                double* __restrict__ r) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) r[j] = b[j] - ax[j];
}

// Device workspace of one solver: (m + 1) Krylov vectors of stride ldv, two
// work vectors, reduction partials, coefficients; a pinned host buffer for
// the dot products.
struct Work {
  double *V, *w, *r, *part, *dots, *coef, *dots_host;
  size_t ldv;
  int m;  // restart length
  hipStream_t st;
};

inline int device_error(hipError_t e, const char* what) {
  static thread_local char msg[256];
  snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
  return ggem_set_error(GGEM_E_DEVICE, msg);
}

#define GM_TRY(expr)                                         \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return gm::device_error(e_, #expr); \
  } while (0)

inline int alloc_work(Work& W, size_t n, int m) {
  memset(&W, 0, sizeof W);
  W.ldv = n;
  W.m = m;
  const size_t m1 = (size_t)m + 1;
  const bool ok = hipMalloc((void**)&W.V, m1 * n * 8) == hipSuccess &&
                  hipMalloc((void**)&W.w, n * 8) == hipSuccess &&
                  hipMalloc((void**)&W.r, n * 8) == hipSuccess &&
                  hipMalloc((void**)&W.part, m1 * kDotBlocks * 8) == hipSuccess &&
                  hipMalloc((void**)&W.dots, m1 * 8) == hipSuccess &&
                  hipMalloc((void**)&W.coef, m1 * 8) == hipSuccess &&
                  hipHostMalloc((void**)&W.dots_host, m1 * 8, 0) == hipSuccess;
  return ok ? GGEM_OK : ggem_set_error(GGEM_E_NOMEM, "device allocation failed");
}

inline void free_work(Work& W) {
  void* ptrs[] = {W.V, W.w, W.r, W.part, W.dots, W.coef};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (W.dots_host) (void)hipHostFree(W.dots_host);
  memset(&W, 0, sizeof W);
}

// k dot products V_i . w (V_i at stride ldv), returned on the host
inline int dots(Work& W, const double* V, size_t ldv, int k, const double* w, int n,
                double* host) {
  dots_partial<<<dim3(kDotBlocks, k), kDotBlock, 0, W.st>>>(n, V, ldv, w, W.part);
  dots_final<<<k, kDotBlock, 0, W.st>>>(W.part, W.dots);
  GM_TRY(hipMemcpyAsync(W.dots_host, W.dots, k * 8, hipMemcpyDeviceToHost, W.st));
  GM_TRY(hipStreamSynchronize(W.st));
  memcpy(host, W.dots_host, k * 8);
  return GGEM_OK;
}

// x += c * p on the device, c a host scalar (the copy is complete before return)
inline int axpy_host(Work& W, int n, double c, const double* p, double* x) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  GM_TRY(hipMemcpyAsync(W.coef, &c, 8, hipMemcpyHostToDevice, W.st));
  multi_axpy<<<nb, 256, 0, W.st>>>(n, 1, p, 0, W.coef, 1.0, x);
  GM_TRY(hipStreamSynchronize(W.st));  // c lives on the caller's stack
  return GGEM_OK;
}

// Solve A x = b from the guess in x.  apply(p, y) computes y = A p (device
// vectors of length n); first(r) may reduce the first residual r (in place,
// updating x to match) before the Krylov cycles start.  Returns the number of
// products A p made inside the cycles and the final relative residual.
template <class Apply, class First>
int solve(Work& W, int n, const double* b, double* x, double tol, int max_iter, Apply apply,
          First first, int* iters, double* rel_res) {
  const int m = W.m;
  const size_t ldv = W.ldv;
  const unsigned nb = (unsigned)((n + 255) / 256);
  double bnorm2;
  if (int rc = dots(W, b, 0, 1, b, n, &bnorm2)) return rc;
  const double bnorm = sqrt(bnorm2);
  if (bnorm == 0.0) {
    scale_copy<<<nb, 256, 0, W.st>>>(n, 0.0, b, x);
    GM_TRY(hipStreamSynchronize(W.st));
    if (iters) *iters = 0;
    if (rel_res) *rel_res = 0.0;
    return GGEM_OK;
  }
  std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 1), h2(m + 1), y(m);
  int total = 0;
  double res = 0.0;
  bool is_first = true;
  for (;;) {
    if (int rc = apply(x, W.w)) return rc;
    sub_into<<<nb, 256, 0, W.st>>>(n, b, W.w, W.r);
    if (is_first) {
      if (int rc = first(W.r)) return rc;
      is_first = false;
    }
    double beta2;
    if (int rc = dots(W, W.r, 0, 1, W.r, n, &beta2)) return rc;
    const double beta = sqrt(beta2);
    res = beta / bnorm;
    if (res <= tol || total >= max_iter) break;
    scale_copy<<<nb, 256, 0, W.st>>>(n, 1.0 / beta, W.r, W.V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    for (; j < m && total < max_iter; ++j) {
      ++total;
      double* Vj = W.V + (size_t)j * ldv;
      if (int rc = apply(Vj, W.w)) return rc;
      // classical Gram-Schmidt, twice
      if (int rc = dots(W, W.V, ldv, j + 1, W.w, n, h.data())) return rc;
      GM_TRY(hipMemcpyAsync(W.coef, h.data(), (j + 1) * 8, hipMemcpyHostToDevice, W.st));
      multi_axpy<<<nb, 256, 0, W.st>>>(n, j + 1, W.V, ldv, W.coef, -1.0, W.w);
      if (int rc = dots(W, W.V, ldv, j + 1, W.w, n, h2.data())) return rc;
      GM_TRY(hipMemcpyAsync(W.coef, h2.data(), (j + 1) * 8, hipMemcpyHostToDevice, W.st));
      multi_axpy<<<nb, 256, 0, W.st>>>(n, j + 1, W.V, ldv, W.coef, -1.0, W.w);
      for (int i = 0; i <= j; ++i) h[i] += h2[i];
      double wn2;
      if (int rc = dots(W, W.w, 0, 1, W.w, n, &wn2)) return rc;
      h[j + 1] = sqrt(wn2);
      if (h[j + 1] > 0.0)
        scale_copy<<<nb, 256, 0, W.st>>>(n, 1.0 / h[j + 1], W.w, W.V + (size_t)(j + 1) * ldv);
      // Givens rotations on the new Hessenberg column
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double den = hypot(h[j], h[j + 1]);
      if (!(den > 0)) break;  // A V_j = 0 within the basis: keep the j columns so far
      cs[j] = h[j] / den;
      sn[j] = h[j + 1] / den;
      h[j] = den;
      h[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) Hm[(size_t)i * m + j] = h[i];
      if (fabs(g[j + 1]) / bnorm <= tol) {
        ++j;
        break;
      }
    }
    // x += V y with H y = g (upper triangular, j columns)
    const int k = j;
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= Hm[(size_t)i * m + l] * y[l];
      y[i] = t / Hm[(size_t)i * m + i];
    }
    if (k > 0) {
      GM_TRY(hipMemcpyAsync(W.coef, y.data(), k * 8, hipMemcpyHostToDevice, W.st));
      multi_axpy<<<nb, 256, 0, W.st>>>(n, k, W.V, ldv, W.coef, 1.0, x);
      GM_TRY(hipGetLastError());
    }
  }
  if (iters) *iters = total;
  if (rel_res) *rel_res = res;
  return GGEM_OK;
}

}  // namespace gm
}  // namespace ggem
