// Interpolation of the global solution to the targets with 4th-order
// Lagrange polynomials, 5 nodes per axis (Sec. 3.2.2: error ~ h^5), and the
// local + global combination (Eq. tot_l_g; Eq. vsigma for the double layer).
//
// Stencil: x nodes i0-2..i0+2 (periodic) with i0 = floor(x/dx + 1/2), z
// likewise; y nodes j0-2..j0+2 of the Gauss-Lobatto grid with
// j0 = clamp(rint(arccos(y/H) (Ny-1)/pi), 2, Ny-3).  Indices and weights are
// formed in FP64 from FP64 positions in both precision modes; the sums run in
// the grid's precision, each stencil row's five z nodes first, then times the
// row's x-y weight.
#include "ggem_internal.h"

namespace ggem {

struct InterpArgs {
  int nt, Nx, Nz, Ny;
  double dx, dz, H;
  const double* y;
  const int* perm;
  const double *tx, *ty, *tz;
  const void* tn;      // sorted normals (T, SoA) for the double layer
  size_t tcap;
  const void* ul;      // local part at sorted targets (kNearSlices x 3 components, T, SoA)
  const void* grid;    // [ncomp][Ny][Nx][Nz] T
  double* out;         // (nt, 3) in input order
};

// G lanes per target (G = 1, 4 or 16, more when there are few targets):
// lane r of a target's group takes the stencil rows (y, x) = r, r + G, ...
// of the 25 rows of 5 contiguous z nodes, and the group adds its partial
// sums in a fixed tree order.  Weights and stencil indices are recomputed by
// every lane of the group from the same FP64 position, so they are identical
// across the group.
template <typename T, bool STRESS, bool GLOBAL, int kGrp>
__global__ void __launch_bounds__(256) interp_combine(InterpArgs a) {
  __shared__ double ly[kMaxNy];
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = gid / kGrp, r = gid % kGrp;
  const bool valid = t < a.nt;
  constexpr int NC = STRESS ? 6 : 3;
  // the Gauss-Lobatto nodes once per block, so the stencil's y nodes come
  // from LDS rather than a global load that waits for the stencil index
  if (GLOBAL) {
    for (int j = threadIdx.x; j < a.Ny; j += blockDim.x) ly[j] = a.y[j];
    __syncthreads();
  }
  // the local part and the output slot, loaded before the gathers so that
  // their latency overlaps them
  const T* ul = (const T*)a.ul;
  double res[3] = {0.0, 0.0, 0.0};
  int slot = 0;
  if (valid && r == 0) {
    slot = a.perm[t];
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int s = 0; s < kNearSlices; ++s) v += (double)ul[(size_t)(3 * s + c) * a.tcap + t];
      res[c] = v;
    }
  }
  T acc[NC];
  for (int c = 0; c < NC; ++c) acc[c] = (T)0;
  if (GLOBAL && valid) {
    const double x = a.tx[t], y = a.ty[t], z = a.tz[t];
    const double fx = floor(x / a.dx + 0.5), fz = floor(z / a.dz + 0.5);
    double wx[5], wz[5], wy[5], ny[5];
    lagrange5_uniform(x / a.dx - fx, wx);
    lagrange5_uniform(z / a.dz - fz, wz);
    const int N = a.Ny - 1;
    int j0 = (int)rint(acos(y / a.H) * N / 3.141592653589793);
    j0 = j0 < 2 ? 2 : (j0 > a.Ny - 3 ? a.Ny - 3 : j0);
    for (int q = 0; q < 5; ++q) ny[q] = ly[j0 - 2 + q];
    lagrange5(y, ny, wy);
    const int i0 = (int)fx, k0 = (int)fz;
    // k0 - 2 + q lies in [-2, Nz + 2] (z in [0, Lz)) and Nz >= 8: one wrap
    int kk[5];
    for (int q = 0; q < 5; ++q) kk[q] = wrap1(k0 - 2 + q, a.Nz);
    const T* g = (const T*)a.grid;
    const size_t fs = (size_t)a.Ny * a.Nx * a.Nz;
    T tz[5];
    for (int q = 0; q < 5; ++q) tz[q] = (T)wz[q];
    for (int row = r; row < 25; row += kGrp) {
      const int qa = row / 5, qb = row % 5;
      const int ii = wrap1(i0 - 2 + qb, a.Nx);
      const size_t base = ((size_t)(j0 - 2 + qa) * a.Nx + ii) * a.Nz;
      const T wab = (T)(wy[qa] * wx[qb]);
      // the row's five z nodes first, then its x-y weight
      for (int c = 0; c < NC; ++c) {
        const T* gc = g + c * fs + base;
        T zr = tz[0] * gc[kk[0]];
        for (int qc = 1; qc < 5; ++qc) zr = fma(tz[qc], gc[kk[qc]], zr);
        acc[c] = fma(wab, zr, acc[c]);
      }
    }
  }
  // fixed-order reduction over the group (lanes r and r + o, o = 8, 4, 2, 1)
  for (int o = kGrp / 2; o > 0; o >>= 1)
    for (int c = 0; c < NC; ++c) acc[c] += __shfl_down(acc[c], o, kGrp);  // none when G = 1
  if (!valid || r != 0) return;
  // res holds the local part: the near-field slices' partial sums, added in
  // slice order
  if (GLOBAL) {
    if (!STRESS) {
      res[0] += acc[0];
      res[1] += acc[1];
      res[2] += acc[2];
    } else {
      const T* tn = (const T*)a.tn;
      const double nx = tn[t], nyv = tn[a.tcap + t], nz = tn[2 * a.tcap + t];
      // acc: xx, yy, zz, xy, xz, yz
      res[0] += acc[0] * nx + acc[3] * nyv + acc[4] * nz;
      res[1] += acc[3] * nx + acc[1] * nyv + acc[5] * nz;
      res[2] += acc[4] * nx + acc[5] * nyv + acc[2] * nz;
    }
  }
  const size_t o = 3 * (size_t)slot;
  a.out[o] = res[0];
  a.out[o + 1] = res[1];
  a.out[o + 2] = res[2];
}

// Large target sets: one thread per target, 256 consecutive sorted targets
// per block (they share one or two cells).  The box of grid nodes that their
// stencils cover is staged in LDS one field at a time and every thread sums
// its 125 nodes from there, in the order of interp_combine.  Blocks whose box
// exceeds 36 KiB of LDS (targets far apart in the sorted order, e.g. across
// a row of cells) gather from global memory as interp_combine does.
constexpr int kBoxBytes = 36 * 1024;

template <typename T, bool STRESS>
__global__ void __launch_bounds__(256) interp_staged(InterpArgs a) {
  extern __shared__ unsigned char smem[];
  T* box = (T*)smem;
  __shared__ double ly[kMaxNy];
  __shared__ int lo[3], hi[3];
  const int t = blockIdx.x * 256 + threadIdx.x;
  const bool valid = t < a.nt;
  constexpr int NC = STRESS ? 6 : 3;
  for (int j = threadIdx.x; j < a.Ny; j += 256) ly[j] = a.y[j];
  if (threadIdx.x < 3) {
    lo[threadIdx.x] = 1 << 30;
    hi[threadIdx.x] = -(1 << 30);
  }
  __syncthreads();
  const T* ul = (const T*)a.ul;
  double res[3] = {0.0, 0.0, 0.0};
  double wx[5], wz[5], wy[5];
  int i0 = 0, k0 = 0, j0 = 2;
  if (valid) {
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int s = 0; s < kNearSlices; ++s) v += (double)ul[(size_t)(3 * s + c) * a.tcap + t];
      res[c] = v;
    }
    const double x = a.tx[t], y = a.ty[t], z = a.tz[t];
    const double fx = floor(x / a.dx + 0.5), fz = floor(z / a.dz + 0.5);
    lagrange5_uniform(x / a.dx - fx, wx);
    lagrange5_uniform(z / a.dz - fz, wz);
    const int N = a.Ny - 1;
    j0 = (int)rint(acos(y / a.H) * N / 3.141592653589793);
    j0 = j0 < 2 ? 2 : (j0 > a.Ny - 3 ? a.Ny - 3 : j0);
    double ny[5];
    for (int q = 0; q < 5; ++q) ny[q] = ly[j0 - 2 + q];
    lagrange5(y, ny, wy);
    i0 = (int)fx - 2;   // first stencil node, unwrapped: in [-2, Nx - 2]
    k0 = (int)fz - 2;
    atomicMin(&lo[0], j0 - 2);
    atomicMax(&hi[0], j0 - 2);
    atomicMin(&lo[1], i0);
    atomicMax(&hi[1], i0);
    atomicMin(&lo[2], k0);
    atomicMax(&hi[2], k0);
  }
  __syncthreads();
  const int bj = hi[0] - lo[0] + 5, bi = hi[1] - lo[1] + 5, bk = hi[2] - lo[2] + 5;
  const int nbox = bj * bi * bk;
  const size_t fs = (size_t)a.Ny * a.Nx * a.Nz;
  const T* g = (const T*)a.grid;
  T acc[NC];
  for (int c = 0; c < NC; ++c) acc[c] = (T)0;
  // weights in T: the z weights and the 25 x-y products (formed in FP64)
  T tz[5], twab[25];
  for (int q = 0; q < 5; ++q) tz[q] = (T)wz[q];
  for (int row = 0; row < 25; ++row) twab[row] = (T)(wy[row / 5] * wx[row % 5]);
  if (nbox * (int)sizeof(T) <= kBoxBytes) {
    const int oj = j0 - 2 - lo[0], oi = i0 - lo[1], ok = k0 - lo[2];
    // A box of at most 256 x UR nodes is held one register per node and
    // thread: the next field's loads are issued before this field's sums,
    // so their memory latency overlaps the arithmetic.  A larger box is
    // staged in batches of eight loads per thread.
    constexpr int UR = 12;
    const bool piped = nbox <= 256 * UR;
    int off[UR];
    T v[UR];
    if (piped) {
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int e = threadIdx.x + 256 * u;
        off[u] = 0;
        if (e < nbox) {
          const int kb = e % bk, r = e / bk, ib = r % bi, jb = r / bi;
          const int gi = wrap1(lo[1] + ib, a.Nx), gk = wrap1(lo[2] + kb, a.Nz);
          off[u] = ((lo[0] + jb) * a.Nx + gi) * a.Nz + gk;
          v[u] = g[off[u]];
        }
      }
    }
    for (int c = 0; c < NC; ++c) {
      if (piped) {
#pragma unroll
        for (int u = 0; u < UR; ++u)
          if (threadIdx.x + 256 * u < nbox) box[threadIdx.x + 256 * u] = v[u];
      } else {
        constexpr int U = 8;
        for (int e0 = threadIdx.x; e0 < nbox; e0 += 256 * U) {
          T w[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = e0 + 256 * u;
            if (e < nbox) {
              const int kb = e % bk, r = e / bk, ib = r % bi, jb = r / bi;
              const int gi = wrap1(lo[1] + ib, a.Nx), gk = wrap1(lo[2] + kb, a.Nz);
              w[u] = g[c * fs + ((size_t)(lo[0] + jb) * a.Nx + gi) * a.Nz + gk];
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (e0 + 256 * u < nbox) box[e0 + 256 * u] = w[u];
        }
      }
      __syncthreads();
      if (piped && c + 1 < NC) {
        const T* gc = g + (size_t)(c + 1) * fs;
#pragma unroll
        for (int u = 0; u < UR; ++u)
          if (threadIdx.x + 256 * u < nbox) v[u] = gc[off[u]];
      }
      if (valid) {
        T sum = (T)0;
        for (int row = 0; row < 25; ++row) {
          const int qa = row / 5, qb = row % 5;
          const int base = ((oj + qa) * bi + oi + qb) * bk + ok;
          T zr = tz[0] * box[base];
          for (int qc = 1; qc < 5; ++qc) zr = fma(tz[qc], box[base + qc], zr);
          sum = fma(twab[row], zr, sum);
        }
        acc[c] = sum;
      }
      __syncthreads();
    }
  } else if (valid) {
    int kk[5];
    for (int q = 0; q < 5; ++q) kk[q] = wrap1(k0 + q, a.Nz);
    for (int row = 0; row < 25; ++row) {
      const int qa = row / 5, qb = row % 5;
      const int ii = wrap1(i0 + qb, a.Nx);
      const size_t base = ((size_t)(j0 - 2 + qa) * a.Nx + ii) * a.Nz;
      for (int c = 0; c < NC; ++c) {
        const T* gc = g + c * fs + base;
        T zr = tz[0] * gc[kk[0]];
        for (int qc = 1; qc < 5; ++qc) zr = fma(tz[qc], gc[kk[qc]], zr);
        acc[c] = fma(twab[row], zr, acc[c]);
      }
    }
  }
  if (!valid) return;
  if (!STRESS) {
    res[0] += acc[0];
    res[1] += acc[1];
    res[2] += acc[2];
  } else {
    const T* tn = (const T*)a.tn;
    const double nx = tn[t], nyv = tn[a.tcap + t], nz = tn[2 * a.tcap + t];
    res[0] += acc[0] * nx + acc[3] * nyv + acc[4] * nz;
    res[1] += acc[3] * nx + acc[1] * nyv + acc[5] * nz;
    res[2] += acc[4] * nx + acc[5] * nyv + acc[2] * nz;
  }
  const size_t o = 3 * (size_t)a.perm[t];
  a.out[o] = res[0];
  a.out[o + 1] = res[1];
  a.out[o + 2] = res[2];
}

template <typename T, int G>
static void launch_interp_g(Plan& p, const InterpArgs& a, int nt, bool stress, bool with_global) {
  const unsigned nb = (unsigned)(((size_t)nt * G + 255) / 256);
  if (!with_global) interp_combine<T, false, false, G><<<nb, 256, 0, p.stream>>>(a);
  else if (stress) interp_combine<T, true, true, G><<<nb, 256, 0, p.stream>>>(a);
  else interp_combine<T, false, true, G><<<nb, 256, 0, p.stream>>>(a);
}

template <typename T>
hipError_t launch_interp(Plan& p, int nt, double* out, bool stress, bool with_global) {
  if (nt <= 0) return hipSuccess;
  InterpArgs a;
  a.nt = nt;
  a.Nx = p.p.Nx;
  a.Nz = p.p.Nz;
  a.Ny = p.p.Ny;
  a.dx = p.dx;
  a.dz = p.dz;
  a.H = p.p.H;
  a.y = p.y;
  a.perm = p.tview->perm;
  a.tx = p.tview->x;
  a.ty = p.tview->y;
  a.tz = p.tview->z;
  a.tn = p.tnrm;
  a.tcap = (size_t)p.p.max_tgt;
  a.ul = p.ul;
  a.grid = p.phys;
  a.out = out;
  if (nt < 65536) {
    launch_interp_g<T, 16>(p, a, nt, stress, with_global);
  } else if (!with_global) {
    launch_interp_g<T, 1>(p, a, nt, stress, with_global);
  } else {
    const unsigned nb = (unsigned)((nt + 255) / 256);
    const size_t lds = kBoxBytes;
    if (stress) interp_staged<T, true><<<nb, 256, lds, p.stream>>>(a);
    else interp_staged<T, false><<<nb, 256, lds, p.stream>>>(a);
  }
  return hipGetLastError();
}

template <typename T>
__global__ void to_f64(const T* __restrict__ in, double* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

template <typename T>
hipError_t launch_grid_to_f64(Plan& p, double* out) {
  const size_t n = (size_t)3 * p.p.Ny * p.p.Nx * p.p.Nz;
  to_f64<T><<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>((const T*)p.phys, out, n);
  return hipGetLastError();
}

template hipError_t launch_interp<double>(Plan&, int, double*, bool, bool);
template hipError_t launch_interp<float>(Plan&, int, double*, bool, bool);
template hipError_t launch_grid_to_f64<double>(Plan&, double*);
template hipError_t launch_grid_to_f64<float>(Plan&, double*);

}  // namespace ggem
