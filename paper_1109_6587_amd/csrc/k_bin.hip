// Cell-list binning by a deterministic, stable counting sort (Sec. 3.2.1:
// neighbours within r_c are found through a cell-linked list; here the list is
// a sorted order plus per-cell ranges, so later kernels read contiguous runs).
// The sort key is (cell, z slab): each cell is cut into nzs slabs along z, so
// a cell stays one contiguous run and a row of cells along z is sorted by slab.
//
//   bin_keys     per chunk: wrap x,z into [0,L), check the slab, bucket key per
//                point, and the chunk's histogram in LDS -> counts[chunk][bucket]
//   bin_cellscan per-bucket running sum over chunks     -> offs[chunk][bucket]
//   bin_scan     exclusive scan over buckets            -> sub_start, cell_start,
//                                                          item_start
//   bin_scatter  one wave per chunk, stable ranks by bitwise key match -> sorted SoA
//
// Points keep their input order inside a bucket, so every later sum over a
// cell's points has a fixed order and results are bitwise reproducible.
#include "ggem_internal.h"

namespace ggem {

__device__ inline double wrap_periodic(double v, double L) {
  double r = fmod(v, L);
  if (r < 0.0) r += L;
  if (r >= L) r = 0.0;
  return r;
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bucket (cell * nzs + z slab) of a (wrapped, finite) position; y is clamped
// into the slit.  z * icz * nzs is exact (nzs is a power of two), so the slab
// floor(z * icz * nzs) always lies inside the cell floor(z * icz).
__device__ inline int bucket_key(const CellGeom& g, double x, double y, double z) {
  int ix = clampi((int)floor(x * g.icx), 0, g.ncx - 1);
  int iy = clampi((int)floor((y + g.H) * g.icy), 0, g.ncy - 1);
  const double tz = z * g.icz;
  int iz = clampi((int)floor(tz), 0, g.ncz - 1);
  int sz = clampi((int)floor(tz * g.nzs) - iz * g.nzs, 0, g.nzs - 1);
  return ((iy * g.ncx + ix) * g.ncz + iz) * g.nzs + sz;
}

// One block per chunk: the chunk's keys and its histogram (counts are
// integers, so the LDS atomics give the same result in any order).
__global__ void bin_keys(int n, int chunk_size, int nb, const double* __restrict__ x,
                         CellGeom g, int is_source, int* __restrict__ keys,
                         int* __restrict__ counts, unsigned* __restrict__ cflags) {
  extern __shared__ int hist[];
  __shared__ unsigned bflags;
  const int chunk = blockIdx.x;
  for (int c = threadIdx.x; c < nb; c += blockDim.x) hist[c] = 0;
  if (threadIdx.x == 0) bflags = 0u;
  __syncthreads();
  const int i0 = chunk * chunk_size;
  const int i1 = min(n, i0 + chunk_size);
  unsigned f = 0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double px = x[3 * (size_t)i], py = x[3 * (size_t)i + 1], pz = x[3 * (size_t)i + 2];
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) {
      f |= kFlagNonFinite;
      px = py = pz = 0.0;
    }
    if (is_source ? !(fabs(py) < g.H) : !(fabs(py) <= g.H)) f |= kFlagOutside;
    px = wrap_periodic(px, g.Lx);
    pz = wrap_periodic(pz, g.Lz);
    const int key = bucket_key(g, px, py, pz);
    keys[i] = key;
    atomicAdd(&hist[key], 1);
  }
  if (f) atomicOr(&bflags, f);
  __syncthreads();
  for (int c = threadIdx.x; c < nb; c += blockDim.x) counts[(size_t)chunk * nb + c] = hist[c];
  if (threadIdx.x == 0) cflags[chunk] = bflags;
}

// counts and offsets are chunk-major ([chunk][bucket]).  A block takes 32
// buckets; its 8 thread rows split the chunks into 8 consecutive runs, sum
// their run, and write the offsets from the sum of the earlier runs (integer
// sums: the same result as one thread walking all chunks).
constexpr int kScanSeg = 8;
__global__ void __launch_bounds__(32 * kScanSeg) bin_cellscan(int nchunks, int nb,
                                                              const int* __restrict__ counts,
                                                              int* __restrict__ offs,
                                                              int* __restrict__ totals) {
  __shared__ int part[kScanSeg][32];
  const int bl = threadIdx.x & 31, seg = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + bl;
  const int per = (nchunks + kScanSeg - 1) / kScanSeg;
  const int k0 = min(nchunks, seg * per), k1 = min(nchunks, k0 + per);
  int s = 0;
  if (c < nb)
    for (int k = k0; k < k1; ++k) s += counts[(size_t)k * nb + c];
  part[seg][bl] = s;
  __syncthreads();
  int run = 0;
  for (int q = 0; q < seg; ++q) run += part[q][bl];
  if (c >= nb) return;
  if (seg == kScanSeg - 1) totals[c] = run + s;
  for (int k = k0; k < k1; ++k) {
    const int v = counts[(size_t)k * nb + c];
    offs[(size_t)k * nb + c] = run;
    run += v;
  }
}

__device__ inline int cell_total(const int* __restrict__ sub, int c, int nzs) {
  int v = 0;
  for (int q = 0; q < nzs; ++q) v += sub[c * nzs + q];
  return v;
}

// Single block: exclusive scans of the per-bucket totals (held in sub_start
// on entry), of the per-cell totals (cell_start) and of the per-cell
// near-field work items ceil(total / kNearBlock) (item_start, and the cell of
// every item in item_cell).  It also
// folds the chunks' domain flags into *flags: the first binning of an
// evaluation overwrites them and clears the pair counters (no kernel of the
// evaluation has touched either yet), later binnings OR into them.
__global__ void __launch_bounds__(1024) bin_scan(int ncells, int nzs, int* __restrict__ sub_start,
                                                 int* __restrict__ cell_start,
                                                 int* __restrict__ item_start,
                                                 int* __restrict__ item_cell, int nchunks,
                                                 const unsigned* __restrict__ cflags,
                                                 unsigned* __restrict__ flags,
                                                 unsigned long long* __restrict__ work,
                                                 int first) {
  __shared__ int sa[16], sb[16];
  __shared__ unsigned fl;
  if (threadIdx.x == 0) fl = 0u;
  __syncthreads();
  if ((int)threadIdx.x < nchunks) {
    const unsigned v = cflags[threadIdx.x];
    if (v) atomicOr(&fl, v);
  }
  const int per = (ncells + 1023) / 1024;
  int t = threadIdx.x;
  int c0 = t * per, c1 = min(ncells, c0 + per);
  int la = 0, lb = 0;
  for (int c = c0; c < c1; ++c) {
    int v = cell_total(sub_start, c, nzs);
    la += v;
    lb += (v + kNearBlock - 1) / kNearBlock;
  }
  // inclusive scan of the 1024 partial sums: within each wave by shuffles,
  // then over the 16 wave totals
  const int lane = t & 63, wv = t >> 6;
  int ia = la, ib = lb;
  for (int o = 1; o < 64; o <<= 1) {
    const int va = __shfl_up(ia, o), vb = __shfl_up(ib, o);
    if (lane >= o) {
      ia += va;
      ib += vb;
    }
  }
  if (lane == 63) {
    sa[wv] = ia;
    sb[wv] = ib;
  }
  __syncthreads();
  int wa = 0, wb = 0;
  for (int q = 0; q < wv; ++q) {
    wa += sa[q];
    wb += sb[q];
  }
  ia += wa;
  ib += wb;
  int ra = ia - la, rb = ib - lb;
  for (int c = c0; c < c1; ++c) {
    cell_start[c] = ra;
    item_start[c] = rb;
    int v = 0;
    for (int q = 0; q < nzs; ++q) {
      const int w = sub_start[c * nzs + q];
      sub_start[c * nzs + q] = ra + v;
      v += w;
    }
    const int ni = (v + kNearBlock - 1) / kNearBlock;
    for (int it = 0; it < ni; ++it) item_cell[rb + it] = c;
    ra += v;
    rb += ni;
  }
  if (t == 1023) {
    cell_start[ncells] = ia;
    sub_start[ncells * nzs] = ia;
    item_start[ncells] = ib;
  }
  if (t == 0) {
    if (first) {
      *flags = fl;
      work[0] = 0ull;
      work[1] = 0ull;
    } else if (fl) {
      *flags |= fl;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(64) bin_scatter(int n, int chunk_size, int nchunks, int nb,
                                                  int kbits,
                                                  CellGeom g,
                                                  const int* __restrict__ keys,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ s,
                                                  const int* __restrict__ sub_start,
                                                  const int* __restrict__ offs,
                                                  int* __restrict__ perm, double* __restrict__ sx,
                                                  double* __restrict__ sy, double* __restrict__ sz,
                                                  T* __restrict__ ss, size_t cap) {
  extern __shared__ int cnt[];
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x;
  for (int c = lane; c < nb; c += 64) cnt[c] = 0;
  __syncthreads();
  const int i0 = chunk * chunk_size;
  const int i1 = min(n, i0 + chunk_size);
  const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int base = i0; base < i1; base += 64) {
    int i = base + lane;
    bool valid = i < i1;
    int key = valid ? keys[i] : 0;
    // the lanes holding the same key, found bit by bit (one ballot per key bit)
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < kbits; ++b) {
      const bool bit = (key >> b) & 1;
      const unsigned long long bm = __ballot(bit);
      m &= bit ? bm : ~bm;
    }
    // rank among the earlier lanes of the key; the key's lowest lane advances
    // the chunk's running count for the later groups
    const int rank = __popcll(m & lt);
    const int before = valid ? cnt[key] : 0;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) cnt[key] = before + __popcll(m);
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      int pos = sub_start[key] + offs[(size_t)chunk * nb + key] + before + rank;
      double px = x[3 * (size_t)i], py = x[3 * (size_t)i + 1], pz = x[3 * (size_t)i + 2];
      if (!(isfinite(px) && isfinite(py) && isfinite(pz))) px = py = pz = 0.0;
      py = fmin(fmax(py, -g.H), g.H);
      perm[pos] = i;
      sx[pos] = wrap_periodic(px, g.Lx);
      sy[pos] = py;
      sz[pos] = wrap_periodic(pz, g.Lz);
      if (s) {
        ss[pos] = (T)s[3 * (size_t)i];
        ss[cap + pos] = (T)s[3 * (size_t)i + 1];
        ss[2 * cap + pos] = (T)s[3 * (size_t)i + 2];
      }
    }
  }
}

__global__ void zero_ints(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

static hipError_t bin_impl(Plan& p, Binned& b, long long n, const double* x, const double* s,
                           bool is_source, size_t cap, bool first) {
  hipStream_t st = p.stream;
  const CellGeom& g = p.cg;
  b.n = (int)n;
  // at most kMaxChunks chunks, at least 256 points each (multiple of 64)
  const long long per = (n + kMaxChunks - 1) / kMaxChunks;
  b.chunk = (int)(per < 256 ? 256 : ((per + 63) / 64) * 64);
  b.nchunks = (int)((n + b.chunk - 1) / b.chunk);
  const int nb = g.nbuckets;
  int kbits = 1;  // bits of the largest bucket key
  while ((1 << kbits) < nb) ++kbits;
  if (n > 0) {
    bin_keys<<<b.nchunks, 256, nb * sizeof(int), st>>>((int)n, b.chunk, nb, x, g,
                                                        is_source ? 1 : 0, b.keys, b.counts,
                                                        b.cflags);
    bin_cellscan<<<(nb + 31) / 32, 32 * kScanSeg, 0, st>>>(b.nchunks, nb, b.counts, b.offs,
                                                          b.sub_start);
  } else {
    zero_ints<<<(nb + 1 + 255) / 256, 256, 0, st>>>(b.sub_start, nb + 1);
  }
  bin_scan<<<1, 1024, 0, st>>>(g.ncells, g.nzs, b.sub_start, b.cell_start, b.item_start, b.item_cell,
                               n > 0 ? b.nchunks : 0, b.cflags, p.flags, p.work, first ? 1 : 0);
  if (n > 0) {
    if (p.fp64)
      bin_scatter<double><<<b.nchunks, 64, nb * sizeof(int), st>>>(
          (int)n, b.chunk, b.nchunks, nb, kbits, g, b.keys, x, s, b.sub_start, b.offs, b.perm,
          b.x, b.y, b.z, (double*)b.s, cap);
    else
      bin_scatter<float><<<b.nchunks, 64, nb * sizeof(int), st>>>(
          (int)n, b.chunk, b.nchunks, nb, kbits, g, b.keys, x, s, b.sub_start, b.offs, b.perm,
          b.x, b.y, b.z, (float*)b.s, cap);
  }
  return hipGetLastError();
}

hipError_t launch_bin(Plan& p, Binned& b, long long n, const double* x, const double* s,
                      const double* /*s2*/, bool is_source, bool first) {
  size_t cap = is_source ? (size_t)p.p.max_src : (size_t)p.p.max_tgt;
  if (&b == &p.wall) cap = 2 * (size_t)p.p.Nx * p.p.Nz;
  return bin_impl(p, b, n, x, s, is_source, cap, first);
}

}  // namespace ggem
