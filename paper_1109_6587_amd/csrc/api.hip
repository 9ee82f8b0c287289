// C-ABI of the GGEM slit library: plan creation (validation, plan-time
// constants, workspace), the two evaluations and the spread diagnostic.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ggem_internal.h"

using namespace ggem;

static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(GGEM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

extern "C" const char* ggem_last_error(void) { return g_last_error.c_str(); }

int ggem_set_error(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

namespace {

bool factor_radices(int n, int* r, int* nr) {
  int k = 0;
  while (n % 8 == 0 && n > 8) {
    r[k++] = 8;
    n /= 8;
  }
  const int ps[5] = {8, 4, 2, 3, 5};
  for (int i = 0; i < 5; ++i)
    while (n % ps[i] == 0) {
      if (k >= 12) return false;
      r[k++] = ps[i];
      n /= ps[i];
    }
  *nr = k;
  return n == 1;
}

// Sub-allocation of a plan's device workspace from one block: every buffer
// starts on a 256-byte boundary.  With base == nullptr only the size is
// computed (the pointers stay null).
struct Carver {
  char* base;
  size_t off;
  void* take_bytes(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* r = base ? (void*)(base + off) : nullptr;
    off += bytes ? bytes : 1;
    return r;
  }
  template <typename T>
  T* take(size_t n) {
    return (T*)take_bytes((n ? n : 1) * sizeof(T));
  }
};

// The same for the host arrays the plan constants are computed in.
struct HostStage {
  char* base;
  size_t off, cap;
  template <typename T>
  T* take(size_t n) {
    off = (off + 63) & ~(size_t)63;
    T* r = (base && off + n * sizeof(T) <= cap) ? (T*)(base + off) : nullptr;
    off += (n ? n : 1) * sizeof(T);
    return r;
  }
};

void carve_binned(Carver& c, Binned& b, long long cap, const CellGeom& g, size_t elt) {
  const size_t nch = kMaxChunks + 1;
  const size_t nb = (size_t)g.nbuckets, ncells = (size_t)g.ncells;
  const size_t n = (size_t)(cap > 0 ? cap : 1);
  b.keys = c.take<int>(n);
  b.counts = c.take<int>(nb * (nch + 1));
  b.offs = c.take<int>(nb * (nch + 1));
  b.sub_start = c.take<int>(nb + 1);
  b.cell_start = c.take<int>(ncells + 1);
  b.cflags = c.take<unsigned>(kMaxChunks + 1);
  b.item_start = c.take<int>(ncells + 1);
  b.item_cell = c.take<int>(n / kNearBlock + ncells + 1);
  b.perm = c.take<int>(n);
  b.x = c.take<double>(n);
  b.y = c.take<double>(n);
  b.z = c.take<double>(n);
  b.s = c.take_bytes(3 * n * elt);
}

// Every device buffer of a plan, in one layout shared by ggem_plan_create
// (one hipMalloc) and ggem_single_layer_noalloc (the static scratch array).
void layout_plan(Plan& p, Carver& c) {
  const ggem_params& q = p.p;
  const size_t elt = p.fp64 ? 8 : 4;
  const size_t Ny = q.Ny, Nx = q.Nx, Nz = q.Nz, nm = (size_t)p.nmodes;
  const size_t MP = ((q.Ny + 15) / 16) * 16, KP = ((q.Ny + 3) / 4) * 4;
  const size_t mt = (size_t)(q.max_tgt > 0 ? q.max_tgt : 1);
  p.y = c.take<double>(Ny);
  p.cf64 = c.take<double>(MP * KP);
  p.ci64 = c.take<double>(MP * KP);
  p.cf32 = c.take<float>(MP * KP);
  p.ci32 = c.take<float>(MP * KP);
  const size_t KP32 = ((q.Ny + 31) / 32) * 32;
  p.cf_hi = c.take<unsigned short>(MP * KP32);
  p.cf_lo = c.take<unsigned short>(MP * KP32);
  p.ci_hi = c.take<unsigned short>(MP * KP32);
  p.ci_lo = c.take<unsigned short>(MP * KP32);
  p.twx = c.take_bytes(2 * Nx * elt);
  p.twz = c.take_bytes(2 * Nz * elt);
  p.infl = c.take<double>(4 * nm);
  p.nconst = c.take<double>(3 * Ny);
  p.sweep = c.take<double>((6 * Ny + 2) * nm);
  p.ul = c.take_bytes(kNearSlices * 3 * mt * elt);
  p.phys = c.take_bytes(6 * Ny * Nx * Nz * elt);
  p.specA = c.take_bytes(6 * Ny * nm * 2 * elt);
  p.specB = c.take_bytes(6 * Ny * nm * 2 * elt);
  p.wall_phys = c.take_bytes(6 * Nx * Nz * elt);
  p.wall_part = c.take_bytes(kWallSlices * 6 * Nx * Nz * elt);
  p.wall_spec = c.take_bytes(6 * nm * 2 * elt);
  p.tau_scr = c.take<double>(2 * 9 * Ny * nm);
  p.gauge = c.take<double>((size_t)(q.max_src / 256 + 4));
  p.flags = c.take<unsigned>(1);
  p.work = c.take<unsigned long long>(2);
  p.wall_pos = c.take<double>(3 * 2 * Nx * Nz);
  p.norder = c.take<int>(mt);
  carve_binned(c, p.src, q.max_src, p.cg, elt);
  carve_binned(c, p.tgt, q.max_tgt, p.cg, elt);
  carve_binned(c, p.wall, 2LL * q.Nx * q.Nz, p.cg, elt);
}

void free_over(Plan& p) {
  if (p.over_block) (void)hipFree(p.over_block);
  delete p.over;
  p.over = nullptr;
  p.over_block = p.over_spec = p.over_phys = p.over_theta = p.cth = nullptr;
  p.interp_mode = GGEM_INTERP_LAGRANGE;
}

void free_plan(Plan& p) {
  free_over(p);
  if (p.block && p.owns_block) (void)hipFree(p.block);
  p.block = nullptr;
  if (p.flags_host && p.owns_flags_host) (void)hipHostFree(p.flags_host);
  p.flags_host = nullptr;
  if (p.side) (void)hipStreamDestroy(p.side);
  hipEvent_t evs[] = {p.ev_fork, p.ev_wall, p.ev_near};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (p.timed_ev) {
    for (int i = 0; i < 2 * p.timed_max; ++i) (void)hipEventDestroy(p.timed_ev[i]);
    delete[] p.timed_ev;
    p.timed_ev = nullptr;
  }
}

// cos(pi * m / N) with the argument reduced exactly (m integer)
double cospi_frac(long m, int N) {
  m %= 2L * N;
  return cos(M_PI * (double)m / (double)N);
}

// bfloat16 of a float, rounded to nearest even, and back (host)
unsigned short bf16_round(float x) {
  unsigned u;
  memcpy(&u, &x, 4);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
double bf16_value(unsigned short h) {
  const unsigned u = (unsigned)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// normals of coinciding targets, in the sources' sorted order
template <typename T>
__global__ void gather_normals(int n, const int* __restrict__ perm, const double* __restrict__ nrm,
                               T* __restrict__ out, size_t cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t j = 3 * (size_t)perm[i];
  out[i] = (T)nrm[j];
  out[cap + i] = (T)nrm[j + 1];
  out[2 * cap + i] = (T)nrm[j + 2];
}

template <typename T>
__global__ void fill_zero(T* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

// FFT twiddles exp(-2 pi i t/n) = cos(pi 2t/n) - i sin(pi 2t/n), t < n,
// as interleaved (re, im) pairs
void fill_twiddles(int n, double* tw) {
  for (int t = 0; t < n; ++t) {
    const long m = (2L * t) % (2L * n);
    tw[2 * t] = cos(M_PI * (double)m / n);
    tw[2 * t + 1] = -sin(M_PI * (double)m / n);
  }
}

// Host arrays of the plan constants, carved from `hs` (a sizing pass with
// hs.base == nullptr gives the bytes needed; GGEM_E_CAPACITY when they do
// not fit).  Then copies them to the device, derives the per-mode tau
// factors and influence matrices, and bins the wall nodes, all on p.stream.
int plan_constants(Plan& p, HostStage& hs) {
  const int Ny = p.p.Ny, N = Ny - 1, Nx = p.p.Nx, Nz = p.p.Nz;
  const int MP = ((Ny + 15) / 16) * 16, KP = ((Ny + 3) / 4) * 4;
  const size_t nw = 2 * (size_t)Nx * Nz;
  double* y = hs.take<double>(Ny);
  double* cf64 = hs.take<double>((size_t)MP * KP);
  double* ci64 = hs.take<double>((size_t)MP * KP);
  float* cf32 = hs.take<float>((size_t)MP * KP);
  float* ci32 = hs.take<float>((size_t)MP * KP);
  const int KP32 = ((Ny + 31) / 32) * 32;
  unsigned short* bsplit = hs.take<unsigned short>(4 * (size_t)MP * KP32);
  double* tw = hs.take<double>(2 * (size_t)(Nx > Nz ? Nx : Nz));
  float* tf = hs.take<float>(2 * (size_t)(Nx > Nz ? Nx : Nz));
  double* nc = hs.take<double>(3 * (size_t)Ny);
  double* wpos = hs.take<double>(3 * nw);
  if (!hs.base) return GGEM_OK;  // sizing pass
  if (hs.off > hs.cap || !wpos) return fail(GGEM_E_CAPACITY, "host staging of the plan constants too small");
  for (int j = 0; j < Ny; ++j) y[j] = p.p.H * cospi_frac(j, N);
  HIP_TRY(hipMemcpy(p.y, y, Ny * sizeof(double), hipMemcpyHostToDevice));
  const double norm = 1.0 / ((double)Nx * (double)Nz);
  for (size_t i = 0; i < (size_t)MP * KP; ++i) cf64[i] = ci64[i] = 0.0;
  for (int n = 0; n < Ny; ++n)
    for (int j = 0; j < Ny; ++j) {
      const double cbn = (n == 0 || n == N) ? 2.0 : 1.0;
      const double cbj = (j == 0 || j == N) ? 2.0 : 1.0;
      const double c = cospi_frac((long)n * j, N);
      // padded (MP x KP) row-major copies of the (Ny x Ny) matrices
      cf64[(size_t)n * KP + j] = 2.0 / (N * cbn * cbj) * c * norm;
      ci64[(size_t)j * KP + n] = c;
    }
  for (size_t i = 0; i < (size_t)MP * KP; ++i) {
    cf32[i] = (float)cf64[i];
    ci32[i] = (float)ci64[i];
  }
  // BF16 hi and lo halves of the two matrices, [MP][KP32], zero padded
  for (size_t i = 0; i < 4 * (size_t)MP * KP32; ++i) bsplit[i] = 0;
  for (int r = 0; r < Ny; ++r)
    for (int k = 0; k < Ny; ++k)
      for (int m = 0; m < 2; ++m) {
        const double v = m == 0 ? cf64[(size_t)r * KP + k] : ci64[(size_t)r * KP + k];
        const unsigned short hi = bf16_round((float)v);
        const unsigned short lo = bf16_round((float)(v - bf16_value(hi)));
        const size_t o = (size_t)r * KP32 + k;
        bsplit[(size_t)(2 * m) * MP * KP32 + o] = hi;
        bsplit[(size_t)(2 * m + 1) * MP * KP32 + o] = lo;
      }
  const size_t nb = (size_t)MP * KP32 * sizeof(unsigned short);
  HIP_TRY(hipMemcpy(p.cf_hi, bsplit, nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.cf_lo, bsplit + (size_t)MP * KP32, nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.ci_hi, bsplit + 2 * (size_t)MP * KP32, nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.ci_lo, bsplit + 3 * (size_t)MP * KP32, nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.cf64, cf64, (size_t)MP * KP * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.ci64, ci64, (size_t)MP * KP * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.cf32, cf32, (size_t)MP * KP * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.ci32, ci32, (size_t)MP * KP * 4, hipMemcpyHostToDevice));
  for (int ax = 0; ax < 2; ++ax) {
    const int n = ax == 0 ? Nx : Nz;
    fill_twiddles(n, tw);
    void* dst = ax == 0 ? p.twx : p.twz;
    if (p.fp64) {
      HIP_TRY(hipMemcpy(dst, tw, 2 * (size_t)n * 8, hipMemcpyHostToDevice));
    } else {
      for (int i = 0; i < 2 * n; ++i) tf[i] = (float)tw[i];
      HIP_TRY(hipMemcpy(dst, tf, 2 * (size_t)n * 4, hipMemcpyHostToDevice));
    }
  }
  for (int i = 0; i < 3 * Ny; ++i) nc[i] = 0.0;
  for (int n = 2; n < Ny; ++n) {
    nc[n] = 1.0 / (4.0 * n * (n - 1));
    nc[Ny + n] = 1.0 / (2.0 * ((double)n * n - 1.0));
    nc[2 * Ny + n] = 1.0 / (4.0 * n * (n + 1));
  }
  HIP_TRY(hipMemcpy(p.nconst, nc, 3 * (size_t)Ny * 8, hipMemcpyHostToDevice));
  HIP_TRY(launch_influence(p));
  // wall nodes (x_i, -H, z_k) then (x_i, +H, z_k), binned once
  for (int w = 0; w < 2; ++w)
    for (int i = 0; i < Nx; ++i)
      for (int k = 0; k < Nz; ++k) {
        const size_t r = (size_t)w * Nx * Nz + (size_t)i * Nz + k;
        wpos[3 * r] = i * p.dx;
        wpos[3 * r + 1] = w ? p.p.H : -p.p.H;
        wpos[3 * r + 2] = k * p.dz;
      }
  HIP_TRY(hipMemcpy(p.wall_pos, wpos, 3 * nw * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(launch_bin(p, p.wall, (long long)nw, p.wall_pos, nullptr, nullptr, false, true));
  HIP_TRY(hipStreamSynchronize(p.stream));
  return GGEM_OK;
}

int check_plan(ggem_plan_t plan) {
  if (!plan) return fail(GGEM_E_ARG, "null plan");
  return GGEM_OK;
}

template <typename T>
int zero_ul(Plan& p, int nt) {
  const size_t n = (size_t)kNearSlices * 3 * p.p.max_tgt;
  if (nt > 0) fill_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>((T*)p.ul, n);
  HIP_TRY(hipGetLastError());
  return GGEM_OK;
}

// With sync_checks the call waits and reports the domain flags; otherwise it
// returns at once and ggem_plan_status reads them later.
int finish(Plan& p) {
  if (!p.p.sync_checks) return GGEM_OK;
  HIP_TRY(hipMemcpyAsync(p.flags_host, p.flags, sizeof(unsigned), hipMemcpyDeviceToHost, p.stream));
  HIP_TRY(hipStreamSynchronize(p.stream));
  const unsigned f = *p.flags_host;
  if (f & kFlagNonFinite) return fail(GGEM_E_DOMAIN, "non-finite input position");
  if (f & kFlagOutside) return fail(GGEM_E_DOMAIN, "point outside the slit");
  return GGEM_OK;
}

// Timing hook: events around the launches of the selected stage.
struct StageScope {
  Plan& p;
  bool on;
  StageScope(Plan& pp, int stage) : p(pp), on(pp.timed_stage == stage && pp.timed_calls < pp.timed_max) {
    if (on) (void)hipEventRecord(p.timed_ev[2 * p.timed_calls], p.stream);
  }
  ~StageScope() {
    if (on) {
      (void)hipEventRecord(p.timed_ev[2 * p.timed_calls + 1], p.stream);
      ++p.timed_calls;
    }
  }
};

void destroy_timer(Plan& p) {
  if (p.timed_ev) {
    for (int i = 0; i < 2 * p.timed_max; ++i) (void)hipEventDestroy(p.timed_ev[i]);
    delete[] p.timed_ev;
  }
  p.timed_ev = nullptr;
  p.timed_max = 0;
  p.timed_calls = 0;
  p.timed_stage = -1;
}

template <typename T>
int evaluate(Plan& p, long long ns, const double* xs, const double* f, long long nt,
             const double* xt, const double* nrm, double* out, int parts, bool dl) {
  {
    StageScope s(p, GGEM_STAGE_BIN);
    HIP_TRY(launch_bin(p, p.src, ns, xs, f, nullptr, true, true));
    if (xt == xs && nt == ns) {
      // targets coincide with the sources: reuse their binning
      p.tview = &p.src;
      if (dl && nt > 0) {
        gather_normals<T><<<(unsigned)((nt + 255) / 256), 256, 0, p.stream>>>(
            (int)nt, p.src.perm, nrm, (T*)p.tgt.s, (size_t)p.p.max_tgt);
        HIP_TRY(hipGetLastError());
      }
    } else {
      HIP_TRY(launch_bin(p, p.tgt, nt, xt, dl ? nrm : nullptr, nullptr, false, false));
      p.tview = &p.tgt;
    }
    p.tnrm = p.tgt.s;
  }
  const bool glob = (parts & GGEM_PART_GLOBAL) != 0 && nt > 0;
  const bool local = (parts & GGEM_PART_LOCAL) != 0;
  const bool spectral = glob && p.interp_mode == GGEM_INTERP_SPECTRAL;
  if (!local) {
    int rc = zero_ul<T>(p, (int)nt);
    if (rc) return rc;
  }
  // side stream: wall data (and gauge, wall-plane FFT), then the local sum at
  // the targets; the main stream meanwhile spreads and transforms.  While the
  // caller's stream is being captured into a graph, or when the plan has no
  // second stream (the allocation-free entry), everything stays on the
  // caller's stream in the same order.
  const hipStream_t main_stream = p.stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(main_stream, &cap));
  const bool fork = cap == hipStreamCaptureStatusNone && p.side != nullptr;
  // Expected work of the local sum against the spread's, from the mean
  // source density: pairs within r_c per target and node updates per node
  // (weighted by their measured relative cost per pair).  A local sum well
  // below the spread finishes before tau starts.
  const double dens = (double)ns / (p.p.Lx * p.p.Lz * 2.0 * p.p.H);
  const double near_cost = (dl ? 8.0 : 5.0) * (double)nt * dens;
  const double spread_cost = (double)p.p.Nx * p.p.Nz * p.p.Ny * dens;
  const bool one_join = local && near_cost < 0.5 * spread_cost;
  if (fork) {
    HIP_TRY(hipEventRecord(p.ev_fork, main_stream));
    HIP_TRY(hipStreamWaitEvent(p.side, p.ev_fork, 0));
    p.stream = p.side;
  }
  int side_rc = GGEM_OK;
  do {
    if (glob) {
      {
        StageScope s(p, GGEM_STAGE_WALL);
        if (launch_wall<T>(p) != hipSuccess || (dl && launch_gauge(p) != hipSuccess)) {
          side_rc = fail(GGEM_E_DEVICE, "wall data launch failed");
          break;
        }
      }
      if (launch_fft_forward<T>(p, p.wall_phys, p.wall_spec, 6) != hipSuccess) {
        side_rc = fail(GGEM_E_DEVICE, "wall FFT launch failed");
        break;
      }
    }
    if (fork && hipEventRecord(p.ev_wall, p.side) != hipSuccess) {
      side_rc = fail(GGEM_E_DEVICE, "event record failed");
      break;
    }
    if (local) {
      StageScope s(p, GGEM_STAGE_NEAR);
      const hipError_t e = dl ? launch_near_dl<T>(p, (int)nt) : launch_near_sl<T>(p, (int)nt);
      if (e != hipSuccess) {
        side_rc = fail(GGEM_E_DEVICE, "local sum launch failed");
        break;
      }
    }
    if (fork && hipEventRecord(p.ev_near, p.side) != hipSuccess)
      side_rc = fail(GGEM_E_DEVICE, "event record failed");
  } while (false);
  p.stream = main_stream;
  if (side_rc) return side_rc;
  if (glob) {
    const int Ny = p.p.Ny;
    {
      StageScope s(p, GGEM_STAGE_SPREAD);
      HIP_TRY(launch_spread<T>(p, 0));
    }
    {
      StageScope s(p, GGEM_STAGE_FFT_FWD);
      HIP_TRY(launch_fft_forward<T>(p, p.phys, p.specA, 3 * Ny));
    }
    {
      StageScope s(p, GGEM_STAGE_CHEB_FWD);
      HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 3, true));
    }
    // tau needs the wall data; when the local sum is expected to be done by
    // then too, one wait for it (it follows the wall data on the second
    // stream) also serves the interpolation
    if (fork) HIP_TRY(hipStreamWaitEvent(p.stream, one_join ? p.ev_near : p.ev_wall, 0));
    {
      StageScope s(p, GGEM_STAGE_TAU);
      HIP_TRY(launch_tau<T>(p, dl));
    }
    const int nf = dl ? 6 : 3;
    if (spectral) {
      // the Chebyshev coefficients stay in y; in x and z they are deconvolved,
      // padded and transformed onto the oversampled grid
      StageScope s(p, GGEM_STAGE_FFT_INV);
      HIP_TRY(launch_nufft_pad<T>(p, nf));
      p.over->stream = p.stream;
      HIP_TRY(launch_fft_inverse<T>(*p.over, p.over_spec, p.over_phys, nf * Ny));
      HIP_TRY(launch_row_gemm<T>(p, (const T*)p.cth, p.th_kp, Ny, p.th_planes, p.over_phys,
                                 p.over_theta, 4L * p.p.Nx * p.p.Nz, nf));
    } else {
      {
        StageScope s(p, GGEM_STAGE_CHEB_INV);
        HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, nf, false));
      }
      {
        StageScope s(p, GGEM_STAGE_FFT_INV);
        HIP_TRY(launch_fft_inverse<T>(p, p.specB, p.phys, nf * Ny));
      }
    }
  }
  if (fork && !(glob && one_join)) HIP_TRY(hipStreamWaitEvent(p.stream, p.ev_near, 0));
  {
    StageScope s(p, GGEM_STAGE_INTERP);
    if (spectral) HIP_TRY(launch_spectral_eval<T>(p, (int)nt, out, dl));
    else HIP_TRY(launch_interp<T>(p, (int)nt, out, dl, glob));
  }
  return finish(p);
}

}  // namespace

namespace ggem {

template <typename T>
int batch_phase_bin(Plan& p, long long ns, const double* xs, const double* f) {
  HIP_TRY(launch_bin(p, p.src, ns, xs, f, nullptr, true, true));
  p.tview = &p.src;
  p.tnrm = p.tgt.s;
  if (ns > 0) launch_near_order_sources(p);
  HIP_TRY(hipGetLastError());
  return GGEM_OK;
}

template <typename T>
int batch_phase_wall(Plan& p) {
  HIP_TRY(launch_wall_sum<T>(p));
  HIP_TRY(launch_fft_forward<T>(p, p.wall_phys, p.wall_spec, 6));
  return GGEM_OK;
}

template <typename T>
int batch_phase_grid(Plan& p) {
  const int Ny = p.p.Ny;
  HIP_TRY(launch_fft_forward<T>(p, p.phys, p.specA, 3 * Ny));
  HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 3, true));
  HIP_TRY(launch_tau<T>(p, false));
  if (p.interp_mode == GGEM_INTERP_SPECTRAL) {
    HIP_TRY(launch_nufft_pad<T>(p, 3));
    p.over->stream = p.stream;
    HIP_TRY(launch_fft_inverse<T>(*p.over, p.over_spec, p.over_phys, 3 * Ny));
    HIP_TRY(launch_row_gemm<T>(p, (const T*)p.cth, p.th_kp, Ny, p.th_planes, p.over_phys,
                               p.over_theta, 4L * p.p.Nx * p.p.Nz, 3));
  } else {
    HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 3, false));
    HIP_TRY(launch_fft_inverse<T>(p, p.specB, p.phys, 3 * Ny));
  }
  return GGEM_OK;
}

template <typename T>
int batch_phase_interp(Plan& p, long long nt, double* out) {
  if (nt <= 0) return GGEM_OK;
  if (p.interp_mode == GGEM_INTERP_SPECTRAL) HIP_TRY(launch_spectral_eval<T>(p, (int)nt, out, false));
  else HIP_TRY(launch_interp<T>(p, (int)nt, out, false, true));
  return GGEM_OK;
}

template int batch_phase_bin<double>(Plan&, long long, const double*, const double*);
template int batch_phase_bin<float>(Plan&, long long, const double*, const double*);
template int batch_phase_wall<double>(Plan&);
template int batch_phase_wall<float>(Plan&);
template int batch_phase_grid<double>(Plan&);
template int batch_phase_grid<float>(Plan&);
template int batch_phase_interp<double>(Plan&, long long, double*);
template int batch_phase_interp<float>(Plan&, long long, double*);

}  // namespace ggem

namespace {


int check_eval(Plan& p, long long ns, const double* xs, const double* f, long long nt,
               const double* xt, double* out, int parts) {
  if (ns < 0 || nt < 0) return fail(GGEM_E_ARG, "negative point count");
  if (ns > p.p.max_src) return fail(GGEM_E_CAPACITY, "ns=%lld exceeds max_src=%lld", ns, p.p.max_src);
  if (nt > p.p.max_tgt) return fail(GGEM_E_CAPACITY, "nt=%lld exceeds max_tgt=%lld", nt, p.p.max_tgt);
  if (ns > 0 && (!xs || !f)) return fail(GGEM_E_ARG, "null source array");
  if (nt > 0 && (!xt || !out)) return fail(GGEM_E_ARG, "null target array");
  if (parts < 1 || parts > 3) return fail(GGEM_E_ARG, "parts must be 1, 2 or 3");
  return GGEM_OK;
}

// Validate the parameters and fill in a plan's geometry (no device work).
int init_plan(Plan& p, const ggem_params* prm, hipStream_t stream) {
  ggem_params q = *prm;
  if (!(q.Lx > 0 && q.Lz > 0 && isfinite(q.Lx) && isfinite(q.Lz)))
    return fail(GGEM_E_ARG, "Lx, Lz must be positive");
  if (!(q.H > 0 && isfinite(q.H))) return fail(GGEM_E_ARG, "H must be positive");
  if (!(q.alpha > 0 && isfinite(q.alpha))) return fail(GGEM_E_ARG, "alpha must be positive");
  if (q.rc == 0) q.rc = 4.0 / q.alpha;
  if (!(q.rc > 0 && isfinite(q.rc))) return fail(GGEM_E_ARG, "rc must be positive");
  const double Lmin = q.Lx < q.Lz ? q.Lx : q.Lz;
  if (!(q.rc < 0.5 * Lmin * (1.0 - 1e-9)))
    return fail(GGEM_E_ARG, "rc=%g must be below half the period (alpha L > 8 at rc = 4/alpha)", q.rc);
  int rx[12], rz[12], nrx = 0, nrz = 0;
  if (q.Nx % 2 || q.Nz % 2 || q.Nx < 8 || q.Nz < 8 || q.Nx > kMaxFFT || q.Nz > kMaxFFT ||
      !factor_radices(q.Nx, rx, &nrx) || !factor_radices(q.Nz, rz, &nrz))
    return fail(GGEM_E_ARG, "Nx, Nz must be even, 8..512 and products of 2, 3, 5");
  if (q.Ny < 5 || q.Ny > kMaxNy) return fail(GGEM_E_ARG, "Ny must be in 5..129");
  if (q.precision != GGEM_FP64 && q.precision != GGEM_MIXED && q.precision != GGEM_MIXED_BF16)
    return fail(GGEM_E_ARG, "precision must be GGEM_FP64, GGEM_MIXED or GGEM_MIXED_BF16");
  if (q.max_src < 0 || q.max_tgt < 0 || q.max_src > (1LL << 30) || q.max_tgt > (1LL << 30))
    return fail(GGEM_E_ARG, "capacities must be in 0..2^30");
  if (!(q.cell_scale >= 0.0 && q.cell_scale <= 4.0)) return fail(GGEM_E_ARG, "cell_scale must be in 0..4");

  memset(&p, 0, sizeof(Plan));
  p.p = q;
  p.stream = stream;
  (void)hipGetDevice(&p.device);
  p.fp64 = q.precision == GGEM_FP64;
  p.bf16 = q.precision == GGEM_MIXED_BF16;
  p.timed_stage = -1;
  p.rc = q.rc;
  p.rc2 = q.rc * q.rc;
  p.dx = q.Lx / q.Nx;
  p.dz = q.Lz / q.Nz;
  p.Nzh = q.Nz / 2 + 1;
  p.nmodes = q.Nx * p.Nzh;
  p.nradx = nrx;
  p.nradz = nrz;
  for (int i = 0; i < 12; ++i) {
    p.radx[i] = i < nrx ? rx[i] : 1;
    p.radz[i] = i < nrz ? rz[i] : 1;
  }
  // cell list: cells strictly larger than rc (times the cell scale), at
  // most kMaxCells of them
  double cs = q.rc * (q.cell_scale > 1.0 ? q.cell_scale : 1.0) * (1.0 + 1e-10);
  CellGeom& g = p.cg;
  for (;;) {
    g.ncx = (int)floor(q.Lx / cs);
    g.ncz = (int)floor(q.Lz / cs);
    g.ncy = (int)floor(2.0 * q.H / cs);
    if (g.ncx < 1) g.ncx = 1;
    if (g.ncz < 1) g.ncz = 1;
    if (g.ncy < 1) g.ncy = 1;
    if ((long)g.ncx * g.ncy * g.ncz <= kMaxCells) break;
    cs *= 1.25;
  }
  g.ncells = g.ncx * g.ncy * g.ncz;
  g.nzs = kMaxZSub;
  while (g.nzs > 1 && (long)g.ncells * g.nzs > kMaxCells) g.nzs >>= 1;
  g.nbuckets = g.ncells * g.nzs;
  g.Lx = q.Lx;
  g.Lz = q.Lz;
  g.H = q.H;
  g.invLx = 1.0 / q.Lx;
  g.invLz = 1.0 / q.Lz;
  g.icx = g.ncx / q.Lx;
  g.icz = g.ncz / q.Lz;
  g.icy = g.ncy / (2.0 * q.H);

  return GGEM_OK;
}

}  // namespace

extern "C" int ggem_plan_create(const ggem_params* prm, void* hip_stream, ggem_plan_t* out) {
  if (!prm || !out) return fail(GGEM_E_ARG, "null argument");
  *out = nullptr;
  ggem_plan_s* h = new (std::nothrow) ggem_plan_s();
  if (!h) return fail(GGEM_E_NOMEM, "host allocation failed");
  Plan& p = h->p;
  if (int rc = init_plan(p, prm, (hipStream_t)hip_stream)) {
    delete h;
    return rc;
  }
  Carver sizing{nullptr, 0};
  layout_plan(p, sizing);
  p.block_bytes = sizing.off;
  p.owns_block = true;
  p.owns_flags_host = true;
  bool ok = hipMalloc(&p.block, p.block_bytes) == hipSuccess;
  if (ok) {
    Carver c{(char*)p.block, 0};
    layout_plan(p, c);
  }
  ok = ok && hipHostMalloc((void**)&p.flags_host, sizeof(unsigned), 0) == hipSuccess &&
       hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking) == hipSuccess &&
       // fork/join events order two streams of this device only: no
       // system-scope fence (device-scope ordering is kept)
       hipEventCreateWithFlags(&p.ev_fork, hipEventDisableTiming | hipEventDisableSystemFence) == hipSuccess &&
       hipEventCreateWithFlags(&p.ev_wall, hipEventDisableTiming | hipEventDisableSystemFence) == hipSuccess &&
       hipEventCreateWithFlags(&p.ev_near, hipEventDisableTiming | hipEventDisableSystemFence) == hipSuccess;
  if (!ok) {
    free_plan(p);
    delete h;
    return fail(GGEM_E_NOMEM, "device allocation failed");
  }
  HostStage sz{nullptr, 0, 0};
  (void)plan_constants(p, sz);
  std::vector<char> host(sz.off + 64);
  HostStage hs{host.data(), 0, host.size()};
  int rc = plan_constants(p, hs);
  if (rc != GGEM_OK) {
    free_plan(p);
    delete h;
    return rc;
  }
  *out = h;
  return GGEM_OK;
}

extern "C" int ggem_plan_destroy(ggem_plan_t plan) {
  if (!plan) return fail(GGEM_E_ARG, "null plan");
  (void)hipStreamSynchronize(plan->p.stream);
  if (plan->p.side) (void)hipStreamSynchronize(plan->p.side);
  free_plan(plan->p);
  delete plan;
  return GGEM_OK;
}

extern "C" int ggem_plan_set_stream(ggem_plan_t plan, void* hip_stream) {
  if (int rc = check_plan(plan)) return rc;
  plan->p.stream = (hipStream_t)hip_stream;
  return GGEM_OK;
}

extern "C" int ggem_plan_status(ggem_plan_t plan) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  HIP_TRY(hipMemcpyAsync(p.flags_host, p.flags, sizeof(unsigned), hipMemcpyDeviceToHost, p.stream));
  HIP_TRY(hipStreamSynchronize(p.stream));
  const unsigned f = *p.flags_host;
  if (f & kFlagNonFinite) return fail(GGEM_E_DOMAIN, "non-finite input position");
  if (f & kFlagOutside) return fail(GGEM_E_DOMAIN, "point outside the slit");
  return GGEM_OK;
}

extern "C" int ggem_single_layer(ggem_plan_t plan, long long ns, const double* xs,
                                 const double* f, long long nt, const double* xt, double* u,
                                 int parts) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  if (int rc = check_eval(p, ns, xs, f, nt, xt, u, parts)) return rc;
  return p.fp64 ? evaluate<double>(p, ns, xs, f, nt, xt, nullptr, u, parts, false)
                : evaluate<float>(p, ns, xs, f, nt, xt, nullptr, u, parts, false);
}

extern "C" int ggem_double_layer(ggem_plan_t plan, long long ns, const double* xs,
                                 const double* q, long long nt, const double* xt,
                                 const double* nrm, double* v, int parts) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  if (int rc = check_eval(p, ns, xs, q, nt, xt, v, parts)) return rc;
  if (nt > 0 && !nrm) return fail(GGEM_E_ARG, "null normal array");
  return p.fp64 ? evaluate<double>(p, ns, xs, q, nt, xt, nrm, v, parts, true)
                : evaluate<float>(p, ns, xs, q, nt, xt, nrm, v, parts, true);
}

extern "C" int ggem_spread_grid(ggem_plan_t plan, long long ns, const double* xs,
                                const double* f, double* grid) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  if (ns < 0) return fail(GGEM_E_ARG, "negative point count");
  if (ns > p.p.max_src) return fail(GGEM_E_CAPACITY, "ns=%lld exceeds max_src", ns);
  if ((ns > 0 && (!xs || !f)) || !grid) return fail(GGEM_E_ARG, "null array");
  HIP_TRY(launch_bin(p, p.src, ns, xs, f, nullptr, true, true));
  if (p.fp64) {
    HIP_TRY(launch_spread<double>(p, 0));
    HIP_TRY(launch_grid_to_f64<double>(p, grid));
  } else {
    HIP_TRY(launch_spread<float>(p, 0));
    HIP_TRY(launch_grid_to_f64<float>(p, grid));
  }
  return finish(p);
}

// Probes: the global problem with the double layer's gauge, its six stress
// components interpolated first, then its velocity and pressure (the
// coefficients tau keeps from the stress pass, transformed back through the
// same buffers), each added onto the local parts.  All on the plan's stream.
template <typename T>
static int probe_eval(Plan& p, long long ns, const double* xs, const double* f, long long nt,
                      const double* xt, double* u, double* pr, double* sigma) {
  const int Ny = p.p.Ny;
  HIP_TRY(launch_bin(p, p.src, ns, xs, f, nullptr, true, true));
  HIP_TRY(launch_wall<T>(p));
  HIP_TRY(launch_gauge(p));
  HIP_TRY(launch_fft_forward<T>(p, p.wall_phys, p.wall_spec, 6));
  HIP_TRY(launch_spread<T>(p, 0));
  HIP_TRY(launch_fft_forward<T>(p, p.phys, p.specA, 3 * Ny));
  HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 3, true));
  HIP_TRY(launch_tau<T>(p, true));
  HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 6, false));
  HIP_TRY(launch_fft_inverse<T>(p, p.specB, p.phys, 6 * Ny));
  HIP_TRY(launch_probe_local(p, (int)nt, xt, f, u, pr, sigma));
  HIP_TRY(launch_probe_interp<T>(p, (int)nt, xt, 6, 6, sigma, 6, nullptr, 0));
  HIP_TRY(launch_tau_export<T>(p));
  HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 4, false));
  HIP_TRY(launch_fft_inverse<T>(p, p.specB, p.phys, 4 * Ny));
  HIP_TRY(launch_probe_interp<T>(p, (int)nt, xt, 4, 3, u, 3, pr, 1));
  return finish(p);
}

extern "C" int ggem_probe(ggem_plan_t plan, long long ns, const double* xs, const double* f,
                          long long nt, const double* xt, double* u, double* pr, double* sigma) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  if (ns < 0 || nt < 0) return fail(GGEM_E_ARG, "negative point count");
  if (ns > p.p.max_src) return fail(GGEM_E_CAPACITY, "ns=%lld exceeds max_src=%lld", ns, p.p.max_src);
  if (nt > p.p.max_tgt) return fail(GGEM_E_CAPACITY, "nt=%lld probes exceed max_tgt=%lld", nt, p.p.max_tgt);
  if (ns > 0 && (!xs || !f)) return fail(GGEM_E_ARG, "null source array");
  if (nt > 0 && (!xt || !u || !pr || !sigma)) return fail(GGEM_E_ARG, "null probe array");
  return p.fp64 ? probe_eval<double>(p, ns, xs, f, nt, xt, u, pr, sigma)
                : probe_eval<float>(p, ns, xs, f, nt, xt, u, pr, sigma);
}

extern "C" int ggem_undisturbed_traction(ggem_plan_t plan, int kind, double rate, long long n,
                                         const double* x, const double* nrm, double* f) {
  if (int rc = check_plan(plan)) return rc;
  if (kind != GGEM_FLOW_SHEAR && kind != GGEM_FLOW_POISEUILLE)
    return fail(GGEM_E_ARG, "unknown flow kind %d", kind);
  if (n < 0 || n > (1LL << 30)) return fail(GGEM_E_ARG, "point count out of range");
  if (n > 0 && (!x || !nrm || !f)) return fail(GGEM_E_ARG, "null array");
  HIP_TRY(launch_undisturbed_traction(plan->p, kind, rate, (int)n, x, nrm, f));
  return GGEM_OK;
}

extern "C" int ggem_plan_time_stage(ggem_plan_t plan, int stage, int max_calls) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  if (stage >= GGEM_NUM_STAGES) return fail(GGEM_E_ARG, "unknown stage %d", stage);
  HIP_TRY(hipStreamSynchronize(p.stream));
  destroy_timer(p);
  if (stage < 0) return GGEM_OK;
  if (max_calls < 1 || max_calls > 1000000) return fail(GGEM_E_ARG, "max_calls out of range");
  p.timed_ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_calls];
  if (!p.timed_ev) return fail(GGEM_E_NOMEM, "host allocation failed");
  for (int i = 0; i < 2 * max_calls; ++i) {
    // timing-only events: no system-scope fence, so recording them around a
    // stage adds no cache write-back between its kernels
    hipError_t e = hipEventCreateWithFlags(&p.timed_ev[i], hipEventDisableSystemFence);
    if (e != hipSuccess) {
      p.timed_max = i / 2;
      destroy_timer(p);
      return fail(GGEM_E_DEVICE, "hipEventCreate failed: %s", hipGetErrorString(e));
    }
  }
  p.timed_max = max_calls;
  p.timed_calls = 0;
  p.timed_stage = stage;
  return GGEM_OK;
}

extern "C" int ggem_plan_stage_time(ggem_plan_t plan, double* total_ms, int* calls) {
  if (int rc = check_plan(plan)) return rc;
  if (!total_ms || !calls) return fail(GGEM_E_ARG, "null output");
  Plan& p = plan->p;
  HIP_TRY(hipStreamSynchronize(p.stream));
  double sum = 0.0;
  for (int i = 0; i < p.timed_calls; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.timed_ev[2 * i], p.timed_ev[2 * i + 1]));
    sum += ms;
  }
  *total_ms = sum;
  *calls = p.timed_calls;
  return GGEM_OK;
}

extern "C" int ggem_plan_work(ggem_plan_t plan, unsigned long long* counts) {
  if (int rc = check_plan(plan)) return rc;
  if (!counts) return fail(GGEM_E_ARG, "null output");
  Plan& p = plan->p;
  HIP_TRY(hipMemcpyAsync(counts, p.work, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         p.stream));
  HIP_TRY(hipStreamSynchronize(p.stream));
  return GGEM_OK;
}

extern "C" int ggem_plan_count_work(ggem_plan_t plan, int on) {
  if (int rc = check_plan(plan)) return rc;
  plan->p.count_work = on != 0;
  return GGEM_OK;
}

extern "C" int ggem_plan_set_interp(ggem_plan_t plan, int mode, int msp) {
  if (int rc = check_plan(plan)) return rc;
  Plan& p = plan->p;
  if (mode != GGEM_INTERP_LAGRANGE && mode != GGEM_INTERP_SPECTRAL)
    return fail(GGEM_E_ARG, "mode must be GGEM_INTERP_LAGRANGE or GGEM_INTERP_SPECTRAL");
  if (!p.owns_block) return fail(GGEM_E_ARG, "plan without its own device memory");
  const int Nx = p.p.Nx, Nz = p.p.Nz, Ny = p.p.Ny, Mx = 2 * Nx, Mz = 2 * Nz;
  int rx[12], rz[12], nrx = 0, nrz = 0;
  if (mode == GGEM_INTERP_SPECTRAL) {
    if (msp < 2 || msp > kMaxMsp || msp > Nx || msp > Nz)
      return fail(GGEM_E_ARG, "msp=%d must be in 2..%d and at most Nx and Nz", msp, kMaxMsp);
    if (Mx > kMaxFFT || Mz > kMaxFFT || !factor_radices(Mx, rx, &nrx) ||
        !factor_radices(Mz, rz, &nrz))
      return fail(GGEM_E_ARG, "spectral evaluation needs Nx, Nz <= %d", kMaxFFT / 2);
  }
  // the previous mode's buffers may still be in use by queued work
  HIP_TRY(hipStreamSynchronize(p.stream));
  if (p.side) HIP_TRY(hipStreamSynchronize(p.side));
  free_over(p);
  if (mode == GGEM_INTERP_LAGRANGE) return GGEM_OK;
  Plan* o = new (std::nothrow) Plan();
  if (!o) return fail(GGEM_E_NOMEM, "host allocation failed");
  memset(o, 0, sizeof(Plan));
  o->p = p.p;
  o->p.Nx = Mx;
  o->p.Nz = Mz;
  o->Nzh = Mz / 2 + 1;
  o->nmodes = Mx * o->Nzh;
  o->nradx = nrx;
  o->nradz = nrz;
  for (int i = 0; i < 12; ++i) {
    o->radx[i] = i < nrx ? rx[i] : 1;
    o->radz[i] = i < nrz ? rz[i] : 1;
  }
  o->fp64 = p.fp64;
  o->device = p.device;
  o->timed_stage = -1;
  const size_t elt = p.fp64 ? 8 : 4;
  Carver sz{nullptr, 0};
  (void)sz.take_bytes(2 * (size_t)Mx * elt);
  (void)sz.take_bytes(2 * (size_t)Mz * elt);
  (void)sz.take_bytes(6 * (size_t)Ny * Mx * o->Nzh * 2 * elt);
  (void)sz.take_bytes(6 * (size_t)Ny * Mx * Mz * elt);
  // theta = arccos(y/H): the Chebyshev series is the even Fourier series
  // sum_n a_n cos(n theta), band |n| <= Ny - 1, gridded on th_m = 2 (2N + 1)
  // nodes; planes j = 0 .. th_m/2 are stored, the rest by symmetry
  const int Nc = Ny - 1, thm = 2 * (2 * Nc + 1), thp = thm / 2 + 1;
  const int kp = (Ny + 3) / 4 * 4, rows = (thp + 143) / 144 * 144;
  (void)sz.take_bytes(6 * (size_t)thp * Mx * Mz * elt);
  (void)sz.take_bytes((size_t)rows * kp * elt);
  if (hipMalloc(&p.over_block, sz.off) != hipSuccess) {
    p.over_block = nullptr;
    delete o;
    return fail(GGEM_E_NOMEM, "device allocation of the oversampled grid failed");
  }
  p.over = o;
  Carver c{(char*)p.over_block, 0};
  o->twx = c.take_bytes(2 * (size_t)Mx * elt);
  o->twz = c.take_bytes(2 * (size_t)Mz * elt);
  p.over_spec = c.take_bytes(6 * (size_t)Ny * Mx * o->Nzh * 2 * elt);
  p.over_phys = c.take_bytes(6 * (size_t)Ny * Mx * Mz * elt);
  p.over_theta = c.take_bytes(6 * (size_t)thp * Mx * Mz * elt);
  p.cth = c.take_bytes((size_t)rows * kp * elt);
  p.th_m = thm;
  p.th_planes = thp;
  p.th_kp = kp;
  p.tau_th = M_PI * msp / (3.0 * (2.0 * Nc + 1.0) * (2.0 * Nc + 1.0));
  {
    // cth[j][n] = (1/th_m) sqrt(pi/tau) exp(n^2 tau) cos(2 pi n j / th_m): the
    // deconvolved coefficients summed on the theta grid (zero padded rows)
    std::vector<double> m((size_t)rows * kp, 0.0);
    const double sc = sqrt(M_PI / p.tau_th) / thm;
    for (int j = 0; j < thp; ++j)
      for (int n = 0; n < Ny; ++n) {
        const long q = (2L * n * j) % (2L * thm);  // cos(pi q / th_m), q reduced exactly
        m[(size_t)j * kp + n] = sc * exp((double)n * n * p.tau_th) * cos(M_PI * (double)q / thm);
      }
    hipError_t e;
    if (p.fp64) {
      e = hipMemcpy(p.cth, m.data(), m.size() * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<float> mf(m.begin(), m.end());
      e = hipMemcpy(p.cth, mf.data(), mf.size() * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      free_over(p);
      return fail(GGEM_E_DEVICE, "%s", hipGetErrorString(e));
    }
  }
  std::vector<double> tw(2 * (size_t)(Mx > Mz ? Mx : Mz));
  std::vector<float> tf(tw.size());
  for (int ax = 0; ax < 2; ++ax) {
    const int n = ax == 0 ? Mx : Mz;
    fill_twiddles(n, tw.data());
    void* dst = ax == 0 ? o->twx : o->twz;
    hipError_t e;
    if (p.fp64) {
      e = hipMemcpy(dst, tw.data(), 2 * (size_t)n * 8, hipMemcpyHostToDevice);
    } else {
      for (int i = 0; i < 2 * n; ++i) tf[i] = (float)tw[i];
      e = hipMemcpy(dst, tf.data(), 2 * (size_t)n * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      free_over(p);
      return fail(GGEM_E_DEVICE, "%s", hipGetErrorString(e));
    }
  }
  p.msp = msp;
  p.tau_x = M_PI * msp / (3.0 * (double)Nx * Nx);
  p.tau_z = M_PI * msp / (3.0 * (double)Nz * Nz);
  p.interp_mode = GGEM_INTERP_SPECTRAL;
  return GGEM_OK;
}

// ---- single layer without device allocation --------------------------------
//
// Workspace of ggem_single_layer_noalloc: one static array per GPU, resident
// until the process ends.  Its name is a host-side stand-in in host code, so
// the device address is looked up with hipGetSymbolAddress once per device
// (with that device current) and only that address is used from then on.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kHostStageBytes = (size_t)2 << 20;

struct StaticSlot {
  char* dev;           // device address of this GPU's scratch (null: not looked up yet)
  bool ready;          // the scratch holds the plan constants for `key`
  ggem_params key;
  Plan plan;
  unsigned flags_host;
};

StaticSlot g_slots[kMaxDevices];
char g_host_stage[kHostStageBytes];
std::mutex g_static_mu;

bool same_params(const ggem_params& a, const ggem_params& b) {
  return a.Lx == b.Lx && a.Lz == b.Lz && a.H == b.H && a.alpha == b.alpha && a.rc == b.rc &&
         a.Nx == b.Nx && a.Nz == b.Nz && a.Ny == b.Ny && a.precision == b.precision &&
         a.sync_checks == b.sync_checks && a.max_src == b.max_src && a.max_tgt == b.max_tgt;
}

}  // namespace

extern "C" int ggem_single_layer_noalloc(const ggem_params* prm, void* hip_stream, long long ns,
                                         const double* xs, const double* f, long long nt,
                                         const double* xt, double* u) {
  if (!prm) return fail(GGEM_E_ARG, "null parameters");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GGEM_E_ARG, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& s = g_slots[dev];
  if (!s.dev) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    s.dev = (char*)ptr;
  }
  if (!(s.ready && same_params(s.key, *prm))) {
    s.ready = false;
    Plan q;
    if (int rc = init_plan(q, prm, (hipStream_t)hip_stream)) return rc;
    Carver sizing{nullptr, 0};
    layout_plan(q, sizing);
    if (sizing.off > kScratchBytes)
      return fail(GGEM_E_CAPACITY,
                  "workspace of %zu bytes for this grid and these capacities exceeds the "
                  "%zu-byte static scratch array",
                  sizing.off, kScratchBytes);
    HostStage hsz{nullptr, 0, 0};
    (void)plan_constants(q, hsz);
    if (hsz.off > kHostStageBytes)
      return fail(GGEM_E_CAPACITY, "plan constants of %zu bytes exceed the %zu-byte host staging",
                  hsz.off, kHostStageBytes);
    Plan& p = s.plan;
    p = q;
    Carver c{s.dev, 0};
    layout_plan(p, c);
    p.block = s.dev;
    p.block_bytes = sizing.off;
    p.owns_block = false;
    p.flags_host = &s.flags_host;
    p.owns_flags_host = false;
    HostStage hs{g_host_stage, 0, kHostStageBytes};
    if (int rc = plan_constants(p, hs)) return rc;
    s.key = *prm;
    s.ready = true;
  }
  Plan& p = s.plan;
  p.stream = (hipStream_t)hip_stream;
  if (int rc = check_eval(p, ns, xs, f, nt, xt, u, GGEM_PART_ALL)) return rc;
  return p.fp64 ? evaluate<double>(p, ns, xs, f, nt, xt, nullptr, u, GGEM_PART_ALL, false)
                : evaluate<float>(p, ns, xs, f, nt, xt, nullptr, u, GGEM_PART_ALL, false);
}
