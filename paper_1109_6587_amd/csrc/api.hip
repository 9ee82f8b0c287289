// C-ABI of the GGEM slit library: plan creation (validation, plan-time
// constants, workspace), the two evaluations and the spread diagnostic.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

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

template <typename T>
bool dev_alloc(T** ptr, size_t count) {
  if (count == 0) count = 1;
  return hipMalloc((void**)ptr, count * sizeof(T)) == hipSuccess;
}

void free_plan(Plan& p) {
  void* ptrs[] = {p.y,         p.cf64,        p.ci64,        p.cf32,       p.ci32,
                  p.twx,       p.twz,         p.infl,        p.ul,         p.phys,
                  p.specA,     p.specB,       p.wall_phys,   p.wall_spec,  p.tau_scr,
                  p.gauge,     p.flags,       p.item_count,  p.src.keys,   p.src.counts,
                  p.src.offs,  p.src.cell_start, p.src.item_start, p.src.perm, p.src.x,
                  p.src.sub_start, p.tgt.sub_start, p.wall.sub_start,
                  p.src.cflags, p.tgt.cflags, p.wall.cflags,
                  p.src.item_cell, p.tgt.item_cell, p.wall.item_cell,
                  p.src.y,     p.src.z,       p.src.s,       p.tgt.keys,   p.tgt.counts,
                  p.tgt.offs,  p.tgt.cell_start, p.tgt.item_start, p.tgt.perm, p.tgt.x,
                  p.tgt.y,     p.tgt.z,       p.tgt.s,       p.nconst,     p.sweep,
                  p.wall.keys, p.wall.counts, p.wall.offs,   p.wall.cell_start,
                  p.wall.item_start, p.wall.perm, p.wall.x,  p.wall.y,     p.wall.z,
                  p.wall.s,    p.work,        p.wall_part};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (p.flags_host) (void)hipHostFree(p.flags_host);
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

bool alloc_binned(Binned& b, long long cap, const CellGeom& g, size_t elt) {
  const long long nch = kMaxChunks + 1;
  const int ncells = g.ncells, nb = g.nbuckets;
  return dev_alloc(&b.keys, (size_t)cap) && dev_alloc(&b.counts, (size_t)nb * (nch + 1)) &&
         dev_alloc(&b.offs, (size_t)nb * (nch + 1)) && dev_alloc(&b.sub_start, nb + 1) &&
         dev_alloc(&b.cell_start, ncells + 1) && dev_alloc(&b.cflags, kMaxChunks + 1) &&
         dev_alloc(&b.item_start, ncells + 1) &&
         dev_alloc(&b.item_cell, (size_t)(cap / kNearBlock) + ncells + 1) &&
         dev_alloc(&b.perm, (size_t)cap) &&
         dev_alloc(&b.x, (size_t)cap) && dev_alloc(&b.y, (size_t)cap) &&
         dev_alloc(&b.z, (size_t)cap) &&
         hipMalloc(&b.s, (size_t)(3 * (cap > 0 ? cap : 1)) * elt) == hipSuccess;
}

// padded (MP x KP) copy of an (Ny x Ny) matrix
template <typename T>
std::vector<T> padded(const std::vector<double>& a, int Ny, int MP, int KP) {
  std::vector<T> o((size_t)MP * KP, (T)0);
  for (int r = 0; r < Ny; ++r)
    for (int c = 0; c < Ny; ++c) o[(size_t)r * KP + c] = (T)a[(size_t)r * Ny + c];
  return o;
}

// cos(pi * m / N) with the argument reduced exactly (m integer)
double cospi_frac(long m, int N) {
  m %= 2L * N;
  return cos(M_PI * (double)m / (double)N);
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

int plan_constants(Plan& p) {
  const int Ny = p.p.Ny, N = Ny - 1, Nx = p.p.Nx, Nz = p.p.Nz;
  std::vector<double> y(Ny);
  for (int j = 0; j < Ny; ++j) y[j] = p.p.H * cospi_frac(j, N);
  HIP_TRY(hipMemcpy(p.y, y.data(), Ny * sizeof(double), hipMemcpyHostToDevice));
  std::vector<double> cf((size_t)Ny * Ny), ci((size_t)Ny * Ny);
  const double norm = 1.0 / ((double)Nx * (double)Nz);
  for (int n = 0; n < Ny; ++n)
    for (int j = 0; j < Ny; ++j) {
      const double cbn = (n == 0 || n == N) ? 2.0 : 1.0;
      const double cbj = (j == 0 || j == N) ? 2.0 : 1.0;
      const double c = cospi_frac((long)n * j, N);
      cf[(size_t)n * Ny + j] = 2.0 / (N * cbn * cbj) * c * norm;
      ci[(size_t)j * Ny + n] = c;
    }
  const int MP = ((Ny + 15) / 16) * 16, KP = ((Ny + 3) / 4) * 4;
  auto cf64 = padded<double>(cf, Ny, MP, KP), ci64 = padded<double>(ci, Ny, MP, KP);
  auto cf32 = padded<float>(cf, Ny, MP, KP), ci32 = padded<float>(ci, Ny, MP, KP);
  HIP_TRY(hipMemcpy(p.cf64, cf64.data(), cf64.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.ci64, ci64.data(), ci64.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.cf32, cf32.data(), cf32.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p.ci32, ci32.data(), ci32.size() * 4, hipMemcpyHostToDevice));
  for (int ax = 0; ax < 2; ++ax) {
    const int n = ax == 0 ? Nx : Nz;
    std::vector<double> tw(2 * (size_t)n);
    for (int t = 0; t < n; ++t) {
      // exp(-2 pi i t/n) = cos(pi 2t/n) - i sin(pi 2t/n)
      const long m = (2L * t) % (2L * n);
      tw[2 * t] = cos(M_PI * (double)m / n);
      tw[2 * t + 1] = -sin(M_PI * (double)m / n);
    }
    void* dst = ax == 0 ? p.twx : p.twz;
    if (p.fp64) {
      HIP_TRY(hipMemcpy(dst, tw.data(), tw.size() * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> tf(tw.begin(), tw.end());
      HIP_TRY(hipMemcpy(dst, tf.data(), tf.size() * 4, hipMemcpyHostToDevice));
    }
  }
  std::vector<double> nc(3 * (size_t)Ny, 0.0);
  for (int n = 2; n < Ny; ++n) {
    nc[n] = 1.0 / (4.0 * n * (n - 1));
    nc[Ny + n] = 1.0 / (2.0 * ((double)n * n - 1.0));
    nc[2 * Ny + n] = 1.0 / (4.0 * n * (n + 1));
  }
  HIP_TRY(hipMemcpy(p.nconst, nc.data(), nc.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(launch_influence(p));
  {
    // wall nodes (x_i, -H, z_k) then (x_i, +H, z_k), binned once
    const size_t nw = 2 * (size_t)Nx * Nz;
    std::vector<double> wpos(3 * nw);
    for (int w = 0; w < 2; ++w)
      for (int i = 0; i < Nx; ++i)
        for (int k = 0; k < Nz; ++k) {
          const size_t r = (size_t)w * Nx * Nz + (size_t)i * Nz + k;
          wpos[3 * r] = i * p.dx;
          wpos[3 * r + 1] = w ? p.p.H : -p.p.H;
          wpos[3 * r + 2] = k * p.dz;
        }
    double* dpos = nullptr;
    HIP_TRY(hipMalloc((void**)&dpos, wpos.size() * sizeof(double)));
    hipError_t e = hipMemcpy(dpos, wpos.data(), wpos.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_bin(p, p.wall, (long long)nw, dpos, nullptr, nullptr, false, true);
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
    (void)hipFree(dpos);
    HIP_TRY(e);
  }
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
  if (!local) {
    int rc = zero_ul<T>(p, (int)nt);
    if (rc) return rc;
  }
  // side stream: wall data (and gauge, wall-plane FFT), then the local sum at
  // the targets; the main stream meanwhile spreads and transforms.  While the
  // caller's stream is being captured into a graph, everything stays on it
  // (in the same order), so a capture never forks into the plan's stream.
  const hipStream_t main_stream = p.stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(main_stream, &cap));
  const bool fork = cap == hipStreamCaptureStatusNone;
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
    {
      StageScope s(p, GGEM_STAGE_CHEB_INV);
      HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, nf, false));
    }
    {
      StageScope s(p, GGEM_STAGE_FFT_INV);
      HIP_TRY(launch_fft_inverse<T>(p, p.specB, p.phys, nf * Ny));
    }
  }
  if (fork && !(glob && one_join)) HIP_TRY(hipStreamWaitEvent(p.stream, p.ev_near, 0));
  {
    StageScope s(p, GGEM_STAGE_INTERP);
    HIP_TRY(launch_interp<T>(p, (int)nt, out, dl, glob));
  }
  return finish(p);
}

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

}  // namespace

extern "C" int ggem_plan_create(const ggem_params* prm, void* hip_stream, ggem_plan_t* out) {
  if (!prm || !out) return fail(GGEM_E_ARG, "null argument");
  *out = nullptr;
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
  if (q.precision != GGEM_FP64 && q.precision != GGEM_MIXED)
    return fail(GGEM_E_ARG, "precision must be GGEM_FP64 or GGEM_MIXED");
  if (q.max_src < 0 || q.max_tgt < 0 || q.max_src > (1LL << 30) || q.max_tgt > (1LL << 30))
    return fail(GGEM_E_ARG, "capacities must be in 0..2^30");

  ggem_plan_s* h = new (std::nothrow) ggem_plan_s();
  if (!h) return fail(GGEM_E_NOMEM, "host allocation failed");
  Plan& p = h->p;
  memset(&p, 0, sizeof(Plan));
  p.p = q;
  p.stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&p.device);
  p.fp64 = q.precision == GGEM_FP64;
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
  // cell list: cells strictly larger than rc, at most kMaxCells of them
  double cs = q.rc * (1.0 + 1e-10);
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

  const size_t elt = p.fp64 ? 8 : 4;
  const size_t Ny = q.Ny, Nx = q.Nx, Nz = q.Nz;
  const int MP = ((q.Ny + 15) / 16) * 16, KP = ((q.Ny + 3) / 4) * 4;
  bool ok = dev_alloc(&p.y, Ny) && dev_alloc(&p.cf64, (size_t)MP * KP) &&
            dev_alloc(&p.ci64, (size_t)MP * KP) && dev_alloc(&p.cf32, (size_t)MP * KP) &&
            dev_alloc(&p.ci32, (size_t)MP * KP) &&
            hipMalloc(&p.twx, 2 * Nx * elt) == hipSuccess &&
            hipMalloc(&p.twz, 2 * Nz * elt) == hipSuccess &&
            dev_alloc(&p.infl, 4 * (size_t)p.nmodes) &&
            hipMalloc(&p.ul, kNearSlices * 3 * (size_t)(q.max_tgt > 0 ? q.max_tgt : 1) * elt) ==
                hipSuccess &&
            hipMalloc(&p.phys, 6 * Ny * Nx * Nz * elt) == hipSuccess &&
            hipMalloc(&p.specA, 6 * Ny * p.nmodes * 2 * elt) == hipSuccess &&
            hipMalloc(&p.specB, 6 * Ny * p.nmodes * 2 * elt) == hipSuccess &&
            hipMalloc(&p.wall_phys, 6 * Nx * Nz * elt) == hipSuccess &&
            hipMalloc(&p.wall_part, kWallSlices * 6 * Nx * Nz * elt) == hipSuccess &&
            hipMalloc(&p.wall_spec, 6 * (size_t)p.nmodes * 2 * elt) == hipSuccess &&
            dev_alloc(&p.tau_scr, 2 * 9 * Ny * (size_t)p.nmodes) &&
            dev_alloc(&p.nconst, 3 * Ny) &&
            dev_alloc(&p.sweep, (6 * Ny + 2) * (size_t)p.nmodes) &&
            dev_alloc(&p.gauge, (size_t)(q.max_src / 256 + 4)) && dev_alloc(&p.flags, 1) &&
            dev_alloc(&p.item_count, 4) && dev_alloc(&p.work, 2) &&
            hipHostMalloc((void**)&p.flags_host, sizeof(unsigned), 0) == hipSuccess &&
            alloc_binned(p.src, q.max_src, g, elt) &&
            alloc_binned(p.tgt, q.max_tgt, g, elt) &&
            alloc_binned(p.wall, 2LL * q.Nx * q.Nz, g, elt) &&
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
  int rc = plan_constants(p);
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
