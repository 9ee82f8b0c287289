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

struct ggem_plan_s {
  Plan p;
};

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

namespace {

bool factor_radices(int n, int* r, int* nr) {
  int k = 0;
  while (n % 4 == 0 && n > 4) {
    r[k++] = 4;
    n /= 4;
  }
  const int ps[4] = {4, 2, 3, 5};
  for (int i = 0; i < 4; ++i)
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
                  p.src.y,     p.src.z,       p.src.s,       p.tgt.keys,   p.tgt.counts,
                  p.tgt.offs,  p.tgt.cell_start, p.tgt.item_start, p.tgt.perm, p.tgt.x,
                  p.tgt.y,     p.tgt.z,       p.tgt.s};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (p.flags_host) (void)hipHostFree(p.flags_host);
}

bool alloc_binned(Binned& b, long long cap, int ncells, size_t elt) {
  const long long nch = (cap + kBinChunk - 1) / kBinChunk;
  return dev_alloc(&b.keys, (size_t)cap) && dev_alloc(&b.counts, (size_t)ncells * (nch + 1)) &&
         dev_alloc(&b.offs, (size_t)ncells * (nch + 1)) && dev_alloc(&b.cell_start, ncells + 1) &&
         dev_alloc(&b.item_start, ncells + 1) && dev_alloc(&b.perm, (size_t)cap) &&
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

__global__ void fill_u32(unsigned* p, unsigned v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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
  HIP_TRY(launch_influence(p));
  HIP_TRY(hipStreamSynchronize(p.stream));
  return GGEM_OK;
}

int check_plan(ggem_plan_t plan) {
  if (!plan) return fail(GGEM_E_ARG, "null plan");
  return GGEM_OK;
}

template <typename T>
int zero_ul(Plan& p, int nt) {
  const size_t n = (size_t)3 * p.p.max_tgt;
  if (nt > 0) fill_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>((T*)p.ul, n);
  HIP_TRY(hipGetLastError());
  return GGEM_OK;
}

int finish(Plan& p) {
  HIP_TRY(hipMemcpyAsync(p.flags_host, p.flags, sizeof(unsigned), hipMemcpyDeviceToHost, p.stream));
  if (!p.p.sync_checks) return GGEM_OK;
  HIP_TRY(hipStreamSynchronize(p.stream));
  const unsigned f = *p.flags_host;
  if (f & kFlagNonFinite) return fail(GGEM_E_DOMAIN, "non-finite input position");
  if (f & kFlagOutside) return fail(GGEM_E_DOMAIN, "point outside the slit");
  return GGEM_OK;
}

template <typename T>
int evaluate(Plan& p, long long ns, const double* xs, const double* f, long long nt,
             const double* xt, const double* nrm, double* out, int parts, bool dl) {
  fill_u32<<<1, 64, 0, p.stream>>>(p.flags, 0u, 1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_bin(p, p.src, ns, xs, f, nullptr, true));
  HIP_TRY(launch_bin(p, p.tgt, nt, xt, dl ? nrm : nullptr, nullptr, false));
  if (parts & GGEM_PART_LOCAL) {
    if (dl) HIP_TRY(launch_near_dl<T>(p, (int)nt));
    else HIP_TRY(launch_near_sl<T>(p, (int)nt));
  } else {
    int rc = zero_ul<T>(p, (int)nt);
    if (rc) return rc;
  }
  const bool glob = (parts & GGEM_PART_GLOBAL) != 0;
  if (glob && nt > 0) {
    const int Ny = p.p.Ny;
    HIP_TRY(launch_wall<T>(p));
    if (dl) HIP_TRY(launch_gauge(p));
    HIP_TRY(launch_spread<T>(p, 0));
    HIP_TRY(launch_fft_forward<T>(p, p.phys, p.specA, 3 * Ny));
    HIP_TRY(launch_fft_forward<T>(p, p.wall_phys, p.wall_spec, 6));
    HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, 3, true));
    HIP_TRY(launch_tau<T>(p, dl));
    const int nf = dl ? 6 : 3;
    HIP_TRY(launch_cheb<T>(p, p.specA, p.specB, nf, false));
    HIP_TRY(launch_fft_inverse<T>(p, p.specB, p.phys, nf * Ny));
  }
  HIP_TRY(launch_interp<T>(p, (int)nt, out, dl, glob));
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
            hipMalloc(&p.ul, 3 * (size_t)(q.max_tgt > 0 ? q.max_tgt : 1) * elt) == hipSuccess &&
            hipMalloc(&p.phys, 6 * Ny * Nx * Nz * elt) == hipSuccess &&
            hipMalloc(&p.specA, 6 * Ny * p.nmodes * 2 * elt) == hipSuccess &&
            hipMalloc(&p.specB, 6 * Ny * p.nmodes * 2 * elt) == hipSuccess &&
            hipMalloc(&p.wall_phys, 6 * Nx * Nz * elt) == hipSuccess &&
            hipMalloc(&p.wall_spec, 6 * (size_t)p.nmodes * 2 * elt) == hipSuccess &&
            dev_alloc(&p.tau_scr, 2 * 7 * Ny * (size_t)p.nmodes) &&
            dev_alloc(&p.gauge, (size_t)(q.max_src / 256 + 4)) && dev_alloc(&p.flags, 1) &&
            dev_alloc(&p.item_count, 4) &&
            hipHostMalloc((void**)&p.flags_host, sizeof(unsigned), 0) == hipSuccess &&
            alloc_binned(p.src, q.max_src, g.ncells, elt) &&
            alloc_binned(p.tgt, q.max_tgt, g.ncells, elt);
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
  fill_u32<<<1, 64, 0, p.stream>>>(p.flags, 0u, 1);
  HIP_TRY(launch_bin(p, p.src, ns, xs, f, nullptr, true));
  if (p.fp64) {
    HIP_TRY(launch_spread<double>(p, 0));
    HIP_TRY(launch_grid_to_f64<double>(p, grid));
  } else {
    HIP_TRY(launch_spread<float>(p, 0));
    HIP_TRY(launch_grid_to_f64<float>(p, grid));
  }
  return finish(p);
}
