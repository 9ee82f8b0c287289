// Internal declarations of the GGEM slit library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ggem.h"

namespace ggem {

// Sum of a per-lane count over the wave, added to *ctr by lane 0.
__device__ inline void wave_count_add(unsigned long long* ctr, unsigned v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr, (unsigned long long)v);
}

constexpr int kMaxCells = 16384;     // counting-sort buckets (LDS histograms)
constexpr int kMaxZSub = 8;          // z sub-slabs per cell (spread candidate windows)
constexpr int kNearSlices = 3;       // blocks per near-field work item (partial sums)
constexpr int kWallSlices = 3;       // blocks per wall-data work item (partial sums)
constexpr int kMaxChunks = 512;      // counting-sort chunks per point set (at most)
constexpr int kNearBlock = 64;       // targets per near-field work item
constexpr int kMaxNy = 129;
constexpr int kMaxFFT = 512;
constexpr int kMaxMsp = 16;   // NUFFT window half-width (spectral_eval holds 2 kMaxMsp weights)

// Domain flags raised on the device.
enum : unsigned { kFlagNonFinite = 1u, kFlagOutside = 2u };

// Geometry of the cell list: cells of size >= rc in x, y (over [-H, H]) and z.
// Each cell is cut into nzs slabs along z; points are sorted by (cell, slab),
// so a cell is still one contiguous run and a run of cells along z is sorted
// by slab, which lets the spread read only the slabs within r_c of its tile.
struct CellGeom {
  double Lx, Lz, H;
  double invLx, invLz;
  double icx, icy, icz;   // inverse cell sizes
  int ncx, ncy, ncz;
  int ncells;
  int nzs;                // z slabs per cell (power of two)
  int nbuckets;           // ncells * nzs
};

// A binned point set: sorted positions (wrapped) and cell ranges.
struct Binned {
  int n;
  int chunk;         // points per counting-sort chunk
  int nchunks;
  int* keys;         // bucket (cell * nzs + slab) per original point
  int* counts;       // [chunk][bucket]
  int* offs;         // [chunk][bucket] exclusive offsets inside the bucket
  int* sub_start;    // nbuckets + 1
  unsigned* cflags;  // per-chunk domain flags (kMaxChunks)
  int* cell_start;   // ncells + 1 (cell c starts at sub_start[c * nzs])
  int* item_start;   // ncells + 1: near-field work items per cell (prefix)
  int* item_cell;    // cell of each near-field work item (cap / kNearBlock + ncells)
  int* perm;         // sorted position -> original index
  double* x;         // sorted wrapped positions (SoA)
  double* y;
  double* z;
  void* s;           // sorted strengths or normals (3 x n, element type T)
  void* s2;          // second sorted vector field (normals for targets)
};

struct Plan {
  ggem_params p;
  hipStream_t stream;
  // the local sums (wall data, then the targets) run on `side`, concurrently
  // with the spread and the transforms on `stream`
  hipStream_t side;
  hipEvent_t ev_fork, ev_wall, ev_near;
  int device;
  bool fp64;
  bool bf16;         // mixed precision with BF16 hi + lo split Chebyshev products
  double rc, rc2;
  double dx, dz;
  int Nzh;           // Nz/2 + 1
  int nmodes;        // Nx * Nzh
  CellGeom cg;
  int nradx, nradz;
  int radx[12], radz[12];

  // plan-time constants on the device
  double* y;          // Gauss-Lobatto nodes (Ny)
  double* cf64;       // forward Chebyshev (Ny x Ny), scaled by 1/(Nx Nz)
  double* ci64;       // inverse Chebyshev (Ny x Ny)
  float* cf32;
  float* ci32;
  unsigned short* cf_hi;   // BF16 hi and lo halves of the two matrices ([MP][KP32])
  unsigned short* cf_lo;
  unsigned short* ci_hi;
  unsigned short* ci_lo;
  void* twx;          // twiddles exp(-2 pi i t/Nx), complex T
  void* twz;
  double* infl;       // per mode: 2x2 inverse influence matrix (4 doubles)
  double* nconst;     // per Chebyshev index: 1/(4n(n-1)), 1/(2(n^2-1)), 1/(4n(n+1))
  double* sweep;      // per mode: tau sweep factors and (b) profiles ((6 Ny + 2) x nmodes)

  // workspace
  Binned src, tgt;
  Binned wall;        // wall nodes of y = -H and y = +H, binned once per plan
  Binned* tview;      // targets of the current call (tgt, or src when they coincide)
  void* tnrm;         // sorted target normals of the current call (3 x max_tgt, T)
  void* ul;           // local result at sorted targets (kNearSlices x 3 x max_tgt, T)
  void* phys;         // physical grid fields (6 x Ny x Nx x Nz, T)
  void* specA;        // spectral fields (6 x Ny x Nx x Nzh, complex T)
  void* specB;
  void* wall_phys;    // wall velocities (2 x 3 x Nx x Nz, T)
  void* wall_part;    // their partial sums (kWallSlices x 2 x 3 x Nx x Nz, T)
  void* wall_spec;    // (2 x 3 x Nx x Nzh, complex T)
  double* tau_scr;    // tau scratch (9 x Ny x nmodes, complex FP64)
  double* gauge;      // gauge partial sums and value
  unsigned* flags;    // device domain flags
  unsigned* flags_host;  // host copy (pinned for plans; static for the allocation-free entry)
  unsigned long long* work;  // [0]: local pairs at the targets, [1]: spread updates (last call)
  double* wall_pos;   // wall node positions (2 Nx Nz x 3), input of their binning
  int* norder;        // targets of each cell in Morton order (near-field items, max_tgt)

  // every device buffer above is carved out of this one block
  void* block;
  size_t block_bytes;
  bool owns_block;    // false: the block is the library's static scratch array
  bool owns_flags_host;

  // stage timing hook (host side)
  int timed_stage;    // -1: off
  int timed_max;
  int timed_calls;
  hipEvent_t* timed_ev;  // 2 * timed_max events
  bool count_work;    // kernels count their work units (pairs, updates)

  // off-mesh evaluation of the global part: GGEM_INTERP_LAGRANGE (the
  // 4th-order stencil on the grid) or GGEM_INTERP_SPECTRAL (the
  // Fourier-Chebyshev series, its x-z sums by Gaussian-gridding NUFFT)
  int interp_mode;
  int msp;            // NUFFT window: msp oversampled nodes on each side
  double tau_x, tau_z;  // Gaussian widths pi msp / (3 N^2) in x and z
  Plan* over;         // FFT descriptor of the 2 Nx x 2 Nz oversampled grid
  void* over_block;   // its device buffers (one allocation of their own):
  void* over_spec;    //   padded spectra (6 x Ny x 2Nx x (Nz+1), complex T)
  void* over_phys;    //   oversampled fields (6 x Ny x 2Nx x 2Nz, T)
  void* over_theta;   //   the fields on the oversampled theta grid (6 x th_planes x 2Nx x 2Nz, T)
  void* cth;          // theta transform (th_rows x th_kp, T): deconvolution, cosines, 1/M_theta
  int th_m;           // oversampled theta nodes over [0, 2 pi): 2 (2 (Ny - 1) + 1)
  int th_planes;      // stored theta planes j = 0 .. th_m / 2 (the series is even in theta)
  int th_kp;          // columns of cth (Ny padded to 4)
  double tau_th;      // Gaussian width in theta
};

// ---- 4th-order Lagrange interpolation (Sec. 3.2.2), shared by the
// interpolation kernels ---------------------------------------------------

// nodes at -2..2: w_q = prod_{p != q} (t - p + 2) / prod_{p != q} (q - p), the
// denominators being 24, -6, 4, -6, 24
__device__ inline void lagrange5_uniform(double t, double* w) {
  const double d0 = t + 2.0, d1 = t + 1.0, d2 = t, d3 = t - 1.0, d4 = t - 2.0;
  const double d01 = d0 * d1, d34 = d3 * d4;
  w[0] = d1 * d2 * d34 * (1.0 / 24.0);
  w[1] = d0 * d2 * d34 * (-1.0 / 6.0);
  w[2] = d01 * d34 * 0.25;
  w[3] = d01 * d2 * d4 * (-1.0 / 6.0);
  w[4] = d01 * d2 * d3 * (1.0 / 24.0);
}

__device__ inline void lagrange5(double t, const double* nd, double* w) {
  double d[5];
  for (int p = 0; p < 5; ++p) d[p] = t - nd[p];
  for (int q = 0; q < 5; ++q) {
    double num = 1.0, den = 1.0;
    for (int p = 0; p < 5; ++p)
      if (p != q) {
        num *= d[p];
        den *= nd[q] - nd[p];
      }
    w[q] = num / den;
  }
}

// v in [-n, 2n) mapped into [0, n)
__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---- kernel launchers (each enqueues on p.stream) -------------------------
// first: this binning opens an evaluation, so its scan also resets the
// pair counters and overwrites the domain flags (later ones OR into them).
hipError_t launch_bin(Plan& p, Binned& b, long long n, const double* x, const double* s,
                      const double* s2, bool is_source, bool first);
template <typename T>
hipError_t launch_near_sl(Plan& p, int nt);
template <typename T>
hipError_t launch_near_dl(Plan& p, int nt);
template <typename T>
hipError_t launch_wall(Plan& p);
hipError_t launch_gauge(Plan& p);
template <typename T>
hipError_t launch_spread(Plan& p, int ncomp_offset);
template <typename T>
hipError_t launch_fft_forward(Plan& p, void* phys, void* spec, int nplanes);
template <typename T>
hipError_t launch_fft_inverse(Plan& p, void* spec, void* phys, int nplanes);
template <typename T>
hipError_t launch_cheb(Plan& p, const void* in, void* out, int nfields, bool forward);
template <typename T>
hipError_t launch_tau(Plan& p, bool stress);
template <typename T>
hipError_t launch_tau_export(Plan& p);
hipError_t launch_influence(Plan& p);
hipError_t launch_probe_local(Plan& p, int nt, const double* xt, const double* f, double* u,
                              double* pr, double* sigma);
template <typename T>
hipError_t launch_probe_interp(Plan& p, int nt, const double* xt, int ncomp, int split,
                               double* out0, int stride0, double* out1, int stride1);
hipError_t launch_undisturbed_traction(Plan& p, int kind, double rate, int n, const double* x,
                                       const double* nrm, double* f);
template <typename T>
hipError_t launch_interp(Plan& p, int nt, double* out, bool stress, bool with_global);
template <typename T>
hipError_t launch_grid_to_f64(Plan& p, double* out);
// The Fredholm solver's stream (its plan's) and capacities.
hipStream_t solver_stream(ggem_solver_t s);
long long solver_max_nodes(ggem_solver_t s);
long long solver_max_tri(ggem_solver_t s);
template <typename T>
hipError_t launch_nufft_pad(Plan& p, int nf);
template <typename T>
hipError_t launch_row_gemm(Plan& p, const T* A, int KP, int Kin, int Mout, const void* in,
                           void* out, long ncols, int nfields);
template <typename T>
hipError_t launch_spectral_eval(Plan& p, int nt, double* out, bool stress);
template <typename T>
hipError_t launch_wall_sum(Plan& p);
const int* launch_near_order_sources(Plan& p);

// Shared launches of a batch: the spread, and the local sums at the targets
// and at the wall nodes, of many plans in one launch each.  The job lists
// (each plan's kernel arguments and block offsets) are uploaded once, when
// the batch is created; a launch then reads them on the device.
int spread_job_blocks(const Plan& p);
bool spread_job_rel(const Plan& p);
size_t spread_job_bytes();
int spread_jobs_upload(const Plan* const* plans, int n, void* dev_args, int* dev_boff);
template <typename T>
hipError_t launch_spread_jobs(hipStream_t s, const void* dev_args, const int* dev_boff, int n,
                              int nblocks, bool rel);
bool near_job_fast(const Plan& p);
size_t near_job_bytes(bool fp64);
int near_job_blocks(const Plan& p, bool wall);
int near_jobs_upload(Plan* const* plans, int n, bool wall, void* dev_jobs, int* dev_boff);
hipError_t launch_near_jobs(hipStream_t s, bool fp64, bool fast, bool wall, const void* dev_jobs,
                            const int* dev_boff, int n, int nblocks);
// The single-layer evaluation of a plan whose targets are its sources, in
// the phases around the shared launches: binning (and the target order of
// the local sum), the wall data after the shared wall-node sums, the grid
// stages after the shared spread, and the interpolation after the shared
// local sums.  Each enqueues on p.stream.
template <typename T>
int batch_phase_bin(Plan& p, long long ns, const double* xs, const double* f);
template <typename T>
int batch_phase_wall(Plan& p);
template <typename T>
int batch_phase_grid(Plan& p);
template <typename T>
int batch_phase_interp(Plan& p, long long nt, double* out);

}  // namespace ggem

// The plan handle of the C ABI.
struct ggem_plan_s {
  ggem::Plan p;
};

// Record a thread-local error message and return code.
int ggem_set_error(int code, const char* msg);
