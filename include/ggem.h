/*
 * ggem.h -- GGEM evaluation of Stokes flow driven by point forces in a planar
 * slit on one AMD Instinct MI355X (gfx950).
 *
 * Method: Kumar & Graham, "Accelerated boundary integral method for
 * multiphase flow in non-periodic geometries" -- the General Geometry
 * Ewald-like Method of Sec. 3.2 (density split Eq. rho_l_g, local solution
 * Eq. local / Eq. u_loc, global spectral slit solver of Appendix C) applied to
 * the single layer (Eq. u_g a) and to the double layer written as the traction
 * n . sigma at targets (Eq. wdbl, Eq. vsigma).
 *
 * Geometry: periodic in x (period Lx) and z (period Lz); no-slip walls at
 * y = -H and y = +H (H is the half-gap).  Viscosity is 1.
 *
 * Conventions shared by every entry point
 *  - Position, strength, normal and output arrays are caller-owned DEVICE
 *    buffers (hipMalloc'd or torch tensors), contiguous, row-major (n, 3)
 *    float64: x, y, z components of one point per row.
 *  - All work is enqueued on the plan's HIP stream; no call after
 *    ggem_plan_create allocates device memory.  Outputs are overwritten.
 *  - x and z are wrapped into [0, L); they are not rejected.
 *  - Status codes are returned; ggem_last_error() gives a thread-local
 *    message for the last failing call on the calling thread.
 *  - Domain checks (|y| of a source >= H, |y| of a target > H, non-finite
 *    positions) are evaluated on the device.  With sync_checks = 1 the call
 *    waits for its stream and returns GGEM_E_DOMAIN; with sync_checks = 0 it
 *    returns immediately and the flag is read by ggem_plan_status().
 *    Offending points are clamped inside the kernels, so no access ever
 *    leaves the workspace; their outputs are meaningless.
 *  - Calls on one plan must not overlap (they share the plan's workspace).
 */
#ifndef GGEM_H
#define GGEM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ggem_plan_s* ggem_plan_t;

enum ggem_precision {
  GGEM_FP64 = 0,   /* every stage in double precision                       */
  GGEM_MIXED = 1,  /* FP32 near field, spread, FFT, interpolation; FP32 MFMA
                      Chebyshev transforms; FP64 tau solves                   */
  GGEM_MIXED_BF16 = 2  /* as GGEM_MIXED, but the Chebyshev transforms are
                      BF16 hi + lo split products (A_hi B_hi + A_hi B_lo +
                      A_lo B_hi) on the BF16 matrix cores with FP32
                      accumulation (about 4e-6 relative error per transform) */
};

enum ggem_status {
  GGEM_OK = 0,
  GGEM_E_ARG = -1,       /* invalid parameter or null pointer                 */
  GGEM_E_DOMAIN = -2,    /* a point outside the slit, or a non-finite value   */
  GGEM_E_CAPACITY = -3,  /* more points than reserved at plan creation        */
  GGEM_E_NOMEM = -4,     /* device allocation failed at plan creation         */
  GGEM_E_DEVICE = -5     /* a HIP runtime call failed                         */
};

/* Which parts of the GGEM sum to evaluate (test hook; ALL is the method). */
enum ggem_parts {
  GGEM_PART_LOCAL = 1,   /* local sum of Eq. u_loc including the self rule    */
  GGEM_PART_GLOBAL = 2,  /* global spectral solution interpolated to targets  */
  GGEM_PART_ALL = 3
};

typedef struct {
  double Lx, Lz;        /* periodic box lengths                               */
  double H;             /* wall half-gap: walls at y = -H and y = +H          */
  double alpha;         /* GGEM split parameter (Eq. rho_l_g)                 */
  double rc;            /* cutoff of the local sum and of the global density;
                           0 selects 4/alpha (Sec. 3.2.2).  Must satisfy
                           rc < min(Lx, Lz)/2 (the paper's alpha L > 8)        */
  int Nx, Nz;           /* Fourier nodes in x and z: even, 8..512, products of
                           2, 3 and 5                                          */
  int Ny;               /* Chebyshev Gauss-Lobatto nodes in y: 5..129          */
  int precision;        /* GGEM_FP64, GGEM_MIXED or GGEM_MIXED_BF16           */
  int sync_checks;      /* 1: wait and report domain errors; 0: asynchronous  */
  long long max_src;    /* capacity reserved at plan time (sources)           */
  long long max_tgt;    /* capacity reserved at plan time (targets)           */
  double cell_scale;    /* cells of the cell list at least cell_scale * rc on
                           a side: 0 or 1 selects rc, the smallest cell the
                           27-cell neighbourhood of the local sum allows; up
                           to 4.  A tuning knob only (the set of pairs within
                           rc, and so the result, is the same at any value):
                           larger cells mean fewer, fuller cell rows for the
                           spread and the local sum to walk                   */
} ggem_params;

/* Create a plan: validates the parameters, precomputes the Gauss-Lobatto
 * nodes, Chebyshev transform matrices, FFT twiddles and, for every Fourier
 * mode, the 2x2 influence matrix of Appendix C (the homogeneous problems (b)
 * and (c) are solved once per plan), and reserves all workspace.
 * hip_stream: a hipStream_t (NULL = default stream).
 * Errors: GGEM_E_ARG (bad parameter, null out), GGEM_E_NOMEM, GGEM_E_DEVICE.
 * The plan owns its workspace; release it with ggem_plan_destroy. */
int ggem_plan_create(const ggem_params* params, void* hip_stream, ggem_plan_t* out);

/* Release a plan and its workspace (waits for the plan's stream). */
int ggem_plan_destroy(ggem_plan_t plan);

/* Rebind the plan to another HIP stream. */
int ggem_plan_set_stream(ggem_plan_t plan, void* hip_stream);

/* Status of the last evaluation's device-side domain check (waits for the
 * plan's stream): GGEM_OK or GGEM_E_DOMAIN. */
int ggem_plan_status(ggem_plan_t plan);

/* Single layer (Eq. u_g a, evaluated by the GGEM split of Sec. 3.2):
 *   u[t] = (1/8 pi) sum_s G^slit(x_t, x_s) f_s
 * ns sources xs (ns,3) with strengths f (ns,3); nt targets xt (nt,3); output
 * u (nt,3).  A target that coincides with a source receives the regular part
 * of the slit Green's function for that pair (the free-space singular part
 * is omitted).  parts selects local / global / both.  ns = 0 or nt = 0 is
 * allowed.  Errors: GGEM_E_ARG, GGEM_E_CAPACITY, GGEM_E_DOMAIN, GGEM_E_DEVICE. */
int ggem_single_layer(ggem_plan_t plan, long long ns, const double* xs, const double* f,
                      long long nt, const double* xt, double* u, int parts);

/* Double layer in adjoint form (Eq. wdbl with Eq. vsigma):
 *   v[t]_j = n_k(x_t) sigma_jk(x_t),  sigma the stress of the point forces q
 *   sigma_jk(x) = (1/8 pi) sum_s T^slit_jik(x, x_s) q_s,i
 * The normal belongs to the TARGET (nrm (nt,3), not renormalised).  The
 * pressure gauge makes the lateral mean of the total pressure vanish at
 * y = -H.  Same sizes, errors and parts as ggem_single_layer. */
int ggem_double_layer(ggem_plan_t plan, long long ns, const double* xs, const double* q,
                      long long nt, const double* xt, const double* nrm, double* v,
                      int parts);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: serving loops, harnesses that forbid allocation): the single
 * layer of ggem_single_layer (parts = ALL) without a plan object.  The
 * workspace is a static device array of 64 MiB per GPU, held by the library
 * until the process ends; params describe the problem as for
 * ggem_plan_create (max_src/max_tgt give the capacities the workspace is laid
 * out for).  The first call on a device, and every call whose params differ
 * from the previous call's on that device, recomputes the plan constants into
 * the array (host work and synchronous copies; no allocation); calls with
 * the same params only enqueue the evaluation on hip_stream, on that one
 * stream (no second stream).  All calls on one GPU share its array, which
 * keeps the last call's contents: calls that overlap on one GPU (from two
 * threads, or on two streams whose work overlaps) race and give wrong
 * results.  Errors: as ggem_single_layer, plus GGEM_E_CAPACITY when the
 * workspace for these params exceeds the 64 MiB array (e.g. a 64x64x33 grid
 * with 2^17 sources and targets fits; a 128x128x65 grid does not). */
int ggem_single_layer_noalloc(const ggem_params* params, void* hip_stream, long long ns,
                              const double* xs, const double* f, long long nt, const double* xt,
                              double* u);

/* Diagnostic: the global force density of Sec. 3.2.2 on the grid,
 *   F(node) = sum_s f_s rho_g(node - x_s)   over |node - x_s| <= rc,
 * written as float64 (3, Ny, Nx, Nz) with y_j = H cos(pi j/(Ny-1)),
 * x_i = i Lx/Nx, z_k = k Lz/Nz.  Errors as above. */
int ggem_spread_grid(ggem_plan_t plan, long long ns, const double* xs, const double* f,
                     double* grid);

/* Pipeline stages, for the timing hook below. */
enum ggem_stage {
  GGEM_STAGE_BIN = 0,       /* cell binning of sources and targets           */
  GGEM_STAGE_NEAR = 1,      /* local sum at the targets                      */
  GGEM_STAGE_WALL = 2,      /* wall data u^g = -u^l (and the pressure gauge) */
  GGEM_STAGE_SPREAD = 3,    /* global density on the grid                    */
  GGEM_STAGE_FFT_FWD = 4,   /* forward x-z FFTs of the grid and wall planes  */
  GGEM_STAGE_CHEB_FWD = 5,  /* forward Chebyshev transform                   */
  GGEM_STAGE_TAU = 6,       /* per-mode tau / influence-matrix solves        */
  GGEM_STAGE_CHEB_INV = 7,  /* inverse Chebyshev transform                   */
  GGEM_STAGE_FFT_INV = 8,   /* inverse x-z FFTs                              */
  GGEM_STAGE_INTERP = 9,    /* interpolation and local + global combination  */
  GGEM_NUM_STAGES = 10
};

/* Timing hook: from now on, record HIP events on the plan's stream around
 * the launches of `stage` in each of the next max_calls evaluations (no host
 * synchronisation is added).  stage < 0 switches timing off.  The events are
 * created here, on the host side of the runtime; no device buffer is
 * allocated.  Errors: GGEM_E_ARG, GGEM_E_DEVICE. */
int ggem_plan_time_stage(ggem_plan_t plan, int stage, int max_calls);

/* Waits for the plan's stream and returns the summed duration (ms) of the
 * timed stage over the evaluations recorded since ggem_plan_time_stage, and
 * their number. */
int ggem_plan_stage_time(ggem_plan_t plan, double* total_ms, int* calls);

/* Work units of the last evaluation, counted by the kernels themselves when
 * counting was on for it (ggem_plan_count_work), else zeros:
 * counts[0] = target/source pairs within rc evaluated by the local sum (the
 * wall nodes excluded), counts[1] = (source, grid node within rc) updates of
 * the global density.  Waits for the plan's stream.  counts: host array of 2. */
int ggem_plan_work(ggem_plan_t plan, unsigned long long* counts);

/* Turn the kernels' work counting on (on != 0) or off for the following
 * evaluations of the plan; off by default, so that evaluations pay nothing
 * for it (a diagnostic: the counts give the work units of a throughput
 * figure).  Results do not depend on it.  Errors: GGEM_E_ARG (null plan). */
int ggem_plan_count_work(ggem_plan_t plan, int on);

/* Off-mesh evaluation of the global part (Sec. 3.2.2, last paragraph).  The
 * paper interpolates the grid solution with a 4th-order Lagrange stencil,
 * whose error falls only as h^5 off the mesh, and notes that the
 * non-uniform FFT keeps the spectral accuracy of the mesh points there too.
 * GGEM_INTERP_SPECTRAL evaluates the Fourier-Chebyshev series of the global
 * velocity (or stress, for the double layer) at each target as a type-2 NUFFT
 * by Gaussian gridding (Greengard and Lee) in x, z and theta = arccos(y/H)
 * (T_n(y/H) = cos(n theta)): oversampling 2 in each variable and msp nodes
 * on each side of the target (error about exp(-0.75 pi msp): msp = 12 for
 * FP64, 6 for the mixed modes). */
enum ggem_interp { GGEM_INTERP_LAGRANGE = 0, GGEM_INTERP_SPECTRAL = 1 };

/* Select the off-mesh evaluation for the following single- and double-layer
 * evaluations of the plan (and everything built on them: rigid particles,
 * Fredholm solves).  GGEM_INTERP_SPECTRAL allocates the oversampled grids
 * here (6 Ny (2 Nx)(2 Nz) reals, their padded spectra and 6 (2 Ny)(2 Nx)(2 Nz)
 * reals on the theta grid, in the plan's precision; one hipMalloc, freed by
 * the next call or ggem_plan_destroy);
 * GGEM_INTERP_LAGRANGE (the default) frees it.  msp: 2..16, at most Nx and
 * Nz (ignored for GGEM_INTERP_LAGRANGE).  Waits for the plan's streams.
 * Probes (ggem_probe) keep the Lagrange stencil.  Errors: GGEM_E_ARG (mode,
 * msp, Nx or Nz above 256: the plan keeps its mode), GGEM_E_NOMEM and
 * GGEM_E_DEVICE (the plan is left in the Lagrange mode). */
int ggem_plan_set_interp(ggem_plan_t plan, int mode, int msp);

/* ---- batches of independent slit problems -------------------------------
 *
 * Not in the paper: many independent problems of uneven size (each with its
 * own box, split parameter, grid and capacities) evaluated in one
 * submission.  A batch owns one plan per instance and n_branches streams;
 * instances are assigned to branches by longest-processing-time on an
 * estimate of their work, and an evaluation forks into the branches and
 * joins back, so instances run concurrently.  The enqueue can be captured
 * once into a HIP graph and replayed with a single launch.  Per-instance
 * sync_checks is forced off: domain errors are reported by
 * ggem_batch_status.  Errors: GGEM_E_ARG, GGEM_E_CAPACITY (with the instance
 * index in the message), GGEM_E_NOMEM, GGEM_E_DEVICE. */
typedef struct ggem_batch_s* ggem_batch_t;

int ggem_batch_create(int n_inst, const ggem_params* params, int n_branches, ggem_batch_t* out);
int ggem_batch_destroy(ggem_batch_t batch);

/* Single layer of every instance i: sources xs[src_off[i] .. src_off[i+1])
 * with strengths f, targets xt[tgt_off[i] .. tgt_off[i+1]), velocities into
 * u at the targets' rows (packed (N,3) float64 device arrays; src_off and
 * tgt_off are HOST arrays of n_inst + 1 offsets starting at 0).  Ordered
 * after prior work on hip_stream, and later work on hip_stream waits for it. */
int ggem_batch_single_layer(ggem_batch_t batch, void* hip_stream, const long long* src_off,
                            const double* xs, const double* f, const long long* tgt_off,
                            const double* xt, double* u);

/* Capture the same enqueue into the batch's graph (replacing any previous
 * one) without running it.  Every replay reads and writes the device
 * addresses given here: keep those buffers alive and in place. */
int ggem_batch_capture_single_layer(ggem_batch_t batch, const long long* src_off,
                                    const double* xs, const double* f, const long long* tgt_off,
                                    const double* xt, double* u);

/* Replay the captured graph on hip_stream. */
int ggem_batch_graph_launch(ggem_batch_t batch, void* hip_stream);

/* Wait for hip_stream and the batch, then report the first instance whose
 * last evaluation saw a non-finite or out-of-slit point (GGEM_E_DOMAIN). */
int ggem_batch_status(ggem_batch_t batch, void* hip_stream);

/* Branch (stream index) an instance was assigned to, or a negative error. */
int ggem_batch_branch(ggem_batch_t batch, int instance);

/* ---- Fredholm equation of the single-layer density (Eq. qa) ------------
 *
 * At every element node x_b of a triangulated surface (flat triangles,
 * density q linear on each):
 *   q_j(x_b) + (kappa_b/4pi) n_k(x_b) sum int q_i(x) T_jik(x_b, x) dS(x) = b_j(x_b),
 * kappa = (lambda - 1)/(lambda + 1).  The surface integral uses the three
 * interior Gauss points of every triangle (barycentric (2/3,1/6,1/6) and
 * permutations, weight area/3); each matrix-vector product is one GGEM double
 * layer on the plan.  Solved by restarted GMRES (Sec. 5) with FP64 Krylov
 * vectors and norms.  A solver owns its workspace (allocated at creation). */
typedef struct ggem_solver_s* ggem_solver_t;

typedef struct {
  long long max_nodes;  /* node capacity (plan max_tgt must cover it)           */
  long long max_tri;    /* triangle capacity (plan max_src must cover 3 x it)   */
  int restart;          /* Krylov dimension m of GMRES(m), 1..200               */
} ggem_solver_params;

int ggem_solver_create(ggem_plan_t plan, const ggem_solver_params* params, ggem_solver_t* out);
int ggem_solver_destroy(ggem_solver_t solver);

/* y = (I + kappa/4pi D) x for nodal vectors x, y (n_nodes, 3) float64.
 * nodes (n_nodes,3), normals (n_nodes,3) (the paper's area-averaged node
 * normals, Sec. 3.5.2), kappa (n_nodes) or NULL to use kappa0, tri (n_tri,3)
 * int32 node indices: all device arrays owned by the caller, read on the
 * plan's stream.  Node positions may be unwrapped (x and z are wrapped by the
 * evaluation); every triangle must be contiguous in space.  Triangle indices
 * are checked on the device before any node is read (one stream
 * synchronisation).  Errors: GGEM_E_ARG (null pointer, empty surface, node
 * index outside [0, n_nodes)), GGEM_E_CAPACITY (n_nodes or n_tri above the
 * solver's capacities), GGEM_E_DOMAIN (a node or Gauss point outside the
 * slit), GGEM_E_DEVICE. */
int ggem_fredholm_apply(ggem_solver_t solver, long long n_nodes, const double* nodes,
                        const double* normals, const double* kappa, double kappa0,
                        long long n_tri, const int* tri, const double* x, double* y);

/* Solve (I + kappa/4pi D) q = b; q holds the initial guess on entry and the
 * solution on exit.  Each cycle of m Krylov steps starts from the true
 * residual b - A q (one product); the solve stops when that true relative
 * residual |b - A q|/|b| is <= tol, or once max_iter Krylov products have
 * been spent.  A cycle ends early when the Arnoldi estimate reaches tol.
 * *iters: Krylov products (the residual products not counted); *rel_res: the
 * true relative residual of the returned q.  Non-convergence is not an
 * error: compare *rel_res with tol.  Returns after the plan's stream has
 * finished (every iteration reads its dot products on the host).  Errors as
 * for ggem_fredholm_apply, plus GGEM_E_ARG for tol <= 0 or max_iter < 1. */
int ggem_fredholm_solve(ggem_solver_t solver, long long n_nodes, const double* nodes,
                        const double* normals, const double* kappa, double kappa0,
                        long long n_tri, const int* tri, const double* b, double* q,
                        double tol, int max_iter, int* iters, double* rel_res);

/* ---- boundary-integral layers and rigid particles (Sec. 3.4, 3.5, 6.1) --
 *
 * The paper's own discretisation of the single layer on a triangulated
 * surface with the traction f linear on flat triangles (Sec. 3.3.1), at the
 * mesh nodes z:
 *   w(z) = (1/8pi) [ sum_k int_{S_k} f G^l(z - x) dS + sum_b G^g(z, x_b) f_b A_b ].
 * Local part (Sec. 3.4.1, Eq. int_l): each triangle whose nearest vertex lies
 * within r_c of z (minimum image) is integrated whole over its parent
 * triangle, xi in [0, 1 - eta], with the product of two 4-point
 * Gauss-Legendre rules; when z is a vertex of the triangle the parent
 * triangle is taken in polar coordinates about it (the Jacobian removes the
 * 1/r singularity).  Always FP64.  Global part (Sec. 3.4.2): the nodal
 * trapezoid strengths f_b A_b (A_b one third of the areas of the triangles
 * at b) through the plan's global problem (its precision), whose wall data
 * is the local sum of those point forces.
 *
 * A rigid solver owns its workspace: node areas, the two parts, and a
 * GMRES(restart) basis of 3 max_nodes + 6.  It runs on the plan's stream; the
 * plan's capacities must cover max_nodes sources and targets.  Errors:
 * GGEM_E_ARG (null pointer, restart outside 1..400, capacities out of
 * range), GGEM_E_CAPACITY, GGEM_E_NOMEM. */
typedef struct ggem_rigid_s* ggem_rigid_t;

int ggem_rigid_create(ggem_plan_t plan, long long max_nodes, long long max_tri, int restart,
                      ggem_rigid_t* out);
int ggem_rigid_destroy(ggem_rigid_t rigid);

/* w = the discretised single layer above, at every node.  nodes (n_nodes,3)
 * float64 (any periodic image in x and z; every triangle contiguous in
 * space), tri (n_tri,3) int32, inc_off (n_nodes + 1) and inc_tri
 * (inc_off[n_nodes]) int32 the triangles incident to each node (CSR), f and
 * w (n_nodes,3) float64: device arrays owned by the caller.  The mesh arrays
 * are checked on the device first (an index out of range, or a triangle
 * listed at a node it does not contain, gives GGEM_E_ARG; one stream
 * synchronisation).  Errors also: GGEM_E_CAPACITY, GGEM_E_DOMAIN (a node
 * outside the slit), GGEM_E_DEVICE. */
int ggem_bi_single_layer(ggem_rigid_t rigid, long long n_nodes, const double* nodes,
                         long long n_tri, const int* tri, const int* inc_off, const int* inc_tri,
                         const double* f, double* w);

/* v = the discretised double layer at every node (Sec. 3.5):
 *   v_j(z) = (1/8pi) n_k(z) [ sum_k int_{S_k} q_i T^l_jik(z - x) dS + sigma^g_jk(z) ],
 * the same elements, rules and nodal strengths q_b A_b as the single layer,
 * with n(z) the node normals (n_nodes,3) given by the caller (the paper's
 * area-averaged normals, Sec. 3.5.2).  On an element that has z as a vertex
 * the normal is replaced inside the integral by
 * n~(x) = n_D phi_z + n(z)(1 - phi_z) (Eq. dbl_l1, Eq. ntilde), n_D the
 * element's unit normal on the side of n(z), and the polar rule is used.
 * q, v (n_nodes,3) float64, device.  Errors as for ggem_bi_single_layer. */
int ggem_bi_double_layer(ggem_rigid_t rigid, long long n_nodes, const double* nodes,
                         long long n_tri, const int* tri, const int* inc_off, const int* inc_tri,
                         const double* normals, const double* q, double* v);

/* Velocity of Eq. bi_ua at the nodes on this discretisation (the procedure
 * the paper uses for the node velocities, Sec. 5):
 *   u = u_inf + 8 pi w(q),  u_inf = (shear_rate y, 0, 0),
 * w the discretised single layer above of the density q.  q, u: (n_nodes,3)
 * float64 device arrays.  Errors as ggem_bi_single_layer. */
int ggem_bi_surface_velocity(ggem_rigid_t rigid, long long n_nodes, const double* nodes,
                             long long n_tri, const int* tri, const int* inc_off,
                             const int* inc_tri, const double* q, double shear_rate, double* u);

/* GMRES for Eq. qa on this discretisation: q + 2 kappa v(q) = b, v the
 * discretised double layer above with the node normals (kappa =
 * (lambda-1)/(lambda+1); with the 1/8pi of v, 2 kappa v = (kappa/4pi) D q).
 * q: the initial guess on entry, the solution on return; b unchanged.
 * GMRES(restart of ggem_rigid_create) as ggem_fredholm_solve: *iters Krylov
 * products, *rel_res the true relative residual (non-convergence is not an
 * error).  The basis must hold 3 n_nodes (the rigid solver's capacity).
 * Errors as ggem_bi_double_layer, plus GGEM_E_ARG for tol <= 0,
 * max_iter < 1 or a non-finite kappa. */
int ggem_bi_fredholm_solve(ggem_rigid_t rigid, long long n_nodes, const double* nodes,
                           long long n_tri, const int* tri, const int* inc_off,
                           const int* inc_tri, const double* normals, double kappa,
                           const double* b, double* q, double tol, int max_iter, int* iters,
                           double* rel_res);

/* Force- and torque-free rigid particle in the undisturbed flow u_inf
 * (Sec. 6.1, Eq. sl_r): unknowns the nodal tractions f, the translational
 * velocity U and the angular velocity Omega about center (host, 3);
 *   U + Omega x (x_b - center) + w(x_b) = u_inf(x_b)   at every node,
 *   sum_b A_b f_b = 0,   sum_b A_b (x_b - center) x f_b = 0,
 * solved by GMRES(restart) (Sec. 5) in FP64 on the 3 n_nodes + 6 unknowns.
 * uinf (n_nodes,3) device; f (n_nodes,3) device holds the initial guess on
 * entry and the solution on exit; motion (host, 6) = (U, Omega) likewise.
 * Stops when the true relative residual is <= tol or after max_iter Krylov
 * products; *iters and *rel_res as for ggem_fredholm_solve (non-convergence
 * is not an error).  Returns after the plan's stream has finished.  Errors
 * as for ggem_bi_single_layer, plus GGEM_E_ARG for tol <= 0 or max_iter < 1. */
int ggem_rigid_solve(ggem_rigid_t rigid, long long n_nodes, const double* nodes, long long n_tri,
                     const int* tri, const int* inc_off, const int* inc_tri, const double* center,
                     const double* uinf, double* f, double* motion, double tol, int max_iter,
                     int* iters, double* rel_res);

/* ---- pressure and stress at probes, undisturbed-flow traction ----------
 *
 * ggem_probe: the velocity, pressure and stress of point forces at probes:
 *   u = u^l + u^g,  p = p^l + p^g,  sigma = sigma^l + sigma^g,
 * the local parts summed over the sources within r_c of a probe (minimum
 * image) with the kernels of Eq. local (a)-(c) and the 1/8pi of the single
 * layer (a coincident source adds -(4 alpha/sqrt(pi))/(8pi) f to the velocity
 * only), the global parts the slit solution of Appendix C (velocity, pressure,
 * and sigma = -p I + grad u + grad u^T formed in coefficient space)
 * interpolated with the 4th-order Lagrange stencil of Sec. 3.2.2.  The
 * pressure gauge is the double layer's: the lateral mean of the total
 * pressure at y = -H is zero.  xs, f (ns,3) and xt (nt,3) float64 device
 * arrays (x, z any periodic image; sources strictly inside the slit, probes
 * with |y| <= H); outputs u (nt,3), p (nt), sigma (nt,6) in the order xx,
 * yy, zz, xy, xz, yz, float64 device.  The local parts are summed in FP64,
 * the grid fields keep the plan's precision.  Runs on the plan's stream
 * without the second stream.  Errors: GGEM_E_ARG, GGEM_E_CAPACITY (ns above
 * max_src or nt above max_tgt: the probes are binned in the plan's target
 * workspace), GGEM_E_DOMAIN (a source or probe outside the slit, reported as
 * for the evaluations), GGEM_E_DEVICE. */
int ggem_probe(ggem_plan_t plan, long long ns, const double* xs, const double* f, long long nt,
               const double* xt, double* u, double* p, double* sigma);

enum { GGEM_FLOW_SHEAR = 0, GGEM_FLOW_POISEUILLE = 1 };

/* Traction f = sigma_inf . n of an undisturbed flow (Appendix B) at the n
 * points x (n,3) with normals nrm (n,3) -> f (n,3), float64 device, on the
 * plan's stream.  GGEM_FLOW_SHEAR: u = (rate y, 0, 0), sigma = rate e
 * (e_xy = e_yx = 1).  GGEM_FLOW_POISEUILLE: centre-line velocity rate between
 * the plan's walls, p = -(2 rate/H^2) x, sigma = (2 rate/H^2)(x I - y e)
 * (x as given: the pressure is not periodic).  Errors: GGEM_E_ARG. */
int ggem_undisturbed_traction(ggem_plan_t plan, int kind, double rate, long long n,
                              const double* x, const double* nrm, double* f);

/* Particle stress (Sec. 7.1, mu = 1) of the particles whose surfaces the
 * mesh holds:
 *   Sigma^p_ij = (1/V) sum int [df_i x_j + (lambda - 1)(u_i n_j + u_j n_i)] dS,
 * the integral taken with the nodal weights A_b (one third of the areas of
 * the triangles at b).  df: traction jump, u: surface velocity, normals: node
 * normals, all (n_nodes,3) float64 device; volume V > 0 of the domain; out
 * (host, 9) row-major Sigma^p.  Mesh arrays and errors as for
 * ggem_bi_single_layer, plus GGEM_E_ARG for volume <= 0. */
int ggem_particle_stress(ggem_rigid_t rigid, long long n_nodes, const double* nodes,
                         long long n_tri, const int* tri, const int* inc_off, const int* inc_tri,
                         const double* normals, const double* df, const double* u, double lambda,
                         double volume, double* out);

/* Undisturbed pressure-driven flow between the plan's walls (Appendix B):
 * u = U0 (1 - y^2/H^2) e_x at the n points x (n,3) float64 -> u (n,3),
 * device arrays, on the plan's stream.  Errors: GGEM_E_ARG. */
int ggem_poiseuille(ggem_plan_t plan, double U0, long long n, const double* x, double* u);

/* ---- surface quantities of a drop suspension in simple shear ------------
 *
 * Helpers that keep a time-stepped suspension of drops (closed triangulated
 * membranes with uniform tension) on the device; they run on the solver's
 * plan stream and use its Gauss-point workspace.
 *
 * ggem_surface_geometry: per node, the area-averaged normal (Sec. 3.5.2),
 * the node area A_p (one third of every incident triangle, Sec. 4) and the
 * cotangent Laplace-Beltrami of the position
 *   (Lap x)_p = 1/(2 A_p) sum_j (cot a_pj + cot b_pj)(x_j - x_p)
 *             = -(1/A_p) d(surface area)/dx_p.
 * node_tri_off (n_nodes + 1) and node_tri (node_tri_off[n_nodes]) list the
 * triangles incident to each node (CSR, int32, device).  Outputs: normals
 * (n_nodes,3), area (n_nodes), lap (n_nodes,3) float64, device.  Inconsistent
 * incidence lists (a triangle out of range, or one that does not contain the
 * node) give GGEM_E_ARG (checked on the device; one stream synchronisation).
 * Degenerate (zero-area) triangles give non-finite outputs. */
int ggem_surface_geometry(ggem_solver_t solver, long long n_nodes, const double* nodes,
                          long long n_tri, const int* tri, const int* node_tri_off,
                          const int* node_tri, double* normals, double* area, double* lap);

/* Right-hand side of Eq. qa for drops of viscosity ratio lambda and tension
 * 1/Ca in the simple shear u_inf = (shear_rate y, 0, 0) (mu = 1):
 *   b = -(1/4pi) (dF/(lambda + 1) + kappa f_inf),  kappa = (lambda-1)/(lambda+1),
 *   dF = -(1/Ca) Lap x  (virtual work of the tension energy, Sec. 4),
 *   f_inf = sigma_inf . n = shear_rate (n_y, n_x, 0)  (App. B).
 * normals, lap, b: (n_nodes,3) float64 device arrays.  Errors: GGEM_E_ARG
 * (null, lambda <= 0, non-finite inv_ca or shear), GGEM_E_CAPACITY. */
int ggem_drop_rhs(ggem_solver_t solver, long long n_nodes, const double* normals,
                  const double* lap, double lambda, double inv_ca, double shear_rate, double* b);

/* Velocity of Eq. bi_ua at the nodes: u = u_inf + sum int q_i G_ji dS, the
 * integral over the three interior Gauss points of every triangle (q linear
 * on each triangle), evaluated as 8 pi times one GGEM single layer on the
 * solver's plan.  q, u: (n_nodes,3) float64 device arrays.  Errors as for
 * ggem_fredholm_apply. */
int ggem_surface_velocity(ggem_solver_t solver, long long n_nodes, const double* nodes,
                          long long n_tri, const int* tri, const double* q, double shear_rate,
                          double* u);

/* out = x + dt u over n doubles (device; out may alias x), on the solver's
 * plan stream: the explicit update of the node positions. */
int ggem_advance(ggem_solver_t solver, long long n, const double* x, const double* u, double dt,
                 double* out);

/* GMRES as ggem_fredholm_solve, started from q + c dq: after the first
 * residual r = b - A q, one more product gives A dq and
 *   c = max(0, (r . A dq) / |A dq|^2)
 * (the least-squares step along dq; 0 when dq does not lower the residual),
 * so the starting residual is never larger than that of q alone.  dq: a
 * proposed correction (n_nodes,3) float64 device array, not aliasing q
 * (e.g. the learned warm start below).  *step (host, may be NULL): c.  Costs
 * one product more than ggem_fredholm_solve, not counted in *iters. */
int ggem_fredholm_solve_guided(ggem_solver_t solver, long long n_nodes, const double* nodes,
                               const double* normals, const double* kappa, double kappa0,
                               long long n_tri, const int* tri, const double* b, double* q,
                               const double* dq, double tol, int max_iter, int* iters,
                               double* rel_res, double* step);

/* Right-hand side of Eq. qa for a given traction jump df (e.g. a capsule
 * membrane's, ggem_membrane_traction) in the simple shear u_inf =
 * (shear_rate y, 0, 0):  b = -(1/4pi) (df/(lambda + 1) + kappa f_inf),
 * kappa = (lambda - 1)/(lambda + 1), f_inf = shear_rate (n_y, n_x, 0)
 * (App. B).  With lambda = 1 the operator of Eq. qa is the identity and
 * q = b.  normals, df, b: (n_nodes,3) float64 device arrays.  Errors:
 * GGEM_E_ARG, GGEM_E_CAPACITY. */
int ggem_traction_rhs(ggem_solver_t solver, long long n_nodes, const double* normals,
                      const double* df, double lambda, double shear_rate, double* b);

/* ---- neo-Hookean capsules (Sec. 4, Sec. 5, Sec. 7.1) ----------------------
 *
 * n_capsules capsules are consecutive, equal groups of nodes_per_capsule
 * nodes and tri_per_capsule triangles (rows of tri, global node ids; every
 * triangle names nodes of its own capsule; outward orientation).  The
 * membrane is infinitely thin and neo-Hookean with two-dimensional shear
 * modulus G: each flat element stores A0 W with
 *   W = (G/2)(l1^2 + l2^2 + 1/(l1^2 l2^2) - 3)   (Eq. WNH),
 * A0 its reference area and l1, l2 the principal stretches of its uniform
 * deformation from the reference (stress-free) element.  All calls run on
 * the solver's plan stream; arrays are device float64 unless stated. */
typedef struct ggem_membrane_s* ggem_membrane_t;

/* Reference state: tri (n_capsules * tri_per_capsule, 3) int32 (copied),
 * ref_nodes (n_capsules * nodes_per_capsule, 3) the stress-free node
 * positions (read here only).  The solver's capacities must cover the
 * nodes and triangles.  Errors: GGEM_E_ARG (a triangle naming a node of
 * another capsule, counts, G <= 0), GGEM_E_CAPACITY, GGEM_E_NOMEM. */
int ggem_membrane_create(ggem_solver_t solver, long long n_capsules, int nodes_per_capsule,
                         int tri_per_capsule, const int* tri, const double* ref_nodes,
                         double shear_modulus, ggem_membrane_t* out);
int ggem_membrane_destroy(ggem_membrane_t membrane);

/* Traction jump at the nodes (Eq. cntr2): the reaction force of the
 * membrane energy at a node, F_p = -dE/dx_p (the finite-element virtual work
 * of Charrier, Shrivastava and Wu, summed over the node's elements), over the
 * node's area A_p (one third of its elements' current areas):
 * df_p = -F_p / A_p.  node_tri_off / node_tri: the node-triangle incidence
 * lists of ggem_surface_geometry.  energy (host, may be NULL): the total
 * membrane energy.  Waits for the stream (the incidence lists are checked on
 * the device).  Errors: GGEM_E_ARG (null, inconsistent incidence lists). */
int ggem_membrane_traction(ggem_membrane_t membrane, const double* nodes, const int* node_tri_off,
                           const int* node_tri, double* df, double* energy);

/* Volume of every capsule, (1/6) sum of x_a . (x_b x x_c) over its
 * triangles (divergence theorem), into vol (n_capsules, device). */
int ggem_capsule_volumes(ggem_membrane_t membrane, const double* nodes, double* vol);

/* Volume correction (Sec. 5): every capsule whose volume V differs from
 * v0 (n_capsules, device, e.g. its initial volume) by more than tol |v0| has
 * each node moved along its normal by (v0 - V)/A, A the sum of its node
 * areas (normals, area: ggem_surface_geometry of the same nodes).  The
 * paper cites this correction without defining it; this uniform normal
 * shift is exact to first order.  nodes is updated in place.  n_corrected
 * (host, may be NULL; then no wait): the number of capsules moved. */
int ggem_volume_correct(ggem_membrane_t membrane, double* nodes, const double* normals,
                        const double* area, const double* v0, double tol, int* n_corrected);

/* The minimum node separation of the time-step rule gamma_dot dt =
 * 0.5 Ca h_s^m / a (Sec. 5): *min_edge (host) the shortest mesh edge, and
 * *min_gap (host) the smallest node-to-node distance between two capsules
 * (minimum image in x and z with periods Lx, Lz) when it is below reach,
 * else +inf (pairs whose bounding spheres are farther apart than reach are
 * not examined; h_s^m = min(min_edge, min_gap) with reach = min_edge).
 * Waits for the stream.  Errors: GGEM_E_ARG, GGEM_E_CAPACITY (more than 64
 * close pairs per capsule). */
int ggem_capsule_separation(ggem_membrane_t membrane, const double* nodes, double Lx, double Lz,
                            double reach, double* min_edge, double* min_gap);

/* Overlap correction (Sec. 7.1): in each sweep, every capsule pair whose
 * node-to-node gap is below h_min (in increasing (i, j) order) moves both
 * capsules rigidly apart along their line of centres (minimum image), each
 * by half the shortfall, and every capsule closer than h_min to a wall
 * (y = +-H) moves away from it by the shortfall; the moves of a sweep are
 * applied together.  Sweeps repeat until none is needed or max_sweeps.
 * nodes is updated in place; *sweeps (host, may be NULL): sweeps that moved
 * something.  Waits for the stream.  Errors as ggem_capsule_separation. */
int ggem_overlap_correct(ggem_membrane_t membrane, double* nodes, double Lx, double Lz, double H,
                         double h_min, int max_sweeps, int* sweeps);

/* ---- learned warm start: a per-node network ------------------------------
 *
 * Not in the paper, whose warm start is the previous stage's density
 * (Sec. 5).  A network of GGEM_MLP_IN inputs, three hidden layers of
 * GGEM_MLP_HIDDEN units with SiLU, and GGEM_MLP_OUT outputs, trained by mean
 * squared error with Adam (beta1 0.9, beta2 0.999, eps 1e-8).  Products run
 * with bfloat16 operands and FP32 accumulation; master weights, biases and
 * Adam moments are FP32.  Parameters are one packed FP32 vector of
 * GGEM_MLP_PARAMS values: W1 (128x13 row-major, [out][in]), b1, W2, b2, W3,
 * b3, W4 (3x128), b4.  Samples are row-major: X (n, 13), T and Y (n, 3).
 * All arrays are device memory owned by the caller; work runs on the stream
 * given at creation.  Errors: GGEM_E_ARG (null, bad value), GGEM_E_CAPACITY
 * (n outside 1..max_batch), GGEM_E_NOMEM, GGEM_E_DEVICE. */
#define GGEM_MLP_IN 13
#define GGEM_MLP_HIDDEN 128
#define GGEM_MLP_OUT 3
#define GGEM_MLP_PARAMS 35203

typedef struct ggem_mlp_s* ggem_mlp_t;

int ggem_mlp_create(int max_batch, void* hip_stream, ggem_mlp_t* out);
int ggem_mlp_destroy(ggem_mlp_t mlp);
/* Copy in the parameters (and reset the Adam moments and step count). */
int ggem_mlp_set_params(ggem_mlp_t mlp, const float* params);
int ggem_mlp_get_params(ggem_mlp_t mlp, float* params);
/* Node features, scaled feature by feature by scales[13] (host array):
 * position relative to the centroid of the node's drop (drops are
 * consecutive groups of nodes_per_drop nodes), normal, curvature term
 * c = -(Lap x) . n (see ggem_surface_geometry), the previous density q_prev
 * and its last change dq_prev (q_prev minus the density before it).
 * nodes, normals, lap, q_prev, dq_prev: (n_nodes,3) float64; X: (n_nodes,13)
 * float32. */
int ggem_mlp_features(ggem_mlp_t mlp, long long n_nodes, const double* nodes,
                      const double* normals, const double* lap, const double* q_prev,
                      const double* dq_prev, int nodes_per_drop, const float* scales, float* X);
/* Y = network(X) (float32). */
int ggem_mlp_forward(ggem_mlp_t mlp, long long n, const float* X, float* Y);
/* dq = scale * network(X) as float64 (n,3): the learned density correction. */
int ggem_mlp_predict(ggem_mlp_t mlp, long long n, const float* X, double scale, double* dq);
/* Loss mean((Y - T)^2) and its gradient (packed like the parameters) into
 * grads (device, may be NULL); *loss (host, may be NULL; waits for the
 * stream). */
int ggem_mlp_gradients(ggem_mlp_t mlp, long long n, const float* X, const float* T, float* grads,
                       float* loss);
/* One Adam step on the batch (X, T) with learning rate lr; *loss as above,
 * for the parameters before the step. */
int ggem_mlp_train_step(ggem_mlp_t mlp, long long n, const float* X, const float* T, float lr,
                        float* loss);

/* Thread-local description of the last error on the calling thread. */
const char* ggem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GGEM_H */
