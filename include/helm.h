/*
 * helm.h -- C ABI of the MI355X fast-diagonalization Helmholtz/Laplace solver.
 *
 * The library solves   (sigma I - Lap_h) u = f   on a 3D tensor-product grid, where
 * Lap_h is the second-order finite-volume Laplacian (Vitoshkin & Gelfgat, Section 3,
 * eqs. 23-29): per axis the 1D operator A_d = -D_dd is eigen-decomposed once on the
 * host (eq. 24), and every solve transforms the right-hand side with E_d^{-1} along
 * x, y and z, divides by lambda_x(a) + lambda_y(b) + lambda_z(c) + sigma (eqs. 26-27)
 * and transforms back with E_d (eq. 29).  The TPT variant replaces the z-direction
 * eigen-transforms by one tridiagonal (Thomas) solve per (a, b) line (end of Section 3).
 *
 * Sign convention: the paper writes the Helmholtz operator as Lap + a I (eq. 27) and
 * H = Lap - I/dt (Section 2); here sigma = -a = 1/dt and eigenvalues lambda = -Lambda >= 0.
 *
 * Memory layout of every grid function: contiguous float64 [nrhs][nz][ny][nx], x fastest.
 * Pointers named f, u, p, b, Hu are DEVICE pointers; grid faces and sigma arrays are HOST
 * pointers.  `stream` is a hipStream_t (NULL = the default stream).  All device work is
 * enqueued on `stream` without host synchronization, except where a call says otherwise.
 *
 * Errors: every call returns helm_status; no C++ exception crosses this boundary.
 * Thread safety: distinct plans may be used concurrently; one plan may be used by
 * several threads at once provided each call has its own workspace and stream.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HELM_OK = 0,
  HELM_EINVAL = 1,        /* bad argument: NULL pointer, size < 2, non-increasing faces, bad enum */
  HELM_ESINGULAR = 2,     /* a denominator lambda_x+lambda_y+lambda_z+sigma is (numerically) zero
                             outside the all-Neumann null mode */
  HELM_ENOMEM = 3,        /* host or device allocation failed */
  HELM_EDEVICE = 4,       /* a HIP runtime call failed (including an asynchronous fault surfaced
                             at a synchronization point) */
  HELM_ENOTCONVERGED = 5, /* iterative refinement or GMRES did not reach its tolerance; the output
                             holds the best iterate */
  HELM_ENONFINITE = 6     /* NaN or Inf detected in a refinement norm */
} helm_status;

/* Boundary condition of one wall (homogeneous). */
enum { HELM_DIRICHLET = 0, HELM_NEUMANN = 1 };
/* Location of the unknowns along one axis: cell centres, or interior faces (a staggered
 * velocity component along its own direction, with wall value 0 on the wall faces). */
enum { HELM_CELL = 0, HELM_FACE = 1 };
/* Arithmetic of the mode products.  The *_IR forms run the products in the low precision
 * and recover FP64 accuracy by iterative refinement with an FP64 7-point residual.
 * BF16X3: each operand split into three bfloat16 pieces, six partial products accumulated
 * in FP32 on the BF16 matrix cores (FP32-class accuracy at the BF16 rate), FP32 storage. */
enum {
  HELM_FP64 = 0, HELM_FP32 = 1, HELM_BF16 = 2, HELM_FP32_IR = 3, HELM_BF16_IR = 4,
  HELM_BF16X3 = 5, HELM_BF16X3_IR = 6
};
/* TPF: eigen-transforms along x, y, z (eq. 29).  TPT_Z: eigen-transforms along x, y and
 * one Thomas tridiagonal solve per z line (end of Section 3).  FFT: TPF in which every
 * uniform axis whose walls give a sine or cosine eigenbasis (cell-centred: any wall pair;
 * face-located: both Dirichlet or both Neumann) and whose transform length 2M has no prime
 * factor above 7 (M <= 512) is transformed by a fast sine/cosine transform in O(N log N)
 * instead of the N x N eigenvector product (the fast-solver route the paper names for
 * uniform grids, Sections 1 and 3); other axes keep the product.  FP64 only. */
enum { HELM_TPF = 0, HELM_TPT_Z = 1, HELM_FFT = 2 };
/* All-Neumann Laplace null mode (eq. 28 discussion): PROJECT sets the zero mode of the
 * solution to 0 (the right-hand side is projected onto the range and u has zero
 * volume-weighted mean); PAPER_EQ28 replaces the zero denominator by 1 as in eq. 28. */
enum { HELM_NULL_PROJECT = 0, HELM_NULL_PAPER_EQ28 = 1 };

typedef struct {
  int n[3];                 /* cells per axis (x, y, z); each >= 2 (>= 3 for HELM_FACE) */
  const double* faces[3];   /* host, n[d] + 1 strictly increasing face coordinates; copied */
  int loc[3];               /* HELM_CELL or HELM_FACE per axis */
} helm_grid;

typedef struct {
  int lo[3];                /* HELM_DIRICHLET / HELM_NEUMANN at the low wall of each axis */
  int hi[3];                /* ... at the high wall */
} helm_bc;

/* Device allocator callback (optional), so that a caller's allocator (e.g. PyTorch's caching
 * allocator) owns the library's device memory.  alloc returns `bytes` bytes of device memory
 * on the current HIP device, at least 256-byte aligned, or NULL on failure (reported as
 * HELM_ENOMEM); dealloc releases a block returned by alloc, with the same size.  Both are
 * called with the device current and may be called from the server's worker threads; they
 * must stay valid until every object created with them is destroyed.  Blocks freed by
 * dealloc may still be read by device work enqueued before the owning object's destroy
 * call: the library synchronizes the device before releasing them. */
typedef void* (*helm_alloc_fn)(size_t bytes, void* ctx);
typedef void (*helm_free_fn)(void* ptr, size_t bytes, void* ctx);

typedef struct {
  int precision;            /* HELM_FP64 (default) ... HELM_BF16X3_IR */
  int method;               /* HELM_TPF (default), HELM_TPT_Z or HELM_FFT (FP64 only) */
  double ir_tol;            /* refinement stops when the correction max|du| / max|u| of a sweep, or
                               its product with the observed contraction factor (the predicted
                               next correction, when that factor is below 1/2), is <= ir_tol
                               (default 1e-11).  0: exactly max_sweeps solves with no norm read
                               back, for callers that know their sweep count (see helm_solve) */
  int max_sweeps;           /* refinement sweep limit, including the first solve (default 12) */
  int null_mode;            /* HELM_NULL_PROJECT (default) or HELM_NULL_PAPER_EQ28 */
  helm_alloc_fn alloc;      /* device allocator for everything the object allocates on the device
                               (plan uploads, pressure-matrix vectors, the server's workspace
                               arena); NULL (default) = hipMalloc / hipFree.  alloc and dealloc
                               are both set or both NULL (else EINVAL).  Plans share their
                               per-axis eigenbases only with plans of the same allocator. */
  helm_free_fn dealloc;
  void* alloc_ctx;          /* passed to alloc and dealloc */
} helm_opts;

typedef struct {
  int sweeps;               /* low-precision solves performed (1 for the plain precisions) */
  double last_correction;   /* max|du| / max|u| of the last refinement sweep (0 if none) */
  int converged;            /* 1 if the refinement tolerance was met (always 1 without IR), 0 if
                               not, -1 if not checked (ir_tol = 0; last_correction is then -1) */
  int iterations;           /* GMRES iterations (pressure-matrix solve only) */
  double residual;          /* final relative residual (pressure-matrix solve only) */
} helm_info;

typedef struct helm_plan helm_plan;
typedef struct helm_pmat helm_pmat;

/* Fills *opts with the defaults listed above. */
void helm_default_opts(helm_opts* opts);

/* Human-readable name of a status code (static string). */
const char* helm_status_str(helm_status s);

/* Builds a solve plan for (sigma I - Lap_h) u = f (eqs. 23-29).  Host work: 1D FV operators
 * from the faces (Section 3, eq. 23), FP64 symmetric-tridiagonal eigen-decomposition of
 * V^{-1/2} K V^{-1/2} per axis (eq. 24, done once), then one upload of E, E^{-1} (FP64,
 * FP32, BF16), the eigenvalues and the 7-point coefficients to the current HIP device.
 * opts may be NULL (defaults).  On success *out owns device memory until helm_destroy.
 * Errors: EINVAL, ESINGULAR (sigma < 0 hits a zero denominator), ENOMEM, EDEVICE. */
helm_status helm_setup(const helm_grid* grid, const helm_bc* bc, double sigma,
                       const helm_opts* opts, helm_plan** out);

/* Bytes of device workspace helm_solve needs for nrhs right-hand sides. */
helm_status helm_workspace_size(const helm_plan* plan, int nrhs, size_t* bytes);

/* Solves for nrhs right-hand sides (1 <= nrhs <= 64).  f, u: device [nrhs][nz][ny][nx]
 * float64; u may equal f only for the non-refined precisions (else EINVAL).
 * sigma_per_rhs: host array of nrhs shifts overriding the plan's sigma, or NULL (the
 * eigenbasis does not depend on sigma; only the denominators change).  ws: device
 * workspace of at least helm_workspace_size bytes (256-byte aligned).  Without
 * refinement the call is fully asynchronous on `stream`.  With refinement each sweep
 * ends with one 16-byte device-to-host copy of the correction norms, so the call
 * returns after the device work is done; with ir_tol = 0 it runs exactly max_sweeps
 * sweeps and reads nothing back, so it is asynchronous too (and launches only kernels,
 * which a caller may capture into a graph).  info (host, nullable) receives the sweep
 * count and final correction.  Errors: EINVAL, ESINGULAR, ENOTCONVERGED (u holds the
 * last iterate), ENONFINITE, EDEVICE. */
helm_status helm_solve(helm_plan* plan, const double* f, double* u, int nrhs,
                       const double* sigma_per_rhs, void* ws, void* stream, helm_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): helm_solve with the workspace taken from a
 * device array the library holds on each GPU (HELM_NOALLOC_MAX_WORKSPACE bytes, created when
 * the library's code is loaded on that GPU and kept until the process ends) instead of a ws
 * argument.  Same arguments, results and asynchrony as helm_solve; the call allocates nothing
 * (no hipMalloc, no pinned memory, no events).  Limits: helm_workspace_size(plan, nrhs) must
 * be <= HELM_NOALLOC_MAX_WORKSPACE (else EINVAL: e.g. a 256^3 FP64 solve with one right-hand
 * side needs 128 MiB, a refined split-BF16 one 192 MiB); refined plans must run a fixed sweep
 * count (ir_tol = 0, else EINVAL: adaptive refinement reads its norms through pinned host
 * memory); stage timing must be off (else EINVAL).  Every call on one GPU uses that GPU's one
 * array, so calls that overlap on one GPU (other threads, other streams) race: serialize them.
 * The array keeps the last call's contents; no call depends on them. */
#define HELM_NOALLOC_MAX_WORKSPACE ((size_t)256 << 20)
helm_status helm_solve_noalloc(helm_plan* plan, const double* f, double* u, int nrhs,
                               const double* sigma_per_rhs, void* stream, helm_info* info);

/* Bit d of *mask is set when axis d of the plan is transformed by the fast sine/cosine
 * transform (HELM_FFT plans with a uniform axis of a supported kind); 0 for other plans. */
helm_status helm_fast_axes(const helm_plan* plan, int* mask);

/* Grouped solve: the right-hand sides of several plans of one shape (different grids of the
 * same cell counts: their own stretching, walls and shifts) solved together, one launch per
 * stage of eqs. 25-29 over all of them; each right-hand side is multiplied by its own plan's
 * eigenbases and divided by its own plan's eigenvalues.  The time stepper's solves and a
 * stream of requests on a few grid sizes are the intended use (Section 5, eqs. 37-40).
 *   plans[i], i < nplans: nrhs[i] right-hand sides each (sum <= 64).  Every plan must be
 *     Cartesian, method HELM_TPF, precision FP64 or BF16X3(_IR), and share the first plan's
 *     unknown counts, device, precision, ir_tol, max_sweeps and null_mode; else EINVAL.
 *   f, u: device, the right-hand sides of plans[0], then plans[1], ... in the layout of
 *     helm_solve ([sum nrhs][nz][ny][nx]); sigma: host, one shift per right-hand side
 *     (nullable: each plan's setup shift).
 *   ws: device workspace of helm_group_workspace_size bytes, 256-byte aligned; it also holds
 *     the per-RHS operand table, which the call writes on `stream` before the products.
 * Semantics, errors and refinement as helm_solve (the refinement loop stops when every
 * right-hand side has converged).  A low-precision group with an all-Neumann plan at
 * sigma = 0 (projection) returns EINVAL: solve that right-hand side on its own.  If every
 * plans[i] is the same plan this is helm_solve with the summed right-hand-side count. */
helm_status helm_group_workspace_size(helm_plan* const* plans, int nplans, const int* nrhs, size_t* bytes);
helm_status helm_solve_group(helm_plan* const* plans, int nplans, const int* nrhs, const double* f, double* u,
                             const double* sigma, void* ws, void* stream, helm_info* info);

/* Hu = (sigma I - Lap_h) u with the FP64 7-point operator (the Kronecker sum of eq. 29),
 * device pointers [nrhs][nz][ny][nx]; asynchronous.  Hu must not alias u. */
helm_status helm_apply(const helm_plan* plan, const double* u, double* Hu, int nrhs,
                       const double* sigma_per_rhs, void* stream);

/* Host copies of one axis' eigenpairs: lam[n], E[n*n] and Einv[n*n] row-major with
 * E[i*n + a] = component i of eigenvector a, so that A_d = E diag(lam) Einv.  Any output
 * pointer may be NULL.  n here is the number of unknowns on that axis. */
helm_status helm_get_eigen(const helm_plan* plan, int axis, int* n, double* lam, double* E,
                           double* Einv);

/* Releases the plan and its device memory (synchronizes the device first). */
void helm_destroy(helm_plan* plan);

/* ---------------------------------------------------------------------------------------
 * Cylindrical coordinates (Section 6, eqs. 41-44): (sigma I - Lap_h) u = f with
 *     Lap u = (1/r) d/dr (r du/dr) + (1/r^2) d^2u/dtheta^2 + d^2u/dz^2
 * discretized by cell-centred finite volumes (face area times normal derivative; the theta
 * derivative taken along the arc at the cell-centre radius).  Per eq. 42 the theta and z
 * operators are eigen-decomposed once; per eq. 44 every (theta mode m, z mode n) pair then
 * leaves one radial tridiagonal system (A_r + lambda_theta(m) / r^2 + lambda_z(n) + sigma) a = g,
 * solved by the Thomas algorithm.  FP64 only.
 *
 * Layout of every grid function of a cylindrical plan: contiguous float64
 * [nrhs][n_r][n_z][n_theta], theta fastest, r slowest (the Thomas direction).  helm_solve,
 * helm_solve_noalloc, helm_apply, helm_workspace_size, helm_get_eigen (axis 0 = theta,
 * 1 = z, 2 = r: the radial operator of the m = 0 mode) and helm_destroy accept such a plan.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  int n[3];                 /* cells along r, theta, z; r >= 2, z >= 2, theta >= 2 (>= 3 periodic) */
  const double* faces[3];   /* host, n[d] + 1 strictly increasing face coordinates (copied):
                               radii r_0 >= 0 (r_0 = 0: the axis, a face of zero area), angles in
                               radians, axial positions */
  int theta_periodic;       /* 1: theta closed on itself (the last cell's upper face is the first
                               cell's lower face; the period is faces[1][n] - faces[1][0]), 0: a
                               sector with walls per bc */
} helm_cyl_grid;

/* Builds a cylindrical plan.  bc->lo/hi[0] are the inner and outer radial walls (the inner one
 * is ignored on the axis), [1] the theta walls of a sector (ignored when periodic), [2] the axial
 * walls.  opts: precision must be HELM_FP64 (else EINVAL); method is ignored (the Thomas form).
 * sigma >= 0 (else EINVAL).  Without any Dirichlet wall of nonzero area and with sigma = 0 the
 * problem is singular: the null mode is handled as in helm_setup (opts->null_mode).  Errors:
 * EINVAL (as helm_setup, plus the above), ENOMEM, EDEVICE. */
helm_status helm_cyl_setup(const helm_cyl_grid* grid, const helm_bc* bc, double sigma, const helm_opts* opts,
                           helm_plan** out);

/* Host-only helpers for the cylindrical axes (kind 0 = radial with walls bc_lo/bc_hi, 1 =
 * periodic theta): rows of A = V^{-1} K and the control volumes (radial: rc dr), and the
 * eigen-decomposition as in helm_host_eigen_1d.  A periodic axis couples its last and first
 * node: lower[0] and upper[m - 1] hold that coupling. */
helm_status helm_host_operator_cyl(int kind, int n, const double* faces, int bc_lo, int bc_hi, int* m_out,
                                   double* lower, double* diag, double* upper, double* vol);
helm_status helm_host_eigen_cyl(int kind, int n, const double* faces, int bc_lo, int bc_hi, int* m_out,
                                double* lam, double* E, double* Einv);

/* Pressure-Laplacian plan used as the pressure-matrix preconditioner (Section 2 and the
 * Neumann case of Section 3, eq. 28): cell-centred, all walls Neumann, sigma = 0.
 * Equivalent to helm_setup with those arguments and null_mode from opts. */
helm_status helm_pressure_setup(const helm_grid* grid, const helm_opts* opts, helm_plan** out);

/* Solves -Lap_h p = f - mean_V(f) and returns p with zero volume-weighted mean. */
helm_status helm_pressure_solve(helm_plan* plan, const double* f, double* p, int nrhs, void* ws,
                                void* stream, helm_info* info);

/* Pressure matrix C of eq. 9 on a MAC grid: C p = -sum_d Div_d H_d^{-1} Grad_d p with
 * H_d = (1/tau) I - Lap_h on the d-velocity grid (no-slip walls) and no pressure
 * boundary values.  p_grid gives the pressure cells (loc ignored); the three velocity
 * plans use opts->precision for their Helmholtz solves, and opts->method when the precision
 * is FP64 (the Thomas variant is FP64 only; other precisions use TPF); the preconditioner is
 * the pressure Laplacian (the Chorin limit of C, end of Section 2).  Errors as helm_setup. */
helm_status helm_pmatrix_setup(const helm_grid* p_grid, double tau, const helm_opts* opts,
                               helm_pmat** out);
/* A helm_pmat holds one pinned host buffer for its Krylov scalars: calls on one helm_pmat
 * (apply, solve, Stokes solve) must not overlap; distinct helm_pmat objects may be used
 * concurrently. */

/* Workspace bytes for helm_pmatrix_apply / helm_pmatrix_solve with restart length m. */
helm_status helm_pmatrix_workspace_size(const helm_pmat* pm, int restart, size_t* bytes);

/* y = C p (one right-hand side), device pointers over the pressure grid. */
helm_status helm_pmatrix_apply(helm_pmat* pm, const double* p, double* y, void* ws, void* stream);

/* Solves C p = b by right-preconditioned flexible GMRES(restart) (the Krylov inverse of C
 * in Section 2).  use_precond: 0 = none; 1 = the inverse pressure Laplacian (the paper's
 * preconditioner, exact in the Chorin limit tau -> 0); 2 = I + (1/tau) A_p^{-1}, where A_p is
 * the pressure Laplacian (Cahouet & Chabard's form: it equals option 1 as tau -> 0 and the
 * identity as tau -> infinity).  b must have zero volume-weighted mean; p is returned with
 * zero volume-weighted mean.  Stops when the relative residual ||b - C p|| / ||b|| <= tol
 * (confirmed with a true residual) or after max_it iterations (ENOTCONVERGED).  info (host,
 * nullable): iterations, the final relative residual, converged, and in `sweeps` the number of
 * Helmholtz solves performed (three per action of C, one per preconditioner application).
 * Synchronizes a few times per iteration (Gram-Schmidt coefficients). */
helm_status helm_pmatrix_solve(helm_pmat* pm, const double* b, double* p, double tol, int max_it,
                               int restart, int use_precond, void* ws, void* stream,
                               helm_info* info);

void helm_pmatrix_destroy(helm_pmat* pm);

/* Workspace bytes for helm_stokes_solve with restart length m (the helm_pmatrix_solve
 * workspace plus one pressure field and a reduction scratch). */
helm_status helm_stokes_workspace_size(const helm_pmat* pm, int restart, size_t* bytes);

/* Stokes system of eq. 8 (Section 2) on the MAC grid of pm, solved by the three steps that
 * follow its LU factorization: velocity solves, the pressure-matrix solve, velocity solves.
 * In the library's signs (the paper's momentum rows times -1, f_d = -R_d):
 *     H_d u_d + Grad_d p = f_d  (d = x, y, z),     sum_d Div_d u_d = g,
 * with H_d = (1/tau) I - Lap_h on the d-velocity grid and zero velocity on every wall.
 *   f[d], u[d]: device FP64 fields on the d-velocity grid, the pressure cell counts with one
 *               fewer along d, [nz'][ny'][nx'] x fastest; u[d] must not alias f[d], g, p or
 *               another u.
 *   g: device FP64 pressure-grid field, or NULL for 0 (the paper's case); its volume-weighted
 *      mean is dropped (the part no wall-bounded velocity can produce).
 *   p: device FP64 pressure-grid output with zero volume-weighted mean.
 *   tol, max_it, restart, use_precond: as helm_pmatrix_solve for step 2.
 *   ws: helm_stokes_workspace_size bytes, 256-byte aligned, owned by the caller.
 * Costs six velocity solves plus the FGMRES iterations (three velocity solves each).
 * Returns the first failing velocity solve's status, else helm_pmatrix_solve's (u is then
 * computed from the best p); info gets the FGMRES iterations and relative residual, and in
 * `sweeps` all Helmholtz solves (the six of steps 1 and 3 plus those of the FGMRES). */
helm_status helm_stokes_solve(helm_pmat* pm, const double* const f[3], const double* g,
                              double* const u[3], double* p, double tol, int max_it, int restart,
                              int use_precond, void* ws, void* stream, helm_info* info);

/* Stage timing (a tracing aid).  When enabled on a plan, every kernel launch made by
 * helm_solve / helm_apply with that plan is bracketed by two HIP events recorded on the
 * call's stream, tagged with its stage below.  helm_profile_read synchronizes those events,
 * adds the elapsed milliseconds and launch counts per stage into ms[HELM_NSTAGES] and
 * launches[HELM_NSTAGES] (host arrays), and clears the records.  Enabling or disabling
 * also clears them.  Not thread-safe with concurrent solves on the same plan. */
enum {
  HELM_STAGE_X_FWD = 0, HELM_STAGE_Y_FWD, HELM_STAGE_Z_FWD_DIV, HELM_STAGE_Z_INV, HELM_STAGE_Y_INV,
  HELM_STAGE_X_INV, HELM_STAGE_THOMAS, HELM_STAGE_NULL_LINE, HELM_STAGE_RESIDUAL, HELM_STAGE_CONVERT,
  HELM_STAGE_APPLY, HELM_STAGE_OTHER, HELM_STAGE_UPDATE,
  /* split-BF16 first solve: the x-forward product reading the FP64 right-hand side, and the
   * z-inverse product writing the solution (FP64, or FP32 into the workspace when refinement
   * sweeps follow) */
  HELM_STAGE_X_FWD_RHS, HELM_STAGE_Z_INV_U, HELM_NSTAGES
};
helm_status helm_profile_enable(helm_plan* plan, int enable);
helm_status helm_profile_read(helm_plan* plan, double* ms, int* launches);
/* Restricts timing to the stages whose bit (1u << stage) is set in stage_mask (default: all),
 * so that a timed run can bracket only the kernel it measures; clears the records.
 * Returns EINVAL for a null plan or a mask with no valid stage bit. */
helm_status helm_profile_stages(helm_plan* plan, unsigned stage_mask);

/* Measurement probes (no solve uses them): the rates the chip sustains on this software stack,
 * beside the datasheet peaks the kernel rooflines are quoted against.
 * helm_probe_mfma launches `blocks` workgroups of four waves, each wave running `iters` steps of
 * `chains` (4, 8 or 16) independent MFMA chains on register operands: kind 0 = BF16 16x16x32
 * with FP32 accumulation, 1 = FP32 16x16x4, 2 = FP64 16x16x4.  out: device buffer of
 * blocks * 256 floats (written, to keep the chains live).  *flops (host, nullable) receives
 * the matrix flops of the launch.  Asynchronous on `stream`; EINVAL for a bad kind or chain
 * count, iters or blocks < 1, or null out.
 * helm_probe_copy copies `bytes` (a multiple of 16) between two 16-byte aligned, non-overlapping
 * device buffers with 16-byte loads and stores on `stream`; EINVAL otherwise. */
helm_status helm_probe_mfma(int kind, int chains, int iters, int blocks, float* out, void* stream,
                            double* flops);
helm_status helm_probe_copy(const void* src, void* dst, long long bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of solve requests on one GPU.
 *
 * Requests (grid, walls, per-RHS shifts, 1..64 right-hand sides, caller-owned device f and u)
 * are queued on submit.  Admission runs inside helm_server_submit and again whenever a slot
 * finishes a request: queued requests are admitted in arrival order while (a) a solve slot is
 * free and (b) the request's device workspace fits in a free range of the server's workspace
 * arena, which is the whole HBM budget allocated once at creation (through opts->alloc when
 * set), and (c) if its solve has 2^23 or more unknowns x right-hand sides (big), no other big
 * solve is running: each kernel of such a solve fills the GPU, so two at once would only share
 * it while every kernel of the smaller requests running beside them waits behind theirs.  A
 * request that is not admissible waits until running requests retire (a later admissible
 * request may pass it only if the head has waited less than `max_bypass_ms`).  The server
 * therefore holds exactly the budget in workspace memory and allocates nothing on the device
 * while requests are in flight.  Each slot owns a HIP stream and a host worker thread, so
 * admitted solves run concurrently on the device and new requests are admitted while others
 * are in flight.  Plans (1D eigenbases) are cached on the device by their axis definition and
 * reused across requests.  When a request is admitted, queued requests on the same plan, or on
 * other grids of its shape that a grouped solve (helm_solve_group) can take, ride along (up to
 * 64 right-hand sides and 2^25 unknowns x right-hand sides in all, below 2^23 while a big solve
 * runs, within the budget, passing earlier requests only under the same bypass rule): they are
 * solved as one solve with each request's shifts, their f and u staged through the workspace
 * (2 x 8 bytes per point and right-hand side more), and their records carry the batch size.  Times are seconds since server
 * creation (steady clock).
 * --------------------------------------------------------------------------------------- */
typedef struct helm_server helm_server;

typedef struct {
  long long id;            /* caller's request id */
  int status;              /* helm_status of the solve */
  int sweeps;              /* refinement sweeps used */
  double last_correction;  /* final refinement correction */
  double t_submit;         /* submit time */
  double t_admit;          /* admission time */
  double t_done;           /* completion time (device work finished) */
  size_t footprint;        /* device workspace bytes charged against the budget (for the whole
                              solve when requests were solved together) */
  int slot;                /* slot that ran it */
  int batch;               /* requests solved together in its multi-RHS solve (1 = alone) */
} helm_request_record;

/* Creates a server with `slots` concurrent solve slots (1..16) and a device-workspace budget
 * of hbm_budget_bytes (allocated at once as the workspace arena: ENOMEM if it cannot be had);
 * opts sets the arithmetic of every solve and the allocator of the arena and of the resident
 * plans (NULL = FP64 TPF, hipMalloc). */
helm_status helm_server_create(size_t hbm_budget_bytes, int slots, double max_bypass_ms, const helm_opts* opts,
                               helm_server** out);
/* Queues one request; returns at once.  f, u: device [nrhs][nz][ny][nx] float64 owned by the
 * caller, untouched until the request's record is returned by helm_server_poll.  sigma: host
 * array of nrhs shifts (copied).  stream: the caller's hipStream_t on which f is produced
 * (NULL = the default stream); an event is recorded on it at submit and the solve waits for
 * that event on the device, so work the caller enqueued before submitting completes before
 * f is read.  u is complete when its record is polled (the slot's stream has finished).
 * Errors: EINVAL (bad arguments, or a footprint larger than the whole budget, which could
 * never be admitted), EDEVICE (the event could not be recorded). */
helm_status helm_server_submit(helm_server* s, const helm_grid* grid, const helm_bc* bc, const double* sigma,
                               int nrhs, const double* f, double* u, long long id, void* stream);
/* Returns up to max completed-request records (oldest first) in out and their count in *n,
 * waiting up to wait_ms milliseconds for at least one (0 = do not wait). */
helm_status helm_server_poll(helm_server* s, helm_request_record* out, int max, int* n, int wait_ms);
/* Blocks until every submitted request has completed (its record stays pollable). */
helm_status helm_server_drain(helm_server* s);
/* Current time on the server clock (seconds since creation). */
double helm_server_now(const helm_server* s);
/* Counters since creation: requests submitted and completed; plan lookups that found a resident
 * plan (hits) or built one (misses: host eigen-decomposition and upload, done inside submit), and
 * the seconds spent building them. */
typedef struct {
  long long submitted, completed, plan_hits, plan_misses;
  double setup_seconds;
} helm_server_stats_t;
helm_status helm_server_stats(helm_server* s, helm_server_stats_t* out);
/* Drains, stops the threads and releases the server and its resident plans.  A server keeps at
 * most 2048 resident plans (least recently used evicted; an evicted plan lives until its queued
 * and running requests complete); the 1D eigenbases are shared across plans per axis. */
void helm_server_destroy(helm_server* s);

/* Host-only simulation of the admission policy on a virtual clock (no device): n requests
 * with arrival times arrival[i], service times service[i], footprints foot[i] and size class
 * big[i] (nonzero: at least 2^23 unknowns x right-hand sides; big may be NULL, no request big)
 * are scheduled on `slots` slots under `budget`; outputs the admission and completion times.
 * Runs the same admission code as the server (riders are not simulated).  Errors: EINVAL. */
helm_status helm_sched_simulate(int n, const double* arrival, const double* service, const size_t* foot,
                                const int* big, int slots, size_t budget, double max_bypass_ms, double* admit,
                                double* done);

/* ---------------------------------------------------------------------------------------
 * Time stepping (Section 5, eqs. 34-40): Boussinesq convection in a box on the MAC grid
 * (pressure and temperature at the cell centres, velocity component d on the interior d-faces,
 * no-slip walls), temperature T_lo at x = 0 and T_hi at x = 1, adiabatic elsewhere, Prandtl
 * number Pr, Grashof number Gr.  One step of the second-order backward, incremental pressure-
 * correction scheme of eqs. 37-40:
 *   (3/(2dt) - kappa Lap) T1 = (4 T0 - Tm)/(2dt) - A_T(v0, T0)            kappa = 1/(Pr Gr^1/2)
 *   (3/(2dt) - nu Lap) v*_d  = (4 v0_d - vm_d)/(2dt) - A_d(v0) - Grad_d p0 + [d = z] T1   nu = Gr^-1/2
 *   -Lap dp = Div v* / dt;   v1 = v* + dt Grad dp;   p1 = p0 - dp
 * with the FV Laplacian of helm_setup (the wall values of T entering through the boundary flux)
 * and conservative central advection: A_T = sum_d (flux_hi - flux_lo) / w_d with face flux
 * v_d times the mean of the two cells; A_d on the d-face control volume, with the flux ubar^2
 * at the cell centres along d (ubar: the mean of the cell's two d-faces) and, across each other
 * direction e, the e-velocity averaged over the two cells beside the d-face times v_d averaged
 * over the two cells beside the e-face.  p1 subtracts dp: the update consistent with eq. 38's
 * -Grad p and the correction of eq. 40 (eq. 40 as printed adds it).
 * Fields are device FP64 arrays, x fastest: cells [nz][ny][nx]; v_d on its face grid (one fewer
 * node along d).  Outputs may alias the step n-1 inputs (T1 = Tm, v1 = vm) and p1 may alias p0.
 * --------------------------------------------------------------------------------------- */
typedef struct helm_ts helm_ts;
typedef struct {
  const double* T0;         /* temperature at step n */
  const double* Tm;         /* ... at step n - 1 */
  const double* v0[3];      /* velocity components at step n */
  const double* vm[3];      /* ... at step n - 1 */
  const double* p0;         /* pressure at step n */
  double* T1;               /* outputs: step n + 1 */
  double* v1[3];
  double* p1;
} helm_ts_fields;

/* Builds the temperature, three velocity and pressure plans (opts: their arithmetic and
 * allocator; NULL = FP64 TPF) for the pressure cells of `grid` (loc ignored, n >= 3 per axis).
 * Errors: EINVAL, ENOMEM, EDEVICE. */
helm_status helm_ts_create(const helm_grid* grid, double Pr, double Gr, double dt, double T_lo, double T_hi,
                           const helm_opts* opts, helm_ts** out);
/* Workspace bytes of helm_ts_step (right-hand sides, divergence, pressure increment, one solve's
 * workspace), 256-byte aligned, owned by the caller. */
helm_status helm_ts_workspace_size(const helm_ts* ts, size_t* bytes);
/* One time step on `stream`.  srv NULL: the five solves run on the stepper's plans, and the call
 * is asynchronous unless the plans refine adaptively.  srv given: they are submitted to that
 * server as requests (the temperature, then the three velocities together, then the pressure),
 * each waited for on the host; the server must serve this stepper only (its completion records
 * are consumed here).  info->sweeps: the low-precision solves performed (5 in FP64). */
helm_status helm_ts_step(helm_ts* ts, const helm_ts_fields* fields, helm_server* srv, void* ws, void* stream,
                         helm_info* info);
void helm_ts_destroy(helm_ts* ts);

/* Host-only helpers (no device needed), for checking the setup stage on any machine. */
/* 1D operator of one axis: lower/diag/upper rows of A = V^{-1} K (each of length m, the
 * number of unknowns) and the control-volume widths vol[m].  Returns m in *m_out. */
helm_status helm_host_operator_1d(int n, const double* faces, int loc, int bc_lo, int bc_hi,
                                  int* m_out, double* lower, double* diag, double* upper,
                                  double* vol);
/* FP64 eigen-decomposition of that operator (eq. 24): lam[m] ascending, E and Einv m*m
 * row-major as in helm_get_eigen. */
helm_status helm_host_eigen_1d(int n, const double* faces, int loc, int bc_lo, int bc_hi,
                               int* m_out, double* lam, double* E, double* Einv);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
