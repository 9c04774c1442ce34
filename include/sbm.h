/*
 * sbm.h -- C ABI of the MI355X (gfx950) matrix-free shifted-boundary (SBM) Poisson library.
 *
 * The library applies v = A u for the high-order SBM discretisation of -Laplace u = f in
 * Omega, u = g on Gamma, posed on the surrogate domain made of the background cells that
 * lie entirely inside Omega (Wichrowski, "Matrix-Free Evaluation of High-Order Shifted
 * Boundary Finite Element Operators", Sec. 2 and Sec. 2.1, Eq. (1)):
 *
 *   a(u,v) = int grad u . grad v - int_{Gam~} (du/dn~) v - int_{Gam~} (dv/dn~) E u
 *            + int_{Gam~} sigma E u v,
 *
 * where E u at a surrogate-face quadrature point x~ is the value of the face's own cell
 * polynomial at the closest point x = x~ + d on the true boundary (Sec. 3.3, Alg. 3).
 * For SBM_DG the Laplace term is replaced by its symmetric interior-penalty (SIPG) form
 * (Sec. 2.1, last display; Sec. 3.2, Alg. 2).  Cells are tensor-product Q_p elements on
 * Gauss-Lobatto-Legendre nodes with lexicographic local numbering (Sec. 3.1); cell
 * integrals use (p+1)^d Gauss points, face integrals (p+1)^(d-1).
 *
 * Conventions common to every entry point:
 *   - Return value: SBM_OK or an error code; sbm_last_error() then holds a message
 *     (thread-local).  No C++ exception crosses this boundary.
 *   - "device" pointers are HIP device allocations of the current device; "host"
 *     pointers are ordinary CPU memory.  The caller owns every buffer it passes in.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).  Device work
 *     is enqueued on it; calls marked "asynchronous" return before the work finishes.
 *   - Vectors have n_dofs entries of the requested precision (double for SBM_F64,
 *     float for SBM_F32), contiguous.
 *   - Supported: dim 2 or 3, p = 1..8, isotropic cells (equal h in every direction).
 */
#ifndef SBM_H
#define SBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbm_ctx *sbm_handle;

typedef enum {
  SBM_OK = 0,
  SBM_EINVAL = 1,        /* invalid argument (bad pointer, size, aliasing, geometry) */
  SBM_ENOMEM = 2,        /* device or host allocation failed */
  SBM_EHIP = 3,          /* a HIP runtime call failed */
  SBM_ENOCONV = 4,       /* solver stopped before reaching the tolerance */
  SBM_EUNSUPPORTED = 5   /* degree, dimension or option outside the built set */
} sbm_status;

enum { SBM_CG = 0, SBM_DG = 1 };      /* continuous Q_p / SIPG discontinuous Q_p */
enum { SBM_F64 = 0, SBM_F32 = 1 };    /* arithmetic and vector precision of an apply */

/* Level-set kinds; the true domain is {phi < 0}. */
enum {
  SBM_LS_SPHERE = 0,       /* |x - centre| - radius (a disk in 2D) */
  SBM_LS_ELLIPSOID = 1,    /* axis-aligned, semi_axes[k], centred at centre */
  SBM_LS_TORUS = 2,        /* 3D only: axis z through centre, major radius R, minor r */
  SBM_LS_SPHERE_UNION = 3, /* union of n_spheres balls (centres n x 3 row-major, radii) */
  SBM_LS_HALFSPACE = 4,    /* normal . x - offset with a unit normal */
  SBM_LS_CALLBACK = 5      /* user phi and grad phi (fields phi, grad, user below); closest
                              points by the level-set Newton iteration of Sec. 4.4,
                              x <- x - phi(x) grad phi(x) / |grad phi(x)|^2 from the surrogate
                              point, until the step |phi| / |grad phi| is at most
                              8 eps max(1, max_k |x_k|) (scale-aware), at most 50 steps,
                              else setup fails with SBM_EINVAL (the point reached is
                              on the boundary, and is the closest one when phi is a distance
                              function or its gradient lines are straight).  The callbacks are
                              called from the thread that calls sbm_setup only, during it. */
};

/* Uniform Cartesian background mesh: n[k] cells on [lo[k], hi[k]], k < dim. */
typedef struct {
  int dim;
  int n[3];
  double lo[3];
  double hi[3];
} sbm_mesh;

typedef struct {
  int kind;
  double centre[3];
  double radius;
  double semi_axes[3];
  double R, r;
  double normal[3];
  double offset;
  int n_spheres;          /* SBM_LS_SPHERE_UNION: the arrays below are copied by sbm_setup */
  const double *centres;  /* host, n_spheres x 3 (the third entry is ignored in 2D) */
  const double *radii;    /* host, n_spheres */
  /* SBM_LS_CALLBACK: phi(x, user) and grad(x, g, user) for a point x of dim coordinates */
  double (*phi)(const double *x, void *user);
  void (*grad)(const double *x, double *g, void *user);
  void *user;
} sbm_levelset;

typedef struct {
  double penalty_gamma;    /* sigma_Gamma = penalty_gamma * p^2 / h  (<= 0 selects 10) */
  double dg_penalty_gamma; /* sigma_F     = dg_penalty_gamma * p^2 / h (<= 0 selects 10) */
  double shift_scale;      /* d is scaled by this factor; 1 = the method, 0 = no shift */
  int flags;               /* SBM_SETUP_HOST_ONLY: build the host-side data only (no device
                              allocation; the handle then serves sbm_info, sbm_dof_points,
                              sbm_rhs_points and the sbm_export_* calls, nothing else);
                              SBM_SETUP_HOST_BUILD: build the geometry, numbering and layout on
                              host threads and upload them (the default for the analytic
                              level-set kinds builds them with device kernels; results are
                              identical; user level sets are always built on the host);
                              SBM_SETUP_NO_GRAPHS: sbm_solve launches every Arnoldi step's
                              kernels one by one instead of replaying them from graphs captured
                              in the second restart cycle (the results are identical) */
} sbm_options;

enum { SBM_SETUP_HOST_ONLY = 1, SBM_SETUP_HOST_BUILD = 2, SBM_SETUP_NO_GRAPHS = 4 };

/*
 * sbm_setup -- build one operator (Sec. 3.4 data structures, Sec. 4.4 initialisation).
 * Classifies the background cells (active: phi < 0 at all 2^d vertices), lists the
 * surrogate faces (faces of active cells whose neighbour is missing or inactive), finds
 * for every surrogate-face Gauss point x~ the exact closest point x on {phi = 0}, stores
 * the shifted reference coordinates xi = xi~ + shift_scale (x - x~) / h, numbers the DoFs
 * and uploads everything to the current device.
 * DoF order: CG -- ranks of the touched lattice points m = p*c + j in lexicographic order
 * (first coordinate fastest); DG -- (rank of the active cell) * (p+1)^d + local index.
 * opts may be NULL (defaults).  On success *out owns all device memory of the operator.
 * Errors: EINVAL (mesh/level set/pointer), EUNSUPPORTED (dim, p), ENOMEM, EHIP.
 */
sbm_status sbm_setup(const sbm_mesh *mesh, const sbm_levelset *ls, int p, int disc,
                     const sbm_options *opts, sbm_handle *out);

/* Counts and the device bytes the handle holds: its operator data and scratch from
 * sbm_setup, plus the solver workspace once a solve has allocated it.  Any output pointer
 * may be NULL. */
sbm_status sbm_info(sbm_handle h, int64_t *n_dofs, int64_t *n_cells, int64_t *n_sbm_faces,
                    int64_t *n_interior_faces, size_t *device_bytes);

/* Releases every resource of h (NULL is ignored).  Waits for the handle's last asynchronous
 * work (apply, diagonal) to finish, and for the last run of every batch of applies
 * (sbm_apply_batch, sbm_batch_run) still pending or not destroyed, then returns its device
 * memory to the library's pool stream-ordered: nothing else on the device is waited for, so
 * other handles' work in flight continues.  Work on h enqueued on a stream after that last
 * call must not exist; a prepared batch that includes h must be destroyed first. */
void sbm_destroy(sbm_handle h);

/* Message of the last failing call on this thread ("" if none). */
const char *sbm_last_error(void);

/*
 * sbm_apply -- v = A u (Sec. 3.5 workflow: cell loop, then surrogate faces; for DG the
 * interior faces are evaluated cell by cell).  u and v are device vectors of n_dofs
 * entries of the precision prec (SBM_F64: double, SBM_F32: float); v is overwritten and
 * must not alias u.  Asynchronous on stream; never synchronises.  A handle owns a scratch
 * buffer used by every apply (surrogate-face results; for CG also the brick-boundary
 * partial sums), so applies of the same handle must be ordered on one stream (applies of
 * different handles may run concurrently).  With the default extension the result is
 * bitwise reproducible: every sum is taken in a fixed order (no atomics).
 * Errors: EINVAL (NULL handle/pointer, u == v, bad prec), EHIP (launch failure).
 */
sbm_status sbm_apply(sbm_handle h, const void *u, void *v, int prec, void *stream);

/*
 * sbm_apply_noalloc -- sbm_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same operator,
 * kernels, arguments and result as sbm_apply (bitwise equal with the default extension), but
 * the apply's scratch is taken from a static device array of 96 MiB held by the library on
 * each device it runs on (until the process ends) instead of the handle's own buffers.  The
 * call allocates nothing and never synchronises.  Every call on one device shares that array
 * and leaves its contents behind: calls that overlap on one device (other streams or threads)
 * race and give wrong results; calls ordered on one stream are safe.  The first call on a
 * device looks up that device's array address (that device must be current).
 * Errors: EINVAL (as sbm_apply, or the handle needs more scratch than 96 MiB in this
 * precision -- the CG brick-boundary sums take 2^dim x boundary DoFs values and the
 * surrogate faces 2 (p+1)^(dim-1) values each: a 64^3 Q4 sphere needs 67 MB in FP64; the
 * message states the size), EHIP.
 */
sbm_status sbm_apply_noalloc(sbm_handle h, const void *u, void *v, int prec, void *stream);

/*
 * sbm_apply_parts -- diagnostic split of sbm_apply: v = (selected parts of A) u, with
 * SBM_PART_CELLS the cell term (for DG including the interior faces) and
 * SBM_PART_SBM_FACES the surrogate-boundary faces; SBM_PART_ALL gives sbm_apply.  v is
 * overwritten in every case.  It exists to time the cell and surrogate-face work separately
 * (the share of time spent in surrogate faces, Sec. 4.3) and to check each term on its own.
 * Same argument rules as sbm_apply.  Asynchronous.
 */
enum { SBM_PART_CELLS = 2, SBM_PART_SBM_FACES = 4, SBM_PART_ALL = 6,
       SBM_PART_NO_ASSEMBLY = 8,  /* CG: skip the final sum over brick-boundary DoFs (those
                                     entries of v are then left unwritten) */
       SBM_PART_REUSE_FACES = 16  /* CG, with SBM_PART_SBM_FACES: do not evaluate the
                                     surrogate faces again; merge the face results of the
                                     previous call with SBM_PART_SBM_FACES on this handle
                                     (same precision; otherwise the result is undefined).
                                     With SBM_PART_ALL | SBM_PART_NO_ASSEMBLY this times the
                                     brick kernel alone. */ };

/*
 * sbm_layout_stats -- CG work decomposition (zeros for DG): number of bricks (blocks of
 * background cells, one workgroup each), DoFs on brick boundaries (assembled by a second
 * pass) and the slots that pass reads.  Any output pointer may be NULL.
 */
sbm_status sbm_layout_stats(sbm_handle h, int64_t *n_bricks, int64_t *n_boundary_dofs,
                            int64_t *n_boundary_slots);
sbm_status sbm_apply_parts(sbm_handle h, const void *u, void *v, int prec, int parts, void *stream);

/*
 * sbm_set_extension_order -- choose the extension E of the surrogate-face term (Eq. 1) for
 * every later sbm_apply, sbm_apply_batch, sbm_diagonal and sbm_solve on h.  Sec. 2.1 defines
 * E by a Taylor expansion of the solution about the surrogate point x~ along the shift
 * d = x - x~.  m < 0 (the default after sbm_setup): the expansion to all orders, i.e. the face
 * cell's polynomial evaluated at the shifted point (Sec. 3.3, Alg. 3).  m >= 0: the
 * expansion kept to total order m, E_m u(x~) = sum over |alpha| <= m of
 * D^alpha u_K(x~) d^alpha / alpha! (m = 1: value plus gradient; m >= dim * p equals the
 * default up to rounding).  With m >= 0 the surrogate faces run in a separate kernel whose
 * per-face results the cell kernels add in their fixed order (bitwise reproducible, as the
 * default), and sbm_apply_parts returns SBM_EUNSUPPORTED.  Does not touch the device; not synchronised with work already
 * enqueued on h (call it between, not during, applies).  Errors: EINVAL (NULL handle).
 */
sbm_status sbm_set_extension_order(sbm_handle h, int m);

/*
 * Batched applies (serving: many operators' applies in few launches; the matrix-free apply
 * of Sec. 3, Alg. 1-3, per operator).  A batch is n independent applies v_i = A_i u_i in one
 * precision.  The operators that share a kernel instantiation (discretisation, dimension,
 * degree) form a group, and each group runs as one launch per stage across all its operators
 * (surrogate faces; cells or bricks; brick-boundary sums), every workgroup finding its
 * operator in a table in device memory.  Each v_i is bitwise the result of sbm_apply(h_i,
 * u_i, v_i).  Operators with a truncated extension (sbm_set_extension_order) have their
 * surrogate faces computed one by one, their other stages in the group launches.
 *
 * Argument rules (every i): as sbm_apply, and further: a handle appears at most once (its
 * scratch serves one apply at a time), no v_i equals another v_j or any u_j (vectors of a
 * batch must not overlap), all handles on the current device.  Errors: EINVAL (any rule
 * broken, NULL arrays with n > 0), EHIP.
 *
 * sbm_batch_create -- validate and prepare (host tables, one device allocation holding them,
 *   uploaded before returning).  max_streams > 1: the groups' launch chains (independent of
 *   each other) are spread over up to max_streams streams owned by the batch (default
 *   priority), forked from the run's stream and joined back to it, so that the launches of
 *   small groups overlap on the device; 1 (or 0): every launch on the run's stream.
 *   graph != 0: the first sbm_batch_run captures the batch's launches (fork and join included)
 *   into a HIP graph (on the stream given to it, which must not be the legacy default stream;
 *   otherwise, or if capture fails, launches are issued directly) and every later run replays
 *   it.  The handles and vectors must stay valid until sbm_batch_destroy; changing a handle's
 *   extension order after creation is not seen by the batch.
 * sbm_batch_run -- enqueue the batch on stream (asynchronous).  A batch is not to be run from
 *   two threads at once, nor concurrently with other work on its handles.
 * sbm_batch_destroy -- waits for the batch's last run, then releases it (NULL: no-op).
 * sbm_apply_batch -- one-shot form: create (no graph, every launch on stream), run, release
 *   the tables once the run has completed (without waiting for it).  n = 0: no-op.
 */
typedef struct sbm_batch_s *sbm_batch;
sbm_status sbm_batch_create(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec,
                            int graph, int max_streams, sbm_batch *out);
sbm_status sbm_batch_run(sbm_batch b, void *stream);
sbm_status sbm_batch_destroy(sbm_batch b);
sbm_status sbm_apply_batch(int n, const sbm_handle *hs, const void *const *u, void *const *v,
                           int prec, void *stream);

/* Physical coordinates of every DoF (host, n_dofs x dim). */
sbm_status sbm_dof_points(sbm_handle h, double *xyz);

/*
 * Points where the caller evaluates the problem data for sbm_rhs (host arrays):
 *   cell_qp:  n_cells x (p+1)^d x dim  Gauss points of every active cell, cell-rank order,
 *             lexicographic point order (first coordinate fastest);
 *   bdry_pts: n_sbm_faces x (p+1)^(d-1) x dim  closest points x on the true boundary of
 *             every surrogate-face Gauss point, in the library's face order.
 * Either pointer may be NULL.
 */
sbm_status sbm_rhs_points(sbm_handle h, double *cell_qp, double *bdry_pts);

/*
 * sbm_rhs -- right-hand side of Eq. (1): b_i = int f psi_i - int_{Gam~} (dpsi_i/dn~) g
 * + int_{Gam~} sigma g psi_i, from f at cell_qp and g at bdry_pts (host arrays laid out
 * as sbm_rhs_points).  b is a device FP64 vector of n_dofs entries.  Synchronous.
 */
sbm_status sbm_rhs(sbm_handle h, const double *f_qp, const double *g_bp, double *b, void *stream);

/*
 * sbm_l2_error -- the L2 error ||u_h - u*|| on the surrogate domain of the FP64 device vector x
 * (the error measure of App. A), by each cell's (p+1)^d-point Gauss rule: u* is given at the
 * cell_qp points of sbm_rhs_points (host array, n_cells x (p+1)^d, evaluated by the caller).
 * Synchronous (copies x to the host).  Errors: EINVAL (NULL argument, host-only handle), EHIP.
 */
sbm_status sbm_l2_error(sbm_handle h, const double *x, const double *ustar_qp, double *err);

/* Solver selection for sbm_solve. */
enum {
  SBM_SOLVE_GMRES_F64 = 0,  /* restarted GMRES(m) in FP64 */
  SBM_SOLVE_GMRES_IR = 1,   /* FP64 iterative refinement around FP32 GMRES(m) */
  SBM_SOLVE_CG_F64 = 2,     /* conjugate gradients in FP64: only for symmetric operators
                               (shift_scale = 0); the shifted operator is nonsymmetric */
  SBM_SOLVE_CG_IR = 3,      /* FP64 iterative refinement around FP32 conjugate gradients:
                               r = b - A x, |r| and x += |r| c in FP64, each inner FP32 CG
                               solves A c = r / |r| to max(1e-6, tol |b| / (2 |r|));
                               symmetric operators only */
  SBM_SOLVE_CG_RR = 4       /* conjugate gradients on the FP32 operator with x in FP64 and
                               FP64 residual replacement: r is recomputed as b - A x with the
                               FP64 operator whenever the recursive residual has dropped by
                               1e3 since the last replacement, without restarting (outer_its
                               counts the replacements); stops on the true residual;
                               symmetric operators only */
};

typedef struct {
  int status;             /* sbm_status of the solve */
  int outer_its;          /* refinement steps (IR) or restart cycles (GMRES) */
  int inner_its;          /* total Krylov iterations */
  int applies_f64;        /* FP64 operator applications */
  int applies_f32;        /* FP32 operator applications */
  double rel_residual;    /* final ||b - A x||_2 / ||b||_2, computed in FP64 on the device */
  double seconds;         /* wall time of the call */
} sbm_solve_info;

/*
 * sbm_solve -- solve A x = b to ||b - A x|| <= rel_tol ||b|| from the initial guess in x.
 * b, x: device FP64 vectors of n_dofs entries (x is read as the initial guess and
 * overwritten).  restart: Krylov dimension m of GMRES (<= 0 selects 50, at most 256).
 * max_it bounds the total Krylov iterations.  jacobi != 0 right-preconditions with the
 * inverse of the operator's diagonal.  The Krylov workspace (GMRES: m + 1 basis vectors per
 * precision used) is allocated on the first solve and kept with the handle; solves on one
 * handle must not overlap.  The solve runs on a stream of the workspace, after the work
 * already enqueued on stream; from the second GMRES restart cycle on, each run of Arnoldi
 * steps between residual checks is replayed from a graph captured at its first use (kept with
 * the workspace; SBM_SETUP_NO_GRAPHS disables this).  Synchronous (returns after the solve's
 * work has finished).
 * Errors: EINVAL, ENOMEM, ENOCONV (info->rel_residual holds what was reached), EHIP.
 */
sbm_status sbm_solve(sbm_handle h, const double *b, double *x, double rel_tol, int max_it,
                     int mode, int restart, int jacobi, void *stream, sbm_solve_info *info);

/*
 * sbm_solve_batch -- n independent solves A_i x_i = b_i (serving), each to
 * ||b_i - A_i x_i|| <= rel_tol ||b_i||, by restarted GMRES in lockstep: mode
 * SBM_SOLVE_GMRES_F64 or SBM_SOLVE_GMRES_IR (others: EUNSUPPORTED), no preconditioner.  At
 * every Krylov step the operator applies of all systems still iterating run as one batch of
 * applies (sbm_batch_*: one launch per stage per group of operators sharing a kernel
 * instantiation, groups on up to four streams); the other kernels of each system are the
 * ones sbm_solve launches, in the same order on that system's own workspace, so x_i and
 * infos[i] are those of sbm_solve(h_i, b_i, x_i, ...) with jacobi = 0 (bit for bit), except
 * the seconds, which are the wall time of the whole call.  Systems leave the lockstep as
 * they converge or reach max_it.  Argument rules as sbm_solve for each i, plus: a handle
 * appears at most once.  Runs on stream (after the work already on it); synchronous.
 * infos: n entries, each filled as sbm_solve fills its info.  Returns SBM_OK when every
 * system converged, else the first failing status (ENOCONV: see infos[i].status and
 * rel_residual).  Errors: EINVAL, ENOMEM, EUNSUPPORTED, EHIP.
 */
sbm_status sbm_solve_batch(int n, const sbm_handle *hs, const double *const *b, double *const *x,
                           double rel_tol, int max_it, int mode, int restart, void *stream,
                           sbm_solve_info *infos);

/*
 * sbm_diagonal -- the diagonal of A (device vector of n_dofs entries, precision prec),
 * computed matrix-free from the cell and face contributions.  Asynchronous.
 */
sbm_status sbm_diagonal(sbm_handle h, void *diag, int prec, void *stream);

/* Upper bound of the device bytes sbm_setup allocates for a problem on this mesh with at
 * most n_cells_hint active cells and n_faces_hint surrogate faces (host-side, no setup; the
 * solver workspace is not included).  0 for invalid arguments. */
size_t sbm_footprint_estimate(const sbm_mesh *mesh, int p, int disc, int64_t n_cells_hint,
                              int64_t n_faces_hint);

/* ---- introspection for setup-parity tests (host outputs) ---- */
/* Active-cell multi-indices (n_cells x dim, int32, cell-rank order). */
sbm_status sbm_export_cells(sbm_handle h, int32_t *cells);
/* Surrogate faces: (cell rank, axis, side) triples (n_sbm_faces x 3, int32, library order). */
sbm_status sbm_export_sbm_faces(sbm_handle h, int32_t *faces);
/* Shifted reference coordinates xi of every face point (n_sbm_faces x (p+1)^(d-1) x dim). */
sbm_status sbm_export_face_xi(sbm_handle h, double *xi);
/* Global DoF id of every local DoF of every active cell (n_cells x (p+1)^d, int64). */
sbm_status sbm_export_cell_dofs(sbm_handle h, int64_t *dofs);

#ifdef __cplusplus
}
#endif
#endif /* SBM_H */
