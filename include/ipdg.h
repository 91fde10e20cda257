/*
 * ipdg.h - C ABI of the MI355X symmetric interior-penalty DG elliptic solver.
 *
 * The library applies and inverts the screened-Poisson operator
 *     A = lambda M - Lap_IPDG
 * discretised with nodal discontinuous Galerkin on triangles of degree N
 * (Karakus, Chalmers, Swirydowicz, Warburton: Sec. 2.1 for the SIPDG
 * Laplacian, Eq. INS_SD_5 and the penalty Eq. Ch2.PenaltyParameter; Sec. 5.2,
 * Eq. ellipticOp1 / ellipticOp3, for the operator A; Sec. 3 for the
 * preconditioned conjugate-gradient solvers).
 *
 * Conventions shared by every entry point
 *   - Every call returns an ipdg_status; no C++ exception crosses the ABI.
 *     On failure ipdg_last_error() (thread-local) describes the cause.
 *   - Field vectors are DEVICE pointers to K*Np contiguous values,
 *     element-major (value i of element e at e*Np + i), node order: row by
 *     row from face 0 (j = 0..N, i = 0..N-j), Warp & Blend nodes on the
 *     bi-unit triangle (-1,-1), (1,-1), (-1,1).  Np = (N+1)(N+2)/2.
 *   - Mesh arrays passed to ipdg_mesh_create are HOST pointers, copied.
 *   - hip_stream is a hipStream_t (NULL = default stream).  apply-type calls
 *     are asynchronous on that stream; solve calls synchronise it before
 *     returning their iteration count and residual.
 *   - A handle is used from one stream at a time; calls on one handle must
 *     not overlap.
 *   - Boundary conditions are homogeneous and imposed through a mirror ghost
 *     state: Dirichlet u+ = -u-, grad u+ = grad u-; Neumann u+ = u-,
 *     n.grad u+ = -n.grad u-.
 *   - tau is the penalty constant c_tau: on face F between E- and E+,
 *     tau_F = c_tau * max(kappa- |F|/|E-|, kappa+ |F|/|E+|) (one-sided on
 *     boundary faces, kappa = 1 unless a coefficient was given).
 *     tau <= 0 selects (N+1)^2.
 */
#ifndef IPDG_H
#define IPDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipdg_mesh_s* ipdg_mesh;

typedef enum {
  IPDG_OK = 0,
  IPDG_NOT_CONVERGED = 1,   /* max_iters reached; x holds the last iterate */
  IPDG_EINVAL = -1,         /* bad argument (null pointer, size, option) */
  IPDG_EMESH = -2,          /* invalid mesh (see ipdg_mesh_create) */
  IPDG_EHIP = -3,           /* HIP runtime error; text has hipGetErrorString */
  IPDG_ENOMEM = -4,         /* device or host allocation failed */
  IPDG_EUNSUPPORTED = -5,   /* degree outside 1..8 or feature not built */
  IPDG_EBREAKDOWN = -6      /* CG breakdown: p^T A p <= 0 or not finite */
} ipdg_status;

typedef enum { IPDG_F64 = 0, IPDG_F32 = 1 } ipdg_dtype;
typedef enum { IPDG_BC_INTERIOR = 0, IPDG_BC_DIRICHLET = 1, IPDG_BC_NEUMANN = 2 } ipdg_bc;
typedef enum { IPDG_PC_NONE = 0, IPDG_PC_JACOBI = 1, IPDG_PC_BLOCK_MASS = 2, IPDG_PC_PMG = 3 } ipdg_pc;
typedef enum { IPDG_PREC_FP64 = 0, IPDG_PREC_MIXED = 1, IPDG_PREC_FP32_OPERATOR = 2 } ipdg_prec;

#define IPDG_MAX_LEVELS 8
#define IPDG_AMG_MAX_LEVELS 12

/* Options of the PCG solvers.  ipdg_default_opts() fills every field. */
typedef struct {
  ipdg_pc pc;              /* preconditioner */
  ipdg_prec prec;          /* FP64 throughout; IPDG_PREC_MIXED: an FP32
                              preconditioner (its operator applications,
                              smoothing, transfers and coarse solve) inside
                              FP64 CG: the outer operator, recurrences, dots and
                              residuals stay FP64; IPDG_PREC_FP32_OPERATOR: the
                              outer operator A p in FP32 as well (x, r, p and
                              the dots FP64), with reliable updates: r = b - A x
                              recomputed in FP64 and the direction restarted
                              whenever |r| fell by reliable_drop (1e-3 when 0) */
  int max_iters;           /* outer iteration limit */
  int check_every;         /* host polls convergence every this many iterations */
  int flexible;            /* 1: flexible CG beta = -(z+, Ap)/(p, Ap);
                              -1: automatic (flexible for PMG or MIXED) */
  /* p-multigrid (pc == IPDG_PC_PMG): degrees[0] must equal the mesh degree,
     strictly decreasing, last level solved by Jacobi-PCG.  n_levels == 0
     chooses the levels by halving the degree down to 1 (7, 3, 1 or
     8, 4, 2, 1), also per mesh in a batch of mixed degrees. */
  int n_levels;
  int degrees[IPDG_MAX_LEVELS];
  int cheb_degree;         /* Chebyshev steps per smoothing (>= 1) */
  double cheb_lo, cheb_hi; /* interval [lo*rho, hi*rho] of D^-1 A */
  double rho[IPDG_MAX_LEVELS]; /* spectral-radius estimates of D^-1 A per
                              level; <= 0: estimated at setup by
                              rho_steps Lanczos (Jacobi-PCG) steps */
  int rho_steps;
  double coarse_tol;       /* coarsest Jacobi-PCG relative tolerance */
  int coarse_max_iters;    /* and iteration cap (tol 0 => exactly this many);
                              < 0 (default): max(20, ceil(0.414 sqrt(K))), per
                              mesh (150 at K = 131,072) */
  double reliable_drop;    /* > 0: also recompute r = b - A x in FP64 whenever
                              |r| fell by this factor since the last recompute
                              (default 0: only when the recurrence stops) */
  int coarse_persistent;   /* 1: run the coarsest-level Jacobi-PCG as one
                              persistent launch with grid-wide barriers
                              (degrees 1..4, single solves only); 0 (default):
                              one short kernel sequence per iteration inside
                              the captured graph, converged iterations skipped */
  /* pMG-AMG (Sec. 3): coarse_amg = 1 replaces the coarsest-level Jacobi-PCG
     by amg_cycles cycles of an aggregation AMG hierarchy below the degree-1
     level (the last p-level must be degree 1): the degree-1 level (smoothed
     as the p-levels), one value per element (the element-block sums of the
     degree-1 operator), then greedy aggregates of maximal independent node
     sets with Galerkin operators, smoothed by Chebyshev of cheb_degree steps
     over [cheb_lo, cheb_hi] times the Gershgorin bound of D^-1 A, until at
     most amg_coarse_size (<= 2048) unknowns remain or 12 levels exist; the
     coarsest level is solved by its inverse.  The cycle is a K-cycle on the
     first amg_kcycle_levels levels (the coarse correction by two flexible-CG
     steps on the next level, each preconditioned by one cycle there; the
     second step skipped once the first reduced the coarse residual norm to
     0.25 of its start) and a V-cycle below.  Built on the host at setup.
     In a batch the solves then keep their own launches. */
  int coarse_amg;          /* 0 (default) or 1 */
  int amg_coarse_size;     /* default 512 */
  int amg_cycles;          /* default 1 */
  int amg_kcycle_levels;   /* default 2 (the paper's two finest levels); 0: V-cycle */
  int amg_top_krylov;      /* 1: the degree-1 level solved by two flexible-CG
                              steps on it, each preconditioned by one AMG
                              cycle (the K-cycle's step one level higher;
                              needs amg_cycles = 1); default 0 */
} ipdg_solve_opts;

/* Result record of a solve (all fields written). */
typedef struct {
  int iters;               /* outer iterations taken */
  double relres;           /* true ||b - A x|| / ||b|| in FP64 at exit */
  int restarts;            /* residual replacements (reliable updates) */
  double rho_used[IPDG_MAX_LEVELS];   /* Chebyshev radii used per level */
  double setup_ms;         /* preconditioner setup wall time */
  double solve_ms;         /* iteration wall time */
  int coarse_iters;        /* iterations of the last coarsest-level solve (0
                              with coarse_amg) */
  int amg_levels;          /* coarse_amg: levels of the algebraic hierarchy,
                              the degree-1 level included (else 0) */
  int amg_n[IPDG_AMG_MAX_LEVELS];   /* unknowns per level, degree-1 level first */
  int64_t precond_bytes;   /* device memory the preconditioner's set-up holds
                              beyond the outer CG's vectors (p-multigrid
                              levels' diagonals and work vectors, coarse-solve
                              work, the algebraic levels' matrices, transfers,
                              inverse and work); 0 for the diagonal ones */
} ipdg_solve_info;

void ipdg_default_opts(ipdg_solve_opts* opts);

/* Build a mesh handle of degree N (1..8) from K counter-clockwise triangles.
 *   VX, VY   : Nv vertex coordinates (host).
 *   EToV     : K*3 vertex ids, 0-based, counter-clockwise (host).
 *   EToB     : K*3 face flags; face f joins vertices f and (f+1)%3; values
 *              ipdg_bc (host).
 *   kappa    : K per-element coefficients > 0, or NULL for kappa = 1 (host).
 * IPDG_EMESH for a non-positive Jacobian, a face shared by more than two
 * elements, an unmatched face flagged interior or a matched face flagged as
 * boundary.  IPDG_EUNSUPPORTED for N outside 1..8.  The mesh's device data
 * live on the device current at creation; later calls on the mesh run there
 * (and restore the caller's current device).  Sec. 2.1 (mesh, degree),
 * Sec. 5.2 (geometric factors of the affine map, Eq. operators2). */
ipdg_status ipdg_mesh_create(int N, int Nv, const double* VX, const double* VY,
                             int K, const int32_t* EToV, const int8_t* EToB,
                             const double* kappa, ipdg_mesh* out);
ipdg_status ipdg_mesh_destroy(ipdg_mesh mesh);
ipdg_status ipdg_mesh_info(ipdg_mesh mesh, int* N, int* Np, int* K);

/* Physical node coordinates, HOST arrays of K*Np values each. */
ipdg_status ipdg_node_coords(ipdg_mesh mesh, double* x, double* y);

/* Replace the per-element coefficient kappa (HOST, K values > 0; NULL = 1). */
ipdg_status ipdg_set_kappa(ipdg_mesh mesh, const double* kappa);

/* y = (lambda M - Lap_IPDG) x for device vectors x, y of the given dtype
 * (Eq. ellipticOp1; computed in the regrouped strong form Eq. ellipticOp3).
 * x and y must not overlap.  Asynchronous on hip_stream. */
ipdg_status ipdg_apply(ipdg_mesh mesh, double lambda, double tau, ipdg_dtype dtype,
                       const void* x, void* y, void* hip_stream);

/* y = M x, the block-diagonal mass matrix J_e M (Eq. elMass, elementOps). */
ipdg_status ipdg_mass_apply(ipdg_mesh mesh, ipdg_dtype dtype, const void* x, void* y,
                            void* hip_stream);

/* Solve A x = b by PCG (Sec. 3).  b, x: device FP64 vectors; x holds x0 on
 * entry and the solution on exit.  Stops when ||r||_2 <= tol ||b||_2 with the
 * true residual confirmed.  info may be NULL. */
ipdg_status ipdg_pcg_solve(ipdg_mesh mesh, double lambda, double tau, const double* b,
                           double* x, double tol, const ipdg_solve_opts* opts,
                           ipdg_solve_info* info, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of ipdg_pcg_solve, same arguments and results, for the identity, Jacobi
 * and block inverse-mass preconditioners in FP64 (opts->prec must be
 * IPDG_PREC_FP64, opts->reliable_drop 0), calling no hipMalloc, hipFree or
 * other allocating routine.  Its work vectors, block partial sums and device
 * scalars live in one file-scope device array of the library (about 50 MB,
 * held on every GPU the library runs on until the process ends), so K*Np
 * must not exceed 1,048,576 (IPDG_EINVAL otherwise).  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  Kernels run
 * directly on hip_stream (no internal stream, no captured graph); the call
 * synchronises hip_stream before returning.  x (device, FP64) holds x0 on
 * entry and the solution on exit, and is the iterate throughout. */
ipdg_status ipdg_pcg_solve_noalloc(ipdg_mesh mesh, double lambda, double tau, const double* b,
                                   double* x, double tol, const ipdg_solve_opts* opts,
                                   ipdg_solve_info* info, void* hip_stream);

/* One application z = B r of the preconditioner that ipdg_pcg_solve would use
 * (device FP64 vectors).  Used to check a single V-cycle. */
ipdg_status ipdg_precond_apply(ipdg_mesh mesh, double lambda, double tau,
                               const ipdg_solve_opts* opts, const double* r, double* z,
                               ipdg_solve_info* info, void* hip_stream);

/* nb independent solves (lambda_i M - Lap) x_i = b_i, one mesh each (Sec. 3:
 * per-component velocity Helmholtz solves), advanced together: every round
 * replays each unfinished solve's captured graph of check_every iterations on
 * that solve's own stream, all launched before any is waited for.  b and x are
 * HOST arrays of nb device FP64 vector pointers; iters and relres are HOST
 * arrays of nb entries (may be NULL).  Each mesh handle may appear once.
 * With IPDG_PC_PMG and at least two solves whose coarsest levels share a
 * degree, those levels are solved together every outer iteration: one
 * launch per coarse-CG iteration covers all solves (their concatenated
 * coarsest levels), between each solve's captured parts before and after
 * it; the environment variable IPDG_BATCH_COARSE=separate keeps each solve's
 * coarsest level on its own launches.  The library keeps the last fused
 * batch's concatenated coarsest levels (about a dozen vectors of the
 * members' degree-1 sizes, plus their metric and connectivity) allocated,
 * for reuse by the next batch of the same solves, until a different batch
 * replaces them.  The persistent single-launch coarse
 * form is never used in a batch (its grids could not all be resident).
 * All meshes must live on one device.  opts NULL: defaults with the
 * block inverse-mass preconditioner.  Returns IPDG_NOT_CONVERGED if any
 * solve stopped at max_iters. */
ipdg_status ipdg_helmholtz_solve_batch(int nb, const ipdg_mesh* meshes, const double* lambdas,
                                       double tau, const double* const* b, double* const* x,
                                       double tol, const ipdg_solve_opts* opts, int* iters,
                                       double* relres, void* hip_stream);

/* dL/dkappa_e = -w^T (dA/dkappa_e) u for device FP64 vectors u, w;
 * dLdkappa is a device array of K doubles.  On a mesh without a
 * coefficient the derivative is taken at kappa = 1 (the mesh is not
 * changed). */
ipdg_status ipdg_kappa_grad(ipdg_mesh mesh, double tau, const double* u, const double* w,
                            double* dLdkappa, void* hip_stream);

/* ---- Semi-Lagrangian subcycling advection (Sec. 2.3, Eq. SS_3 and
 * INS_CUB_N; Sec. 5.3, Eq. KSS_3, Alg. SSV and SSS).  Device FP64 vectors of
 * K*Np values, asynchronous on hip_stream unless stated; outputs must not
 * overlap inputs.  The operator is
 *   (v, N~)_E = -(grad v, Ubar (x) U~)_E + (v, n . F~*)_dE,
 *   n . F~* = {n . (Ubar (x) U~)} + (Lambda / 2) (U~- - U~+),
 *   Lambda = max(|n . Ubar-|, |n . Ubar+|) at each face cubature point,
 * integrated with the volume rule (collapsed Gauss product, q^2 points,
 * q = floor(3N/2) + 1, exact for the volume integrand) and the q-point
 * Gauss-Legendre rule on faces.  Boundary faces: Ubar+ = Ubar-; U~+ = g on
 * Dirichlet faces (nodal data, face nodes read; NULL = 0), U~+ = U~- on
 * Neumann faces. ---- */

/* nu, nv = the selected parts of N~(Ubar, U~): parts = 1 the volume term
 * (Alg. SSV), 2 the surface term (Alg. SSS), 3 both (Eq. KSS_3).
 * IPDG_EINVAL for parts outside 1..3 or a null required vector. */
ipdg_status ipdg_subcycle_rhs(ipdg_mesh mesh, const double* ubar, const double* vbar, const double* u,
                              const double* v, const double* gu, const double* gv, int parts, double* nu,
                              double* nv, void* hip_stream);

/* Ns steps of the five-stage fourth-order low-storage Runge-Kutta scheme
 * (Carpenter and Kennedy) over [0, T] for dU~/dtau = -N~(Ubar(tau), U~)
 * (Eq. SS_3), with Ubar(tau) = ubar0 + tau ubar1 and Dirichlet data
 * g(tau) = g0 + tau g1 (ubar1, vbar1, gu1, gv1 may be NULL: constant in tau;
 * gu0, gv0 NULL: zero data).  (u, v) hold U~(0) on entry and U~(T) when
 * the work enqueued on hip_stream has run.  The mesh keeps 4 K Np doubles of
 * Runge-Kutta registers after the first call (allocated then, freed with the
 * mesh); calls on one mesh must not overlap.  IPDG_EINVAL for Ns < 1 or T not
 * finite. */
ipdg_status ipdg_subcycle(ipdg_mesh mesh, const double* ubar0, const double* vbar0, const double* ubar1,
                          const double* vbar1, const double* gu0, const double* gv0, const double* gu1,
                          const double* gv1, double T, int Ns, double* u, double* v, void* hip_stream);

/* ---- Around the elliptic solves of the algebraic splitting scheme (Sec. 2.2,
 * Eq. INS_TD_3); device FP64 vectors of K*Np values, asynchronous on
 * hip_stream, outputs must not overlap inputs.  Boundary faces take the
 * mesh's flags as velocity conditions: on Dirichlet faces u* = g_D and
 * p* = p-, on Neumann (outflow) faces u* = u- and p* = 0 (Sec. 2.1). ---- */

/* DG gradient with the central flux p* = {p} (Sec. 2.1, Eq. INS_SD_4_1):
 * (gx, gy) = G p. */
ipdg_status ipdg_grad(ipdg_mesh mesh, const double* p, double* gx, double* gy, void* hip_stream);

/* Nodal Lax-Friedrichs advection term of the splitting scheme's explicit
 * stage (Sec. 2.1, Eq. INS_SD_2 / INS_SD_3), per velocity component c:
 *   N_c = div(u_c u) + LIFT (|F|/|E|) (n . F_c* - n . F_c(u-)),
 *   n . F_c* = {n . F_c} + (Lambda / 2) (u_c- - u_c+),
 *   Lambda = 2 max(|n . u-|, |n . u+|),
 * the flux products taken at the nodes.  Dirichlet faces take u+ = g (gu, gv
 * nodal fields, face nodes read; NULL = 0), Neumann faces u+ = u-.
 * (nu, nv) = N(u, v). */
ipdg_status ipdg_advect(ipdg_mesh mesh, const double* u, const double* v, const double* gu, const double* gv,
                        double* nu, double* nv, void* hip_stream);

/* DG divergence with the central flux u* = {u} (Eq. INS_SD_4_2):
 * out = D (u, v).  gu, gv: Dirichlet data g_D as nodal fields (only their
 * values on Dirichlet face nodes are read), or NULL for g_D = 0. */
ipdg_status ipdg_div(ipdg_mesh mesh, const double* u, const double* v, const double* gu,
                     const double* gv, double* out, void* hip_stream);

/* b += the right-hand-side terms of inhomogeneous Dirichlet data g for the
 * SIPDG operator of ipdg_apply (Sec. 2.1, Eq. INS_SD_5 with its boundary
 * rules: the mirror ghost 2 g - u- on Dirichlet faces, so that u* = g):
 * -kappa (g, d_n l_i)_F + 2 tau_F (g, l_i)_F over the mesh's Dirichlet
 * faces, tau_F = c_tau kappa |F|/|E| (c_tau = tau, or (N+1)^2 when tau <= 0).
 * g: nodal field whose face-node values on Dirichlet faces are the data;
 * the operator's solution then takes the trace g there. */
ipdg_status ipdg_dirichlet_rhs(ipdg_mesh mesh, double tau, const double* g, double* b, void* hip_stream);

/* Right-hand sides of the two solves, mass-weighted for the SIPDG operator
 * (lambda M - Lap_IPDG) of ipdg_apply / ipdg_pcg_solve:
 *   velocity (Eq. INS_TD_3_2), lambda = gamma / (nu dt), per component:
 *     (bu, bv) = M (U^ / (nu dt) - G sigmaP / nu);
 *   pressure increment (Eq. INS_TD_3_3), lambda = 0 on a mesh with the
 *     swapped boundary flags (velocity Dirichlet faces are pressure Neumann
 *     faces and vice versa):  b = -(gamma / dt) M D (U^^). */
ipdg_status ipdg_ins_velocity_rhs(ipdg_mesh mesh, double nu, double dt, const double* uhat,
                                  const double* vhat, const double* sigma_p, double* bu, double* bv,
                                  void* hip_stream);
ipdg_status ipdg_ins_pressure_rhs(ipdg_mesh mesh, double gamma, double dt, const double* u,
                                  const double* v, const double* gu, const double* gv, double* b,
                                  void* hip_stream);

/* Correction (Eq. INS_TD_3_4): u_out = u - (dt / gamma) Gx dp,
 * v_out = v - (dt / gamma) Gy dp, p_out = dp + sigma_p. */
ipdg_status ipdg_ins_correct(ipdg_mesh mesh, double gamma, double dt, const double* u, const double* v,
                             const double* dp, const double* sigma_p, double* u_out, double* v_out,
                             double* p_out, void* hip_stream);

/* One step of the algebraic splitting scheme (Sec. 2.2, Eq. INS_TD_3), first
 * order in time (gamma = beta_0 = alpha_0 = 1), the pressure increment taken
 * over sigma P = 2 P^n - P^{n-1}:
 *   U^ = U^n - dt N(U^n)  (nodal Lax-Friedrichs advection, data gu_n, gv_n),
 *   (M / (nu dt) - Lap) U^^ = M (U^ / (nu dt) - G sigmaP / nu) + Dirichlet
 *     terms of gu_1, gv_1 (the data at t^{n+1}), PCG on `mesh`,
 *   -Lap dP = -(1 / dt) D(U^^; gu_1, gv_1), PCG on `pmesh` (the same
 *     triangles with the boundary flags swapped; without Dirichlet faces the
 *     right-hand side's constant component is removed first),
 *   U^{n+1} = U^^ - dt G dP,  P^{n+1} = dP + sigma P.
 * All vectors are device FP64 (K*Np); gu_*, gv_* may be NULL (zero data).
 * tol: relative tolerance of the three solves; vel_opts / pres_opts may be
 * NULL (defaults); iters (3 ints: the u, v and pressure solves) may be NULL.
 * Synchronous: returns when the step is done. */
ipdg_status ipdg_ins_step(ipdg_mesh mesh, ipdg_mesh pmesh, double nu, double dt, double tau,
                          const double* u_n, const double* v_n, const double* p_n, const double* p_nm1,
                          const double* gu_n, const double* gv_n, const double* gu_1, const double* gv_1,
                          double* u_1, double* v_1, double* p_1, double tol, const ipdg_solve_opts* vel_opts,
                          const ipdg_solve_opts* pres_opts, int* iters, void* hip_stream);

/* The same step with the semi-Lagrangian subcycling of Sec. 2.3 at first
 * order (S = 0) in place of the explicit advection step:
 *   U^ = U~(t^{n+1}),  dU~/dt = -N~(U^n, U~),  U~(t^n) = U^n,
 * advanced by `subcycles` substeps of ipdg_subcycle (cubature operator of
 * Eq. KSS_3, five-stage fourth-order low-storage Runge-Kutta), the Dirichlet
 * data of U~ linear in time from (gu_n, gv_n) to (gu_1, gv_1).  The rest of
 * the step is that of ipdg_ins_step.  Uses the Runge-Kutta registers the mesh
 * keeps for ipdg_subcycle: calls on one mesh must not overlap.  IPDG_EINVAL
 * for subcycles < 1. */
ipdg_status ipdg_ins_step_subcycled(ipdg_mesh mesh, ipdg_mesh pmesh, double nu, double dt, double tau,
                                    int subcycles, const double* u_n, const double* v_n, const double* p_n,
                                    const double* p_nm1, const double* gu_n, const double* gv_n,
                                    const double* gu_1, const double* gv_1, double* u_1, double* v_1,
                                    double* p_1, double tol, const ipdg_solve_opts* vel_opts,
                                    const ipdg_solve_opts* pres_opts, int* iters, void* hip_stream);

/* Host-only validation of a mesh, without any device use: the same checks
 * and face matching as ipdg_mesh_create.  EToE (neighbour element, -1 on a
 * boundary face) and EToF (neighbour's face index, -1 on a boundary face)
 * are HOST arrays of K*3 entries, or NULL. */
ipdg_status ipdg_mesh_check(int N, int Nv, const double* VX, const double* VY, int K,
                            const int32_t* EToV, const int8_t* EToB, int32_t* EToE,
                            int8_t* EToF);

/* Host-only: reference nodes r, s (Np each) and the reference operators of
 * Sec. 5.2, Eq. elMass / elLift on the bi-unit triangle: D_r, D_s, M
 * (Np x Np, row-major) and LIFT (Np x 3 Nfp).  Any output may be NULL. */
ipdg_status ipdg_reference_element(int N, double* r, double* s, double* Dr, double* Ds,
                                   double* M, double* LIFT);

/* Operator-kernel variants.  Every call that applies the operator at degree
 * N in a given precision (ipdg_apply and the solvers' operator launches)
 * uses the variant set for (N, dtype), process-wide: bit 1 = the element's
 * own nodal values staged through LDS for coalesced loads and stores, bit
 * 2 = raised occupancy (fewer registers per lane).  Degrees 1..5 take
 * variants 0..3; degrees 6..8 variants 0 and 1.  All variants give identical results
 * (same arithmetic in the same order); they differ in speed only.  Solves
 * already captured into a graph keep the variant they were captured with.
 * Defaults come from sweeps of the 524,288-triangle operator workload; the
 * environment variable IPDG_AX_VARIANT, read once, overrides them for all
 * degrees <= 5.  Returns IPDG_EINVAL for N outside 1..8, a bad dtype or a
 * variant the degree does not have. */
ipdg_status ipdg_ax_variant_get(int N, ipdg_dtype dtype, int* variant);
ipdg_status ipdg_ax_variant_set(int N, ipdg_dtype dtype, int variant);

/* Autotuner: times every operator variant of this mesh's degree in dtype on
 * this mesh (one warm-up apply, then reps applies, on hip_stream, with the
 * given lambda and tau), selects the fastest for (N, dtype) as by
 * ipdg_ax_variant_set and returns it in *chosen.  times_ms (HOST, 4
 * entries, may be NULL) receives the mean time per apply of variants 0..3
 * (-1 for a variant the degree does not have).  reps <= 0 selects 20.
 * Allocates two device vectors of K*Np values for the duration of the call
 * and synchronises hip_stream.  On failure the previous variant is kept. */
ipdg_status ipdg_autotune_apply(ipdg_mesh mesh, double lambda, double tau, ipdg_dtype dtype,
                                int reps, int* chosen, double* times_ms, void* hip_stream);

/* Empirical roofs of the current device (Sec. 5.1: the kernels are judged
 * against a measured device-to-device copy rate).  ipdg_probe_copy: GB/s of
 * read + write traffic of a vectorised (16 bytes per lane) copy kernel moving
 * `bytes` per copy, rotating over `sets` source/destination pairs (sets *
 * 2 * bytes larger than the last-level cache measures HBM) for `reps`
 * copies on hip_stream.  ipdg_probe_fma: TFLOP/s (two per multiply-add) of
 * independent FP64 or FP32 multiply-add chains with wave-uniform
 * multipliers, every SIMD occupied.  Both allocate their buffers for the
 * duration of the call and synchronise hip_stream. */
ipdg_status ipdg_probe_copy(size_t bytes, int sets, int reps, double* gbs, void* hip_stream);
ipdg_status ipdg_probe_fma(ipdg_dtype dtype, int reps, double* tflops, void* hip_stream);

/* Message of the last failed call on this thread ("" after a success). */
const char* ipdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IPDG_H */
