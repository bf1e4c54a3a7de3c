/*
 * ibpm.h -- C ABI of the MI355X immersed-boundary projection library.
 *
 * The library advances the discrete incompressible Navier-Stokes equations
 * with an immersed boundary by the projection method of Taira & Colonius as
 * used in Layton, Krishnan & Barba, "cuIBM -- A GPU-accelerated Immersed
 * Boundary Method" (arXiv:1109.3524), Sec. 2: per time step
 *     A q*            = r1                     (Eq. 11a, velocity solve)
 *     Q^T B^N Q lambda = Q^T q* - r2           (Eq. 11b, pressure + forces)
 *     q^{n+1}         = q* - B^N Q lambda      (Eq. 11c, projection)
 * with Q = [G, E^T], E the regularised-delta interpolation (Eqs. 5-7),
 * lambda = (phi, f~), B^1 = dt Mf^{-1} (first-order approximation of A^{-1}).
 * Every step runs on the GPU in hand-written HIP kernels for gfx950.
 *
 * Conventions shared by all calls
 *  - Grid: nx x ny cells with face lines xf[0..nx], yf[0..ny] (strictly
 *    increasing, non-uniform allowed; uniform under every delta support).
 *  - Flux vector q (length n_q = (nx-1)*ny + nx*(ny-1)): first the u faces
 *    u_{i,j} at (xf[i], yc_j), i = 1..nx-1, j = 0..ny-1, x index fastest,
 *    stored as q = u * dy_j; then the v faces v_{i,j} at (xc_i, yf[j]),
 *    i = 0..nx-1, j = 1..ny-1, stored as q = v * dx_i.
 *  - lambda (length n_lambda = nx*ny + 2*nb): cell pressures phi (x fastest),
 *    then the nb x-forces, then the nb y-forces on the Lagrangian points.
 *    One pressure cell (ibpm_params.pin_cell, default 0) is pinned: its row
 *    and column carry only the diagonal (Sec. 2, last paragraph), so
 *    phi[pin_cell] = 0 when rhs[pin_cell] = 0.
 *  - Device pointers are HIP device memory owned by the caller (for example
 *    torch tensors); they must stay valid until the work queued on the
 *    context's stream has completed.  Host pointers are read during the
 *    call only.
 *  - Every call queues work on the stream given to ibpm_build_operators.
 *    The solves (ibpm_solve_poisson, ibpm_solve_velocity and the solves
 *    inside ibpm_step) wait for the stream: their iterations are queued in
 *    chunks, and the host reads the device status (a few bytes) after each
 *    chunk to decide how many more to queue.  The other calls return without
 *    waiting, except where a host output (stats, forces, walls) is
 *    requested: then they wait for the stream.
 *  - Return codes: IBPM_OK or a negative IBPM_E* code; ibpm_last_error()
 *    returns a text description.  No C++ exception crosses this boundary.
 *  - One context serves one stream; calls on one context must not overlap.
 */
#ifndef IBPM_H
#define IBPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IBPM_OK        0
#define IBPM_EINVAL   -1   /* bad shape or parameter, delta support on a non-uniform patch */
#define IBPM_ENOMEM   -2   /* device or host allocation failed */
#define IBPM_ENOTCONV -3   /* iteration limit reached; outputs hold the last iterate */
#define IBPM_EHIP     -4   /* a HIP runtime call failed */
#define IBPM_ENAN     -5   /* a residual norm became NaN or Inf */

/* Poisson solvers (Sec. 3: CG with diagonal or smoothed-aggregation AMG
 * preconditioning).  The velocity solve always uses Jacobi-PCG. */
#define IBPM_SOLVER_JACOBI_PCG       0
#define IBPM_SOLVER_AMG_PCG          1
#define IBPM_SOLVER_AMG_PCG_MIXED    2   /* FP32 inner AMG-PCG inside FP64 iterative refinement */
#define IBPM_SOLVER_AMG_FCG_LEARNED  3   /* flexible CG, AMG V-cycle plus a learned stage */
#define IBPM_SOLVER_AMG_FCG_MIXED_LEARNED 4  /* FP32 inner flexible CG with the learned stage
                                                inside FP64 iterative refinement */
#define IBPM_SOLVER_AMG_PCG_FP32_CYCLE 5     /* FP64 CG whose V-cycle runs in FP32 (the
                                                residual rounded to FP32 on entry) */
#define IBPM_SOLVER_AMG_PCG_FP32_CYCLE_GUESS 6  /* solver 5 started from the learned initial
                                                   guess x0 + w N(b - K x0) (network weights
                                                   required, see below) */

/* Wall kinds (ibpm_params.bc_kind, per side: left x = xf[0], right
 * x = xf[nx], bottom y = yf[0], top y = yf[ny]). */
#define IBPM_BC_DIRICHLET  0   /* the wall velocity is (bc_u, bc_v) of that side at all times */
#define IBPM_BC_CONVECTIVE 1   /* right wall only: du/dt + U du/dx = 0 with U = uinf cos(alpha)
                                  (Sec. 5.2), explicit in time from the adjacent interior
                                  values; the wall starts at the freestream (uinf, alpha), and
                                  its normal velocity is shifted uniformly each step so that
                                  the net flux through the walls is zero */

typedef struct ibpm_ctx ibpm_ctx;

typedef struct ibpm_params {
    int32_t nx, ny;              /* cells per direction, >= 4 */
    const double *xf, *yf;       /* host, nx+1 and ny+1 face coordinates */
    int32_t nb;                  /* Lagrangian points, >= 0 */
    const double *xb, *yb;       /* host, nb point positions */
    const double *ubx, *uby;     /* host, nb prescribed body velocity; NULL means 0 */
    double nu;                   /* kinematic viscosity, > 0 */
    double dt;                   /* time step, > 0 */
    double uinf, alpha;          /* freestream speed and inflow angle (radians) */
    int32_t bn_order;            /* order N of B^N, the N-term series of A^{-1} (Sec. 2, after
                                    Eq. 11): 1 or 3 (the two of Sec. 5.1; B^2 is indefinite
                                    where (nu dt / 2) rho(L Mf^{-1}) > 1).  N = 1 (B^1 = dt Mf^{-1}, diagonal)
                                    keeps K matrix-free; N > 1 forms K = Q^T B^N Q on the
                                    device by sliced sparse products (Sec. 4) and supports the
                                    Jacobi-PCG and AMG-PCG Poisson solvers */
    double vel_rtol;             /* velocity solve: ||r|| <= vel_rtol ||b|| */
    int32_t vel_maxit;
    int32_t poisson_solver;      /* IBPM_SOLVER_* */
    double poisson_rtol;
    int32_t poisson_maxit;
    double amg_theta;            /* strength threshold (0 = every connection strong) */
    int32_t amg_pre, amg_post;   /* Jacobi sweeps before / after the coarse correction */
    int32_t amg_coarse_max;      /* stop coarsening at or below this many unknowns */
    int32_t amg_max_levels;
    double inner_rtol;           /* refinement (solvers 2, 4): floor of the relative tolerance
                                    of an inner FP32 solve; 0 selects 1e-5 */
    int32_t learned_every;       /* solvers 3, 4: the network runs on every learned_every-th
                                    preconditioner application, the V-cycle alone on the
                                    others; 0 or 1 = every application */
    int32_t fcg_depth;           /* solvers 3, 4: directions kept by the truncated flexible
                                    CG, FCG(m); 0 selects 4, at most 8 */
    int32_t use_graphs;          /* 1: replay the launches of CG iterations as HIP graphs
                                    (recorded once per solve kind and operand set on a
                                    stream of the context's own); 0: launch them one by one */
    int32_t fuse_transfers;      /* 1: the V-cycle folds the residual into the restriction
                                    (R b - (R A) x) on every CSR level and on a finest level of
                                    at most 600,000 unknowns, and the prolongation into the
                                    first post-sweep on CSR levels of at most 200,000 unknowns,
                                    with R A and A P formed at build time; 0: separate kernels
                                    (the same V-cycle, other rounding) */
    int32_t pin_cell;            /* pressure cell (j * nx + i) whose value is pinned: its row
                                    and column of K carry only the diagonal and its right-hand
                                    side entry is 0 (Sec. 2, last paragraph); 0..nx*ny-1 */
    int32_t bc_kind[4];          /* IBPM_BC_* of the left, right, bottom and top walls.  The
                                    paper's cylinder runs: DIRICHLET at the freestream on the
                                    left, bottom and top, CONVECTIVE on the right (Sec. 5.2).
                                    Without a convective wall the Dirichlet walls must carry
                                    zero net flux (else IBPM_EINVAL) */
    double bc_u[4], bc_v[4];     /* wall velocity (u, v) of each Dirichlet side (same order);
                                    ignored for a convective side */
    double fcg_stall_fall;       /* solvers 3, 4: fraction by which ||r|| must fall within 16
                                    iterations for the flexible iteration to count as making
                                    progress (else it falls back to AMG-PCG); 0 selects 0.05,
                                    1 makes every 16 iterations a stall; 0..1 */
    double body_ramp;            /* time over which the prescribed body velocity (ubx, uby) rises
                                    from rest as sin^2(pi t / (2 body_ramp)), t the time the step
                                    advances to; 0: the full velocity from the first step (the
                                    impulsive start of Sec. 5.1); >= 0 */
    int32_t moving_body;         /* 1: the points may move between steps (ibpm_move_body, Sec. 6):
                                    the level-0 K is stored and re-assembled on the device at
                                    every move; B^1 only, Jacobi-PCG or AMG-PCG.  0: fixed body */
    int32_t amg_rebuild_every;   /* moving body with AMG-PCG: at every n-th move (n >= 1) the
                                    smoothed-aggregation hierarchy is formed anew from the moved K,
                                    on the device, keeping the aggregates and smoothing weights of
                                    the first set-up (the levels of the dense coarse cycle are
                                    formed on the host); in between it is re-used with only its
                                    finest level following K (Sec. 4).  0: never formed anew */
} ibpm_params;

typedef struct ibpm_solve_stats {
    int32_t iters;        /* Krylov iterations */
    int32_t status;       /* IBPM_OK, IBPM_ENOTCONV or IBPM_ENAN */
    double relres;        /* true residual ||b - K x|| / ||b|| recomputed at exit */
    double ms;            /* wall time of the call */
    int32_t outer_iters;  /* refinement steps (mixed precision), else 1 */
    int32_t fallbacks;    /* switches to the plain AMG-PCG (learned stage), else 0 */
} ibpm_solve_stats;

typedef struct ibpm_step_stats {
    int32_t steps;              /* steps taken */
    int32_t vel_iters;          /* summed over the steps */
    int32_t poisson_iters;      /* summed over the steps */
    int32_t last_vel_iters, last_poisson_iters;
    double vel_relres_max;      /* largest true relative residual over the steps */
    double poisson_relres_max;
    double fx, fy;              /* body force of the last step (sum of f~), C_d = 2 fx / (U^2 D) */
    double ms;                  /* wall time of the call */
    double vel_ms, poisson_ms;  /* wall time of the solves, summed over the steps */
} ibpm_step_stats;

/* Build every operator of Sec. 2 for the given grid and body, the
 * smoothed-aggregation hierarchy when an AMG solver is selected (Sec. 3),
 * and upload them to the current HIP device.  `stream` is a hipStream_t
 * (NULL = the null stream) on which all later work of the context is
 * queued.  On success *out owns all device memory of the context.
 * Errors: IBPM_EINVAL (shapes, parameters, delta support not uniform),
 * IBPM_ENOMEM, IBPM_EHIP. */
int ibpm_build_operators(const ibpm_params *p, void *stream, ibpm_ctx **out);

/* Free the context and all its device memory (waits for its stream). */
int ibpm_destroy(ibpm_ctx *ctx);

/* Text of the last error on this context ("" if none; also valid for NULL). */
const char *ibpm_last_error(const ibpm_ctx *ctx);

/* Sizes of the flux and lambda vectors. */
int ibpm_sizes(const ibpm_ctx *ctx, int64_t *n_q, int64_t *n_lambda);

/* Impulsive start (Sec. 5.2): q = freestream (uinf, alpha) everywhere
 * (device, n_q), conv_prev = 0 (device, n_q), lambda = 0 (device, n_lambda),
 * the Dirichlet walls at their (bc_u, bc_v), a convective wall at the
 * freestream, and the step counter reset to 0. */
int ibpm_init_state(ibpm_ctx *ctx, double *q, double *conv_prev, double *lambda);

/* Advance nsteps time steps of Eq. (11) in place.
 *   q         device n_q, in: q^n, out: q^{n+nsteps}
 *   conv_prev device n_q, in: N(q^{n-1}) (ignored on step 0, where the
 *             Adams-Bashforth history is taken as N(q^0)), out: N(q^{n+nsteps-1})
 *   lambda    device n_lambda, in: warm start, out: last (phi, f~)
 *   stats     host, may be NULL (then the call does not wait).
 * Returns IBPM_ENOTCONV / IBPM_ENAN if a solve failed (the step is still
 * completed with the last iterate). */
int ibpm_step(ibpm_ctx *ctx, int32_t nsteps, double *q, double *conv_prev,
              double *lambda, ibpm_step_stats *stats);

/* Solve K lambda = rhs with K = Q^T B^1 Q pinned (Eq. 11b) by the selected
 * Poisson solver.  rhs device n_lambda; lambda device n_lambda, in: initial
 * guess, out: solution.  stats host, may be NULL. */
int ibpm_solve_poisson(ibpm_ctx *ctx, const double *rhs, double *lambda,
                       ibpm_solve_stats *stats);

/* Solve A q = rhs (Eq. 11a) by Jacobi-PCG; q in: initial guess, out: solution. */
int ibpm_solve_velocity(ibpm_ctx *ctx, const double *rhs, double *q,
                        ibpm_solve_stats *stats);

/* ibpm_solve_velocity without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the Jacobi-PCG work vectors, partial
 * sums and status live in a file-scope device array of the library
 * (5 * 2^20 + 3 * 3 * 32768 doubles plus the status, about 42 MB per device,
 * held from the library's first use on a device until the process ends;
 * its address is looked up once per device by ibpm_build_operators).  The
 * iterations are launched one by one (no graph is recorded); the results
 * are those of ibpm_solve_velocity, bit for bit.  Limit: n_q <= 2^20
 * (1,048,576 flux unknowns, e.g. a 724 x 724 grid), else IBPM_EINVAL.  Every
 * context on a device shares that device's array: calls that overlap on one
 * device (two streams, two threads) race and must not be made.  Other
 * errors as ibpm_solve_velocity. */
int ibpm_solve_velocity_static(ibpm_ctx *ctx, const double *rhs, double *q,
                               ibpm_solve_stats *stats);

/* The pinned Poisson operator K = Q^T B^N Q as the context holds it on the
 * host (for N > 1: the product formed on the device; for a moving body: the
 * device K of the current positions, read back): *nnz receives its stored
 * entries; ptr (n_lambda + 1), col and val (nnz each), host arrays, receive
 * its CSR rows (sorted columns) when not NULL. */
int ibpm_get_poisson_matrix(ibpm_ctx *ctx, int64_t *nnz, int32_t *ptr, int32_t *col, double *val);

/* Sizes of the B^N operators: stored entries of K and of B^N (n_q for the
 * diagonal B^1), and for N > 1 the device memory of the sliced triple
 * product -- the largest slice (its B^N Q rows, its K rows and its rows of
 * Q^T) against the rows of B^N Q over all slices, which an unsliced product
 * would hold at once (0 for N = 1).  Host outputs, each may be NULL. */
int ibpm_bn_info(const ibpm_ctx *ctx, int64_t *nnz_K, int64_t *nnz_B, int64_t *peak_bytes,
                 int64_t *unsliced_bytes);

/* A body in prescribed motion (Sec. 6; the per-step update of the forcing
 * rows of Q that Sec. 4 keeps apart from the rest of the solve): the nb
 * Lagrangian points move to (xb, yb) with velocities (ubx, uby), host arrays
 * of nb each, taken as those at the time the next step advances to (the
 * body_ramp start-up scales the velocities as for a fixed body).  Needs a
 * context built with moving_body = 1.  E and every row of K that couples to
 * the forces are formed anew on the device (K is re-assembled in place as
 * one CSR with the fixed pressure rows), and with AMG-PCG the hierarchy is
 * formed anew at every amg_rebuild_every-th move.  Synchronises the stream.
 * Points whose delta support leaves the uniform cells around them or the
 * grid, or non-finite values: IBPM_EINVAL, the context unchanged. */
int ibpm_move_body(ibpm_ctx *ctx, const double *xb, const double *yb, const double *ubx,
                   const double *uby);

/* Moving body: the moves made, the hierarchies formed anew since set-up,
 * and box (4 entries: i0, i1, j0, j1) the cells whose faces E reaches at the
 * current positions.  Host outputs, each may be NULL; IBPM_EINVAL for a
 * fixed-body context. */
int ibpm_moving_info(const ibpm_ctx *ctx, int64_t *moves, int64_t *refreshes, int32_t *box);

/* ------------------------------------------------------------------------
 * The three-dimensional extension (Sec. 7 names the 7-point pressure stencil
 * in three dimensions as the method's next step): Eqs. 6-11 carried over
 * axis by axis on an nx x ny x nz staggered grid.  Unknowns x fastest, then
 * y, then z: q = [u faces (x_1..x_{nx-1}); v faces; w faces] as fluxes
 * (velocity times face area), lambda = [nx ny nz cell pressures; 3 nb forces
 * (x, y, z components)].  A context built here answers the calls below and
 * ibpm_solve_poisson, ibpm_apply_K, ibpm_get_poisson_matrix,
 * ibpm_hierarchy_info, ibpm_sizes, ibpm_destroy and ibpm_last_error; the
 * two-dimensional time-step calls return IBPM_EINVAL on it.  The momentum
 * right-hand side (convection, wall values) is the caller's: the library
 * carries the linear algebra of a step, Eq. 11.
 * ------------------------------------------------------------------------ */
typedef struct ibpm3d_params {
    int32_t nx, ny, nz;          /* cells per axis, >= 2 */
    const double *xf, *yf, *zf;  /* host face coordinates (n + 1 each), strictly increasing */
    int32_t nb;                  /* Lagrangian points (>= 0) */
    const double *xb, *yb, *zb;  /* host point coordinates; every delta support must lie on
                                    uniform cells inside the grid, else IBPM_EINVAL */
    double nu, dt;               /* viscosity and time step (> 0) */
    double vel_rtol;             /* velocity solve: Jacobi-PCG relative residual */
    int32_t vel_maxit;
    int32_t poisson_solver;      /* IBPM_SOLVER_JACOBI_PCG or IBPM_SOLVER_AMG_PCG */
    double poisson_rtol;
    int32_t poisson_maxit;
    double amg_theta;            /* smoothed aggregation as in two dimensions (Sec. 3) */
    int32_t amg_pre, amg_post, amg_coarse_max, amg_max_levels;
    int32_t pin_cell;            /* pressure value pinned: cell (k ny + j) nx + i */
    int32_t use_graphs;          /* 1: CG iterations replayed as HIP graphs */
} ibpm3d_params;

/* Operators on the host (A, Q^T = [-D; E], B^1 = dt R M^-1, K = Q^T B^1 Q
 * pinned, the SA hierarchy of K), then stored on the device as CSR; the
 * context as ibpm_build_operators. */
int ibpm3d_build_operators(const ibpm3d_params *p, void *stream, ibpm_ctx **out);

/* q: A q = rhs by Jacobi-PCG from q (Eq. 11a); device n_q vectors. */
int ibpm3d_solve_velocity(ibpm_ctx *ctx, const double *rhs, double *q, ibpm_solve_stats *stats);

/* y = A x, device n_q vectors, distinct. */
int ibpm3d_apply_A(ibpm_ctx *ctx, const double *x, double *y);

/* rhs = Q^T q* - r2 with the pinned entry cleared (Eq. 11b); q* device n_q,
 * r2 and rhs device n_lambda, distinct. */
int ibpm3d_poisson_rhs(ibpm_ctx *ctx, const double *qstar, const double *r2, double *rhs);

/* qout = q* - B^1 Q lambda (Eq. 11c); device vectors, qout may be q*. */
int ibpm3d_project(ibpm_ctx *ctx, const double *qstar, const double *lambda, double *qout);

/* The linear algebra of one time step, Eq. 11: q* from A q* = r1 (starting
 * from q), lambda from K lambda = Q^T q* - r2 (starting from lambda), then
 * q = q* - B^1 Q lambda written over q.  Device vectors (r1, q: n_q; r2,
 * lambda: n_lambda).  Stats of both solves (each may be NULL); returns the
 * first solve's failure code, if any.  Synchronises the stream. */
int ibpm3d_linear_step(ibpm_ctx *ctx, const double *r1, const double *r2, double *q, double *lambda,
                       ibpm_solve_stats *vel_stats, ibpm_solve_stats *poisson_stats);

/* y = K x (pinned Q^T B^N Q), x and y device n_lambda, distinct. */
int ibpm_apply_K(ibpm_ctx *ctx, const double *x, double *y);

/* y = A x (Mf/dt - nu/2 L on interior faces), x and y device n_q, distinct. */
int ibpm_apply_A(ibpm_ctx *ctx, const double *x, double *y);

/* Single stages of one step, for checking each kernel:
 *   walls:   wall values n -> n+1 from q^n (convective outflow + mass balance)
 *            into the context's "next" walls (does not swap them in);
 *   rhs1:    r1 (device n_q) and N(q^n) (conv_now, device n_q) from q^n and
 *            conv_prev, using the current and next walls; conv_prev is only
 *            read (step counter 0 means N(q^{-1}) = N(q^n));
 *   rhs2:    Poisson right-hand side [-D q* + bc2 ; E q* - u_B] (pinned
 *            entry zeroed) with the next walls;
 *   project: q_out = q* - B^1 Q lambda (Eq. 11c); q_out may alias qstar. */
int ibpm_stage_walls(ibpm_ctx *ctx, const double *q);
int ibpm_stage_rhs1(ibpm_ctx *ctx, const double *q, const double *conv_prev,
                    double *r1, double *conv_now);
int ibpm_stage_rhs2(ibpm_ctx *ctx, const double *qstar, double *rhs);
int ibpm_stage_project(ibpm_ctx *ctx, const double *qstar, const double *lambda,
                       double *q_out);

/* Wall values, packed on the host as
 *   uL[ny] uR[ny] vB[nx] vT[nx] uBt[nx+1] uTt[nx+1] vLt[ny+1] vRt[ny+1]
 * (4*nx + 4*ny + 4 doubles).  which = 0: current walls, 1: next walls. */
int ibpm_get_walls(ibpm_ctx *ctx, int32_t which, double *host);
int ibpm_set_walls(ibpm_ctx *ctx, int32_t which, const double *host);

/* Step counter (0 = the next step is the first, AB2 start-up). */
int ibpm_get_step(const ibpm_ctx *ctx, int64_t *step);
int ibpm_set_step(ibpm_ctx *ctx, int64_t step);

/* Body force (sum of f~ over the points) of the last step or stage project. */
int ibpm_get_forces(ibpm_ctx *ctx, double *fx, double *fy);

/* Smoothed-aggregation hierarchy: number of levels, and per level (host
 * arrays of length >= levels) the unknowns and stored non-zeros. */
int ibpm_hierarchy_info(const ibpm_ctx *ctx, int32_t *levels, int64_t *sizes,
                        int64_t *nnz);

/* Aggregate index of every unknown of `level` (host, sizes[level] int32s). */
int ibpm_get_aggregates(const ibpm_ctx *ctx, int32_t level, int32_t *agg);

/* Host-only preview of the set-up of Sec. 3 for the parameters p: the
 * operators and the smoothed-aggregation hierarchy that
 * ibpm_build_operators would build, formed on the host without touching the
 * GPU (p->poisson_solver must select an AMG solver).  Outputs (host, each
 * may be NULL): *levels the level count; per level, in arrays with room for
 * `cap` levels, the unknowns (sizes), the stored non-zeros (nnz) and the
 * estimate rho of the spectral radius of D^{-1} A behind that level's
 * Jacobi weights 4 / (3 rho); agg the aggregate of every unknown of level
 * agg_level (sizes[agg_level] int32s, agg_level < levels - 1); *seconds the
 * host set-up time.  err (may be NULL) receives up to errlen bytes of an
 * error text.  Returns IBPM_OK, IBPM_EINVAL (bad parameters, a cap below
 * the level count, agg_level out of range) or IBPM_ENOMEM. */
int ibpm_plan_hierarchy(const ibpm_params *p, int32_t cap, int32_t *levels, int64_t *sizes,
                        int64_t *nnz, double *rho, int32_t agg_level, int32_t *agg,
                        double *seconds, char *err, int32_t errlen);

/* Kernels that ibpm_time_kernel can time (the launch configuration and
 * operands are those of the time step). */
#define IBPM_KERNEL_K0_JACOBI     0   /* damped Jacobi sweep with K, finest AMG level */
#define IBPM_KERNEL_K0_PCG_SPMV   1   /* p = z + beta p; q = K p; p . q */
#define IBPM_KERNEL_A_PCG_SPMV    2   /* velocity: p = D^{-1} r + beta p; q = A p; p . q */
#define IBPM_KERNEL_K0_RESIDUAL   3   /* r = b - K x, finest AMG level (in the cycle only where
                                         the restriction does not fold it in) */
#define IBPM_KERNEL_RESTRICT0     4   /* b1 = P0^T (b - K x) = P0^T b - (P0^T K) x with the
                                         product formed at setup (finest levels up to 600,000
                                         unknowns), else b1 = P0^T r */
#define IBPM_KERNEL_PROLONG0      5   /* x += P0 x1 */
#define IBPM_KERNEL_PCG_UPDATE_K  6   /* x += a p; r -= a q; r . r */
#define IBPM_KERNEL_COARSE_CYCLE  7   /* the V-cycle on the small levels as one dense product */
#define IBPM_KERNEL_PRESMOOTH0    8   /* two damped Jacobi sweeps from zero on the finest level */
#define IBPM_KERNEL_STREAM_COPY   9   /* y = x over 2^25 doubles (256 MiB each way): the
                                         reference for bandwidth and for traffic counters */
#define IBPM_KERNEL_UPDATE_PRESMOOTH0 10 /* the PCG update (x += a p; r' = r - a q) and two damped
                                             Jacobi sweeps from zero for r' on the finest level in
                                             one pass (where the iteration folds them together) */
#define IBPM_KERNEL_L1_JACOBI     11  /* damped Jacobi sweep with the stored (CSR) operator of
                                         AMG level 1 */
#define IBPM_KERNEL_COPY_LEVEL0   12  /* y = x over n_lambda doubles (one finest-level vector each
                                         way): the bandwidth a streaming kernel of the level-0
                                         vectors' size reaches */
#define IBPM_KERNEL_PROLONG_POST0 13  /* the prolongation and both post-smoothing sweeps of the
                                            finest level in one pass (strips, plus three small
                                            passes over the box coupled to the forces), where the
                                            iteration uses it (post = 2, grids of 2^22 cells and
                                            more) */
#define IBPM_NUM_KERNELS          14

/* Launches per PCG iteration that the FP64 AMG-PCG solve of this context
 * makes of each kernel ibpm_time_kernel can time: counts[k] for kernel id
 * k < min(ncounts, IBPM_NUM_KERNELS) (host array).  Level 1 counts its plain
 * damped-Jacobi sweeps only (not its fused two-sweep pass, restriction and
 * prolongation); levels >= 2 and the one-block reductions are not counted.
 * Needs an AMG context with B^1. */
int ibpm_iteration_launches(const ibpm_ctx *ctx, int32_t ncounts, int32_t *counts);

/* Time `reps` back-to-back launches of one kernel of the solver on the
 * context's stream with HIP events and return the mean duration of one
 * launch (ms) and the algorithmic bytes of one launch (every operand read
 * once, every result written once).
 *   min_footprint 0: every launch uses the solver's own work vectors (what
 *     one launch leaves in the L2 and last-level caches the next one finds);
 *   min_footprint > 0: the kernel's vector operands are replicated into as
 *     many operand sets as make up at least min_footprint bytes (at least
 *     two, at most 256), allocated for the call and freed before it returns, and
 *     consecutive launches take consecutive sets, so that with a footprint
 *     above the 256 MB last-level cache a launch finds none of its vectors
 *     in the caches; matrices, aggregates, metrics and partial sums are
 *     shared by the sets.  reps is raised to the number of sets if smaller.
 * Overwrites the context's work vectors (not the caller's).  Needs an AMG
 * context for kernels 0, 3, 4, 5, 7, 8.  The copy kernel's own buffers are
 * allocated on its first use and kept until ibpm_destroy.  Errors:
 * IBPM_EINVAL (unknown kernel, reps < 1, min_footprint < 0), IBPM_ENOMEM,
 * IBPM_EHIP. */
int ibpm_time_kernel(ibpm_ctx *ctx, int32_t kernel, int32_t reps, int64_t min_footprint,
                     double *avg_ms, double *bytes);

/* ------------------------------------------------------------------------
 * Learned preconditioner stage (an addition to the paper's method).
 * A network of six 3x3 convolutions on the cell grid (input 5 channels:
 * pressure residual, the two force residuals spread to cell centres with the
 * delta of Eq. 6, log of the two cell widths over the finest width; 32
 * hidden channels with ReLU; 3 output channels: pressure correction and two
 * force fields interpolated back to the points), no biases, zero padding,
 * BF16 operands and FP32 accumulation.  Its input is scaled by the RMS s of
 * the residual and its output by s / dt.  Solver IBPM_SOLVER_AMG_FCG_LEARNED
 * uses it in flexible CG: M(r) = z0 + w N(r - K z0) with z0 the AMG V-cycle
 * and w = (d . r1) / (d . K d), each new direction K-orthogonal to the
 * last fcg_depth ones; when the residual stalls (16 or more iterations
 * without falling 5 % -- fcg_stall_fall -- below its value at the last such
 * fall) or turns NaN
 * the solve falls back to plain AMG-PCG from the current iterate
 * (ibpm_solve_stats.fallbacks).
 * Weights are given per layer as [out][in][3][3] FP32, layers concatenated:
 * IBPM_NN_PARAMS values in all.  Images are ny x nx x channels (channel
 * fastest) FP32 device arrays.
 * ------------------------------------------------------------------------ */
#define IBPM_NN_PARAMS 39168

/* Allocate the network of this context and draw He-normal weights from a
 * seeded counter-based generator. */
int ibpm_nn_init(ibpm_ctx *ctx, uint64_t seed);
int ibpm_nn_get_weights(ibpm_ctx *ctx, float *host, int64_t n);
int ibpm_nn_set_weights(ibpm_ctx *ctx, const float *host, int64_t n);

/* One layer on the device, for checking the matrix-core kernels:
 *   mode 0: out = conv(x, W) (pre-activation, ny x nx x 32; x has 8
 *           channels for layer 0, 32 otherwise, BF16-representable values)
 *   mode 1: out = input gradient of conv for the output gradient dy masked
 *           by mask > 0 (mask optional, ny x nx x 32), ny x nx x 32
 *   mode 2: out = weight gradient for input x and output gradient dy (masked),
 *           the layer's [out][in][3][3] FP32 (device) */
int ibpm_nn_layer(ibpm_ctx *ctx, int32_t layer, int32_t mode, const float *x, const float *dy,
                  const float *mask, float *out);

/* e = learned correction for the residual r (lambda layout, FP64 device). */
int ibpm_nn_apply(ibpm_ctx *ctx, const double *r, double *e);

/* One pass of Adam (lr, betas 0.9/0.999) over the samples order[0..norder)
 * in batches: r1 and e1 hold nsamples (residual after the V-cycle, remaining
 * error, K e1 = r1) pairs in lambda layout, FP32 device.  The loss per sample
 * is the share of the energy-norm error that the optimally scaled correction
 * d = ibpm_nn_apply(r1) removes, -(d.r1)^2 / ((d.K d)(r1.e1)), in [-1, 0];
 * *mean_loss (host) receives the mean over the pass. */
int ibpm_nn_train(ibpm_ctx *ctx, const float *r1, const float *e1, int32_t nsamples,
                  const int32_t *order, int32_t norder, int32_t batch, float lr,
                  double *mean_loss);

/* One Adam step (Kingma & Ba; betas 0.9 / 0.999, eps 1e-8, bias-corrected
 * with the context's step count, which ibpm_nn_train advances too and
 * ibpm_nn_init / ibpm_nn_set_weights reset) on the FP32 master weights for
 * the gradient grad (host, IBPM_NN_PARAMS values in the layout of
 * ibpm_nn_get_weights) with learning rate lr > 0; the BF16 copies the
 * kernels use are refreshed.  Waits for the stream. */
int ibpm_nn_adam_step(ibpm_ctx *ctx, const float *grad, float lr);

/* Loss of one pair (r1, e1: FP32 device, lambda layout, as for training) in
 * *loss (host) and its gradient with respect to every weight in grad (host,
 * IBPM_NN_PARAMS values, layout of ibpm_nn_get_weights); no update. */
int ibpm_nn_loss_grad(ibpm_ctx *ctx, const float *r1, const float *e1, double *loss,
                      float *grad);

/* Training pairs from an AMG-PCG solve of K x = rhs started at x (device,
 * updated): before each of the first npairs iterations it stores
 * r1 = r - K V(r) and e1 = x* - x - V(r) (FP32, lambda layout, pair k at
 * offset k * n_lambda), x* being the converged solution given by the caller.
 * *nout (host) receives the number of pairs (fewer if the solve converged). */
int ibpm_harvest(ibpm_ctx *ctx, const double *rhs, double *x, const double *xstar,
                 int32_t npairs, float *r1_out, float *e1_out, int32_t *nout);

#ifdef __cplusplus
}
#endif

#endif /* IBPM_H */
