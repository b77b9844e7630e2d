/*
 * nhsem.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * element-based Galerkin nonhydrostatic model of Kang, Giraldo & Camp
 * (arXiv 2504.08157): the right-hand side of the perturbation-form Euler
 * equations on hexahedral LGL spectral elements, its direct stiffness
 * summation, and SSP-RK stage updates.
 *
 * Conventions (every entry point):
 *   - Return value: nh_status; NH_OK on success.  No exception crosses the
 *     ABI and the library never exits the process.  Arguments are validated
 *     before any device work; a failed HIP call makes the context sticky
 *     (NH_ESTATE for every later call); nh_last_error returns the text.
 *   - Memory: the library never allocates device memory.  The caller sizes a
 *     workspace with nh_workspace_bytes, allocates it (e.g. a torch uint8
 *     tensor) and passes its device address; every pointer is borrowed and
 *     must stay valid while the context uses it.
 *   - Streams: a context is bound to one HIP stream (hipStream_t passed as
 *     void*; NULL = default stream).  Calls enqueue asynchronously; only
 *     calls that return host data synchronise that stream.
 *   - Threading: a context is not thread-safe.
 *   - Layout: states and node fields are FP64, field-major [f][U] with fields
 *     (rho', u, v, w, theta') and unique node index
 *     I = ix + n_x (iy + n_y iz), x fastest.  Element-local vectors
 *     ("E-vectors") are [f][e][k][j][i] with e = ex + nel_x (ey + nel_y ez).
 *   - Mesh: an axis-aligned box of nel_x x nel_y x nel_z hexahedra with
 *     strictly increasing element edges (the paper's limited-area domain is
 *     such a box, Sec. 4.1).  x and y are periodic or no-flux walls; z is
 *     always no-flux at z = 0 and z = H.  Lattice sizes:
 *     n_x = nel_x N + (periodic_x ? 0 : 1), n_y likewise, n_z = nel_z N + 1.
 */
#ifndef NHSEM_H
#define NHSEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nh_status;
#define NH_OK 0
#define NH_EINVAL (-1)        /* invalid argument; nothing was enqueued */
#define NH_ESTATE (-2)        /* context is in a sticky error state */
#define NH_EHIP (-3)          /* a HIP runtime call failed */
#define NH_ENOCONV (-4)       /* an iterative solve did not converge */
#define NH_ENONFINITE (-5)    /* NaN or Inf found in the state */
#define NH_EUNSUPPORTED (-6)  /* valid request the library does not support */
#define NH_ESPACE (-7)        /* workspace too small */

#define NH_FP64 0             /* all element arithmetic in FP64 */
#define NH_FP32_MIXED 1       /* element contractions and fluxes in FP32; EOS,
                                 reference subtraction, DSS sums and RK
                                 accumulation in FP64; every array stays FP64 */

#define NH_DSS_SUM 0          /* out_I = sum_{(e,l)->I} in_(e,l) */
#define NH_DSS_MASS_AVG 1     /* out_I = sum w_i w_j w_k J^e in_(e,l) / M_I */

typedef struct nh_ctx nh_ctx;

typedef struct {
    int32_t nel[3];           /* elements per direction, >= 1 */
    int32_t order;            /* polynomial order N, 2..6 */
    const double *xe;         /* host, nel[0]+1 strictly increasing edges */
    const double *ye;         /* host, nel[1]+1 */
    const double *ze;         /* host, nel[2]+1 */
    int32_t periodic[2];      /* x, y: 1 periodic, 0 no-flux walls */
    int32_t precision;        /* NH_FP64 or NH_FP32_MIXED */
} nh_mesh_desc;

typedef struct {
    double g, R, cp, cv, p_a; /* gravity, gas constant, heat capacities,
                                 reference pressure of the EOS (Sec. 2.1) */
    double f;                 /* f-plane Coriolis parameter [1/s] */
    double sponge_z0;         /* Rayleigh sponge bottom [m] */
    double sponge_tau;        /* sponge maximum rate [1/s]; 0 disables.
                                 tau(z) = tau_max sin^2(pi/2 (z-z0)/(H-z0)),
                                 applied to u, v, w, theta' */
} nh_physics;

/* Library version string (static storage). */
const char *nh_version(void);

/* Bytes of device workspace a context for this mesh needs.
   NH_EINVAL for an invalid descriptor. */
nh_status nh_workspace_bytes(const nh_mesh_desc *mesh, size_t *bytes);

/* Create a context: LGL basis (Sec. 2.2), lattice numbering (the implicit
   form of Algorithm 1's intma for a tensor box), per-direction metric and
   DSS weights, diagonal mass (Eq. governing:matrix).  dev_ws: device
   workspace of at least nh_workspace_bytes (256-byte aligned).  The state
   starts at zero, the reference state is unset (nh_set_reference is
   required before nh_rhs / nh_rk_step).  On error *out is NULL. */
nh_status nh_init_mesh(const nh_mesh_desc *mesh, const nh_physics *phys, void *dev_ws,
                       size_t ws_bytes, void *hip_stream, nh_ctx **out);

/* Rebind the context to another HIP stream. */
nh_status nh_set_stream(nh_ctx *ctx, void *hip_stream);

/* Switch element arithmetic between NH_FP64 and NH_FP32_MIXED. */
nh_status nh_set_precision(nh_ctx *ctx, int32_t precision);

/* Workgroup tile of the stage kernel (columns per workgroup from
   nh_tile_shape): variant 0 (default) rows of ~32 lattice columns, a few
   element rows deep; variant 1 a squarer ~16 x 16 tile.  Variants 0 and 1
   compute every node with the same arithmetic in the same order, so results
   are bitwise identical.  Variant 2 (order 4 only; other orders run variant
   0) is variant 0's tile with the nodes assigned to threads by node class and
   the x/y derivatives written per element (a different order of the same
   sums: equal to variants 0 and 1 to rounding).  Chosen by the caller's tuner
   from measured times.  NH_EINVAL for any other value. */
nh_status nh_set_tile(nh_ctx *ctx, int32_t variant);

/* Columns per tile (tx x ty) of a variant for order N (no context needed). */
nh_status nh_tile_shape(int32_t order, int32_t variant, int32_t *tx, int32_t *ty);

/* Sizes: U unique nodes, L local nodes (E (N+1)^3), lattice n[3]. */
nh_status nh_sizes(const nh_ctx *ctx, int64_t *U, int64_t *L, int32_t n[3]);

/* Host copies of the lattice coordinates x[n_x], y[n_y], z[n_z]. */
nh_status nh_lattice_coords(const nh_ctx *ctx, double *x, double *y, double *z);

/* Reference state per lattice level (host arrays of n_z doubles):
   rho0(z), theta0(z) in hydrostatic balance (Sec. 2.1).  The library sets
   p0 = p_a (rho0 R theta0 / p_a)^gamma so that a resting reference has
   p' = 0 exactly, and the discrete vertical derivative of theta0. */
nh_status nh_set_reference(nh_ctx *ctx, const double *rho0_z, const double *theta0_z);

/* Prescribed forcing added to the tendency of one field: field 4 is the
   heating source S_theta of Eq. governing:theta (observed heating in the
   paper, Sec. 4.1; synthetic snapshots here); any field is accepted (e.g.
   manufactured solutions).  nsnap snapshots at host times t_snap (strictly
   increasing), device array dev_snap [nsnap][U] (BORROWED, not copied).  The
   value at time t is the linear interpolation between the bracketing
   snapshots, held constant outside [t_0, t_last].  nsnap = 0 removes it. */
nh_status nh_set_forcing(nh_ctx *ctx, int32_t field, int32_t nsnap, const double *t_snap,
                         const double *dev_snap);

/* Copy a device state [5][U] into / out of the context. */
nh_status nh_set_state(nh_ctx *ctx, const double *dev_q);
nh_status nh_get_state(const nh_ctx *ctx, double *dev_q);

/* Device pointer to the context's current state [5][U] (borrowed). */
nh_status nh_state_ptr(nh_ctx *ctx, double **dev_q);

/* dq/dt = M^{-1} DSS(w J S(q)) at time t (Eq. governing:matrix with S of
   Eq. governing, hyper-diffusion excluded), with the wall-normal velocity
   tendency zeroed on no-flux boundaries.  dev_q, dev_dqdt: device [5][U],
   must not overlap. */
nh_status nh_rhs(nh_ctx *ctx, double t, const double *dev_q, double *dev_dqdt);

/* Advance the context state nsteps SSP-RK3 steps of size dt from time t:
     q1 = q + dt R(q, t); q2 = 3/4 q + 1/4 (q1 + dt R(q1, t+dt));
     q  = 1/3 q + 2/3 (q2 + dt R(q2, t+dt/2)). */
nh_status nh_rk_step(nh_ctx *ctx, double t, double dt, int32_t nsteps);

/* Direct stiffness summation (Algorithm 3, gather): dev_E [nfields][L]
   element-local values -> dev_out [nfields][U] (mode NH_DSS_SUM or
   NH_DSS_MASS_AVG).  Contributions of a node are summed in ascending
   element order (deterministic, no atomics). */
nh_status nh_dss(nh_ctx *ctx, int32_t nfields, int32_t mode, const double *dev_E, double *dev_out);

/* Global-to-local scatter (Algorithm 1 gather, Algorithm 3 scatter):
   dev_E[f][e][k][j][i] = dev_U[f][intma(i,j,k,e)]. */
nh_status nh_scatter(nh_ctx *ctx, int32_t nfields, const double *dev_U, double *dev_E);

/* Diagonal mass M_I [U] into device memory. */
nh_status nh_mass(nh_ctx *ctx, double *dev_M);

/* Diagnostics of the current state (synchronises the stream), host out[8]:
   0 sum M rho', 1 max|u|, 2 max|v|, 3 max|w|, 4 min theta', 5 max theta',
   6 sum M theta', 7 number of non-finite values. */
nh_status nh_diagnostics(nh_ctx *ctx, double out[8]);

/* NH_ENONFINITE if the state holds a NaN or Inf (synchronises). */
nh_status nh_check_finite(nh_ctx *ctx);

/* ------------------------------------------------------------------
 * Tensor hyper-diffusion (section on tensor-based hyper-diffusion):
 * H_q = -(div tau grad)^2 q (order alpha = 2) on all five fields, with
 * tau = (J E) diag(nu_i lambda_i^-1) (J E)^T from the eigendecomposition of
 * the metric tensor G = J^-1 J^-T and nu_i = c_i^(1/2) dx_i^2 / dt^(1/2),
 * dx_i the element extent along principal axis i (repeated eigenvalues:
 * axes in x, y, z order).  The Laplacian is the continuous-Galerkin weak
 * form with the LGL quadrature, direct stiffness summation and the inverse
 * diagonal mass (no boundary term).  On the lattice's box elements it is
 * applied as one assembled (2N+1)-tap operator per direction.
 * ------------------------------------------------------------------ */

/* Device workspace nh_set_hyperdiffusion needs (a state-sized array and the
   operator rows). */
nh_status nh_hyperdiffusion_workspace_bytes(const nh_ctx *ctx, size_t *bytes);

/* Enable H_q with coefficients c[3] (dimensionless, >= 0, for the principal
   axes in ascending order of the metric eigenvalues, i.e. descending element
   extent) and time step dt: computes the operator rows into dev_ws (borrowed,
   256-byte aligned, at least nh_hyperdiffusion_workspace_bytes) and adds
   H_q(q^s) to the tendency in nh_rhs, nh_rk_step and the explicit part of
   nh_hevi_step, with its wall-normal velocity rows zeroed (u on x walls, v
   on y walls, w at the bottom and top: the no-flux walls are imposed on the
   whole tendency).  c == NULL disables it.  NH_EUNSUPPORTED if the order of the
   element extents (x, y, z) changes across the mesh; NH_EINVAL for c_i < 0
   or not finite, dt not finite and > 0, a null or misaligned workspace;
   NH_ESPACE for a small one.  The workspace must stay valid while the term
   is on. */
nh_status nh_set_hyperdiffusion(nh_ctx *ctx, const double *c, double dt, void *dev_ws, size_t bytes);

/* dev_H = H_q(dev_q) on device [5][U] arrays (distinct), the term as it
   enters the tendency: wall-normal velocity rows zero.  Needs
   nh_set_hyperdiffusion.  Asynchronous on the context's stream. */
nh_status nh_hyperdiffusion(nh_ctx *ctx, const double *dev_q, double *dev_H);

/* ------------------------------------------------------------------
 * RI-velocity diagnostic (section on the RI velocity): u_RI is the maximum
 * over radius and height of the azimuthal mean of the tangential speed
 * u_theta = |(I - e_r e_r^T - e_z e_z^T) u| about the centre of each level,
 * the centre being the speed-weighted mean position of the level (LGL
 * quadrature; a level at rest takes the domain midpoint), and the azimuthal
 * mean the arithmetic mean over the lattice nodes of an open annulus
 * j eps < r < (j+1) eps, eps = rmax / nstrips (the paper uses 50 strips).
 * Strip membership is decided in FP64 on squared radii (dx*dx + dy*dy
 * against (j*eps)*(j*eps), no fused multiply-add); nodes on a strip edge and
 * the centre itself belong to no strip.
 * ------------------------------------------------------------------ */

/* Device workspace nh_ri_velocity needs for nstrips strips (1..4096). */
nh_status nh_ri_workspace_bytes(const nh_ctx *ctx, int32_t nstrips, size_t *bytes);

/* Diagnostic of the device state dev_q [5][U], asynchronous on the
   context's stream.  Device outputs (caller-allocated):
     dev_center [2][n_z]  x_c then y_c per level; an input instead when
                          center_given != 0;
     dev_ubar [n_z][nstrips]   strip means of u_theta (0 for an empty strip);
     dev_count [n_z][nstrips]  nodes per strip;
     dev_result [4]  u_RI (the largest mean of a populated strip, the first in
                     (level, strip) order on ties), the radius of its strip
                     centre ((j + 1/2) eps), the height of its level (both -1
                     if no strip is populated), and the maximum horizontal
                     speed max sqrt(u^2 + v^2).
   dev_ws: borrowed, 256-byte aligned, nh_ri_workspace_bytes.  Strip sums
   are accumulated in an unordered way, so means may differ in the last bits
   between calls.  Errors: NH_EINVAL (nstrips outside 1..4096, rmax not
   finite and > 0, a null array, a misaligned workspace), NH_ESPACE (workspace
   too small); nothing is launched then. */
nh_status nh_ri_velocity(nh_ctx *ctx, const double *dev_q, int32_t nstrips, double rmax, int32_t center_given,
                         double *dev_center, double *dev_ubar, int32_t *dev_count, double *dev_result,
                         void *dev_ws, size_t bytes);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   diagnostic, arguments and outputs as nh_ri_velocity, with its partial sums
   in a fixed 8 MiB scratch array that the library holds in device memory,
   one copy per GPU, until the process ends (no workspace argument; no
   hipMalloc, hipFree or allocating library call).  The scratch address of
   the context's device is resolved in nh_init_mesh.  Every call on one GPU
   shares that GPU's scratch: calls that overlap on one GPU (other streams,
   other threads, other contexts on the same device) race and must be
   ordered by the caller.  NH_ESPACE, with nothing launched, when the
   partial sums would exceed the scratch (n_z * nb * (32 + 12 nstrips) bytes
   in 256-byte aligned blocks, nb = ceil(n_x n_y / 4096) chunks per level, at
   most 256: on a 512 x 512 x 81 lattice up to about 130 strips); other
   errors as nh_ri_velocity. */
nh_status nh_ri_velocity_noalloc(nh_ctx *ctx, const double *dev_q, int32_t nstrips, double rmax,
                                 int32_t center_given, double *dev_center, double *dev_ubar, int32_t *dev_count,
                                 double *dev_result);

/* ------------------------------------------------------------------
 * 1D-IMEX (HEVI) step (Sec. 2.3: IMEX split S = (S - L) + L with the fast
 * waves implicit, ARK2 "ARK(2,3,2)b", matrix-free GMRES).  Here L = L_v, the
 * linearisation of S about the resting reference restricted to vertical
 * derivatives; every lattice column is an independent implicit system in
 * (rho', w, theta').
 * ------------------------------------------------------------------ */
typedef struct nh_mlp nh_mlp;
typedef struct {
    int32_t restart;          /* Krylov vectors per cycle, 1..40 (paper: < 20) */
    int32_t max_restarts;     /* restarts before NH_ENOCONV */
    double rtol;              /* stop when ||b - A x||_2 <= rtol ||b||_2 */
    int32_t schur;            /* 0: GMRES on the column system in (rho', w, theta');
                                 1: GMRES on its Schur complement in the interior w
                                 values (rho', theta' eliminated per column, then
                                 reconstructed); same stopping test on the full
                                 system; restart 10 and n_z <= 130 only
                                 (NH_EUNSUPPORTED otherwise) */
    int32_t precondition;     /* global (3D-IMEX) solves only, ignored by the
                                 column solves: 1 = right-precondition with the
                                 column systems (I - alpha L_v), solved by the
                                 column GMRES(10) to rtol 1e-6 (flexible GMRES:
                                 the preconditioned vectors are kept) */
    int32_t guess_pick;       /* column solves started from a given guess (dev_x0,
                                 or the MLP guess of nh_hevi_step), restart 10 forms:
                                 1 = per column, compare the residual of the guess
                                 with that of the default start x0 = b and start
                                 from the smaller (one more operator application
                                 per column, not counted as an Arnoldi step) */
} nh_gmres_opts;
typedef struct {
    int64_t columns;          /* columns per solve */
    int64_t solves;           /* solves of the call, each over `columns` columns */
    int64_t iters_total;      /* Arnoldi steps summed over all column solves */
    int64_t iters_max;        /* most Arnoldi steps of one column solve */
    int64_t not_converged;    /* column solves that missed rtol */
} nh_solve_stats;

/* Device workspace the HEVI calls need (8 state-sized arrays + counters). */
nh_status nh_hevi_workspace_bytes(const nh_ctx *ctx, size_t *bytes);

/* Attach that workspace (borrowed, 256-byte aligned). */
nh_status nh_hevi_attach(nh_ctx *ctx, void *dev_ws, size_t bytes);

/* y = L_v x on device [5][U] arrays (u, v rows of y are zero; w rows zero at
   z = 0 and z = H). */
nh_status nh_lv_apply(nh_ctx *ctx, const double *dev_x, double *dev_y);

/* Solve (I - alpha L_v) x = b in every column by restarted matrix-free
   GMRES (one wavefront per column; with restart 10 and 3 n_z <= 256 the
   Krylov basis is held in registers, otherwise in LDS).  dev_b, dev_x:
   [5][U]; the u, v fields of x are copied from b.  dev_x0: initial guess of
   (rho', w, theta') as [3][U], or NULL for x0 = b.  dev_iters: optional
   device int32 [n_x n_y] receiving the Arnoldi steps per column (negative:
   -steps-1 when the column did not converge).  stats (host, optional)
   synchronises the stream.  NH_ENOCONV if any column missed rtol. */
nh_status nh_column_solve(nh_ctx *ctx, double alpha, const double *dev_b, const double *dev_x0,
                          double *dev_x, const nh_gmres_opts *opts, nh_solve_stats *stats,
                          int32_t *dev_iters);

/* One HEVI ARK2 step of the context state from t to t + dt: stages
   (I - dt At_ii L_v) Q_i = q^n + dt sum_{j<i} [A_ij (S - L_v)(Q_j) + At_ij L_v(Q_j)],
   q^{n+1} = q^n + dt sum_j b_j S(Q_j).  guess: a trained column MLP giving
   the initial GMRES guess, or NULL (x0 = right-hand side).  The Krylov solve
   always runs to opts->rtol.  stats (optional, host) synchronises. */
nh_status nh_hevi_step(nh_ctx *ctx, double t, double dt, const nh_gmres_opts *opts, nh_mlp *guess,
                       nh_solve_stats *stats);

/* Device pointers (into the HEVI workspace, valid until the next HEVI call)
   to the right-hand sides and solutions of the two implicit stages of the
   last nh_hevi_step, [5][U] each; *alpha_per_dt = At_22 = At_33, so the
   solves used alpha = dt * (*alpha_per_dt).  For collecting training data. */
nh_status nh_hevi_last_solves(nh_ctx *ctx, const double **R2, const double **X2, const double **R3,
                              const double **X3, double *alpha_per_dt, double *reserved);

/* ------------------------------------------------------------------
 * 3D-IMEX step (Sec. 2.3 with the linear operator over all directions):
 * L is the linearisation of S about the resting reference in x, y and z
 * (acoustic and gravity terms, p'_L = gamma p0 (rho'/rho0 + theta'/theta0)),
 *   L_rho' = -d/dx(rho0 u) - d/dy(rho0 v) - d/dz(rho0 w),
 *   L_u = -(1/rho0) dp'_L/dx,  L_v = -(1/rho0) dp'_L/dy,
 *   L_w = -(1/rho0) dp'_L/dz - g rho'/rho0 - tau(z) w,
 *   L_theta' = -w dtheta0/dz,
 * discretised like S (DSS'd derivative stencils, the walls of S); the
 * damping of w in the absorbing layer is implicit, that of u, v and theta'
 * stays in the explicit part.  Each implicit stage solves one global system
 * (I - dt At_ii L) Q = R in 5U unknowns by restarted matrix-free GMRES
 * (classical Gram-Schmidt with a second pass when needed, fixed-order
 * device reductions).  nh_gmres_opts: restart 1..32, schur must be 0
 * (NH_EUNSUPPORTED), stop when ||R - A Q||_2 <= rtol ||R||_2 (global).
 * ------------------------------------------------------------------ */

/* Device workspace of nh_global_solve and nh_imex3d_step for a restart
   length (restart + 1 Krylov vectors, restart preconditioned vectors, one
   scratch vector and, for the step, eight state-sized arrays, 5U doubles
   each; plus the block partial sums and the solver's device state). */
nh_status nh_imex3d_workspace_bytes(const nh_ctx *ctx, int32_t restart, size_t *bytes);

/* dev_y = L dev_x on device [5][U] arrays (distinct; NH_EINVAL otherwise or
   without a reference state). */
nh_status nh_l3_apply(nh_ctx *ctx, const double *dev_x, double *dev_y);

/* Solve (I - alpha L) dev_x = dev_b (alpha >= 0) from dev_x0 (NULL: dev_b);
   dev_b and dev_x distinct.  The Hessenberg problem and the convergence
   test run on the device; the host queues each Arnoldi step while the one
   before runs, waits on an event of the stream every step and synchronises
   the stream once per solve (the call returns with the solve complete).  The
   first 3D-IMEX call on a context creates a small host-mapped status block
   and two events, released by nh_destroy.  stats (optional):
   columns = 1, solves = 1, iters = Arnoldi steps.  NH_ENOCONV when the
   residual test fails after max_restarts restarts (dev_x holds the last
   iterate); NH_EINVAL for bad options (restart outside 1..32, rtol outside
   (0, 1), negative max_restarts or alpha, aliased arrays), NH_EUNSUPPORTED
   for schur != 0 or a column preconditioner on n_z > 130, NH_ESPACE for a
   small workspace. */
nh_status nh_global_solve(nh_ctx *ctx, double alpha, const double *dev_b, const double *dev_x0, double *dev_x,
                          const nh_gmres_opts *opts, void *dev_ws, size_t bytes, nh_solve_stats *stats);

/* One 3D-IMEX ARK2 step of the context state from t to t + dt: the same
   tableau and stage structure as nh_hevi_step with L in place of L_v (two
   global solves per step).  stats as for nh_global_solve, summed over the
   two solves; NH_ENOCONV if either missed rtol (the step is completed). */
nh_status nh_imex3d_step(nh_ctx *ctx, double t, double dt, const nh_gmres_opts *opts, void *dev_ws, size_t bytes,
                         nh_solve_stats *stats);

/* ------------------------------------------------------------------
 * Batched instances: many contexts (uneven meshes, orders 2..6, one
 * precision) advanced by SSP-RK3 together.  Per stage, one grouped launch
 * per order covers every instance of that order, its workgroups taking
 * (instance, tile) items sorted longest-column-first; K steps of launches are
 * captured once into a hipGraph and replayed (the per-stage descriptors of
 * the next K steps are uploaded with one copy before each replay).  Each
 * instance computes bitwise the same as nh_rk_step on its own.
 * Restrictions: reference set on every context, forcing only on theta',
 * hyper-diffusion off (NH_EUNSUPPORTED at create and step otherwise).
 * The batch owns no context; contexts must outlive it.
 * ------------------------------------------------------------------ */
typedef struct nh_batch nh_batch;
nh_status nh_batch_workspace_bytes(nh_ctx *const *ctxs, int32_t n, int32_t steps_per_graph, size_t *bytes);

/* tile_variant: optional [7] array indexed by order (tuner's choice per
   order), kept by the batch (the contexts' own tile settings are neither
   used nor changed); hip_stream must be a non-default stream (graph
   capture). */
nh_status nh_batch_create(nh_ctx *const *ctxs, int32_t n, int32_t steps_per_graph, const int32_t *tile_variant,
                          void *dev_ws, size_t bytes, void *hip_stream, nh_batch **out);

/* Launch form of the next graph capture (the current graph, if any, is
   dropped).  persistent = 1: per (order group, stage) one launch of at most
   one workgroup per compute unit, whose workgroups take (instance, tile)
   items from the cost-sorted list through a device counter in the batch
   workspace, zeroed by a fill kernel at the start of each graph replay
   (persistent = 0: one workgroup per item).  concurrent_groups = 1: each
   order group's chain of stage launches is captured on a stream of its own
   (forked from and joined back to the batch stream), so the groups'
   launches may overlap; otherwise they run in step, stage, group order.
   Results do not depend on the form.  Default 0, 0.  NH_EINVAL for flags
   other than 0 or 1. */
nh_status nh_batch_set_mode(nh_batch *b, int32_t persistent, int32_t concurrent_groups);

/* Advance every instance nsteps (a multiple of steps_per_graph) from t.
   Re-checks every context first: NH_EUNSUPPORTED if one has since turned on
   hyper-diffusion or forcing of fields 0..3, NH_EINVAL if its precision
   changed, NH_ESTATE if it is in an error state; nothing is launched then. */
nh_status nh_batch_step(nh_batch *b, double t, double dt, int32_t nsteps);
nh_status nh_batch_last_error(const nh_batch *b, char *buf, size_t n);
nh_status nh_batch_destroy(nh_batch *b);

/* ------------------------------------------------------------------
 * Column MLP for the initial guess of the HEVI column solves (trained on
 * solves the method itself produces; the Krylov solve still runs to the
 * same tolerance).  Network 208 -> 256 -> 256 -> 256 with SiLU and a
 * linear bypass, y = W3 h2 + b3 + S x; FP16 weights and activations on MFMA
 * with FP32 accumulation in the forward pass, FP32 backward, Adam on FP32
 * master weights.  Parameters, in order: W1 [256][208], b1 [256],
 * W2 [256][256], b2 [256], W3 [256][256], b3 [256], S [256][208].
 * Inputs x: FP16 [batch][208] (features of nh_mlp_samples); outputs y: FP32
 * [batch][256] (the first 3 x 65 are used).  batch: multiple of 64, at most the capacity given at
 * creation.
 * ------------------------------------------------------------------ */
nh_status nh_mlp_workspace_bytes(int64_t max_batch, size_t *bytes);

/* Create with Glorot-uniform weights from `seed` (last layer zero, so the
   untrained guess equals the default guess). */
nh_status nh_mlp_create(int64_t max_batch, uint64_t seed, void *dev_ws, size_t bytes, void *hip_stream,
                        nh_mlp **out);

/* Forward pass; keeps the activations for nh_mlp_backward.  dev_y may be
   NULL. */
nh_status nh_mlp_forward(nh_mlp *m, int64_t batch, const void *dev_x_f16, float *dev_y);

/* Gradients of sum(y * dy) with respect to every parameter for the last
   forward pass (FP32, overwritten). */
nh_status nh_mlp_backward(nh_mlp *m, int64_t batch, const void *dev_x_f16, const float *dev_dy);

/* forward, mean-squared-error loss against dev_t [batch][256], backward,
   Adam (Kingma & Ba, bias-corrected).  dev_loss (device float, optional). */
nh_status nh_mlp_train_step(nh_mlp *m, int64_t batch, const void *dev_x_f16, const float *dev_t, float lr,
                            float b1, float b2, float eps, float *dev_loss);

/* One Adam step (Kingma & Ba, bias-corrected with the step count kept since
   creation or nh_mlp_set_params) on the FP32 masters with the gradients of
   the last nh_mlp_backward, then the FP16 copies refreshed: the update that
   nh_mlp_train_step applies.  NH_EINVAL for lr <= 0, b1 or b2 outside
   [0, 1), eps <= 0. */
nh_status nh_mlp_adam_step(nh_mlp *m, float lr, float b1, float b2, float eps);

/* Copy FP32 master parameters and/or gradients to device arrays; *n = count. */
nh_status nh_mlp_params(nh_mlp *m, float *dev_master, float *dev_grad, int64_t *n);

/* Replace the FP32 master parameters (FP16 copies refreshed, Adam reset). */
nh_status nh_mlp_set_params(nh_mlp *m, const float *dev_master);

/* Training samples / features for columns [col0, col0 + ncol) of ctx: the
   right-hand side b of (I - alpha L_v) x = b and, if dev_x is given, the
   solution x.  Without dev_x0 the samples are those of the default start
   b: features of its residual alpha L_v b, targets x - b; with dev_x0
   (device [3][U], rho', w, theta': a guess, e.g. the network's first pass)
   those of the start x0: features of its residual b - (I - alpha L_v) x0,
   targets x - x0 (the samples of a refinement pass).  dev_feat FP16
   [ncol][208], dev_scale double [ncol] (the column scale: RMS of the
   dimensionless residual), dev_tgt float [ncol][256] (the scaled
   dimensionless correction on the 65 canonical levels per field, zero
   past 195; needs dev_x), dev_tmp device [5][U] scratch. */
nh_status nh_mlp_samples(nh_mlp *m, nh_ctx *ctx, double alpha, const double *dev_b, const double *dev_x,
                         int64_t col0, int64_t ncol, void *dev_feat, double *dev_scale, float *dev_tgt,
                         double *dev_tmp, const double *dev_x0);

/* Decoupled weight decay (Loshchilov & Hutter, AdamW) applied by every
   later Adam step (nh_mlp_adam_step, nh_mlp_train_step) to the hidden
   path's parameters W1, b1, W2, b2, W3, b3 -- not to the bypass S:
   w -= lr (m_hat / (sqrt(v_hat) + eps) + wd w).  Default 0 (plain Adam).
   NH_EINVAL for wd < 0 or non-finite. */
nh_status nh_mlp_set_decay(nh_mlp *m, float wd);

/* Network applications per initial guess (default 1): pass 1 predicts the
   correction of the default start b from its residual alpha L_v b; each
   further pass applies the same network to the residual
   r = b - (I - alpha L_v) x0 of the guess so far (whose exact correction
   (I - alpha L_v)^-1 r is the same linear map) and adds its prediction.
   Used by nh_mlp_guess and by nh_hevi_step with this network.  NH_EINVAL
   for passes outside 1 .. 4. */
nh_status nh_mlp_set_passes(nh_mlp *m, int32_t passes);

/* The initial guess x0 of (I - alpha L_v) x = b in every column of ctx, as
   used by nh_hevi_step: features of the default start's residual
   alpha L_v b (dimensionless, divided by its column RMS s), the network,
   and x0 = b + D s (output resampled to the lattice levels), the w correction
   zero on the walls and a non-finite prediction replaced by x0 = b; then
   the refinement passes set by nh_mlp_set_passes (alpha > 0 only).
   dev_b device [5][U] (fields rho', w, theta' are used), dev_tmp device
   [5][U] scratch (receives L_v b, or the residual of the last refinement
   pass, in fields 0, 3, 4), dev_x0 device [3][U]
   (rho', w, theta').  Asynchronous on the context's stream.  NH_EINVAL for
   null arguments, alpha < 0 or non-finite, or a context without reference
   state. */
nh_status nh_mlp_guess(nh_mlp *m, nh_ctx *ctx, double alpha, const double *dev_b, double *dev_tmp,
                       double *dev_x0);
nh_status nh_mlp_last_error(const nh_mlp *m, char *buf, size_t n);
nh_status nh_mlp_destroy(nh_mlp *m);

/* Text of the last error (always NUL-terminated when n > 0). */
nh_status nh_last_error(const nh_ctx *ctx, char *buf, size_t n);

/* Destroy the context (host memory, and the 3D-IMEX status block and events
   if a global solve made them; the workspace stays the caller's). */
nh_status nh_destroy(nh_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* NHSEM_H */
