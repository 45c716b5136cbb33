/*
 * ibm.h -- C ABI of the MI355X (gfx950) solver for the discrete-forcing
 * immersed-boundary, fractional-step incompressible Navier-Stokes method of
 * Sundar, Majumdar, Shah & Sarkar (arXiv 2402.17337).
 *
 * The method (paper Sec. 2.1-2.3, Eqs. 1-4): a rigid ellipse (thickness /
 * chord 0.12) plunging as y = h sin(k t) in a uniform stream, on a Cartesian
 * staggered grid that is uniform around the body and stretched outward.  Each
 * time step classifies mesh points as fluid or solid, forms the momentum
 * predictor (Adams-Bashforth convection, Crank-Nicolson diffusion), applies
 * the immersed-boundary forcing f at the solid points, solves the implicit
 * velocity equations and the pressure-correction Poisson equation with
 * red-black Gauss-Seidel SOR, and projects.
 *
 * Discrete reading used here (the paper prints no formulas):
 *   - faces xf[0..nx], yf[0..ny]; p at cell centres (nx*ny), u at x-faces
 *     ((nx+1)*ny), v at y-faces (nx*(ny+1)); every array row-major, x fastest;
 *   - channel boundaries: inflow u = u_inf and v = 0 on the x = xf[0] face,
 *     slip walls at y = yf[0], yf[ny], convective outflow for u and zero
 *     gradient for v at x = xf[nx]; the pressure correction phi is Neumann
 *     except phi = 0 on the outlet face;
 *   - incremental pressure: A phi = V (D(u^) - q)/dt with A = V D G,
 *     u^{n+1} = u^ - dt G phi, p^{n+1} = p^n + phi - dt/(2 Re) L phi;
 *   - forced nodes are those strictly inside the ellipse; those with an
 *     outside 4-neighbour take a target by linear extrapolation through the
 *     boundary crossing on each grid line (weight d_f/d_o capped at
 *     alpha_max), the others the body velocity; f = (target - u~)/dt;
 *   - mass source q (Eq. 4): divergence of (u^ - body velocity) over a cell's
 *     forced faces, so the Poisson source sees forced faces moving with the
 *     body;
 *   - forces F = -sum f dV + pi a b (0, a_body); C = 2 F / (u_inf^2 chord).
 *
 * Conventions for every entry point:
 *   - return IBM_OK (0) on success, a positive soft status or a negative
 *     error code; ibm_last_error() gives a message for the context;
 *   - "host" pointers are ordinary CPU memory and are copied; "device"
 *     pointers are HIP device memory on the context's device, borrowed for the
 *     duration of the call only;
 *   - all GPU work is enqueued on the HIP stream given to ibm_init and is
 *     ordered with the caller's other work on that stream;
 *   - a context is not thread-safe; distinct contexts are independent.
 */
#ifndef IBM_H
#define IBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IBM_OK 0
#define IBM_NOT_CONVERGED 1 /* soft: an iterative solve stopped at its iteration limit */
#define IBM_ERR_INVALID (-1) /* invalid argument; nothing was enqueued */
#define IBM_ERR_HIP (-2)     /* a HIP runtime call failed */
#define IBM_ERR_STATE (-3)   /* context in a state that forbids the call */
#define IBM_ERR_NAN (-5)     /* a residual became NaN or Inf; the state is not usable */

/* boundary conditions */
#define IBM_BC_CHANNEL 0
/* Periodic in x and y (the Taylor-Green vortex test of the time integrator;
 * not a configuration of the paper): no body, the two ends of each direction
 * are neighbours (centre distance (dx[0] + dx[nx-1]) / 2), u face nx and v
 * face row ny mirror face 0 and row 0.  The pressure operator is singular:
 * every Poisson solve uses the zero-sum part of V b and returns the solution
 * of zero volume-weighted mean.  Red-black SOR runs colour by colour (the
 * blocked sweeps are for the channel), or PCG; no mixed-precision sweeps, no
 * learned guess, no batch. */
#define IBM_BC_PERIODIC 1

/* pressure solvers */
#define IBM_SOLVER_RBSOR 0 /* red-black SOR, red = (i+j) even updated first */
#define IBM_SOLVER_PCG 1   /* conjugate gradients on -A, Jacobi preconditioner */
/* Red-black SOR with single-precision sweeps and double-precision refinement:
 * each check interval solves the correction equation A e = r (r the double
 * residual, rounded to float) by float SOR sweeps from e = 0, then phi += e
 * and the residual and stop test are evaluated in double.  Same omega, stop
 * test and check interval as IBM_SOLVER_RBSOR; it uses the blocked sweep's
 * tile shape (IBM_OPT_TB_*). */
#define IBM_SOLVER_RBSOR_MP 2
/* Jacobi-PCG in the one-reduction form (Chronopoulos and Gear, 1989): the
 * search direction's product s = M p is carried by its own recurrence, so
 * both inner products of an iteration come from one reduction and an
 * iteration is one kernel.  The same iterates as IBM_SOLVER_PCG in exact
 * arithmetic (not bitwise); the same stop test and confirmation. */
#define IBM_SOLVER_CG1 3

/* initial guess of the pressure correction at each step */
#define IBM_INIT_ZERO 0
#define IBM_INIT_PREVIOUS 1
/* Learned warm start (an extension; the paper starts from the previous
 * solution): phi^n plus the prediction of the network attached with
 * ibm_set_warm_start.  The solve still runs to p_tol, so the guess changes
 * the iteration count, never the stop test. */
#define IBM_INIT_LEARNED 2

/* arithmetic of the sweeps */
#define IBM_PREC_FP64 0

/* Problem and solver parameters.  Lengths in chords, velocities in u_inf. */
typedef struct ibm_params {
    int32_t nx, ny;          /* cells in x and y; both even and >= 8 */
    int32_t bc_mode;         /* IBM_BC_CHANNEL or IBM_BC_PERIODIC */
    int32_t body;            /* 1: ellipse present; 0: no body */
    double re;               /* Reynolds number u_inf c / nu, > 0 */
    double dt;               /* time step, > 0 */
    double u_inf;            /* free-stream (inflow) velocity */
    double chord;            /* ellipse major axis (= 2a) */
    double thickness;        /* thickness / chord (minor axis = thickness * chord) */
    double x0, y0;           /* centre of the ellipse at rest position */
    double amp, freq, phase; /* plunge y_c = y0 + amp sin(2 pi freq t + phase) (Eqs. 1-2, k = 2 pi freq) */
    int32_t p_method;        /* IBM_SOLVER_RBSOR, IBM_SOLVER_PCG, IBM_SOLVER_RBSOR_MP or IBM_SOLVER_CG1 */
    int32_t p_max_iter;      /* iteration limit of one pressure solve, >= 1 */
    int32_t p_check_every;   /* SOR: residual tested every this many iterations, >= 1 */
    int32_t p_init;          /* IBM_INIT_ZERO, IBM_INIT_PREVIOUS or IBM_INIT_LEARNED */
    double p_omega;          /* SOR relaxation factor, 0 < omega < 2 */
    double p_tol;            /* stop when ||V b - A phi||_2 <= p_tol ||V b||_2 */
    double uv_omega;         /* relaxation factor of the implicit velocity solves */
    double uv_tol;           /* their relative residual tolerance (tested every iteration) */
    int32_t uv_max_iter;     /* their iteration limit, >= 1 */
    int32_t q_mode;          /* 1: mass source in cells with forced faces; 0: q = 0 */
    double alpha_max;        /* cap of the extrapolation weight d_f/d_o, >= 0 */
    int32_t precision;       /* IBM_PREC_FP64 */
    int32_t reserved;        /* must be 0 */
} ibm_params;

/* Statistics of the last step of an ibm_step call. */
typedef struct ibm_step_stats {
    int32_t status;                   /* worst status of the step */
    int32_t p_iters;                  /* pressure iterations */
    int32_t u_iters, v_iters;         /* implicit velocity iterations */
    int32_t n_forced_u, n_forced_v;   /* forced u and v nodes */
    int32_t n_msrc;                   /* cells with a forced face */
    int32_t n_net;                    /* network guesses and corrections applied */
    double p_r0;                      /* initial residual / ||V b|| of the pressure solve */
    double p_rel;                     /* final residual / ||V b|| */
    double cd, cl;                    /* drag and lift coefficients */
    double t;                         /* time reached */
    double seconds;                   /* host wall time of the whole ibm_step call */
    double net_step;                  /* mean step a of those (see ibm_set_warm_start) */
} ibm_step_stats;

/* Options of a stand-alone Poisson solve. */
typedef struct ibm_solve_opts {
    int32_t method;       /* IBM_SOLVER_RBSOR, IBM_SOLVER_PCG, IBM_SOLVER_RBSOR_MP or IBM_SOLVER_CG1 */
    int32_t max_iter;     /* iteration limit, >= 1 */
    int32_t check_every;  /* SOR residual test interval, >= 1 (PCG tests every iteration) */
    int32_t fixed_iters;  /* > 0: run exactly this many iterations, tol ignored */
    double omega;         /* SOR relaxation factor */
    double tol;           /* relative residual tolerance */
} ibm_solve_opts;

typedef struct ibm_solve_stats {
    int32_t status;       /* IBM_OK, IBM_NOT_CONVERGED or IBM_ERR_NAN */
    int32_t iters;        /* iterations performed */
    int32_t reserved0, reserved1;
    double r0_rel;        /* initial residual / ||V b|| */
    double rel;           /* final residual / ||V b|| */
    double seconds;       /* GPU time of the solve (HIP events on the context stream) */
} ibm_solve_stats;

typedef struct ibm_ctx ibm_ctx;

/* Device workspace a context needs for prm, in bytes (0 if prm is invalid).
 * Paper: the fields and solver arrays of the staggered-grid method of
 * Sec. 2.2 on the grid of Sec. 2.3, held resident on the device (Sec. 3.4.4,
 * data management).  Pure function; no GPU call. */
size_t ibm_workspace_bytes(const ibm_params* prm);

/* Create a context.
 * Paper: the problem of Sec. 2.1 (rigid ellipse, thickness/chord 0.12,
 * plunge y = h sin(k t), Eqs. 1-2) in the domain of Sec. 2.3 (Cartesian grid
 * uniform around the body, stretched outward; channel boundary conditions),
 * with the flow parameters of Sec. 4.1 (Re, plunge amplitude and frequency).
 *   xf[nx+1], yf[ny+1]     host; strictly increasing face coordinates;
 *   u0[(nx+1)*ny], v0[nx*(ny+1)], p0[nx*ny]
 *                          host initial fields, or NULL for u = u_inf, v = 0,
 *                          p = 0; the inflow u and wall v are always reset to
 *                          their boundary values;
 *   workspace              device memory of at least ibm_workspace_bytes(prm)
 *                          bytes, 256-byte aligned, owned by the caller, which
 *                          must keep it alive until ibm_destroy; the library
 *                          never frees it;
 *   hip_stream             hipStream_t (NULL = the null stream), borrowed.
 * Errors: IBM_ERR_INVALID for odd or too small nx/ny, non-increasing faces,
 * dt <= 0, re <= 0, omega outside (0, 2), a body whose range of motion comes
 * within two cells of the boundary, an unknown bc_mode, IBM_BC_PERIODIC with
 * a body, IBM_SOLVER_RBSOR_MP or IBM_INIT_LEARNED, an unsupported precision, a
 * small or misaligned workspace; IBM_ERR_HIP if the device rejects the setup.
 * Validation happens before any GPU call. */
int32_t ibm_init(const ibm_params* prm, const double* xf, const double* yf, const double* u0,
                 const double* v0, const double* p0, void* workspace, size_t workspace_bytes,
                 void* hip_stream, ibm_ctx** out);

/* Advance nsteps (>= 1) time steps.
 * Paper: one time-marching step of Sec. 2.2 (Eqs. 3-4: momentum forcing f and
 * mass source q; semi-implicit fractional step with Adams-Bashforth and
 * Crank-Nicolson terms; fluid/solid flagging at the start of every step;
 * red-black SOR for the velocity and pressure equations), whose four hot
 * spots are those of Table 1 (Sec. 3.4.1).  Each step: classification at
 * t^{n+1}, momentum predictor, forcing, implicit velocity solves, pressure
 * Poisson solve (p_method, from zero or the previous phi), projection,
 * pressure update, forces.  Returns the worst status; IBM_NOT_CONVERGED is
 * soft (the step completed at the iteration limit), IBM_ERR_NAN stops the
 * call.  last (nullable) receives the statistics of the last step. */
int32_t ibm_step(ibm_ctx* ctx, int32_t nsteps, ibm_step_stats* last);

/* Solve the cell-centred Poisson problem (D G) x = rhs on the context's grid
 * and boundary conditions (the pressure-correction operator A / V).
 * Paper: the pressure-correction equation of the fractional step (Sec. 2.2)
 * and its red-black SOR solver (Sec. 2.2, Sec. 3.1), the "P iterative
 * solver" of Table 1 (54.7 % of the serial step).
 *   rhs_dev[nx*ny]  device, per unit volume, natural layout; read only;
 *   x_dev[nx*ny]    device; initial guess on entry, solution on exit.
 * Stream-ordered; returns after the solve has finished.  rhs = 0 gives
 * x = 0 with 0 iterations.  Does not touch the time-stepping state. */
int32_t ibm_poisson_solve(ibm_ctx* ctx, const double* rhs_dev, double* x_dev, const ibm_solve_opts* opts,
                          ibm_solve_stats* stats);

/* Allocation-free variant of ibm_poisson_solve, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, iterates, stop test,
 * statistics and results as ibm_poisson_solve with opts->method =
 * IBM_SOLVER_RBSOR (bit for bit: the same kernels in the same launch shape),
 * but the solve's working arrays (the red/black split copies of x and of
 * V rhs, the residual partials and the control block) live in a static array
 * of the library's own device memory instead of the context's workspace:
 * 6 * 393216 + 33792 doubles plus 256 bytes (about 19.2 MB), one copy per
 * device, held until the process ends, its address resolved by ibm_init.
 * The call allocates no device memory and creates no events (kernel timing
 * with ibm_profile is suspended for its duration).  Limits: nx * ny <=
 * 1024 * 768 cells and at most 8192 tiles of the blocked sweep
 * (IBM_OPT_TB_TILE_X / _Y); IBM_ERR_INVALID beyond them, for another method
 * or invalid options, with nothing enqueued; IBM_ERR_HIP if the runtime could
 * not resolve the array on this device.  Every call on a device shares that
 * device's array and leaves its contents behind (each call rewrites what it
 * reads before reading it): calls that overlap on one device, from two
 * contexts or two threads, race and give wrong results. */
int32_t ibm_poisson_solve_noalloc(ibm_ctx* ctx, const double* rhs_dev, double* x_dev, const ibm_solve_opts* opts,
                                  ibm_solve_stats* stats);

/* Drag and lift coefficients of the last completed step (0 before the
 * first).  Paper: the aerodynamic force coefficients of Sec. 4.1 (Fig. 4);
 * the force is the reaction of the forcing f of Eq. 3 plus the inertia of the
 * fluid inside the rigid body.  Synchronizes the context stream. */
int32_t ibm_forces(ibm_ctx* ctx, double* cd, double* cl);

/* Host copies of the current fields; each pointer is nullable.
 * Paper: the velocity and pressure of Eqs. 3-4 on the staggered grid of
 * Sec. 2.2.
 * u[(nx+1)*ny], v[nx*(ny+1)], p[nx*ny], phi[nx*ny].  Synchronizes. */
int32_t ibm_get_fields(ibm_ctx* ctx, double* u, double* v, double* p, double* phi);

/* The right-hand side V b of the pressure-correction equation A phi = V b
 * that the last time step solved.  Paper: the pressure correction of the
 * fractional-step method (Sec. 2.2) with the mass source q of Eq. 4:
 * V b = V (D(u^) - q) / dt, V the cell area; in the periodic mode after its
 * zero-mean projection.  vb[nx*ny] (natural layout, row j at j*nx), host or
 * device memory; the copy runs on the context stream and the call returns
 * when it is done.  To solve the same system with ibm_poisson_solve, divide by
 * the cell areas (that call takes b per unit area).  IBM_ERR_INVALID (message
 * in ibm_last_error) when no step's right-hand side is held: before the first
 * step, and after a stand-alone solve (ibm_poisson_solve or its noalloc form,
 * which use the same storage) or ibm_set_state, until the next step. */
int32_t ibm_get_poisson_rhs(ibm_ctx* ctx, double* vb);

/* Immersed-boundary data of the last step (each pointer nullable).
 * Paper: the solid/fluid flags of Sec. 2.2 (Table 1, "fluid/solid
 * flagging"), the cells of the mass source q (Eq. 4) and the forcing f
 * (Eq. 3; Table 1, "body force interpolation"):
 * flu[(nx+1)*ny], flv[nx*(ny+1)] (0 fluid, 1 forcing, 2 deep),
 * msrc[nx*ny] (1 = cell with a forced face), fu, fv (forcing f, full-size
 * arrays, zero away from forced nodes).  Synchronizes. */
int32_t ibm_get_ibm(ibm_ctx* ctx, uint8_t* flu, uint8_t* flv, uint8_t* msrc, double* fu, double* fv);

/* Checkpoint: bytes needed, then a host copy of the complete state (fields,
 * the time-stepping state of Sec. 2.2; checkpointing itself is not in the
 * paper),
 * phi, convection history, time, step count, forces) and its restore.  A run
 * restored from a checkpoint continues bit for bit as the uninterrupted run.
 * IBM_ERR_INVALID if bytes is too small or the blob does not match the grid. */
size_t ibm_state_bytes(const ibm_ctx* ctx);
int32_t ibm_get_state(ibm_ctx* ctx, void* host, size_t bytes);
int32_t ibm_set_state(ibm_ctx* ctx, const void* host, size_t bytes);

/* Replay schedule of pressure iterations (a test aid, not in the paper:
 * the stop test of Sec. 2.2's SOR is reproduced iteration for iteration):
 * the next n steps each run exactly
 * iters[k] pressure iterations (tolerance ignored), e.g. to reproduce the
 * iteration sequence of a reference run.  n = 0 clears the schedule.  host
 * array, copied. */
int32_t ibm_set_poisson_schedule(ibm_ctx* ctx, const int32_t* iters, int32_t n);

/* Learned guess and correction of the pressure solve (an extension of the
 * method, not in the paper; it changes only the initial guess and iterates
 * of the Sec. 2.2 pressure solve, whose stop test still decides; the network
 * is declared in ibm_unet.h).  The network works on the
 * grid coarsened by F = IBM_OPT_NET_FACTOR in both directions: coarse cell
 * (I, J) averages the fine cells [F I, F I + F) x [F J, F J + F).  For the
 * current phi it sees three coarse maps, each divided by its RMS over the
 * coarse grid:
 *   0: r = V b - A phi, the residual of phi;
 *   1: phi;
 *   2: the fraction of the block's cell centres inside the body at t^{n+1};
 * and predicts the coarse average of the remaining change of phi in units of
 * out_scale * s_r, s_r = RMS(map 0 before scaling); every fine cell of a
 * coarse cell receives its block's value:
 *   phi <- phi + out_scale * s_r * net(maps).
 * It is applied to phi^n before the solve when p_init is IBM_INIT_LEARNED
 * (the learned warm start), and, with IBM_OPT_NET_EVERY = M > 0, after every
 * M red-black SOR iterations that did not meet the stop test (the learned
 * correction; SOR and mixed-precision SOR only).  Every SOR segment ends on
 * the method's own stop test, so the network never decides convergence.
 * ibm_set_warm_start attaches a network (borrowed; NULL detaches) whose
 * image shape is (ny / F, nx / F) and whose stream is the context's stream;
 * IBM_ERR_INVALID otherwise, or for out_scale <= 0.  A step that would use a
 * network while none (or one of another shape) is attached returns
 * IBM_ERR_STATE before anything is enqueued. */
typedef struct ibm_unet ibm_unet;
int32_t ibm_set_warm_start(ibm_ctx* ctx, ibm_unet* net, double out_scale);

/* Training snapshots: while set, every step writes the maps above into
 * feat_dev (device float, (3, ny / F, nx / F)) and, after the solve, the
 * target: the coarse average of (phi^{n+1} - phi_s) / (out_scale * s_r) into
 * target_dev (device float, (ny / F, nx / F)).  phi_s is phi^n when
 * IBM_OPT_SNAPSHOT_ITER is 0, whatever the initial guess; with
 * IBM_OPT_SNAPSHOT_ITER = k > 0 (SOR methods) it is the iterate after k SOR
 * iterations from the step's initial guess, after which PCG completes the
 * solve.  Both pointers are borrowed until they are replaced or cleared
 * (both NULL). */
int32_t ibm_set_snapshot(ibm_ctx* ctx, float* feat_dev, float* target_dev, double out_scale);

/* Batches (an extension, not in the paper: many plunging-foil problems of
 * Sec. 2.1 on their own grids of Sec. 2.3 at once): the pressure solves of
 * many independent contexts (cases of
 * different grids) advanced together, one blocked red-black SOR launch per
 * IBM_OPT_TB_SWEEPS iterations sweeping the tiles of every case through one
 * work list, with the stop test of every case taken in one check launch; a
 * case that has met its stop test skips its tiles while the others go on.
 * Each case's iterates, iteration counts and results are those of ibm_step on
 * that context alone (its own tile shape, omega, tolerance and limit).
 * ibm_batch_create: n >= 1 distinct contexts (borrowed, kept alive by the
 * caller), all on one stream, either all IBM_SOLVER_RBSOR with the
 * register-resident blocked sweep (IBM_SOR_TEMPORAL) or all
 * IBM_SOLVER_RBSOR_MP (then each refinement runs as one launch over the row
 * blocks of every case, and the float sweeps as one launch over all their
 * tiles), the same IBM_OPT_TB_SWEEPS and p_check_every, at most 512 tiles
 * each, no network correction or snapshot, and either one p_max_iter shared
 * by all contexts or limits that are all multiples of p_check_every (the
 * batch advances in whole check intervals, so only then does every case stop
 * at its own limit); IBM_ERR_INVALID otherwise.  It
 * allocates a small descriptor array on the device and pinned host memory for
 * the check snapshots.
 * ibm_batch_step: nsteps time steps of every case; each step runs every
 * case's steps before and after its pressure solve in turn and one batched
 * pressure solve between.  last (nullable): n statistics of the last step
 * (seconds: the whole batched step).  Returns the worst status; after an
 * error the contexts' states are not usable. */
typedef struct ibm_batch ibm_batch;
int32_t ibm_batch_create(int32_t n, ibm_ctx* const* ctxs, ibm_batch** out);
int32_t ibm_batch_step(ibm_batch* batch, int32_t nsteps, ibm_step_stats* last);

/* Graph replay of the batched pressure solve.  intervals > 0 (even, at most
 * 1000): the launches of that many check intervals (the blocked sweeps and
 * the stop tests of all cases) are captured once into a HIP graph, on a
 * private stream of the batch, and each stretch of the solve replays it on
 * the contexts' stream after a one-thread launch that sets the stretch's
 * iteration base; the host waits on one event per stretch instead of one per
 * interval.  The final intervals that do not fill a stretch (up to the
 * largest p_max_iter) are launched one by one.  Results, iteration counts
 * and statuses are bit for bit those without the graph; a case that finishes
 * inside a stretch leaves the rest of the stretch's launches to skip its
 * tiles.  The graph is captured at the next ibm_batch_step and again when
 * the cases' tile counts change.  intervals = 0 (the default): no graph.
 * A batch of IBM_SOLVER_RBSOR_MP contexts captures, per interval, its float
 * sweep launches, the refinement and the stop tests; its stretches start
 * after an even number of intervals.  IBM_ERR_INVALID for odd or
 * out-of-range counts; IBM_ERR_HIP if the stream or the 8-byte device cursor
 * cannot be made (then the setting is unchanged). */
int32_t ibm_batch_set_graph(ibm_batch* batch, int32_t intervals);
void ibm_batch_destroy(ibm_batch* batch);
const char* ibm_batch_last_error(const ibm_batch* batch);

/* Kernel timing with HIP events on the context stream (the per-kernel view
 * of the profiling of Sec. 3.4.1).  sample_every > 0
 * brackets every sample_every-th launch of each timed kernel with a pair of
 * events; 0 switches it off and clears the samples.
 * ibm_profile_query: kernel id (IBM_KERNEL_*), average duration of the
 * sampled launches in ms, number of samples, number of launches, and the
 * algorithmic bytes one launch moves on this grid.  Launches that only
 * observed a finished solve (the tail enqueued ahead of the convergence
 * test) are not sampled.  Synchronizes. */
#define IBM_KERNEL_SOR_SWEEP 0      /* one colour of an SOR iteration: 24 B per cell updated */
#define IBM_KERNEL_SOR_RESIDUAL 1   /* residual check: 16 B per cell (phi, V b) */
#define IBM_KERNEL_PCG_DIR_SPMV 2   /* p = z + beta p, q = M p: 32 B per cell (z, p in; p, q out) */
#define IBM_KERNEL_PCG_UPDATE 3     /* x, r, z = r/d: 64 B per cell (x, r, p, q, d in; x, r, z out) */
#define IBM_KERNEL_SOR_TB 4         /* blocked SOR (either variant): 24 B per cell and iteration */
#define IBM_KERNEL_SOR_MP 5         /* mixed-precision sweeps: 12 B per cell and iteration (float e, r) */
#define IBM_KERNEL_SOR_MP_REFINE 6  /* its refinement: 32 B per cell (phi, e, V b in; phi, r out) */
#define IBM_KERNEL_CG1_ITER 7       /* one-reduction CG iteration: 88 B per cell (x, p, r, w, s, 1/d in;
                                       x, p, r, w, s out) */
#define IBM_KERNEL_COUNT 8
int32_t ibm_profile(ibm_ctx* ctx, int32_t sample_every);
/* Phase split of ibm_step (the four hot spots of Table 1, Sec. 3.4.1, with
 * the other parts of a step beside them): while kernel timing is on
 * (sample_every > 0), every ibm_step records HIP events on the context stream
 * at the phase boundaries and adds each phase's GPU time (ms) to a running
 * sum; ibm_profile resets the sums.  ibm_profile_phases copies the first n
 * sums (n <= IBM_PHASE_COUNT; later entries 0) and the number of steps
 * summed.  Batched steps are not phase-timed.  Synchronizes. */
#define IBM_PHASE_FLAGGING 0     /* fluid/solid classification ("flagging") */
#define IBM_PHASE_MOMENTUM 1     /* explicit momentum predictor */
#define IBM_PHASE_FORCING 2      /* body-force interpolation, forces, outlet */
#define IBM_PHASE_UV_SOLVE 3     /* implicit velocity solves ("U-V solver") */
#define IBM_PHASE_POISSON_RHS 4  /* Poisson source and the initial guess */
#define IBM_PHASE_P_SOLVE 5      /* pressure Poisson solve ("P solver") */
#define IBM_PHASE_PROJECTION 6   /* projection, pressure update, statistics */
#define IBM_PHASE_COUNT 7
int32_t ibm_profile_phases(ibm_ctx* ctx, double* ms, int32_t n, int64_t* steps);
int32_t ibm_profile_query(ibm_ctx* ctx, int32_t kernel, double* avg_ms, int64_t* samples, int64_t* launches,
                          double* bytes_per_launch);

/* Tuning options (not in the paper) of the red-black SOR sweeps of
 * Sec. 2.2 (they change the launch shape,
 * never the arithmetic: every choice gives bit-identical iterates).
 *   IBM_OPT_SOR_KERNEL  IBM_SOR_TEMPORAL (default): one launch performs
 *                       IBM_OPT_TB_SWEEPS iterations on a tile with halos
 *                       held in registers; IBM_SOR_TEMPORAL_LDS: the same
 *                       with the tile in LDS; IBM_SOR_PER_COLOUR: one launch
 *                       per colour sweep;
 *   IBM_OPT_TB_SWEEPS   iterations per blocked launch S, 1..12 (default 10);
 *   IBM_OPT_TB_TILE_X   interior tile width, even (default 76);
 *   IBM_OPT_TB_TILE_Y   interior tile height, even (default 44).
 * The loaded tile (interior plus a halo of 2 S + 2 on each side, clamped to
 * the grid) must fit 128 x 96 cells (one block of 16 waves, 6 rows per wave).
 * IBM_ERR_INVALID for an unknown option or a tile shape whose loaded tile
 * does not fit.  Applies to solves started after the call; the options
 * apply to the mixed-precision sweeps and the batched solves as well. */
#define IBM_OPT_SOR_KERNEL 0
#define IBM_OPT_TB_SWEEPS 1
#define IBM_OPT_TB_TILE_X 2
#define IBM_OPT_TB_TILE_Y 3
/* Options of the learned guess and correction (see ibm_set_warm_start):
 *   IBM_OPT_NET_FACTOR     coarsening factor F of the network's grid: 1, 2,
 *                          4, 8 or 16, dividing nx and ny (default 1);
 *   IBM_OPT_NET_EVERY      SOR iterations between network corrections, a
 *                          multiple of p_check_every; 0 (default): none;
 *   IBM_OPT_SNAPSHOT_ITER  SOR iterations before the snapshot, a multiple of
 *                          p_check_every; 0 (default): at the start. */
#define IBM_OPT_NET_FACTOR 4
#define IBM_OPT_NET_EVERY 5
#define IBM_OPT_SNAPSHOT_ITER 6
#define IBM_OPT_NET_SMOOTH 7  /* binomial [1 2 1]/4 passes (x then y) over the
                                 network output on the coarse grid, 0..16 (default 4) */
#define IBM_OPT_NET_STEP 8    /* step rule of a guess or correction e (default ENERGY):
   IBM_NET_STEP_ENERGY     a = min(1, 2 alpha), alpha = e.r / e.(A e) the step
                           minimising the energy norm of the error: the full
                           step unless it would increase that norm;
   IBM_NET_STEP_BACKTRACK  a = 1, halved whenever an SOR segment ends with a
                           larger residual than the previous one; below 1/64
                           the solve continues as plain SOR. */
#define IBM_NET_STEP_ENERGY 0
#define IBM_NET_STEP_BACKTRACK 1
#define IBM_OPT_NET_MAPS 9    /* maps given to the network, bit k = map k, 1..7
                                 (default 7); the others are zero, also in
                                 snapshots */
#define IBM_SOR_TEMPORAL 0
#define IBM_SOR_PER_COLOUR 1
#define IBM_SOR_TEMPORAL_LDS 2
int32_t ibm_set_option(ibm_ctx* ctx, int32_t option, int64_t value);

/* Release the context (not the workspace).  Synchronizes the stream first. */
void ibm_destroy(ibm_ctx* ctx);

/* Static text of a status code. */
const char* ibm_status_string(int32_t status);

/* Last error message of the context ("" if none); valid until the next call. */
const char* ibm_last_error(const ibm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* IBM_H */
