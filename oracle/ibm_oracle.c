/*
 * ibm_oracle.c -- plain, slow FP64 CPU reference ("oracle") for the
 * discrete-forcing immersed-boundary, fractional-step incompressible
 * Navier-Stokes solver of Sundar, Majumdar, Shah & Sarkar,
 * "Massive parallelization and performance enhancement of an immersed
 * boundary method based unsteady flow solver" (arXiv 2402.17337).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library, and neither calls the other.
 *
 * What the paper fixes (Sec. 2.1-2.3, Eqs. 1-4):
 *   - a 2-D rigid ellipse, thickness/chord 0.12, plunging as
 *     y(t) = h sin(k t), dy/dt = k h cos(k t)                     (Eqs. 1-2)
 *   - the non-dimensional N-S equations with a momentum forcing f that
 *     imposes no-slip on the body and a mass source q in the continuity
 *     equation                                                     (Eqs. 3-4)
 *   - fluid/solid flagging of mesh points at the start of every step
 *   - a finite-volume, staggered, semi-implicit fractional-step method with
 *     Adams-Bashforth (convection) and Crank-Nicolson (viscous) terms
 *   - red-black Gauss-Seidel SOR for the velocity and pressure equations.
 *
 * The paper prints no discrete formula.  The readings taken here (and by the
 * GPU library, written separately) are:
 *   grid      faces xf[0..nx], yf[0..ny]; dx_i, centres xc_i; centre
 *             distances dxu_i (u-face i sits between cells i-1 and i), with
 *             half cells dx_0/2 and dx_{nx-1}/2 at the two x ends; same in y.
 *   storage   p, phi at centres (nx*ny); u at x-faces ((nx+1)*ny); v at
 *             y-faces (nx*(ny+1)); row-major, x fastest.
 *   BCs       channel: inflow u = U, v = 0 on the face (half-cell distance);
 *             slip walls (v = 0, zero u flux); convective outlet for u,
 *             zero-gradient v; pressure Neumann except phi = 0 on the outlet
 *             face.  Periodic: both directions periodic (uniform grids only,
 *             used for the Taylor-Green check).
 *   momentum  R = u^n + dt[-(3/2 N^n - 1/2 N^{n-1}) - G p^n + 1/(2Re) L u^n],
 *             N^{-1} := N^0, N in divergence form with arithmetic averages;
 *             explicit predictor u~ = R + dt/(2Re) L u^n;
 *             (I - dt/(2Re) L) u^ = R + dt f  solved by red-black SOR.
 *   IBM       nodes strictly inside the ellipse are forced; a forced node
 *             with an outside 4-neighbour gets its target by linear
 *             extrapolation through the boundary crossing on each grid line
 *             (alpha = d_f/d_o capped at alpha_max), averaged over outside
 *             neighbours; deeper nodes take the body velocity;
 *             f = (V - u~)/dt.  Cells with a forced face carry the mass
 *             source q = divergence of (u^ - body velocity) over their forced
 *             faces, so D(u^) - q is the divergence with forced faces moving
 *             with the body (q_mode 1).  q_mode 2 keeps the other reading for
 *             comparison: q = D(u^) in cells with at least one forced and one
 *             free face, so their Poisson source vanishes (it lets mass
 *             appear in the cut cells and is unstable); q_mode 0: q = 0.
 *   pressure  incremental: A phi = V (D(u^) - q)/dt, A = V D G (5-point FV),
 *             u^{n+1} = u^ - dt G phi, p^{n+1} = p^n + phi - dt/(2Re) L phi.
 *   Poisson   red-black SOR, red = (i+j) even first, stop when
 *             ||Vb - A phi||_2 <= tol ||Vb||_2 tested every K iterations;
 *             or Jacobi-preconditioned CG on -A.
 *   forces    F = -sum_forced f dV + pi a b (0, a_body); C = 2F/(U^2 c).
 *
 * Built -O2 -ffp-contract=off.  OpenMP (when enabled) only splits loops whose
 * iterations are independent (one colour of a red-black sweep, pointwise
 * kernels); every reduction is a sequential compensated sum in row-major
 * order, so the threaded result equals the serial result bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CHANNEL 0
#define ORC_PERIODIC 1
#define ORC_SOR 0
#define ORC_PCG 1
#define ORC_SOR_MP 2
#define ORC_CG1 3     /* Jacobi-PCG with one reduction per iteration */
#define ORC_PCG_MP 4  /* single-precision CG with double reliable updates */
#define ORC_MP_DROP 0.1  /* reliable update once the float residual drops by this factor */

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_INVALID -1
#define ORC_ERR_NAN -5

/* Grids smaller than this run every loop on one thread (thread start-up
 * would cost more than the loop). */
#define ORC_OMP_MIN_CELLS 32768

#define FL_FLUID 0
#define FL_FORCING 1
#define FL_DEEP 2

/* Parameter block, mirrored field by field in oracle.py. */
typedef struct {
    int32_t nx, ny, bc, body;
    double re, dt, uinf;
    double chord, thick, x0, y0, amp, freq, phase;
    int32_t p_method, p_max_iter, p_check, p_init_prev;
    double p_omega, p_tol;
    double uv_omega, uv_tol;
    int32_t uv_max_iter, q_mode;
    double alpha_max;
} orc_params;

typedef struct {
    int32_t status, iters, pad0, pad1;
    double r0_rel, rel;
} orc_solve_stats;

typedef struct {
    int32_t status, p_iters, u_iters, v_iters;
    int32_t n_forced_u, n_forced_v, n_msrc, pad;
    double p_r0, p_rel, cd, cl, t;
} orc_step_stats;

typedef struct orc_ctx {
    orc_params P;
    int nx, ny, per;
    double *xf, *yf, *dx, *dy, *xc, *yc, *dxu, *dyv;
    double *u, *v, *p, *phi;
    double *nu, *nv;
    int have_hist;
    double *ru, *rv, *ut, *vt, *fu, *fv, *nwu, *nwv;
    unsigned char *flu, *flv, *msrc;
    double *vb, *w0, *w1, *w2, *w3, *w4, *w5, *w6;
    long step;
    double t, cd, cl;
} orc_ctx;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static int wrapi(int k, int n) {
    k %= n;
    return k < 0 ? k + n : k;
}

/* u at x-face (i, j); periodic mode wraps both indices (u[nx] mirrors u[0]). */
static double U(const orc_ctx *c, int i, int j) {
    if (c->per) { i = wrapi(i, c->nx); j = wrapi(j, c->ny); }
    return c->u[(size_t)j * (c->nx + 1) + i];
}
/* v at y-face (i, j); periodic mode wraps (v row ny mirrors row 0). */
static double V(const orc_ctx *c, int i, int j) {
    if (c->per) { i = wrapi(i, c->nx); j = wrapi(j, c->ny); }
    return c->v[(size_t)j * c->nx + i];
}
/* a cell-centred field a at (i, j). */
static double C(const orc_ctx *c, const double *a, int i, int j) {
    if (c->per) { i = wrapi(i, c->nx); j = wrapi(j, c->ny); }
    return a[(size_t)j * c->nx + i];
}
static double DX(const orc_ctx *c, int i) { return c->dx[c->per ? wrapi(i, c->nx) : i]; }
static double DY(const orc_ctx *c, int j) { return c->dy[c->per ? wrapi(j, c->ny) : j]; }

static size_t iu(const orc_ctx *c, int i, int j) { return (size_t)j * (c->nx + 1) + i; }
static size_t iv(const orc_ctx *c, int i, int j) { return (size_t)j * c->nx + i; }
static size_t ic(const orc_ctx *c, int i, int j) { return (size_t)j * c->nx + i; }

/* Sequential Neumaier-compensated sum of squares, row-major order. */
static double sumsq(const double *a, size_t n) {
    double s = 0.0, comp = 0.0;
    for (size_t k = 0; k < n; ++k) {
        double x = a[k] * a[k];
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x;
        else comp += (x - t) + s;
        s = t;
    }
    return s + comp;
}
static double sumv(const double *a, size_t n) {
    double s = 0.0, comp = 0.0;
    for (size_t k = 0; k < n; ++k) {
        double x = a[k];
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x;
        else comp += (x - t) + s;
        s = t;
    }
    return s + comp;
}
static double dot(const double *a, const double *b, size_t n) {
    double s = 0.0, comp = 0.0;
    for (size_t k = 0; k < n; ++k) {
        double x = a[k] * b[k];
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x;
        else comp += (x - t) + s;
        s = t;
    }
    return s + comp;
}

/* Range of u unknowns in x: channel faces 1..nx-1 (0 is the inflow, nx the
 * outlet, both set by boundary conditions); periodic faces 0..nx-1. */
static int u_i0(const orc_ctx *c) { return c->per ? 0 : 1; }
static int u_i1(const orc_ctx *c) { return c->nx; } /* exclusive */
static int v_j0(const orc_ctx *c) { return c->per ? 0 : 1; }
static int v_j1(const orc_ctx *c) { return c->ny; } /* exclusive */

static void sync_periodic(orc_ctx *c) {
    if (!c->per) return;
    const int nx = c->nx, ny = c->ny;
    for (int j = 0; j < ny; ++j) c->u[iu(c, nx, j)] = c->u[iu(c, 0, j)];
    for (int i = 0; i < nx; ++i) c->v[iv(c, i, ny)] = c->v[iv(c, i, 0)];
}

/* ------------------------------------------------------------------------ */
/* Pressure operator A = V D G (cell-centred 5-point finite volume).         */
/* Returns s = sum a_nb x_nb and stores the diagonal d = sum a_nb (+ outlet  */
/* term) so that (A x)_ij = s - d x_ij.  Neumann faces carry no coefficient; */
/* the outlet face holds phi = 0 at half-cell distance and only adds to d.   */
/* ------------------------------------------------------------------------ */
static double A_row(const orc_ctx *c, const double *x, int i, int j, double *diag) {
    const int nx = c->nx, ny = c->ny, per = c->per;
    double s = 0.0, d = 0.0, a;
    if (per || i < nx - 1) { a = c->dy[j] / c->dxu[i + 1]; s += a * C(c, x, i + 1, j); d += a; }
    else { d += c->dy[j] / c->dxu[nx]; }
    if (per || i > 0) { a = c->dy[j] / c->dxu[i]; s += a * C(c, x, i - 1, j); d += a; }
    if (per || j < ny - 1) { a = c->dx[i] / c->dyv[j + 1]; s += a * C(c, x, i, j + 1); d += a; }
    if (per || j > 0) { a = c->dx[i] / c->dyv[j]; s += a * C(c, x, i, j - 1); d += a; }
    *diag = d;
    return s;
}

void orc_apply_A(const orc_ctx *c, const double *x, double *y) {
    const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double d, s = A_row(c, x, i, j, &d);
            y[ic(c, i, j)] = s - d * x[ic(c, i, j)];
        }
}

static double poisson_resid_norm(const orc_ctx *c, const double *x, const double *vb, double *r) {
    const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double d, s = A_row(c, x, i, j, &d);
            r[ic(c, i, j)] = vb[ic(c, i, j)] - (s - d * x[ic(c, i, j)]);
        }
    return sqrt(sumsq(r, (size_t)nx * ny));
}

/* One colour of a red-black SOR sweep: colour 0 = (i+j) even ("red"). */
static void poisson_sor_colour(const orc_ctx *c, double *x, const double *vb, double omega, int colour) {
    const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = (j + colour) & 1; i < nx; i += 2) {
            double d, s = A_row(c, x, i, j, &d);
            double g = (s - vb[ic(c, i, j)]) / d;
            x[ic(c, i, j)] = (1.0 - omega) * x[ic(c, i, j)] + omega * g;
        }
}

/* Periodic (singular) mode: make the volume-weighted right-hand side sum to
 * zero, and the solution have zero volume-weighted mean. */
static void periodic_project_rhs(const orc_ctx *c, double *vb) {
    const size_t n = (size_t)c->nx * c->ny;
    double *vol = c->w4;
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) vol[ic(c, i, j)] = c->dx[i] * c->dy[j];
    double sb = sumv(vb, n), sv = sumv(vol, n);
    for (size_t k = 0; k < n; ++k) vb[k] -= (sb / sv) * vol[k];
}
static void periodic_zero_mean(const orc_ctx *c, double *x) {
    const size_t n = (size_t)c->nx * c->ny;
    double *vol = c->w4, *tmp = c->w3;
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            vol[ic(c, i, j)] = c->dx[i] * c->dy[j];
            tmp[ic(c, i, j)] = vol[ic(c, i, j)] * x[ic(c, i, j)];
        }
    double m = sumv(tmp, n) / sumv(vol, n);
    for (size_t k = 0; k < n; ++k) x[k] -= m;
}

/* Red-black SOR on A x = vb.  Iterations are counted in full red+black
 * sweeps; the residual is tested after iterations K, 2K, ... (and once
 * before the first).  fixed > 0 runs exactly that many iterations. */
static int poisson_sor(const orc_ctx *c, const double *vb, double *x, double omega, double tol,
                       int max_iter, int check, int fixed, orc_solve_stats *st) {
    const size_t n = (size_t)c->nx * c->ny;
    double *r = c->w0;
    double bn = sqrt(sumsq(vb, n));
    st->iters = 0; st->r0_rel = 0.0; st->rel = 0.0; st->status = ORC_OK;
    if (!isfinite(bn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (bn == 0.0) { memset(x, 0, n * sizeof(double)); return ORC_OK; }
    if (fixed > 0) { max_iter = fixed; tol = -1.0; }
    if (check < 1) check = 1;
    double rn = poisson_resid_norm(c, x, vb, r);
    st->r0_rel = rn / bn; st->rel = rn / bn;
    if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    int it = 0;
    if (rn <= tol * bn) return ORC_OK;
    while (it < max_iter) {
        int m = check < max_iter - it ? check : max_iter - it;
        for (int k = 0; k < m; ++k) {
            poisson_sor_colour(c, x, vb, omega, 0);
            poisson_sor_colour(c, x, vb, omega, 1);
        }
        it += m;
        rn = poisson_resid_norm(c, x, vb, r);
        st->iters = it; st->rel = rn / bn;
        if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
        if (rn <= tol * bn) return ORC_OK;
    }
    if (fixed > 0) return ORC_OK;
    st->status = ORC_NOT_CONVERGED;
    return ORC_NOT_CONVERGED;
}

/* Mixed precision: red-black SOR with single-precision sweeps and
 * double-precision refinement.  Every check interval of m iterations solves
 * the correction equation A e = r of the current residual r = vb - A x with
 * m SOR iterations from e = 0 in single precision (coefficients, right-hand
 * side and e rounded to float, float arithmetic), then x += e and the residual
 * and the stop test are evaluated in double precision.  SOR is a stationary
 * iteration, so in exact arithmetic restarting it on the correction equation
 * reproduces the double-precision iterates; rounding is relative to the size
 * of the correction, which shrinks as x converges.  Single-precision SOR alone
 * stalls where its rounding error reaches the residual (set refine = 0 to run
 * it without refinement, x += e once at the end). */
static void sor_colour_f32(const orc_ctx *c, float *e, const float *r32, float omega, int colour) {
    const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = (j + colour) & 1; i < nx; i += 2) {
            float s = 0.0f, d = 0.0f, a;
            if (i < nx - 1) { a = (float)(c->dy[j] / c->dxu[i + 1]); s += a * e[ic(c, i + 1, j)]; d += a; }
            else { d += (float)(c->dy[j] / c->dxu[nx]); }
            if (i > 0) { a = (float)(c->dy[j] / c->dxu[i]); s += a * e[ic(c, i - 1, j)]; d += a; }
            if (j < ny - 1) { a = (float)(c->dx[i] / c->dyv[j + 1]); s += a * e[ic(c, i, j + 1)]; d += a; }
            if (j > 0) { a = (float)(c->dx[i] / c->dyv[j]); s += a * e[ic(c, i, j - 1)]; d += a; }
            float g = (s - r32[ic(c, i, j)]) / d;
            e[ic(c, i, j)] = (1.0f - omega) * e[ic(c, i, j)] + omega * g;
        }
}

static int poisson_sor_mp(const orc_ctx *c, const double *vb, double *x, double omega, double tol,
                          int max_iter, int check, int fixed, int refine, orc_solve_stats *st) {
    const size_t n = (size_t)c->nx * c->ny;
    double *r = c->w0;
    float *e = (float *)c->w1, *r32 = (float *)c->w2;
    const float om = (float)omega;
    double bn = sqrt(sumsq(vb, n));
    st->iters = 0; st->r0_rel = 0.0; st->rel = 0.0; st->status = ORC_OK;
    if (!isfinite(bn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (bn == 0.0) { memset(x, 0, n * sizeof(double)); return ORC_OK; }
    if (fixed > 0) { max_iter = fixed; tol = -1.0; }
    if (check < 1) check = 1;
    double rn = poisson_resid_norm(c, x, vb, r);
    st->r0_rel = rn / bn; st->rel = rn / bn;
    if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (rn <= tol * bn) return ORC_OK;
    int it = 0;
    if (!refine) {
        for (size_t k = 0; k < n; ++k) { r32[k] = (float)r[k]; e[k] = 0.0f; }
        for (; it < max_iter; ++it) {
            sor_colour_f32(c, e, r32, om, 0);
            sor_colour_f32(c, e, r32, om, 1);
        }
        for (size_t k = 0; k < n; ++k) x[k] += (double)e[k];
        rn = poisson_resid_norm(c, x, vb, r);
        st->iters = it; st->rel = rn / bn;
        return ORC_OK;
    }
    while (it < max_iter) {
        int m = check < max_iter - it ? check : max_iter - it;
        for (size_t k = 0; k < n; ++k) { r32[k] = (float)r[k]; e[k] = 0.0f; }
        for (int k = 0; k < m; ++k) {
            sor_colour_f32(c, e, r32, om, 0);
            sor_colour_f32(c, e, r32, om, 1);
        }
        for (size_t k = 0; k < n; ++k) x[k] += (double)e[k];
        it += m;
        rn = poisson_resid_norm(c, x, vb, r);
        st->iters = it; st->rel = rn / bn;
        if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
        if (rn <= tol * bn) return ORC_OK;
    }
    if (fixed > 0) return ORC_OK;
    st->status = ORC_NOT_CONVERGED;
    return ORC_NOT_CONVERGED;
}

/* Jacobi-preconditioned conjugate gradients on M x = c with M = -A (SPD in
 * channel mode), c = -vb; the preconditioner is diag(M) = sum of the
 * neighbour coefficients plus the outlet term.  The stop test uses the
 * recursively updated residual and is confirmed with the true residual; on a
 * failed confirmation the residual is replaced by the true one and the search
 * direction restarts. */
static int poisson_pcg(const orc_ctx *c, const double *vb, double *x, double tol, int max_iter,
                       int fixed, orc_solve_stats *st) {
    const int nx = c->nx, ny = c->ny;
    const size_t n = (size_t)nx * ny;
    double *r = c->w0, *z = c->w1, *pp = c->w2, *q = c->w3, *dg = c->w4;
    double bn = sqrt(sumsq(vb, n));
    st->iters = 0; st->r0_rel = 0.0; st->rel = 0.0; st->status = ORC_OK;
    if (!isfinite(bn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (bn == 0.0) { memset(x, 0, n * sizeof(double)); return ORC_OK; }
    if (fixed > 0) { max_iter = fixed; tol = -1.0; }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) { double d; A_row(c, x, i, j, &d); dg[ic(c, i, j)] = d; }
    /* r = c - M x = -vb + A x */
    orc_apply_A(c, x, q);
    for (size_t k = 0; k < n; ++k) r[k] = -vb[k] + q[k];
    double rn = sqrt(sumsq(r, n));
    st->r0_rel = rn / bn; st->rel = rn / bn;
    if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (rn <= tol * bn) return ORC_OK;
    for (size_t k = 0; k < n; ++k) { z[k] = r[k] / dg[k]; pp[k] = z[k]; }
    double rz = dot(r, z, n);
    int it = 0;
    while (it < max_iter) {
        orc_apply_A(c, pp, q);
        for (size_t k = 0; k < n; ++k) q[k] = -q[k];       /* q = M p */
        double pq = dot(pp, q, n);
        double alpha = rz / pq;
        for (size_t k = 0; k < n; ++k) { x[k] += alpha * pp[k]; r[k] -= alpha * q[k]; }
        ++it;
        rn = sqrt(sumsq(r, n));
        st->iters = it; st->rel = rn / bn;
        if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
        if (rn <= tol * bn) {
            orc_apply_A(c, x, q);
            for (size_t k = 0; k < n; ++k) r[k] = -vb[k] + q[k];
            rn = sqrt(sumsq(r, n));
            st->rel = rn / bn;
            if (rn <= tol * bn) return ORC_OK;
            for (size_t k = 0; k < n; ++k) { z[k] = r[k] / dg[k]; pp[k] = z[k]; }
            rz = dot(r, z, n);
            continue;
        }
        for (size_t k = 0; k < n; ++k) z[k] = r[k] / dg[k];
        double rz1 = dot(r, z, n);
        double beta = rz1 / rz;
        rz = rz1;
        for (size_t k = 0; k < n; ++k) pp[k] = z[k] + beta * pp[k];
    }
    if (fixed > 0) {
        orc_apply_A(c, x, q);
        for (size_t k = 0; k < n; ++k) r[k] = -vb[k] + q[k];
        st->rel = sqrt(sumsq(r, n)) / bn;
        return ORC_OK;
    }
    st->status = ORC_NOT_CONVERGED;
    return ORC_NOT_CONVERGED;
}

/* y = M x = -A x for the Jacobi-PCG solvers. */
static void apply_M(const orc_ctx *c, const double *x, double *y) {
    const size_t n = (size_t)c->nx * c->ny;
    orc_apply_A(c, x, y);
    for (size_t k = 0; k < n; ++k) y[k] = -y[k];
}

/* Jacobi-preconditioned CG on M x = -vb (M = -A) in the form with one
 * reduction per iteration (Chronopoulos and Gear, 1989): besides the
 * direction p it carries s = M p by its own recurrence, so the two inner
 * products of an iteration, gamma = (r, u) and delta = (M u, u) with
 * u = D^-1 r, are taken together:
 *   beta_i = gamma_i / gamma_{i-1},
 *   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
 *   p_i = u_i + beta_i p_{i-1},  s_i = M u_i + beta_i s_{i-1},
 *   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i.
 * In exact arithmetic its iterates are those of poisson_pcg.  Stop test and
 * confirmation as there: the recursive residual, then the true one (on a
 * failed confirmation the recurrences restart from it). */
static int poisson_cg1(const orc_ctx *c, const double *vb, double *x, double tol, int max_iter, int fixed,
                       orc_solve_stats *st) {
    const int nx = c->nx, ny = c->ny;
    const size_t n = (size_t)nx * ny;
    double *r = c->w0, *u = c->w1, *w = c->w2, *pp = c->w3, *ss = c->w4, *dg = c->w5, *q = c->w6;
    double bn = sqrt(sumsq(vb, n));
    st->iters = 0; st->r0_rel = 0.0; st->rel = 0.0; st->status = ORC_OK;
    if (!isfinite(bn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (bn == 0.0) { memset(x, 0, n * sizeof(double)); return ORC_OK; }
    if (fixed > 0) { max_iter = fixed; tol = -1.0; }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) { double d; A_row(c, x, i, j, &d); dg[ic(c, i, j)] = d; }
    orc_apply_A(c, x, q);
    for (size_t k = 0; k < n; ++k) r[k] = -vb[k] + q[k];
    double rn = sqrt(sumsq(r, n));
    st->r0_rel = rn / bn; st->rel = rn / bn;
    if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
    if (rn <= tol * bn) return ORC_OK;
    int it = 0, start = 1;
    double gamma_old = 0.0, alpha = 0.0;
    for (;;) {
        /* u = D^-1 r, w = M u, gamma, delta; then the new direction */
        for (size_t k = 0; k < n; ++k) u[k] = r[k] / dg[k];
        apply_M(c, u, w);
        double gamma = dot(r, u, n), delta = dot(w, u, n);
        if (start) {
            alpha = gamma / delta;
            for (size_t k = 0; k < n; ++k) { pp[k] = u[k]; ss[k] = w[k]; }
            start = 0;
        } else {
            double beta = gamma / gamma_old;
            alpha = gamma / (delta - beta * gamma / alpha);
            for (size_t k = 0; k < n; ++k) { pp[k] = u[k] + beta * pp[k]; ss[k] = w[k] + beta * ss[k]; }
        }
        gamma_old = gamma;
        if (it >= max_iter) break;
        for (size_t k = 0; k < n; ++k) { x[k] += alpha * pp[k]; r[k] -= alpha * ss[k]; }
        ++it;
        rn = sqrt(sumsq(r, n));
        st->iters = it; st->rel = rn / bn;
        if (!isfinite(rn)) { st->status = ORC_ERR_NAN; return ORC_ERR_NAN; }
        if (rn <= tol * bn) {
            orc_apply_A(c, x, q);
            for (size_t k = 0; k < n; ++k) r[k] = -vb[k] + q[k];
            rn = sqrt(sumsq(r, n));
            st->rel = rn / bn;
            if (rn <= tol * bn) return ORC_OK;
            start = 1;  /* restart from the true residual */
        }
    }
    if (fixed > 0) {
        orc_apply_A(c, x, q);
        for (size_t k = 0; k < n; ++k) r[k] = -vb[k] + q[k];
        st->rel = sqrt(sumsq(r, n)) / bn;
        return ORC_OK;
    }
    st->status = ORC_NOT_CONVERGED;
    return ORC_NOT_CONVERGED;
}

/* y = M x in single precision: M = -A with the coefficients of A rounded to
 * float, summed in the order E, W, N, S (outlet term with E), float
 * arithmetic throughout. */
static void apply_M_f32(const orc_ctx *c, const float *x, float *y) {
    const int nx = c->nx, ny = c->ny;

#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            float s = 0.0f, d = 0.0f, a;
            if (i < nx - 1) { a = (float)(c->dy[j] / c->dxu[i + 1]); s += a * x[ic(c, i + 1, j)]; d += a; }
            else { d += (float)(c->dy[j] / c->dxu[nx]); }
            if (i > 0) { a = (float)(c->dy[j] / c->dxu[i]); s += a * x[ic(c, i - 1, j)]; d += a; }
            if (j < ny - 1) { a = (float)(c->dx[i] / c->dyv[j + 1]); s += a * x[ic(c, i, j + 1)]; d += a; }
            if (j > 0) { a = (float)(c->dx[i] / c->dyv[j]); s += a * x[ic(c, i, j - 1)]; d += a; }
            y[ic(c, i, j)] = d * x[ic(c, i, j)] - s;
        }
}
/* Diagonal of the single-precision M. */
static void diag_M_f32(const orc_ctx *c, float *d) {
    const int nx = c->nx, ny = c->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            float dd = 0.0f;
            if (i < nx - 1) dd += (float)(c->dy[j] / c->dxu[i + 1]);
            else dd += (float)(c->dy[j] / c->dxu[nx]);
            if (i > 0) dd += (float)(c->dy[j] / c->dxu[i]);
            if (j < ny - 1) dd += (float)(c->dx[i] / c->dyv[j + 1]);
            if (j > 0) dd += (float)(c->dx[i] / c->dyv[j]);
            d[ic(c, i, j)] = dd;
        }
}
/* Inner product of two float vectors: every product exactly in double
 * (a float times a float fits), summed in double. */
static double dot_f32(const float *a, const float *b, size_t n) {
    double s = 0.0, comp = 0.0;
    for (size_t k = 0; k < n; ++k) {
        double x = (double)a[k] * (double)b[k];
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x;
        else comp += (x - t) + s;
        s = t;
    }
    return s + comp;
}

/* Mixed precision Jacobi-PCG with reliable updates: the one-reduction CG of
 * poisson_cg1 runs in single precision on the correction equation M e = -r of
 * the current double x (vectors e, r, u = D^-1 r, w = M u, p, s and the
 * operator in float; inner products in double; alpha and beta rounded to
 * float for the vector updates), and the recurrences are never restarted.
 * Whenever the float residual has dropped to ORC_MP_DROP times the largest
 * one since the last update, after at most `every` iterations, and when it
 * passes the stop test, x += e in double, e = 0, the double residual
 * r = vb - A x is formed and tested, and its float rounding replaces the
 * recursive residual (residual replacement, as in reliable-update CG): the
 * search direction and its product s = M p carry on, so the Krylov space is
 * kept, while the residual the iteration works on stays the true one up to
 * float rounding.  Iterations count CG iterations.  refine = 0: single
 * precision alone, no replacement; the solve ends when the float residual
 * passes the test or at max_iter, then x += e. */
static int poisson_pcg_mp(const orc_ctx *c, const double *vb, double *x, double tol, int max_iter, int every,
                          int refine, orc_solve_stats *st) {
    const size_t n = (size_t)c->nx * c->ny;
    double *r = c->w0;
    float *fr = calloc(n, sizeof(float)), *fu = calloc(n, sizeof(float)), *fw = calloc(n, sizeof(float));
    float *fp = calloc(n, sizeof(float)), *fs = calloc(n, sizeof(float)), *fe = calloc(n, sizeof(float));
    float *fd = calloc(n, sizeof(float));
    int rc = ORC_OK;
    double bn = sqrt(sumsq(vb, n));
    st->iters = 0; st->r0_rel = 0.0; st->rel = 0.0; st->status = ORC_OK;
    if (!fr || !fu || !fw || !fp || !fs || !fe || !fd) { rc = ORC_ERR_INVALID; goto out; }
    if (!isfinite(bn)) { st->status = rc = ORC_ERR_NAN; goto out; }
    if (bn == 0.0) { memset(x, 0, n * sizeof(double)); goto out; }
    diag_M_f32(c, fd);
    double rn = poisson_resid_norm(c, x, vb, r);
    st->r0_rel = rn / bn; st->rel = rn / bn;
    if (!isfinite(rn)) { st->status = rc = ORC_ERR_NAN; goto out; }
    if (refine && rn <= tol * bn) goto out;
    for (size_t k = 0; k < n; ++k) { fr[k] = (float)(-r[k]); fe[k] = 0.0f; }
    int it = 0, start = 1, since = 0;
    double rmax = sqrt(dot_f32(fr, fr, n));  /* largest float residual since the last update */
    double gamma_old = 0.0, alpha = 0.0;
    for (;;) {
        for (size_t k = 0; k < n; ++k) fu[k] = fr[k] / fd[k];
        apply_M_f32(c, fu, fw);
        double gamma = dot_f32(fr, fu, n), delta = dot_f32(fw, fu, n);
        if (start) {
            alpha = gamma / delta;
            for (size_t k = 0; k < n; ++k) { fp[k] = fu[k]; fs[k] = fw[k]; }
            start = 0;
        } else {
            double beta = gamma / gamma_old;
            alpha = gamma / (delta - beta * gamma / alpha);
            const float fb = (float)beta;
            for (size_t k = 0; k < n; ++k) { fp[k] = fu[k] + fb * fp[k]; fs[k] = fw[k] + fb * fs[k]; }
        }
        gamma_old = gamma;
        if (it >= max_iter) break;
        const float fa = (float)alpha;
        for (size_t k = 0; k < n; ++k) { fe[k] += fa * fp[k]; fr[k] -= fa * fs[k]; }
        ++it; ++since;
        double rin = sqrt(dot_f32(fr, fr, n));
        if (!isfinite(rin)) { st->iters = it; st->status = rc = ORC_ERR_NAN; goto out; }
        const int passed = rin <= tol * bn;
        if (!refine) { if (passed || it >= max_iter) break; continue; }
        if (rin > rmax) rmax = rin;
        if (passed || rin <= ORC_MP_DROP * rmax || (every > 0 && since >= every) || it >= max_iter) {
            /* reliable update: x += e, the double residual, its test, and
             * the float residual replaced by it */
            for (size_t k = 0; k < n; ++k) { x[k] += (double)fe[k]; fe[k] = 0.0f; }
            rn = poisson_resid_norm(c, x, vb, r);
            st->iters = it; st->rel = rn / bn;
            if (!isfinite(rn)) { st->status = rc = ORC_ERR_NAN; goto out; }
            if (rn <= tol * bn) goto out;
            if (it >= max_iter) break;
            for (size_t k = 0; k < n; ++k) fr[k] = (float)(-r[k]);
            since = 0;
            rmax = sqrt(dot_f32(fr, fr, n));
        }
    }
    if (!refine) {
        for (size_t k = 0; k < n; ++k) x[k] += (double)fe[k];
        rn = poisson_resid_norm(c, x, vb, r);
        st->iters = it; st->rel = rn / bn;
        goto out;
    }
    st->status = rc = ORC_NOT_CONVERGED;
out:
    free(fr); free(fu); free(fw); free(fp); free(fs); free(fe); free(fd);
    return rc;
}

static int poisson_solve_vb(orc_ctx *c, double *vb, double *x, int method, double omega, double tol,
                            int max_iter, int check, int fixed, orc_solve_stats *st) {
    int rc;
    if ((method == ORC_SOR_MP || method == ORC_PCG_MP) && c->per) return ORC_ERR_INVALID;  /* channel only */
    if (c->per) periodic_project_rhs(c, vb);
    if (method == ORC_PCG) rc = poisson_pcg(c, vb, x, tol, max_iter, fixed, st);
    else if (method == ORC_SOR_MP) rc = poisson_sor_mp(c, vb, x, omega, tol, max_iter, check, fixed, 1, st);
    else if (method == ORC_CG1) rc = poisson_cg1(c, vb, x, tol, max_iter, fixed, st);
    else if (method == ORC_PCG_MP) {
        if (fixed > 0) return ORC_ERR_INVALID;
        rc = poisson_pcg_mp(c, vb, x, tol, max_iter, check, 1, st);
    }
    else rc = poisson_sor(c, vb, x, omega, tol, max_iter, check, fixed, st);
    if (c->per && rc >= 0) periodic_zero_mean(c, x);
    return rc;
}

/* Stand-alone solve of the cell-centred Poisson problem  (D G) x = b  with the
 * context's grid and boundary conditions: b is per unit volume, the solver
 * works on A x = V b.  x holds the initial guess on entry. */
int orc_poisson_solve(orc_ctx *c, const double *b, double *x, int method, double omega, double tol,
                      int max_iter, int check, int fixed, orc_solve_stats *st) {
    const int nx = c->nx, ny = c->ny;
    double *vb = c->vb;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) vb[ic(c, i, j)] = (c->dx[i] * c->dy[j]) * b[ic(c, i, j)];
    return poisson_solve_vb(c, vb, x, method, omega, tol, max_iter, check, fixed, st);
}

/* Single-precision SOR without refinement (the stall that refinement
 * removes): `iters` float iterations on the correction of x, then x += e. */
int orc_poisson_sor_f32(orc_ctx *c, const double *b, double *x, double omega, int iters, orc_solve_stats *st) {
    const int nx = c->nx, ny = c->ny;
    double *vb = c->vb;
    if (c->per || iters < 1) return ORC_ERR_INVALID;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) vb[ic(c, i, j)] = (c->dx[i] * c->dy[j]) * b[ic(c, i, j)];
    return poisson_sor_mp(c, vb, x, omega, -1.0, iters, iters, iters, 0, st);
}

/* Single-precision CG without refinement: one inner solve of `iters`
 * iterations on the correction of x, then x += e. */
int orc_poisson_pcg_f32(orc_ctx *c, const double *b, double *x, int iters, orc_solve_stats *st) {
    const int nx = c->nx, ny = c->ny;
    double *vb = c->vb;
    if (c->per || iters < 1) return ORC_ERR_INVALID;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) vb[ic(c, i, j)] = (c->dx[i] * c->dy[j]) * b[ic(c, i, j)];
    return poisson_pcg_mp(c, vb, x, -1.0, iters, 0, 0, st);
}

/* ------------------------------------------------------------------------ */
/* Momentum operators on the staggered grid.                                 */
/* ------------------------------------------------------------------------ */

/* Viscous operator L u at an x-face unknown (i, j), finite-volume form over
 * the face control volume dxu_i x dy_j; slip walls carry no flux. */
static double Lu_at(const orc_ctx *c, int i, int j) {
    const int ny = c->ny, per = c->per;
    double uP = U(c, i, j);
    double L = (U(c, i + 1, j) - uP) / (DX(c, i) * c->dxu[i]) + (U(c, i - 1, j) - uP) / (DX(c, i - 1) * c->dxu[i]);
    if (per || j < ny - 1) L += (U(c, i, j + 1) - uP) / (c->dyv[j + 1] * c->dy[j]);
    if (per || j > 0) L += (U(c, i, j - 1) - uP) / (c->dyv[j] * c->dy[j]);
    return L;
}

/* Viscous operator L v at a y-face unknown (i, j); at the inflow v = 0 sits on
 * the face (half-cell distance), at the outlet v has zero gradient. */
static double Lv_at(const orc_ctx *c, int i, int j) {
    const int nx = c->nx, per = c->per;
    double vP = V(c, i, j);
    double L = (V(c, i, j + 1) - vP) / (DY(c, j) * c->dyv[j]) + (V(c, i, j - 1) - vP) / (DY(c, j - 1) * c->dyv[j]);
    if (per || i < nx - 1) L += (V(c, i + 1, j) - vP) / (c->dxu[i + 1] * c->dx[i]);
    if (per || i > 0) L += (V(c, i - 1, j) - vP) / (c->dxu[i] * c->dx[i]);
    else L += (0.0 - vP) / (c->dxu[0] * c->dx[0]);
    return L;
}

/* Convection N(u) = d(uu)/dx + d(vu)/dy at x-face (i, j), divergence form:
 * uu at cell centres from the two neighbouring faces, vu at the cell corners
 * from two v and two u values; zero flux through the slip walls. */
static double Nu_at(const orc_ctx *c, int i, int j) {
    const int ny = c->ny, per = c->per;
    double uP = U(c, i, j);
    double ue = 0.5 * (uP + U(c, i + 1, j));
    double uw = 0.5 * (U(c, i - 1, j) + uP);
    double nxp = (ue * ue - uw * uw) / c->dxu[i];
    double fn = 0.0, fs = 0.0;
    if (per || j < ny - 1) {
        double vc = 0.5 * (V(c, i - 1, j + 1) + V(c, i, j + 1));
        double uc = 0.5 * (uP + U(c, i, j + 1));
        fn = vc * uc;
    }
    if (per || j > 0) {
        double vc = 0.5 * (V(c, i - 1, j) + V(c, i, j));
        double uc = 0.5 * (U(c, i, j - 1) + uP);
        fs = vc * uc;
    }
    return nxp + (fn - fs) / c->dy[j];
}

/* Convection N(v) = d(uv)/dx + d(vv)/dy at y-face (i, j). */
static double Nv_at(const orc_ctx *c, int i, int j) {
    const int nx = c->nx, per = c->per;
    double vP = V(c, i, j);
    double vn = 0.5 * (vP + V(c, i, j + 1));
    double vs = 0.5 * (V(c, i, j - 1) + vP);
    double nyp = (vn * vn - vs * vs) / c->dyv[j];
    double ue = 0.5 * (U(c, i + 1, j - 1) + U(c, i + 1, j));
    double ve = (per || i < nx - 1) ? 0.5 * (vP + V(c, i + 1, j)) : vP;
    double uw = 0.5 * (U(c, i, j - 1) + U(c, i, j));
    double vw = (per || i > 0) ? 0.5 * (V(c, i - 1, j) + vP) : 0.0;
    return (ue * ve - uw * vw) / c->dx[i] + nyp;
}

static double Gu_at(const orc_ctx *c, const double *p, int i, int j) {
    return (C(c, p, i, j) - C(c, p, i - 1, j)) / c->dxu[i];
}
static double Gv_at(const orc_ctx *c, const double *p, int i, int j) {
    return (C(c, p, i, j) - C(c, p, i, j - 1)) / c->dyv[j];
}

/* Evaluate N, G p and L at every unknown for the current fields (used by the
 * operator consistency checks).  Non-unknown entries are left at zero. */
void orc_momentum_terms(const orc_ctx *c, double *Nu, double *Gu, double *Lu, double *Nv, double *Gv,
                        double *Lv) {
    const int nx = c->nx, ny = c->ny;
    memset(Nu, 0, sizeof(double) * (nx + 1) * ny);
    memset(Gu, 0, sizeof(double) * (nx + 1) * ny);
    memset(Lu, 0, sizeof(double) * (nx + 1) * ny);
    memset(Nv, 0, sizeof(double) * nx * (ny + 1));
    memset(Gv, 0, sizeof(double) * nx * (ny + 1));
    memset(Lv, 0, sizeof(double) * nx * (ny + 1));
    for (int j = 0; j < ny; ++j)
        for (int i = u_i0(c); i < u_i1(c); ++i) {
            Nu[iu(c, i, j)] = Nu_at(c, i, j);
            Gu[iu(c, i, j)] = Gu_at(c, c->p, i, j);
            Lu[iu(c, i, j)] = Lu_at(c, i, j);
        }
    for (int j = v_j0(c); j < v_j1(c); ++j)
        for (int i = 0; i < nx; ++i) {
            Nv[iv(c, i, j)] = Nv_at(c, i, j);
            Gv[iv(c, i, j)] = Gv_at(c, c->p, i, j);
            Lv[iv(c, i, j)] = Lv_at(c, i, j);
        }
}

/* Cell divergence D(u)_ij = (u_{i+1,j}-u_ij)/dx_i + (v_{i,j+1}-v_ij)/dy_j. */
static double div_at(const orc_ctx *c, int i, int j) {
    return (U(c, i + 1, j) - U(c, i, j)) / c->dx[i] + (V(c, i, j + 1) - V(c, i, j)) / c->dy[j];
}
void orc_divergence(const orc_ctx *c, double *out) {
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) out[ic(c, i, j)] = div_at(c, i, j);
}

/* ------------------------------------------------------------------------ */
/* Helmholtz (implicit viscous) solves  (I - beta L) x = rhs  by red-black   */
/* SOR, in place on the u or v array.  Boundary values (inflow, outlet,      */
/* walls) are held fixed.  Tested every iteration against                    */
/* ||rhs - (I - beta L) x||_2 <= tol ||rhs||_2 (||rhs|| = 0 -> absolute).    */
/* ------------------------------------------------------------------------ */
static void helm_u_colour(orc_ctx *c, const double *rhs, double beta, double omega, int colour) {
    const int ny = c->ny, per = c->per;
    const int i0 = u_i0(c), i1 = u_i1(c);
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j) {
        int is = i0 + (((i0 + j + colour) & 1) ? 1 : 0);
        for (int i = is; i < i1; i += 2) {
            double ce = 1.0 / (DX(c, i) * c->dxu[i]);
            double cw = 1.0 / (DX(c, i - 1) * c->dxu[i]);
            double s = ce * U(c, i + 1, j) + cw * U(c, i - 1, j);
            double cs = ce + cw;
            if (per || j < ny - 1) { double a = 1.0 / (c->dyv[j + 1] * c->dy[j]); s += a * U(c, i, j + 1); cs += a; }
            if (per || j > 0) { double a = 1.0 / (c->dyv[j] * c->dy[j]); s += a * U(c, i, j - 1); cs += a; }
            double g = (rhs[iu(c, i, j)] + beta * s) / (1.0 + beta * cs);
            c->u[iu(c, i, j)] = (1.0 - omega) * c->u[iu(c, i, j)] + omega * g;
        }
    }
    if (per) for (int j = 0; j < ny; ++j) c->u[iu(c, c->nx, j)] = c->u[iu(c, 0, j)];
}
static void helm_v_colour(orc_ctx *c, const double *rhs, double beta, double omega, int colour) {
    const int nx = c->nx, per = c->per;
    const int j0 = v_j0(c), j1 = v_j1(c);
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = j0; j < j1; ++j) {
        for (int i = (j + colour) & 1; i < nx; i += 2) {
            double cn = 1.0 / (DY(c, j) * c->dyv[j]);
            double cso = 1.0 / (DY(c, j - 1) * c->dyv[j]);
            double s = cn * V(c, i, j + 1) + cso * V(c, i, j - 1);
            double cs = cn + cso;
            if (per || i < nx - 1) { double a = 1.0 / (c->dxu[i + 1] * c->dx[i]); s += a * V(c, i + 1, j); cs += a; }
            if (per || i > 0) { double a = 1.0 / (c->dxu[i] * c->dx[i]); s += a * V(c, i - 1, j); cs += a; }
            else { double a = 1.0 / (c->dxu[0] * c->dx[0]); s += a * 0.0; cs += a; }
            double g = (rhs[iv(c, i, j)] + beta * s) / (1.0 + beta * cs);
            c->v[iv(c, i, j)] = (1.0 - omega) * c->v[iv(c, i, j)] + omega * g;
        }
    }
    if (per) for (int i = 0; i < nx; ++i) c->v[iv(c, i, c->ny)] = c->v[iv(c, i, 0)];
}
static double helm_u_resid(orc_ctx *c, const double *rhs, double beta, double *rnorm_rhs) {
    const int ny = c->ny;
    const int i0 = u_i0(c), i1 = u_i1(c), w = i1 - i0;
    double *r = c->w0, *b = c->w1;
    for (int j = 0; j < ny; ++j)
        for (int i = i0; i < i1; ++i) {
            size_t k = (size_t)j * w + (i - i0);
            r[k] = rhs[iu(c, i, j)] - (U(c, i, j) - beta * Lu_at(c, i, j));
            b[k] = rhs[iu(c, i, j)];
        }
    *rnorm_rhs = sqrt(sumsq(b, (size_t)w * ny));
    return sqrt(sumsq(r, (size_t)w * ny));
}
static double helm_v_resid(orc_ctx *c, const double *rhs, double beta, double *rnorm_rhs) {
    const int nx = c->nx;
    const int j0 = v_j0(c), j1 = v_j1(c), h = j1 - j0;
    double *r = c->w0, *b = c->w1;
    for (int j = j0; j < j1; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)(j - j0) * nx + i;
            r[k] = rhs[iv(c, i, j)] - (V(c, i, j) - beta * Lv_at(c, i, j));
            b[k] = rhs[iv(c, i, j)];
        }
    *rnorm_rhs = sqrt(sumsq(b, (size_t)h * nx));
    return sqrt(sumsq(r, (size_t)h * nx));
}
static int helm_solve(orc_ctx *c, int comp, const double *rhs, double beta, int *iters) {
    const double omega = c->P.uv_omega, tol = c->P.uv_tol;
    const int max_iter = c->P.uv_max_iter;
    double bn, rn = comp == 0 ? helm_u_resid(c, rhs, beta, &bn) : helm_v_resid(c, rhs, beta, &bn);
    double den = bn > 0.0 ? bn : 1.0;
    *iters = 0;
    if (!isfinite(rn) || !isfinite(bn)) return ORC_ERR_NAN;
    if (rn <= tol * den) return ORC_OK;
    for (int it = 1; it <= max_iter; ++it) {
        if (comp == 0) { helm_u_colour(c, rhs, beta, omega, 0); helm_u_colour(c, rhs, beta, omega, 1); }
        else { helm_v_colour(c, rhs, beta, omega, 0); helm_v_colour(c, rhs, beta, omega, 1); }
        rn = comp == 0 ? helm_u_resid(c, rhs, beta, &bn) : helm_v_resid(c, rhs, beta, &bn);
        *iters = it;
        if (!isfinite(rn)) return ORC_ERR_NAN;
        if (rn <= tol * den) return ORC_OK;
    }
    return ORC_NOT_CONVERGED;
}

/* ------------------------------------------------------------------------ */
/* Body: kinematics, classification, forcing                                */
/* ------------------------------------------------------------------------ */

/* Plunge kinematics (Eqs. 1-2) with k = 2 pi f (c = U = 1 scaling):
 * y_c = y0 + h sin(2 pi f t + phase), its velocity and acceleration. */
static void kinematics(const orc_params *P, double t, double *yb, double *vb, double *ab) {
    const double pi = 3.14159265358979323846;
    double om = 2.0 * pi * P->freq, ph = om * t + P->phase;
    *yb = P->y0 + P->amp * sin(ph);
    *vb = om * P->amp * cos(ph);
    *ab = -om * om * P->amp * sin(ph);
}

/* Strict inside test of the ellipse with semi-axes a (x) and b (y). */
static int inside(double x, double y, double xb, double yb, double a, double b) {
    double ex = (x - xb) / a, ey = (y - yb) / b;
    return ex * ex + ey * ey < 1.0;
}

typedef struct { double xb, yb, a, b; } body_pos;

static int in_u(const orc_ctx *c, const body_pos *bp, int i, int j) {
    return inside(c->xf[i], c->yc[j], bp->xb, bp->yb, bp->a, bp->b);
}
static int in_v(const orc_ctx *c, const body_pos *bp, int i, int j) {
    return inside(c->xc[i], c->yf[j], bp->xb, bp->yb, bp->a, bp->b);
}

/* Number of forced faces of cell (i, j) under the current flags. */
static int forced_faces(const orc_ctx *c, int i, int j) {
    return (c->flu[iu(c, i, j)] != 0) + (c->flu[iu(c, i + 1, j)] != 0) + (c->flv[iv(c, i, j)] != 0) +
           (c->flv[iv(c, i, j + 1)] != 0);
}

/* Flag every u and v unknown (fluid / forcing / deep) and every cell (mass
 * source or not) for the body at bp.  Forcing = inside with at least one of
 * its four same-component neighbours outside; deep = all four inside; a
 * mass-source cell has at least one forced face. */
static void classify(orc_ctx *c, const body_pos *bp, int *nfu, int *nfv, int *nms) {
    const int nx = c->nx, ny = c->ny;
    memset(c->flu, 0, (size_t)(nx + 1) * ny);
    memset(c->flv, 0, (size_t)nx * (ny + 1));
    memset(c->msrc, 0, (size_t)nx * ny);
    *nfu = *nfv = *nms = 0;
    if (!c->P.body) return;
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            if (!in_u(c, bp, i, j)) continue;
            int all = in_u(c, bp, i + 1, j) && in_u(c, bp, i - 1, j) && in_u(c, bp, i, j + 1) && in_u(c, bp, i, j - 1);
            c->flu[iu(c, i, j)] = all ? FL_DEEP : FL_FORCING;
            ++*nfu;
        }
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (!in_v(c, bp, i, j)) continue;
            int all = in_v(c, bp, i + 1, j) && in_v(c, bp, i - 1, j) && in_v(c, bp, i, j + 1) && in_v(c, bp, i, j - 1);
            c->flv[iv(c, i, j)] = all ? FL_DEEP : FL_FORCING;
            ++*nfv;
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (forced_faces(c, i, j) > 0) { c->msrc[ic(c, i, j)] = 1; ++*nms; }
}

/* Interpolation weight along one grid line: the forced node sits d_f inside
 * the boundary crossing, the outside node d_o outside it. */
static double alpha_of(double df, double dout, double amax) {
    double al = dout > 0.0 ? df / dout : amax;
    if (al > amax) al = amax;
    if (al < 0.0) al = 0.0;
    return al;
}

/* Forcing target at a forcing u node: for each outside neighbour (E, W, N, S)
 * linear extrapolation through the boundary value ub at the crossing,
 * V_o = ub + (ub - ut_o) alpha; the mean over outside neighbours. */
static double target_u(const orc_ctx *c, const body_pos *bp, const double *ut, int i, int j, double ub) {
    const double amax = c->P.alpha_max;
    double sum = 0.0;
    int cnt = 0;
    double sy = 1.0 - ((c->yc[j] - bp->yb) / bp->b) * ((c->yc[j] - bp->yb) / bp->b);
    if (sy < 0.0) sy = 0.0;
    double sx = 1.0 - ((c->xf[i] - bp->xb) / bp->a) * ((c->xf[i] - bp->xb) / bp->a);
    if (sx < 0.0) sx = 0.0;
    if (!in_u(c, bp, i + 1, j)) {
        double xbd = bp->xb + bp->a * sqrt(sy);
        double al = alpha_of(xbd - c->xf[i], c->xf[i + 1] - xbd, amax);
        sum += ub + (ub - ut[iu(c, i + 1, j)]) * al; ++cnt;
    }
    if (!in_u(c, bp, i - 1, j)) {
        double xbd = bp->xb - bp->a * sqrt(sy);
        double al = alpha_of(c->xf[i] - xbd, xbd - c->xf[i - 1], amax);
        sum += ub + (ub - ut[iu(c, i - 1, j)]) * al; ++cnt;
    }
    if (!in_u(c, bp, i, j + 1)) {
        double ybd = bp->yb + bp->b * sqrt(sx);
        double al = alpha_of(ybd - c->yc[j], c->yc[j + 1] - ybd, amax);
        sum += ub + (ub - ut[iu(c, i, j + 1)]) * al; ++cnt;
    }
    if (!in_u(c, bp, i, j - 1)) {
        double ybd = bp->yb - bp->b * sqrt(sx);
        double al = alpha_of(c->yc[j] - ybd, ybd - c->yc[j - 1], amax);
        sum += ub + (ub - ut[iu(c, i, j - 1)]) * al; ++cnt;
    }
    return sum / cnt;
}

static double target_v(const orc_ctx *c, const body_pos *bp, const double *vt, int i, int j, double vb) {
    const double amax = c->P.alpha_max;
    double sum = 0.0;
    int cnt = 0;
    double sy = 1.0 - ((c->yf[j] - bp->yb) / bp->b) * ((c->yf[j] - bp->yb) / bp->b);
    if (sy < 0.0) sy = 0.0;
    double sx = 1.0 - ((c->xc[i] - bp->xb) / bp->a) * ((c->xc[i] - bp->xb) / bp->a);
    if (sx < 0.0) sx = 0.0;
    if (!in_v(c, bp, i + 1, j)) {
        double xbd = bp->xb + bp->a * sqrt(sy);
        double al = alpha_of(xbd - c->xc[i], c->xc[i + 1] - xbd, amax);
        sum += vb + (vb - vt[iv(c, i + 1, j)]) * al; ++cnt;
    }
    if (!in_v(c, bp, i - 1, j)) {
        double xbd = bp->xb - bp->a * sqrt(sy);
        double al = alpha_of(c->xc[i] - xbd, xbd - c->xc[i - 1], amax);
        sum += vb + (vb - vt[iv(c, i - 1, j)]) * al; ++cnt;
    }
    if (!in_v(c, bp, i, j + 1)) {
        double ybd = bp->yb + bp->b * sqrt(sx);
        double al = alpha_of(ybd - c->yf[j], c->yf[j + 1] - ybd, amax);
        sum += vb + (vb - vt[iv(c, i, j + 1)]) * al; ++cnt;
    }
    if (!in_v(c, bp, i, j - 1)) {
        double ybd = bp->yb - bp->b * sqrt(sx);
        double al = alpha_of(c->yf[j] - ybd, ybd - c->yf[j - 1], amax);
        sum += vb + (vb - vt[iv(c, i, j - 1)]) * al; ++cnt;
    }
    return sum / cnt;
}

static void body_at(const orc_ctx *c, double t, body_pos *bp, double *vb, double *ab) {
    double yb;
    kinematics(&c->P, t, &yb, vb, ab);
    bp->xb = c->P.x0;
    bp->yb = yb;
    bp->a = 0.5 * c->P.chord;
    bp->b = 0.5 * c->P.thick * c->P.chord;
}

/* ------------------------------------------------------------------------ */
/* One time step                                                            */
/* ------------------------------------------------------------------------ */
static int worst(int a, int b) {
    if (a < 0 || b < 0) return a < b ? a : b;
    return a > b ? a : b;
}

/* Convective outflow (channel mode): the outlet velocity of row j advected
 * with the free-stream speed, u* = u^n - dt U (u^n_nx - u^n_{nx-1}) / dx_{nx-1}
 * (a first-order upwind step of du/dt + U du/dx = 0 at the outlet face). */
static double outlet_predictor(const orc_ctx *c, int j) {
    const int nx = c->nx;
    double uo = U(c, nx, j), ui = U(c, nx - 1, j);
    return uo - c->P.dt * c->P.uinf * (uo - ui) / c->dx[nx - 1];
}

static int step_once(orc_ctx *c, orc_step_stats *st) {
    const int nx = c->nx, ny = c->ny, per = c->per;
    const double dt = c->P.dt, re = c->P.re, beta = dt / (2.0 * re);
    const double t1 = (double)(c->step + 1) * dt;
    int status = ORC_OK;
    memset(st, 0, sizeof(*st));

    /* body at the new time level, flags */
    body_pos bp;
    double vbody, abody;
    body_at(c, t1, &bp, &vbody, &abody);
    int nfu, nfv, nms;
    classify(c, &bp, &nfu, &nfv, &nms);
    st->n_forced_u = nfu; st->n_forced_v = nfv; st->n_msrc = nms;

    /* explicit momentum: N^n, then R and the predictor u~ */
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = u_i0(c); i < u_i1(c); ++i) c->nwu[iu(c, i, j)] = Nu_at(c, i, j);
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = v_j0(c); j < v_j1(c); ++j)
        for (int i = 0; i < nx; ++i) c->nwv[iv(c, i, j)] = Nv_at(c, i, j);
    if (!c->have_hist) {
        memcpy(c->nu, c->nwu, sizeof(double) * (nx + 1) * ny);
        memcpy(c->nv, c->nwv, sizeof(double) * nx * (ny + 1));
        c->have_hist = 1;
    }
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j)
        for (int i = u_i0(c); i < u_i1(c); ++i) {
            size_t k = iu(c, i, j);
            double L = Lu_at(c, i, j);
            double R = c->u[k] + dt * (-(1.5 * c->nwu[k] - 0.5 * c->nu[k]) - Gu_at(c, c->p, i, j) + (0.5 / re) * L);
            c->ru[k] = R;
            c->ut[k] = R + beta * L;
        }
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = v_j0(c); j < v_j1(c); ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = iv(c, i, j);
            double L = Lv_at(c, i, j);
            double R = c->v[k] + dt * (-(1.5 * c->nwv[k] - 0.5 * c->nv[k]) - Gv_at(c, c->p, i, j) + (0.5 / re) * L);
            c->rv[k] = R;
            c->vt[k] = R + beta * L;
        }
    memcpy(c->nu, c->nwu, sizeof(double) * (nx + 1) * ny);
    memcpy(c->nv, c->nwv, sizeof(double) * nx * (ny + 1));

    /* convective outlet: u* = u^n - dt U (u^n_nx - u^n_{nx-1}) / dx_{nx-1} */
    if (!per) {
        for (int j = 0; j < ny; ++j) c->ut[iu(c, nx, j)] = outlet_predictor(c, j);
        for (int j = 0; j < ny; ++j) c->u[iu(c, nx, j)] = c->ut[iu(c, nx, j)];
    }

    /* discrete forcing at forced nodes, R += dt f */
    memset(c->fu, 0, sizeof(double) * (nx + 1) * ny);
    memset(c->fv, 0, sizeof(double) * nx * (ny + 1));
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            size_t k = iu(c, i, j);
            if (c->flu[k] == FL_FLUID) continue;
            double Vt = c->flu[k] == FL_DEEP ? 0.0 : target_u(c, &bp, c->ut, i, j, 0.0);
            c->fu[k] = (Vt - c->ut[k]) / dt;
            c->ru[k] += dt * c->fu[k];
        }
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = iv(c, i, j);
            if (c->flv[k] == FL_FLUID) continue;
            double Vt = c->flv[k] == FL_DEEP ? vbody : target_v(c, &bp, c->vt, i, j, vbody);
            c->fv[k] = (Vt - c->vt[k]) / dt;
            c->rv[k] += dt * c->fv[k];
        }

    /* implicit viscous half: (I - beta L) u^ = R + dt f, in place from u^n */
    int it;
    int rc = helm_solve(c, 0, c->ru, beta, &it);
    st->u_iters = it; status = worst(status, rc);
    rc = helm_solve(c, 1, c->rv, beta, &it);
    st->v_iters = it; status = worst(status, rc);
    if (status < 0) { st->status = status; return status; }

    /* Poisson right-hand side  V b = V (D(u^) - q) / dt.  The mass source q
     * is the part of the divergence carried by forced faces in excess of the
     * body velocity, so D(u^) - q is the divergence of u^ with every forced
     * face replaced by the body velocity (0, vbody). */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double d = div_at(c, i, j);
            double q = 0.0;
            if (c->P.q_mode == 1 && c->msrc[ic(c, i, j)]) {
                double fe = c->flu[iu(c, i + 1, j)] ? U(c, i + 1, j) - 0.0 : 0.0;
                double fw = c->flu[iu(c, i, j)] ? U(c, i, j) - 0.0 : 0.0;
                double fn = c->flv[iv(c, i, j + 1)] ? V(c, i, j + 1) - vbody : 0.0;
                double fs = c->flv[iv(c, i, j)] ? V(c, i, j) - vbody : 0.0;
                q = (fe - fw) / c->dx[i] + (fn - fs) / c->dy[j];
            } else if (c->P.q_mode == 2 && c->msrc[ic(c, i, j)] && forced_faces(c, i, j) < 4) {
                /* the alternative reading kept for comparison: q is the whole
                 * divergence of a cut cell (at least one forced and one free
                 * face), so the Poisson source vanishes there */
                q = d;
            }
            c->vb[ic(c, i, j)] = (c->dx[i] * c->dy[j]) * ((d - q) / dt);
        }

    /* pressure-correction solve */
    if (!c->P.p_init_prev) memset(c->phi, 0, sizeof(double) * nx * ny);
    orc_solve_stats ss;
    rc = poisson_solve_vb(c, c->vb, c->phi, c->P.p_method, c->P.p_omega, c->P.p_tol, c->P.p_max_iter,
                          c->P.p_check, 0, &ss);
    st->p_iters = ss.iters; st->p_r0 = ss.r0_rel; st->p_rel = ss.rel;
    status = worst(status, rc);
    if (status < 0) { st->status = status; return status; }

    /* projection and pressure update */
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = 0; j < ny; ++j) {
        for (int i = u_i0(c); i < u_i1(c); ++i) c->u[iu(c, i, j)] -= dt * Gu_at(c, c->phi, i, j);
        if (!per) c->u[iu(c, nx, j)] -= dt * (0.0 - C(c, c->phi, nx - 1, j)) / c->dxu[nx];
    }
#pragma omp parallel for schedule(static) if (c->nx * c->ny >= ORC_OMP_MIN_CELLS)
    for (int j = v_j0(c); j < v_j1(c); ++j)
        for (int i = 0; i < nx; ++i) c->v[iv(c, i, j)] -= dt * Gv_at(c, c->phi, i, j);
    sync_periodic(c);
    orc_apply_A(c, c->phi, c->w0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = ic(c, i, j);
            c->p[k] += c->phi[k] - beta * (c->w0[k] / (c->dx[i] * c->dy[j]));
        }

    /* aerodynamic forces from the forcing (sequential, row-major) */
    double fx = 0.0, fy = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i)
            if (c->flu[iu(c, i, j)]) fx -= c->fu[iu(c, i, j)] * (c->dxu[i] * c->dy[j]);
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (c->flv[iv(c, i, j)]) fy -= c->fv[iv(c, i, j)] * (c->dx[i] * c->dyv[j]);
    if (c->P.body) {
        const double pi = 3.14159265358979323846;
        fy += pi * bp.a * bp.b * abody;
    }
    double uref = c->P.uinf != 0.0 ? c->P.uinf : 1.0;
    double qn = 0.5 * uref * uref * c->P.chord;
    c->cd = qn > 0.0 ? fx / qn : 0.0;
    c->cl = qn > 0.0 ? fy / qn : 0.0;

    c->step += 1;
    c->t = t1;
    st->cd = c->cd; st->cl = c->cl; st->t = c->t;
    st->status = status;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Public interface                                                         */
/* ------------------------------------------------------------------------ */

static void *xalloc(size_t n) {
    void *p = calloc(n ? n : 1, 1);
    return p;
}

void orc_destroy(orc_ctx *c) {
    if (!c) return;
    double *ds[] = {c->xf, c->yf, c->dx, c->dy, c->xc, c->yc, c->dxu, c->dyv, c->u, c->v, c->p, c->phi,
                    c->nu, c->nv, c->ru, c->rv, c->ut, c->vt, c->fu, c->fv, c->nwu, c->nwv, c->vb, c->w0,
                    c->w1, c->w2, c->w3, c->w4, c->w5, c->w6};
    for (size_t k = 0; k < sizeof(ds) / sizeof(ds[0]); ++k) free(ds[k]);
    free(c->flu); free(c->flv); free(c->msrc);
    free(c);
}

/* Create a context.  xf[nx+1], yf[ny+1]: face coordinates (strictly
 * increasing).  u0, v0, p0 may be NULL (then u = U, v = 0, p = 0); the
 * Dirichlet values (u at the inflow face, v on the walls) are always
 * overwritten by the boundary conditions in channel mode. */
int orc_create(const orc_params *P, const double *xf, const double *yf, const double *u0, const double *v0,
               const double *p0, orc_ctx **out) {
    *out = NULL;
    if (!P || P->nx < 4 || P->ny < 4 || (P->nx & 1) || (P->ny & 1) || !(P->dt > 0.0) || !(P->re > 0.0))
        return ORC_ERR_INVALID;
    if (P->bc != ORC_CHANNEL && P->bc != ORC_PERIODIC) return ORC_ERR_INVALID;
    if (P->q_mode < 0 || P->q_mode > 2) return ORC_ERR_INVALID;
    const int nx = P->nx, ny = P->ny;
    for (int i = 0; i < nx; ++i) if (!(xf[i + 1] > xf[i])) return ORC_ERR_INVALID;
    for (int j = 0; j < ny; ++j) if (!(yf[j + 1] > yf[j])) return ORC_ERR_INVALID;
    orc_ctx *c = (orc_ctx *)xalloc(sizeof(orc_ctx));
    c->P = *P;
    c->nx = nx; c->ny = ny; c->per = P->bc == ORC_PERIODIC;
    size_t nu = (size_t)(nx + 1) * ny, nv = (size_t)nx * (ny + 1), nc = (size_t)nx * ny;
    size_t nw = nu > nv ? nu : nv;
    c->xf = xalloc(sizeof(double) * (nx + 1)); c->yf = xalloc(sizeof(double) * (ny + 1));
    c->dx = xalloc(sizeof(double) * nx); c->dy = xalloc(sizeof(double) * ny);
    c->xc = xalloc(sizeof(double) * nx); c->yc = xalloc(sizeof(double) * ny);
    c->dxu = xalloc(sizeof(double) * (nx + 1)); c->dyv = xalloc(sizeof(double) * (ny + 1));
    c->u = xalloc(sizeof(double) * nu); c->v = xalloc(sizeof(double) * nv);
    c->p = xalloc(sizeof(double) * nc); c->phi = xalloc(sizeof(double) * nc);
    c->nu = xalloc(sizeof(double) * nu); c->nv = xalloc(sizeof(double) * nv);
    c->nwu = xalloc(sizeof(double) * nu); c->nwv = xalloc(sizeof(double) * nv);
    c->ru = xalloc(sizeof(double) * nu); c->rv = xalloc(sizeof(double) * nv);
    c->ut = xalloc(sizeof(double) * nu); c->vt = xalloc(sizeof(double) * nv);
    c->fu = xalloc(sizeof(double) * nu); c->fv = xalloc(sizeof(double) * nv);
    c->vb = xalloc(sizeof(double) * nc);
    c->w0 = xalloc(sizeof(double) * nw); c->w1 = xalloc(sizeof(double) * nw);
    c->w2 = xalloc(sizeof(double) * nw); c->w3 = xalloc(sizeof(double) * nw);
    c->w4 = xalloc(sizeof(double) * nw);
    c->w5 = xalloc(sizeof(double) * nw); c->w6 = xalloc(sizeof(double) * nw);
    c->flu = xalloc(nu); c->flv = xalloc(nv); c->msrc = xalloc(nc);

    memcpy(c->xf, xf, sizeof(double) * (nx + 1));
    memcpy(c->yf, yf, sizeof(double) * (ny + 1));
    for (int i = 0; i < nx; ++i) { c->dx[i] = xf[i + 1] - xf[i]; c->xc[i] = 0.5 * (xf[i] + xf[i + 1]); }
    for (int j = 0; j < ny; ++j) { c->dy[j] = yf[j + 1] - yf[j]; c->yc[j] = 0.5 * (yf[j] + yf[j + 1]); }
    for (int i = 1; i < nx; ++i) c->dxu[i] = c->xc[i] - c->xc[i - 1];
    for (int j = 1; j < ny; ++j) c->dyv[j] = c->yc[j] - c->yc[j - 1];
    if (c->per) {
        c->dxu[0] = c->dxu[nx] = 0.5 * (c->dx[nx - 1] + c->dx[0]);
        c->dyv[0] = c->dyv[ny] = 0.5 * (c->dy[ny - 1] + c->dy[0]);
    } else {
        c->dxu[0] = 0.5 * c->dx[0]; c->dxu[nx] = 0.5 * c->dx[nx - 1];
        c->dyv[0] = 0.5 * c->dy[0]; c->dyv[ny] = 0.5 * c->dy[ny - 1];
    }

    if (P->body) {
        double a = 0.5 * P->chord, b = 0.5 * P->thick * P->chord, amp = fabs(P->amp);
        if (!(a > 0.0) || !(b > 0.0) || c->per) { orc_destroy(c); return ORC_ERR_INVALID; }
        /* the body's whole range of motion stays two cells clear of the boundary */
        if (!(P->x0 - a > xf[2]) || !(P->x0 + a < xf[nx - 2]) || !(P->y0 - amp - b > yf[2]) ||
            !(P->y0 + amp + b < yf[ny - 2])) {
            orc_destroy(c);
            return ORC_ERR_INVALID;
        }
    }

    for (size_t k = 0; k < nu; ++k) c->u[k] = u0 ? u0[k] : P->uinf;
    for (size_t k = 0; k < nv; ++k) c->v[k] = v0 ? v0[k] : 0.0;
    for (size_t k = 0; k < nc; ++k) c->p[k] = p0 ? p0[k] : 0.0;
    if (!c->per) {
        for (int j = 0; j < ny; ++j) c->u[iu(c, 0, j)] = P->uinf;
        for (int i = 0; i < nx; ++i) { c->v[iv(c, i, 0)] = 0.0; c->v[iv(c, i, ny)] = 0.0; }
    } else {
        sync_periodic(c);
    }
    c->have_hist = 0;
    c->step = 0;
    c->t = 0.0;
    *out = c;
    return ORC_OK;
}

int orc_step(orc_ctx *c, int nsteps, orc_step_stats *stats) {
    int status = ORC_OK;
    for (int s = 0; s < nsteps; ++s) {
        orc_step_stats st;
        int rc = step_once(c, &st);
        if (stats) stats[s] = st;
        status = worst(status, rc);
        if (rc < 0) break;
    }
    return status;
}

void orc_get_fields(const orc_ctx *c, double *u, double *v, double *p, double *phi) {
    const int nx = c->nx, ny = c->ny;
    if (u) memcpy(u, c->u, sizeof(double) * (nx + 1) * ny);
    if (v) memcpy(v, c->v, sizeof(double) * nx * (ny + 1));
    if (p) memcpy(p, c->p, sizeof(double) * nx * ny);
    if (phi) memcpy(phi, c->phi, sizeof(double) * nx * ny);
}

/* V b of the last pressure solve (a time step's, after the zero-mean
 * projection in the periodic mode, or orc_poisson_solve's), natural layout. */
void orc_get_rhs(const orc_ctx *c, double *vb) {
    memcpy(vb, c->vb, sizeof(double) * c->nx * c->ny);
}

void orc_set_fields(orc_ctx *c, const double *u, const double *v, const double *p) {
    const int nx = c->nx, ny = c->ny;
    if (u) memcpy(c->u, u, sizeof(double) * (nx + 1) * ny);
    if (v) memcpy(c->v, v, sizeof(double) * nx * (ny + 1));
    if (p) memcpy(c->p, p, sizeof(double) * nx * ny);
    sync_periodic(c);
}

/* Flags and forcing of the last step: flu, flv (0 fluid, 1 forcing, 2 deep),
 * msrc (1 = mass-source cell), fu, fv (forcing per unit mass). */
void orc_get_ibm(const orc_ctx *c, unsigned char *flu, unsigned char *flv, unsigned char *msrc, double *fu,
                 double *fv) {
    const int nx = c->nx, ny = c->ny;
    if (flu) memcpy(flu, c->flu, (size_t)(nx + 1) * ny);
    if (flv) memcpy(flv, c->flv, (size_t)nx * (ny + 1));
    if (msrc) memcpy(msrc, c->msrc, (size_t)nx * ny);
    if (fu) memcpy(fu, c->fu, sizeof(double) * (nx + 1) * ny);
    if (fv) memcpy(fv, c->fv, sizeof(double) * nx * (ny + 1));
}

/* Classify for the body at time t (no state change besides the flag arrays). */
void orc_classify_at(orc_ctx *c, double t, int32_t *counts) {
    body_pos bp;
    double vb, ab;
    int a, b, m;
    body_at(c, t, &bp, &vb, &ab);
    classify(c, &bp, &a, &b, &m);
    if (counts) { counts[0] = a; counts[1] = b; counts[2] = m; }
}

/* Forcing targets for given predictor fields ut, vt with the body at time t
 * (classifies first).  Vu, Vv receive the target at every forced node. */
void orc_targets_at(orc_ctx *c, double t, const double *ut, const double *vt, double *Vu, double *Vv) {
    const int nx = c->nx, ny = c->ny;
    body_pos bp;
    double vbody, ab;
    int a, b, m;
    body_at(c, t, &bp, &vbody, &ab);
    classify(c, &bp, &a, &b, &m);
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            size_t k = iu(c, i, j);
            if (c->flu[k] == FL_FLUID) continue;
            Vu[k] = c->flu[k] == FL_DEEP ? 0.0 : target_u(c, &bp, ut, i, j, 0.0);
        }
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = iv(c, i, j);
            if (c->flv[k] == FL_FLUID) continue;
            Vv[k] = c->flv[k] == FL_DEEP ? vbody : target_v(c, &bp, vt, i, j, vbody);
        }
}

/* Implicit viscous solve of one component (0: u, 1: v) on the current
 * fields: (I - beta L) x = rhs by the step's red-black SOR, in place from the
 * current u or v, boundary values held fixed.  rhs has the shape of u or v
 * (entries off the unknowns are ignored).  Returns the status; *iters the
 * iterations taken. */
int orc_helm_solve(orc_ctx *c, int comp, const double *rhs, double beta, int *iters) {
    if (comp != 0 && comp != 1) return ORC_ERR_INVALID;
    return helm_solve(c, comp, rhs, beta, iters);
}

/* Convective-outlet predictor u* of every row for the current fields
 * (channel mode; out[ny]). */
int orc_outlet_predictor(const orc_ctx *c, double *out) {
    if (c->per) return ORC_ERR_INVALID;
    for (int j = 0; j < c->ny; ++j) out[j] = outlet_predictor(c, j);
    return ORC_OK;
}

/* Body centre height, velocity and acceleration at time t (Eqs. 1-2). */
void orc_kinematics(const orc_ctx *c, double t, double *yb, double *vb, double *ab) {
    kinematics(&c->P, t, yb, vb, ab);
}

void orc_forces(const orc_ctx *c, double *cd, double *cl) {
    *cd = c->cd;
    *cl = c->cl;
}

double orc_time(const orc_ctx *c) { return c->t; }
long orc_step_count(const orc_ctx *c) { return c->step; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Sizes of the parameter and stats blocks, so the Python mirror can check
 * its layout. */
int orc_sizeof_params(void) { return (int)sizeof(orc_params); }
int orc_sizeof_step_stats(void) { return (int)sizeof(orc_step_stats); }
int orc_sizeof_solve_stats(void) { return (int)sizeof(orc_solve_stats); }
