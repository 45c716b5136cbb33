// ibm_device.hpp -- device-side types and helpers shared by the gfx950 kernels
// of the immersed-boundary fractional-step solver (arXiv 2402.17337).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibm {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kBlock = 256;     // threads per block of the 2-D kernels (64 x 4)
constexpr int kBlockRows = 4;   // rows per block of the 2-D kernels

// Device view of the grid metrics.  All arrays live in the workspace.
//   dx[i] = xf[i+1]-xf[i], xc[i] cell centre, dxu[i] centre distance across
//   x-face i (half cells dx[0]/2, dx[nx-1]/2 at the ends); same in y.
// Pressure operator A = V D G, row (i, j):
//   a_E = dy_j pcE[i], a_W = dy_j pcW[i], a_N = dx_i pcN[j], a_S = dx_i pcS[j]
//   (zero on Neumann faces), outlet diagonal term dy_j pcD[i] at i = nx-1;
//   (A x)_ij = sum a_nb x_nb - (sum a_nb + outlet) x_ij.
// Viscous operator L (finite volume, per unit control volume):
//   u node (i, j): L u = uce[i](uE-uP) + ucw[i](uW-uP) + ucn[j](uN-uP) + ucs[j](uS-uP)
//   v node (i, j): L v = vcn[j](vN-vP) + vcs[j](vS-vP) + vce[i](vE-vP) + vcw[i](vW-vP)
//   with ucn/ucs zero at the slip walls, vce zero at the outlet (zero
//   gradient) and vcw[0] pointing at v = 0 on the inflow face.
// Periodic mode (per = 1, both directions periodic, no body): every
// coefficient is nonzero, the centre distances across the two ends are
// (dx[nx-1] + dx[0]) / 2 and (dy[ny-1] + dy[0]) / 2, neighbours wrap
// (cell nx-1's east neighbour is cell 0), u faces 0..nx-1 and v faces
// 0..ny-1 are the unknowns, and u face nx / v face row ny mirror face 0.
struct Grid {
    int nx, ny, nh;  // nh = nx / 2 (cells of one colour in a row)
    int per;         // 0: channel boundaries; 1: periodic
    const double *xf, *yf, *dx, *dy, *xc, *yc, *dxu, *dyv;
    const double *pcE, *pcW, *pcD, *pcN, *pcS;
    const double *uce, *ucw, *ucn, *ucs;
    const double *vce, *vcw, *vcn, *vcs;
};

// Body position of the current step.
struct Body {
    double xb, yb, a, b;  // centre and semi-axes
    double vb, ab;        // plunge velocity and acceleration
    int present;
};

// Control block of one iterative solve.  Written only by the finalising
// block of a reduction kernel, read by every kernel of the solve.
enum : int { kRunning = 0, kDone = 1 };
enum : int { kStOk = 0, kStNotConverged = 1, kStNan = -5, kStConfirm = 7 };

struct Ctl {
    int done;       // 1: the solve has finished (converged, limit or NaN)
    int status;     // kSt*
    int iters;      // iterations when it finished (or latest check)
    int zero_rhs;   // 1: ||rhs|| = 0, solution is 0
    double bn;      // ||rhs||
    double r0;      // initial residual norm
    double rn;      // latest residual norm
    double rz[2];   // PCG: r.z of iteration k in rz[k & 1]
    double al[2];   // one-reduction CG: alpha of iteration k in al[k & 1]
};

// Host-mapped snapshot of a control block after a check.
struct Slot {
    int done, status, iters, zero_rhs;
    double bn, r0, rn;
};

// ---------------------------------------------------------------------------
// reductions (deterministic for a fixed launch shape)
// ---------------------------------------------------------------------------
// Cross-lane move of a double by a DPP control (both 32-bit halves); lanes
// with no source, and the lanes of rows outside ROWS, receive 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_move_d(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROWS, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave (every lane active), returned in every lane: prefix sums
// within each row of 16 lanes (row_shr 1, 2, 4, 8), then row 0's total into
// row 1 and row 2's into row 3 (row_bcast:15), then lane 31 into rows 2 and 3
// (row_bcast:31); lane 63 holds the total.  A fixed order, so deterministic.
template <int N>
__device__ inline void wave_sum(double (&v)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double x = v[k];
        x += dpp_move_d<0x111, 0xf>(x);
        x += dpp_move_d<0x112, 0xf>(x);
        x += dpp_move_d<0x114, 0xf>(x);
        x += dpp_move_d<0x118, 0xf>(x);
        x += dpp_move_d<0x142, 0xa>(x);
        x += dpp_move_d<0x143, 0xc>(x);
        const long long bits = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_readlane((int)bits, kWave - 1);
        const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), kWave - 1);
        v[k] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}

// Sum over the block; the result is valid in every lane of wave 0.
// lds must hold N * (blockDim.x / 64) doubles.
template <int N>
__device__ inline void block_sum(double (&v)[N], double* lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    wave_sum(v);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[k * nw + w] = v[k];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = lane < nw ? lds[k * nw + lane] : 0.0;
        wave_sum(v);
    }
}

// Cross-block reductions without fences: a producer kernel writes one
// partial per block with plain stores; a later kernel in the stream (after
// the kernel boundary has made them visible) sums the nb partials in index
// order.  Deterministic for a fixed launch shape.  Reduction kernels use at
// most kRedMax blocks (grid-stride loops), so a consumer can afford to sum
// all partials in every block.
constexpr int kRedMax = 256;      // blocks of a reduction kernel
constexpr int kRedThreads = 1024; // threads per block of a reduction kernel

template <int N>
__device__ inline void block_partials(double (&v)[N], double* partials, int nb, int slot, double* lds) {
    block_sum(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) partials[(size_t)k * nb + slot] = v[k];
    }
}

// Sum of the nb partials of each of N quantities; valid in wave 0.
template <int N>
__device__ inline void sum_partials(double (&v)[N], const double* partials, int nb, double* lds) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += partials[(size_t)k * nb + q];
    }
    block_sum(v, lds);
}

__device__ inline void publish(const Ctl* ctl, Slot* hs) {
    if (!hs) return;
    hs->done = ctl->done;
    hs->status = ctl->status;
    hs->iters = ctl->iters;
    hs->zero_rhs = ctl->zero_rhs;
    hs->bn = ctl->bn;
    hs->r0 = ctl->r0;
    hs->rn = ctl->rn;
    __threadfence_system();
}

// Stop test shared by every residual check.  phase 0: first check (sets bn,
// r0); later phases: after `it` iterations.  den0 selects the denominator used
// when ||rhs|| = 0 (1: absolute test, 0: the solution is zero).
__device__ inline void check_finish(Ctl* ctl, double r2, double b2, int phase, int it, int max_iter,
                                    double tol, int fixed, int den_one_if_zero) {
    const double rn = sqrt(r2);
    ctl->rn = rn;
    if (phase == 0) {
        const double bn = sqrt(b2);
        ctl->bn = bn;
        ctl->r0 = rn;
        ctl->iters = 0;
        ctl->zero_rhs = 0;
        if (!isfinite(rn) || !isfinite(bn)) { ctl->done = kDone; ctl->status = kStNan; return; }
        if (bn == 0.0 && !den_one_if_zero) { ctl->done = kDone; ctl->status = kStOk; ctl->zero_rhs = 1; return; }
        const double den = bn > 0.0 ? bn : 1.0;
        if (rn <= tol * den) { ctl->done = kDone; ctl->status = kStOk; return; }
        ctl->done = kRunning;
        ctl->status = kStOk;
        return;
    }
    ctl->iters = it;
    const double den = ctl->bn > 0.0 ? ctl->bn : 1.0;
    if (!isfinite(rn)) { ctl->done = kDone; ctl->status = kStNan; return; }
    if (rn <= tol * den) { ctl->done = kDone; ctl->status = kStOk; return; }
    if (it >= max_iter) { ctl->done = kDone; ctl->status = fixed ? kStOk : kStNotConverged; return; }
}


// Strict inside test of the ellipse, evaluated without contraction so that it
// takes exactly the decision of a plain IEEE evaluation.
__device__ inline bool inside(double x, double y, const Body& B) {
#pragma clang fp contract(off)
    const double ex = (x - B.xb) / B.a, ey = (y - B.yb) / B.b;
    return ex * ex + ey * ey < 1.0;
}

}  // namespace ibm
