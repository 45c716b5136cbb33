// ibm_kernels.hpp -- gfx950 kernels of one time step of the discrete-forcing
// immersed-boundary fractional-step solver (arXiv 2402.17337, Sec. 2.2).
//
// Layouts (FP64, row-major, x fastest):
//   u[(nx+1)*ny] x-faces, v[nx*(ny+1)] y-faces, p/phi/vb[nx*ny] centres.
//   Red-black split storage for the pressure sweeps: row j of the red array
//   holds the nx/2 cells with (i+j) even, i = 2m + (j&1); the black array the
//   cells with (i+j) odd, i = 2m + 1 - (j&1).  Both colours of a row are
//   contiguous, so a colour sweep reads and writes unit-stride rows.
//
// The pointwise kernels of the step (momentum, forcing, right-hand side,
// projection) evaluate their formulas without floating-point contraction, in
// the operand order of a plain evaluation; the sweeps and reductions of the
// iterative solvers use fused multiply-adds.
#pragma once

#include "ibm_device.hpp"

namespace ibm {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void k_ctl_reset(Ctl* ctl, int n) {
    const int t = threadIdx.x;
    if (t < n) {
        Ctl c = {};
        ctl[t] = c;
    }
}

__global__ void k_fill(double* a, size_t n, double val) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = val;
}

__global__ void k_fill_u8(uint8_t* a, size_t n) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = 0;
}

// Natural -> red/black split (optionally multiplied by the cell volume).
__global__ __launch_bounds__(kBlock) void k_split(Grid g, const double* __restrict__ nat, double* __restrict__ red,
                                                  double* __restrict__ black, int by_volume) {
#pragma clang fp contract(off)
    const int m = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    if (m >= g.nh || j >= g.ny) return;
    const int ir = 2 * m + (j & 1), ib = 2 * m + 1 - (j & 1);
    const size_t k = (size_t)j * g.nh + m;
    const double xr = nat[(size_t)j * g.nx + ir], xb = nat[(size_t)j * g.nx + ib];
    if (by_volume) {
        red[k] = (g.dx[ir] * g.dy[j]) * xr;
        black[k] = (g.dx[ib] * g.dy[j]) * xb;
    } else {
        red[k] = xr;
        black[k] = xb;
    }
}

__global__ __launch_bounds__(kBlock) void k_merge(Grid g, const double* __restrict__ red,
                                                  const double* __restrict__ black, double* __restrict__ nat) {
    const int m = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    if (m >= g.nh || j >= g.ny) return;
    const int ir = 2 * m + (j & 1), ib = 2 * m + 1 - (j & 1);
    const size_t k = (size_t)j * g.nh + m;
    nat[(size_t)j * g.nx + ir] = red[k];
    nat[(size_t)j * g.nx + ib] = black[k];
}

// ---------------------------------------------------------------------------
// Pressure Poisson: red-black SOR on A phi = V b in split storage
// ---------------------------------------------------------------------------
// Neighbour sum and diagonal of row (i, j) of A with explicit fused
// multiply-adds, so that every kernel that forms them rounds alike:
//   sum = aE xE + aW xW + aN xN + aS xS   (absent neighbours: a = 0, x = 0)
//   d   = (((aE + aD) + aW) + aN) + aS    (aD: outlet term, nonzero at i = nx-1)
// with aE = dy_j pcE_i, aW = dy_j pcW_i, aD = dy_j pcD_i, aN = dx_i pcN_j,
// aS = dx_i pcS_j; the coefficient arrays are zero on Neumann faces.  The CG
// kernels and the refinement of the mixed-precision solve use this form.
__device__ inline double rb_sum(double aE, double xE, double aW, double xW, double aN, double xN, double aS,
                                double xS) {
    double sum = aE * xE;
    sum = __fma_rn(aW, xW, sum);
    sum = __fma_rn(aN, xN, sum);
    return __fma_rn(aS, xS, sum);
}
__device__ inline double rb_diag(double aE, double aD, double aW, double aN, double aS) {
    return (((aE + aD) + aW) + aN) + aS;
}
__device__ inline float rb_diag(float aE, float aD, float aW, float aN, float aS) {
    return (((aE + aD) + aW) + aN) + aS;
}

// The red-black SOR kernels (every sweep and the residual of their stop
// test) take the neighbour sum with the grid spacings factored out,
//   sum = dy_j (pcE_i xE + pcW_i xW) + dx_i (pcN_j xN + pcS_j xS),
// three multiplications and three fused multiply-adds, and the update
//   phi <- (sum - V b) wrd + (1 - omega) phi,   wrd = omega (1/d),
// three more; 1/d is the reciprocal of rb_diag of the products above.
__device__ inline double sor_sum(double dy, double cE, double xE, double cW, double xW, double dx, double pn,
                                 double xN, double ps, double xS) {
    const double ew = __fma_rn(cW, xW, cE * xE);
    const double ns = __fma_rn(ps, xS, pn * xN);
    return __fma_rn(dx, ns, dy * ew);
}
__device__ inline double sor_step(double x, double sum, double b, double wrd, double omx) {
    return __fma_rn(sum - b, wrd, omx * x);
}
// The same two operations in single precision (the mixed-precision sweeps).
__device__ inline float sor_sum(float dy, float cE, float xE, float cW, float xW, float dx, float pn, float xN,
                                float ps, float xS) {
    const float ew = __fmaf_rn(cW, xW, cE * xE);
    const float ns = __fmaf_rn(ps, xS, pn * xN);
    return __fmaf_rn(dx, ns, dy * ew);
}
__device__ inline float sor_step(float x, float sum, float b, float wrd, float omx) {
    return __fmaf_rn(sum - b, wrd, omx * x);
}

// Neighbour sum (sor_sum) and diagonal of row (i, j) of A, reading the other
// colour (split index k of the cell, s = its position parity in the row).
__device__ inline double rb_row(const Grid& g, const double* __restrict__ other, int i, int j, size_t k, int s,
                                double& d) {
    const double dyj = g.dy[j], dxi = g.dx[i];
    const double pE = g.pcE[i], pW = g.pcW[i], pN = g.pcN[j], pS = g.pcS[j];
    // periodic mode wraps: cell nx-1's east neighbour is position 0 of the
    // row, cell 0's west neighbour position nh-1, rows ny-1 and 0 are
    // neighbours (same position: the colours alternate, nx and ny are even)
    const size_t nh = g.nh, top = (size_t)(g.ny - 1) * g.nh;
    const double xE = i < g.nx - 1 ? other[k + s] : (g.per ? other[k + 1 - nh] : 0.0);
    const double xW = i > 0 ? other[k + s - 1] : (g.per ? other[k + nh - 1] : 0.0);
    const double xN = j < g.ny - 1 ? other[k + nh] : (g.per ? other[k - top] : 0.0);
    const double xS = j > 0 ? other[k - nh] : (g.per ? other[k + top] : 0.0);
    d = rb_diag(dyj * pE, dyj * g.pcD[i], dyj * pW, dxi * pN, dxi * pS);
    return sor_sum(dyj, pE, xE, pW, xW, dxi, pN, xN, pS, xS);
}

// One colour of a red-black SOR iteration (one launch per colour):
//   phi_P <- (1 - omega) phi_P + omega (sum a_nb phi_nb - V b_P) / (sum a_nb + a_D)
// COLOR 0 updates the red cells ((i+j) even), COLOR 1 the black cells.  A
// thread owns split position m and walks kSwRows rows of it (a block: 64
// positions by kBlockRows such strips), keeping the other colour's values at
// its position in rows j-1, j and j+1 in registers: per cell it loads phi,
// V b, the other colour one row up and the one east/west neighbour that is
// not at its own position, and stores phi; the x coefficients of its two
// cells (i = 2m and 2m + 1) are loaded once.  Each cell's arithmetic is that
// of rb_row and sor_step, so the iterates are those of every other SOR kernel.
constexpr int kSwRows = 8;

template <int S>
__device__ inline void sweep_cell(const Grid& g, double* __restrict__ self, const double* __restrict__ other,
                                  const double* __restrict__ bself, double wom, double omx, int m, int j,
                                  const double (&cdx)[2], const double (&cE)[2], const double (&cW)[2],
                                  const double (&cD)[2], double& xS, double& xC) {
    // periodic mode wraps: cell nx-1's east neighbour is position 0 of the
    // row, cell 0's west neighbour position nh-1, rows ny-1 and 0 are
    // neighbours (same position: the colours alternate, nx and ny are even)
    const size_t nh = g.nh, k = (size_t)j * nh + m;
    const int i = 2 * m + S;
    const double xN = j < g.ny - 1 ? other[k + nh] : (g.per ? other[m] : 0.0);
    double xE, xW;
    if (S) {
        xW = xC;
        xE = i < g.nx - 1 ? other[k + 1] : (g.per ? other[k + 1 - nh] : 0.0);
    } else {
        xE = xC;
        xW = i > 0 ? other[k - 1] : (g.per ? other[k + nh - 1] : 0.0);
    }
    const double dyj = g.dy[j], dxi = cdx[S], pN = g.pcN[j], pS = g.pcS[j];
    const double d = rb_diag(dyj * cE[S], dyj * cD[S], dyj * cW[S], dxi * pN, dxi * pS);
    const double sum = sor_sum(dyj, cE[S], xE, cW[S], xW, dxi, pN, xN, pS, xS);
    self[k] = sor_step(self[k], sum, bself[k], wom * (1.0 / d), omx);
    xS = xC;
    xC = xN;
}

template <int COLOR>
__global__ __launch_bounds__(kBlock) void k_sor_sweep(Grid g, double* __restrict__ self,
                                                      const double* __restrict__ other,
                                                      const double* __restrict__ bself, double omega,
                                                      const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int m = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j0 = (blockIdx.y * kBlockRows + threadIdx.x / kWave) * kSwRows;  // even
    if (m >= g.nh || j0 >= g.ny) return;
    const int j1 = min(j0 + kSwRows, g.ny);
    double cdx[2], cE[2], cW[2], cD[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = 2 * m + q;
        cdx[q] = g.dx[i];
        cE[q] = g.pcE[i];
        cW[q] = g.pcW[i];
        cD[q] = g.pcD[i];
    }
    const size_t nh = g.nh;
    double xS = j0 > 0 ? other[(size_t)(j0 - 1) * nh + m] : (g.per ? other[(size_t)(g.ny - 1) * nh + m] : 0.0);
    double xC = other[(size_t)j0 * nh + m];
    const double omx = 1.0 - omega;
    // rows in pairs: the even row's cell sits at position parity COLOR, the
    // odd row's at the other one
#pragma unroll 2
    for (int j = j0; j < j1; j += 2) {
        sweep_cell<COLOR & 1>(g, self, other, bself, omega, omx, m, j, cdx, cE, cW, cD, xS, xC);
        if (j + 1 < j1) sweep_cell<(COLOR + 1) & 1>(g, self, other, bself, omega, omx, m, j + 1, cdx, cE, cW, cD, xS, xC);
    }
}

// Residual r = V b - A phi over both colours: per-block partial sums of r^2
// and (V b)^2 (grid-stride over the split positions, at most kRedMax blocks).
__global__ __launch_bounds__(kRedThreads) void k_sor_residual(Grid g, const double* __restrict__ red,
                                                              const double* __restrict__ black,
                                                              const double* __restrict__ bred,
                                                              const double* __restrict__ bblack, const Ctl* ctl,
                                                              double* partials) {
    __shared__ double lds[2 * kRedThreads / kWave];
    if (ctl->done) return;
    double acc[2] = {0.0, 0.0};
    const size_t n = (size_t)g.nh * g.ny;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / g.nh), m = (int)(k - (size_t)j * g.nh);
        {
            const int s = j & 1, i = 2 * m + s;
            double d;
            const double sum = rb_row(g, black, i, j, k, s, d);
            const double r = bred[k] - (sum - d * red[k]);
            acc[0] += r * r;
            acc[1] += bred[k] * bred[k];
        }
        {
            const int s = (j + 1) & 1, i = 2 * m + s;
            double d;
            const double sum = rb_row(g, red, i, j, k, s, d);
            const double r = bblack[k] - (sum - d * black[k]);
            acc[0] += r * r;
            acc[1] += bblack[k] * bblack[k];
        }
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// One block: sum the residual partials (r^2, b^2) and run the stop test of a
// solve (phase 0 = before the first iteration).  den_one: ||rhs|| = 0 turns
// the test absolute instead of meaning a zero solution.
__global__ __launch_bounds__(kRedThreads) void k_check(Ctl* ctl, const double* __restrict__ partials, int nb,
                                                       int phase, int it, int max_iter, double tol, int fixed,
                                                       int den_one, Slot* hs) {
    __shared__ double lds[2 * kRedThreads / kWave];
    if (ctl->done) {
        if (threadIdx.x == 0) publish(ctl, hs);
        return;
    }
    double acc[2];
    sum_partials(acc, partials, nb, lds);
    if (threadIdx.x == 0) {
        check_finish(ctl, acc[0], acc[1], phase, it, max_iter, tol, fixed, den_one);
        publish(ctl, hs);
    }
}

// ---------------------------------------------------------------------------
// Temporally blocked red-black SOR.  One block per tile: the tile interior
// plus a halo of depth H (clamped to the domain) is loaded into LDS in split
// layout, S red-black iterations run there, and the interior is written back.
// After h half-sweeps only cells farther than h-1 from the loaded edge are
// still exact, so with H >= 2S (+1 when the residual of the interior is
// summed at the end) the interior equals S global iterations bit for bit: each
// cell is updated by sor_step with the same neighbour values.  The tiles
// read one pair of split arrays and write the other (a tile's halo is another
// tile's interior, and blocks of one launch run in no fixed order).  Half-sweep h
// updates the rows within e_h = 2S - h (+1) of the interior, whole: a cell of
// such a row farther than e_h in x takes a value that is no exact iterate,
// but inexact values spread one cell per half-sweep from the loaded edge and
// stop two cells short of the interior (H = 2S + 2); at a domain edge the LDS
// holds a ring of zeros (the coefficient of an absent neighbour is zero as
// well), and lanes without a cell hold phi = V b = 1/d = 0, which the update
// keeps at zero.
//
// Work layout: lane l of every wave owns split column l of the loaded tile
// (at most 64 columns, i.e. a loaded width of 128 cells); wave w owns rows
// w + 16 r (r < kTbRows), so the position parity of a wave's colour-C cell
// is the same in all its rows and the x coefficients of a lane are fixed per
// colour.  A thread keeps phi, V b and 1/d of its cells in registers (it is
// the only writer of phi); the LDS copy of phi serves the neighbours.  The LDS
// pitch is fixed, so every neighbour address is a register plus a constant.
// ---------------------------------------------------------------------------
constexpr int kTbThreads = 1024;
// the stop tests (k_check, the check block of a sweep launch, the batched
// checks) all sum partials with this many threads, so in the same order
static_assert(kTbThreads == kRedThreads, "one thread count for every stop test");
constexpr int kTbWaves = kTbThreads / kWave;   // 16
constexpr int kTbRows = 6;                     // rows per wave (even): loaded height <= 96
constexpr int kTbCols = kWave;                 // split columns: loaded width <= 128
constexpr int kTbPitch = kTbCols + 2;          // LDS row: ghost, 64 columns, ghost
constexpr int kTbLdsRows = kTbWaves * kTbRows + 2;
constexpr int kTbLds = kTbLdsRows * kTbPitch;  // doubles per colour
constexpr int kTbGroup = 2;                    // rows whose reads are issued together
static_assert(kTbRows % 2 == 0 && kTbRows % kTbGroup == 0, "strips start on even rows; rows go in groups");

struct TbShape {
    int tx, ty;    // interior tile size (tx even)
    int halo;      // H = 2S + 2
    int ntx, nty;  // tiles in x and y
    int per;       // tiles per XCD band: block b takes tile (b % 8) * per + b / 8
};

// Stop test of the previous check interval, carried by the first blocked
// launch of the next one (nb = 0: none in this launch).
struct TbCheck {
    const double* partials;  // residual partials of that interval: nb sums of r^2, then nb of b^2
    int nb;
    int it;                  // iterations at the test
    int max_iter, fixed;
    double tol;
    Slot* slot;              // host-visible snapshot of the decision
};

// Start of a tile block of a blocked launch: the solve's stop flag as the
// control block holds it when the block starts (block-uniform).
__device__ inline int tb_begin(const Ctl* ctl, int* s_flag) {
    if (threadIdx.x == 0) *s_flag = ctl->done;
    __syncthreads();
    return *s_flag;
}

// The carried test of a blocked launch, taken by one extra block of the
// launch (block 8 * per, past the tiles) so that no tile block waits for it:
// it sums the previous interval's partials in the order k_check's callers
// use (a kTbThreads block) and records the stop decision in ctl and in the
// host-visible snapshot.  The tiles of the same launch do not wait for the
// decision: after a finishing test they still sweep into the other pair of
// phi arrays, which does not hold the result, and every later launch of the
// solve returns at once.
__device__ inline void tb_check_block(Ctl* ctl, const TbCheck& chk, double* lds, int* s_flag) {
    if (threadIdx.x == 0) *s_flag = ctl->done;
    __syncthreads();
    if (!*s_flag) {
        double acc[2];
        sum_partials(acc, chk.partials, chk.nb, lds);
        if (threadIdx.x == 0) check_finish(ctl, acc[0], acc[1], 1, chk.it, chk.max_iter, chk.tol, chk.fixed, 0);
    }
    if (threadIdx.x == 0) publish(ctl, chk.slot);
}

// Whether this block of a blocked launch is its check block.
__device__ inline bool tb_is_check_block(const TbCheck& chk, const TbShape& ts) {
    return chk.nb > 0 && (int)blockIdx.x == 8 * ts.per;
}

// Tile of block b.  Blocks are dispatched to the 8 XCDs round-robin, so each
// XCD gets a contiguous band of tiles and the halos its tiles share stay in
// its L2.  The launch has 8 * per blocks; those past the last tile return.
__device__ inline int tb_tile(const TbShape& ts) { return (blockIdx.x & 7) * ts.per + (blockIdx.x >> 3); }

__global__ __launch_bounds__(kTbThreads) void k_sor_tb(Grid g, const double* __restrict__ red,
                                                       const double* __restrict__ black, double* __restrict__ ored,
                                                       double* __restrict__ oblack, const double* __restrict__ bred,
                                                       const double* __restrict__ bblack,
                                                       double omega, Ctl* ctl, TbCheck chk, TbShape ts,
                                                       int nsweep, int residual, double* __restrict__ partials) {
    __shared__ double tile[2 * kTbLds];
    __shared__ double lds[2 * kTbWaves];
    __shared__ int s_flag;
    if (tb_is_check_block(chk, ts)) {
        tb_check_block(ctl, chk, lds, &s_flag);
        return;
    }
    const int nt = ts.ntx * ts.nty;
    const int t = tb_tile(ts);
    if (t >= nt) return;
    if (tb_begin(ctl, &s_flag)) return;
    const int txi = t % ts.ntx, tyi = t / ts.ntx;
    const int X0 = txi * ts.tx, Y0 = tyi * ts.ty;
    const int X1 = min(X0 + ts.tx, g.nx), Y1 = min(Y0 + ts.ty, g.ny);
    const int H = ts.halo;
    const int xa = max(0, X0 - H), xb = min(g.nx, X1 + H);
    const int ya = max(0, Y0 - H), yb = min(g.ny, Y1 + H);
    const int lxh = (xb - xa) >> 1, ly = yb - ya;
    const int m0 = xa >> 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave index, uniform
    const bool col = lane < lxh;

    // zero ring (and everything outside the loaded tile)
    for (int k = threadIdx.x; k < 2 * kTbLds; k += kTbThreads) tile[k] = 0.0;

    // per colour C: position parity s of the lane's cells, their x
    // coefficients and their x distance from the interior (far if no cell)
    const int ic = 2 * (m0 + lane);
    double cdx[2], cE[2], cW[2], cD[2];
    int sC[2], dist[2];
    const double omx = 1.0 - omega;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        sC[c] = (ya + w + c) & 1;
        const int i = ic + sC[c];
        const int ii = col ? i : 0;
        cdx[c] = g.dx[ii];
        cE[c] = g.pcE[ii];
        cW[c] = g.pcW[ii];
        cD[c] = g.pcD[ii];
        dist[c] = col ? max(max(X0 - i, i - (X1 - 1)), 0) : (1 << 20);
    }
    // per row: wave-uniform coefficients and y distance from the interior
    double rdy[kTbRows], rpn[kTbRows], rps[kTbRows];
    int rdist[kTbRows];
    double x[2][kTbRows], b[2][kTbRows], wrd[2][kTbRows];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTbRows; ++r) {
        const int jl = w + kTbWaves * r;
        const int j = min(ya + jl, g.ny - 1);
        rdy[r] = g.dy[j];
        rpn[r] = g.pcN[j];
        rps[r] = g.pcS[j];
        rdist[r] = jl < ly ? max(max(Y0 - j, j - (Y1 - 1)), 0) : (1 << 20);
#pragma unroll
        for (int c = 0; c < 2; ++c) x[c][r] = b[c][r] = wrd[c][r] = 0.0;
        if (jl < ly && col) {
            const size_t kg = (size_t)(ya + jl) * g.nh + m0 + lane;
            x[0][r] = red[kg];
            x[1][r] = black[kg];
            b[0][r] = bred[kg];
            b[1][r] = bblack[kg];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double d = rb_diag(rdy[r] * cE[c], rdy[r] * cD[c], rdy[r] * cW[c], cdx[c] * rpn[r],
                                         cdx[c] * rps[r]);
                wrd[c][r] = omega * (1.0 / d);
            }
            const int p = (jl + 1) * kTbPitch + lane + 1;
            tile[p] = x[0][r];
            tile[kTbLds + p] = x[1][r];
        }
    }
    __syncthreads();

    const int p0 = (w + 1) * kTbPitch + lane + 1;  // LDS position of row 0 of this thread
    const int extra = residual ? 1 : 0;
    for (int it = 0; it < nsweep; ++it) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // red half-sweep h = 2 it + 1, black h = 2 it + 2: cells within e of the interior
            const int e = 2 * nsweep - (2 * it + 1 + c) + extra;
            double* self = tile + c * kTbLds;
            const double* other = tile + (1 - c) * kTbLds;
            const int pe = p0 + sC[c];  // east neighbour of row 0 in the other colour
            // rows in groups of kTbGroup: the group's reads, then its updates
#pragma unroll
            for (int r0 = 0; r0 < kTbRows; r0 += kTbGroup) {
                double vE[kTbGroup], vW[kTbGroup], vN[kTbGroup], vS[kTbGroup];
#pragma unroll
                for (int q = 0; q < kTbGroup; ++q) {
                    // in bounds for every row slot (ghost rows 0 and 65)
                    const int o = (r0 + q) * kTbWaves * kTbPitch;
                    vE[q] = other[pe + o];
                    vW[q] = other[pe + o - 1];
                    vN[q] = other[p0 + o + kTbPitch];
                    vS[q] = other[p0 + o - kTbPitch];
                }
#pragma unroll
                for (int q = 0; q < kTbGroup; ++q) {
                    const int r = r0 + q;
                    if (rdist[r] <= e) {
                        const double sum = sor_sum(rdy[r], cE[c], vE[q], cW[c], vW[q], cdx[c], rpn[r], vN[q],
                                                   rps[r], vS[q]);
                        x[c][r] = sor_step(x[c][r], sum, b[c][r], wrd[c][r], omx);
                        self[p0 + r * kTbWaves * kTbPitch] = x[c][r];
                    }
                }
            }
            __syncthreads();
        }
    }

    // interior back to global memory (both colours), and its residual
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kTbRows; ++r) {
        const int jl = w + kTbWaves * r;
        const int j = ya + jl;
        if (rdist[r] != 0) continue;  // rows of the interior only
        const size_t kg = (size_t)j * g.nh + m0 + lane;
        const int o = r * kTbWaves * kTbPitch;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (dist[c] != 0) continue;
            (c ? oblack : ored)[kg] = x[c][r];
            if (residual) {
                const double* other = tile + (1 - c) * kTbLds;
                const double xE = other[p0 + sC[c] + o], xW = other[p0 + sC[c] + o - 1];
                const double xN = other[p0 + o + kTbPitch], xS = other[p0 + o - kTbPitch];
                const double d = rb_diag(rdy[r] * cE[c], rdy[r] * cD[c], rdy[r] * cW[c], cdx[c] * rpn[r],
                                         cdx[c] * rps[r]);
                const double sum = sor_sum(rdy[r], cE[c], xE, cW[c], xW, cdx[c], rpn[r], xN, rps[r], xS);
                const double bb = b[c][r];
                const double rres = bb - (sum - d * x[c][r]);
                acc[0] += rres * rres;
                acc[1] += bb * bb;
            }
        }
    }
    if (residual) block_partials(acc, partials, nt, t, lds);
}

// ---------------------------------------------------------------------------
// Register-resident variant of the blocked sweep.  Same tile, halo, shrinking
// update region and arithmetic as k_sor_tb, so the interior again equals S
// global iterations bit for bit; only the data movement differs.  Wave w owns
// the kTbRows consecutive tile rows starting at kTbRows * w, lane l split
// column l (both colours), all in registers:
//   north/south neighbours: the thread's own next/previous row, or (at the
//     ends of the wave's strip) the neighbouring wave's edge row, exchanged
//     through LDS once per half-sweep;
//   east/west neighbours: the other colour in the same row, either in the
//     same lane or in the adjacent lane (a cross-lane move; lanes 0 and 63
//     read zero, the ghost value at a domain edge).
// ---------------------------------------------------------------------------
// Cross-lane moves over the whole wave: lane l receives lane l-1
// (from_lower_lane) or lane l+1 (from_upper_lane); the lane without a source
// receives 0.
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ inline float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <class T>
__device__ inline T from_lower_lane(T v) { return dpp_move<0x138>(v); }  // wave_shr:1
template <class T>
__device__ inline T from_upper_lane(T v) { return dpp_move<0x130>(v); }  // wave_shl:1

constexpr int kTrSlots = 2 * kTbWaves + 2;  // edge rows: zero, (first, last) per wave, zero

// The helpers below take the position parity P of the strip's first row as a
// template argument (the kernels use even tile heights, so P = 0): every index
// into the thread's small arrays is then a constant and the arrays stay in
// registers.

// A wave-uniform value as such (held in scalar registers: the row
// coefficients of a strip are the same in every lane).
__device__ inline double wave_uniform(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)bits), hi = __builtin_amdgcn_readfirstlane((int)(bits >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float wave_uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Stores the interior cells of v (colour 0 to o0, colour 1 to o1); row r of
// the strip is at split index kg0 + r nh.
template <int P, class T, class U>
__device__ inline void tbr_store(const T (&v)[2][kTbRows], U* __restrict__ o0, U* __restrict__ o1, size_t kg0,
                                 size_t nh, const int (&dq)[2], const int (&rdist)[kTbRows]) {
#pragma unroll
    for (int r = 0; r < kTbRows; ++r) {
        if (rdist[r] != 0) continue;  // rows of the interior only
        const int s0 = (P + r) & 1;   // position parity of the colour-0 cell
        if (dq[s0] == 0) o0[kg0 + r * nh] = v[0][r];
        if (dq[s0 ^ 1] == 0) o1[kg0 + r * nh] = v[1][r];
    }
}

// Sum of the neighbours of the colour-C cell of row r (position parity
// s = (P + r + C) & 1) in the thread's registers; xS0 / xNR are the other
// colour's rows below the strip and above it.  T = double, or float for the
// single-precision sweeps of the mixed-precision solve.
template <int C, int P, int R, class T>
__device__ inline T tbr_sum(const T (&x)[2][kTbRows], T xS0, T xNR, const T (&cdx)[2], const T (&cE)[2],
                            const T (&cW)[2], T dy, T pn, T ps) {
    constexpr int O = 1 - C;
    constexpr int s = (P + R + C) & 1;
    const T xo = x[O][R];
    T xE, xW;
    if (s) {
        xE = from_upper_lane(xo);
        xW = xo;
    } else {
        xE = xo;
        xW = from_lower_lane(xo);
    }
    const T xN = (R + 1 < kTbRows) ? x[O][R + 1 < kTbRows ? R + 1 : R] : xNR;
    const T xS = (R > 0) ? x[O][R > 0 ? R - 1 : 0] : xS0;
    return sor_sum(dy, cE[s], xE, cW[s], xW, cdx[s], pn, xN, ps, xS);
}

// Update of the colour-C cell of row R (whole rows: see the blocked sweep's
// notes); wrd = omega / d per cell, omx = 1 - omega.
template <int C, int P, int R, class T>
__device__ inline void tbr_row(T (&x)[2][kTbRows], const T (&b)[2][kTbRows], const T (&wrd)[2][kTbRows], T xS0,
                               T xNR, const T (&cdx)[2], const T (&cE)[2], const T (&cW)[2],
                               const T (&rdy)[kTbRows], const T (&rpn)[kTbRows], const T (&rps)[kTbRows],
                               const int (&rdist)[kTbRows], int e, T omx) {
    if (rdist[R] > e) return;  // wave-uniform
    const T sum = tbr_sum<C, P, R>(x, xS0, xNR, cdx, cE, cW, rdy[R], rpn[R], rps[R]);
    x[C][R] = sor_step(x[C][R], sum, b[C][R], wrd[C][R], omx);
}

// Rows R..R1-1 of one colour's half-sweep (unrolled at compile time, so every
// index into the thread's arrays is a constant).
template <int C, int P, class T, int R, int R1>
__device__ inline void tbr_rows(T (&x)[2][kTbRows], const T (&b)[2][kTbRows], const T (&wrd)[2][kTbRows], T xS0,
                                T xNR, const T (&cdx)[2], const T (&cE)[2], const T (&cW)[2],
                                const T (&rdy)[kTbRows], const T (&rpn)[kTbRows], const T (&rps)[kTbRows],
                                const int (&rdist)[kTbRows], int e, T omx) {
    if constexpr (R < R1) {
        tbr_row<C, P, R>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx);
        tbr_rows<C, P, T, R + 1, R1>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx);
    }
}

// One colour's half-sweep over the strip, and the store of its two strip-end
// rows into `edge` for the neighbouring waves.  The cells of one colour do not
// depend on each other, so the row order is free: half of the inner rows
// first, as the strip-end rows need the other waves' rows, read from LDS just
// before the half-sweep (the inner rows hide that read's latency); then the
// strip-end rows and their store; then the other inner rows, which hide the
// store's latency before the barrier that ends the half-sweep.
template <int C, int P, class T>
__device__ inline void tbr_half(T (&x)[2][kTbRows], const T (&b)[2][kTbRows], const T (&wrd)[2][kTbRows], T xS0,
                                T xNR, const T (&cdx)[2], const T (&cE)[2], const T (&cW)[2],
                                const T (&rdy)[kTbRows], const T (&rpn)[kTbRows], const T (&rps)[kTbRows],
                                const int (&rdist)[kTbRows], int e, T omx, T (&edge)[2][kTrSlots][kWave], int w,
                                int lane) {
    static_assert(kTbRows >= 3, "the strip needs inner rows");
    constexpr int M = 1 + (kTbRows - 2) / 2;
    tbr_rows<C, P, T, 1, M>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx);
    tbr_row<C, P, 0>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx);
    tbr_row<C, P, kTbRows - 1>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx);
    edge[C][2 * w + 1][lane] = x[C][0];
    edge[C][2 * w + 2][lane] = x[C][kTbRows - 1];
    tbr_rows<C, P, T, M, kTbRows - 1>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx);
}

// S red-black iterations on the thread's registers with the shrinking update
// region (rows within e = 2 S - h + extra at half-sweep h), exchanging the
// strip-end rows through `edge` after each half-sweep.  On entry `edge`
// holds both colours.
template <int P, class T>
__device__ inline void tbr_sweeps(T (&x)[2][kTbRows], const T (&b)[2][kTbRows], const T (&wrd)[2][kTbRows],
                                  const T (&cdx)[2], const T (&cE)[2], const T (&cW)[2], const T (&rdy)[kTbRows],
                                  const T (&rpn)[kTbRows], const T (&rps)[kTbRows], const int (&rdist)[kTbRows],
                                  T (&edge)[2][kTrSlots][kWave], int w, int lane, int nsweep, int extra, T omx) {
    for (int it = 0; it < nsweep; ++it) {
        {   // red half-sweep h = 2 it + 1
            const int e = 2 * nsweep - (2 * it + 1) + extra;
            const T xS0 = edge[1][2 * w][lane], xNR = edge[1][2 * w + 3][lane];
            tbr_half<0, P>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx, edge, w, lane);
            __syncthreads();
        }
        {   // black half-sweep h = 2 it + 2
            const int e = 2 * nsweep - (2 * it + 2) + extra;
            const T xS0 = edge[0][2 * w][lane], xNR = edge[0][2 * w + 3][lane];
            tbr_half<1, P>(x, b, wrd, xS0, xNR, cdx, cE, cW, rdy, rpn, rps, rdist, e, omx, edge, w, lane);
            __syncthreads();
        }
    }
}

// Writes both colours' strip-end rows (and, from wave 0, the zero slots).
template <class T>
__device__ inline void tbr_edges(const T (&x)[2][kTbRows], T (&edge)[2][kTrSlots][kWave], int w, int lane) {
    if (w == 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            edge[c][0][lane] = T(0);
            edge[c][kTrSlots - 1][lane] = T(0);
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        edge[c][2 * w + 1][lane] = x[c][0];
        edge[c][2 * w + 2][lane] = x[c][kTbRows - 1];
    }
}

// Residual b - (sum - d x) of the colour-C cell of row R, with d from the
// lane's coefficients.
template <int C, int P, int R>
__device__ inline double tbr_rvalue(const double (&x)[2][kTbRows], double bv, double xS0, double xNR,
                                    const double (&cdx)[2], const double (&cE)[2], const double (&cW)[2],
                                    const double (&cD)[2], const double (&rdy)[kTbRows],
                                    const double (&rpn)[kTbRows], const double (&rps)[kTbRows]) {
    constexpr int s = (P + R + C) & 1;
    const double sum = tbr_sum<C, P, R>(x, xS0, xNR, cdx, cE, cW, rdy[R], rpn[R], rps[R]);
    const double dy = rdy[R];
    const double d = rb_diag(dy * cE[s], dy * cD[s], dy * cW[s], cdx[s] * rpn[R], cdx[s] * rps[R]);
    return bv - (sum - d * x[C][R]);
}

// Residual contribution of the colour-C cell of row R (interior cells only).
template <int C, int P, int R>
__device__ inline void tbr_resid(const double (&x)[2][kTbRows], const double (&b)[2][kTbRows], double xS0, double xNR,
                                 const double (&cdx)[2], const double (&cE)[2], const double (&cW)[2],
                                 const double (&cD)[2], const int (&dq)[2], const double (&rdy)[kTbRows],
                                 const double (&rpn)[kTbRows], const double (&rps)[kTbRows],
                                 const int (&rdist)[kTbRows], double (&acc)[2]) {
    if (rdist[R] != 0) return;
    constexpr int s = (P + R + C) & 1;
    const double rres = tbr_rvalue<C, P, R>(x, b[C][R], xS0, xNR, cdx, cE, cW, cD, rdy, rpn, rps);
    if (dq[s] != 0) return;
    const double bb = b[C][R];
    acc[0] += rres * rres;
    acc[1] += bb * bb;
}

// Residual contributions of both colours of rows R..kTbRows-1.
template <int P, int R = 0>
__device__ inline void tbr_residual(const double (&x)[2][kTbRows], const double (&b)[2][kTbRows],
                                    const double (&xS0)[2], const double (&xNR)[2], const double (&cdx)[2],
                                    const double (&cE)[2], const double (&cW)[2], const double (&cD)[2],
                                    const int (&dq)[2], const double (&rdy)[kTbRows], const double (&rpn)[kTbRows],
                                    const double (&rps)[kTbRows], const int (&rdist)[kTbRows], double (&acc)[2]) {
    tbr_resid<0, P, R>(x, b, xS0[1], xNR[1], cdx, cE, cW, cD, dq, rdy, rpn, rps, rdist, acc);
    tbr_resid<1, P, R>(x, b, xS0[0], xNR[0], cdx, cE, cW, cD, dq, rdy, rpn, rps, rdist, acc);
    if constexpr (R + 1 < kTbRows)
        tbr_residual<P, R + 1>(x, b, xS0, xNR, cdx, cE, cW, cD, dq, rdy, rpn, rps, rdist, acc);
}

// One tile t of the register-resident blocked sweep (the body of k_sor_tbr and
// of its batched form): loads the tile with its halo, takes the stop test,
// performs nsweep iterations, stores the interior and, with residual, writes
// the tile's residual partials (slot t of nt).
__device__ __forceinline__ void tbr_tile(const Grid& g, const double* __restrict__ red,
                                         const double* __restrict__ black, double* __restrict__ ored,
                                         double* __restrict__ oblack, const double* __restrict__ bred,
                                         const double* __restrict__ bblack, double omega, Ctl* ctl,
                                         const TbCheck& chk, const TbShape& ts, int t, int nsweep, int residual,
                                         double* __restrict__ partials, double (&edge)[2][kTrSlots][kWave],
                                         double* lds, int* s_flag_ptr) {
    int& s_flag = *s_flag_ptr;
    const int nt = ts.ntx * ts.nty;
    const int txi = t % ts.ntx, tyi = t / ts.ntx;
    const int X0 = txi * ts.tx, Y0 = tyi * ts.ty;
    const int X1 = min(X0 + ts.tx, g.nx), Y1 = min(Y0 + ts.ty, g.ny);
    const int H = ts.halo;
    const int xa = max(0, X0 - H), xb = min(g.nx, X1 + H);
    const int ya = max(0, Y0 - H), yb = min(g.ny, Y1 + H);
    const int lxh = (xb - xa) >> 1, ly = yb - ya;
    const int m0 = xa >> 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave index, uniform
    const bool col = lane < lxh;
    const int jw = kTbRows * w;       // first tile row of the wave's strip
    // position parity of colour C in row r of the strip: (P + r + C) & 1; the
    // tile height is even, so the strip's first row ya + 4 w is even
    constexpr int P = 0;

    // x coefficients and distance from the interior of the lane's two cells,
    // by position parity q (cell i = ic + q)
    const int ic = 2 * (m0 + lane);
    double cdx[2], cE[2], cW[2], cD[2];
    int dq[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = ic + q;
        const int ii = col ? i : 0;
        cdx[q] = g.dx[ii];
        cE[q] = g.pcE[ii];
        cW[q] = g.pcW[ii];
        cD[q] = g.pcD[ii];
        dq[q] = col ? max(max(X0 - i, i - (X1 - 1)), 0) : (1 << 20);
    }
    double rdy[kTbRows], rpn[kTbRows], rps[kTbRows];
    int rdist[kTbRows];
    double x[2][kTbRows], b[2][kTbRows], wrd[2][kTbRows];
#pragma unroll
    for (int r = 0; r < kTbRows; ++r) {
        const int jl = jw + r;
        const int j = min(ya + jl, g.ny - 1);
        rdy[r] = wave_uniform(g.dy[j]);
        rpn[r] = wave_uniform(g.pcN[j]);
        rps[r] = wave_uniform(g.pcS[j]);
        rdist[r] = jl < ly ? max(max(Y0 - j, j - (Y1 - 1)), 0) : (1 << 20);
#pragma unroll
        for (int c = 0; c < 2; ++c) x[c][r] = b[c][r] = 0.0;
        if (jl < ly && col) {
            const size_t kg = (size_t)(ya + jl) * g.nh + m0 + lane;
            x[0][r] = red[kg];
            x[1][r] = black[kg];
            b[0][r] = bred[kg];
            b[1][r] = bblack[kg];
        }
        // omega / d of the thread's cells, formed while the loads are in
        // flight (colour c of row r sits at position parity (P + r + c) & 1)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int q = (P + r + c) & 1;
            const double d = rb_diag(rdy[r] * cE[q], rdy[r] * cD[q], rdy[r] * cW[q], cdx[q] * rpn[r],
                                     cdx[q] * rps[r]);
            wrd[c][r] = (jl < ly && col) ? omega * (1.0 / d) : 0.0;
        }
    }
    // The stop flag is read after the tile's loads are issued, so that its
    // latency overlaps theirs (a finished solve only wastes the loads).
    if (tb_begin(ctl, &s_flag)) return;
    // edge rows of both colours; slots 0 and kTrSlots-1 stay zero
    tbr_edges(x, edge, w, lane);
    __syncthreads();
    tbr_sweeps<P>(x, b, wrd, cdx, cE, cW, rdy, rpn, rps, rdist, edge, w, lane, nsweep, residual ? 1 : 0, 1.0 - omega);

    // interior back to global memory (both colours), and its residual
    const size_t kg0 = (size_t)(ya + jw) * g.nh + m0 + lane;
    tbr_store<P>(x, ored, oblack, kg0, (size_t)g.nh, dq, rdist);
    if (residual) {
        double acc[2] = {0.0, 0.0};
        const double xS0[2] = {edge[0][2 * w][lane], edge[1][2 * w][lane]};
        const double xNR[2] = {edge[0][2 * w + 3][lane], edge[1][2 * w + 3][lane]};
        tbr_residual<P>(x, b, xS0, xNR, cdx, cE, cW, cD, dq, rdy, rpn, rps, rdist, acc);
        block_partials(acc, partials, nt, t, lds);
    }
}

__global__ __launch_bounds__(kTbThreads) void k_sor_tbr(Grid g, const double* __restrict__ red,
                                                        const double* __restrict__ black, double* __restrict__ ored,
                                                        double* __restrict__ oblack, const double* __restrict__ bred,
                                                        const double* __restrict__ bblack,
                                                        double omega, Ctl* ctl, TbCheck chk, TbShape ts,
                                                        int nsweep, int residual, double* __restrict__ partials) {
    __shared__ double edge[2][kTrSlots][kWave];
    __shared__ double lds[2 * kTbWaves];
    __shared__ int s_flag;
    if (tb_is_check_block(chk, ts)) {
        tb_check_block(ctl, chk, lds, &s_flag);
        return;
    }
    const int t = tb_tile(ts);
    if (t >= ts.ntx * ts.nty) return;
    tbr_tile(g, red, black, ored, oblack, bred, bblack, omega, ctl, chk, ts, t, nsweep, residual, partials, edge,
             lds, &s_flag);
}

// Many independent grids ("cases") swept by one launch: case c's tiles are
// the global tiles [tile0, tile0 + ntiles) of a work list over all cases,
// taken by the blocks with the same XCD banding as one grid's tiles.  A case
// whose control block says it has finished skips its tiles.  Every case uses
// the pair `flip` of its split phi arrays as input and the other as output,
// and partial set `pbuf`; the iterates of each case are those of k_sor_tbr on
// that case alone.
struct TbCase {
    Grid g;
    double* ph[2][2];  // [pair][colour]
    const double *bred, *bblack;
    double* partials[2];
    Ctl* ctl;
    TbShape ts;
    double omega, tol;
    int tile0, ntiles, nb0, max_iter;
    int fixed;  // 1: max_iter is a replayed iteration count (tolerance ignored)
};

__global__ __launch_bounds__(kTbThreads) void k_sor_tbr_batch(const TbCase* __restrict__ cases, int ncase,
                                                              int ntotal, int per, int flip, int nsweep,
                                                              int residual, int pbuf) {
    __shared__ double edge[2][kTrSlots][kWave];
    __shared__ double lds[2 * kTbWaves];
    __shared__ int s_flag;
    const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (t >= ntotal) return;
    int lo = 0, hi = ncase - 1;  // last case with tile0 <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cases[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    const TbCase& C = cases[__builtin_amdgcn_readfirstlane(lo)];
    const TbCheck none = {nullptr, 0, 0, 0, 0, 0.0, nullptr};
    tbr_tile(C.g, C.ph[flip][0], C.ph[flip][1], C.ph[flip ^ 1][0], C.ph[flip ^ 1][1], C.bred, C.bblack, C.omega,
             C.ctl, none, C.ts, t - C.tile0, nsweep, residual, C.partials[pbuf], edge, lds, &s_flag);
}

// The stop tests of all cases of a batch, one block per case (blockDim: the
// block size of the check the single-grid solve would use, so that the sums
// and decisions are the same): phase 0 sums the nb0 partials of the initial
// residual, later phases the ntiles partials of set pbuf after `it`
// iterations.  Finished cases only republish.  With a cursor (cur non-null:
// {iteration base, snapshot entry}, written by k_batch_cursor) `it` counts
// from the base and the snapshots go to entry cur[1] of the slot ring, so
// that one captured sequence of launches serves every stretch of the solve.
__global__ __launch_bounds__(kTbThreads) void k_check_batch(const TbCase* __restrict__ cases, int phase, int it,
                                                            int pbuf, Slot* slots, const int* __restrict__ cur) {
    __shared__ double lds[2 * kTbWaves];
    if (cur) {
        it += cur[0];
        slots += (size_t)cur[1] * gridDim.x;
    }
    const TbCase& C = cases[blockIdx.x];
    if (C.ctl->done) {
        if (threadIdx.x == 0) publish(C.ctl, slots + blockIdx.x);
        return;
    }
    double acc[2];
    sum_partials(acc, phase == 0 ? C.partials[0] : C.partials[pbuf], phase == 0 ? C.nb0 : C.ntiles, lds);
    if (threadIdx.x == 0) {
        check_finish(C.ctl, acc[0], acc[1], phase, it, C.max_iter, C.tol, C.fixed, 0);
        publish(C.ctl, slots + blockIdx.x);
    }
}

// Sets the cursor read by the checks of a captured stretch of a batched solve.
__global__ void k_batch_cursor(int* cur, int base, int entry) {
    if (threadIdx.x == 0) {
        cur[0] = base;
        cur[1] = entry;
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision red-black SOR: single-precision sweeps on the correction
// equation, double-precision refinement.  A check interval of K iterations
// solves A e = r32 from e = 0 (e_zero on its first launch) with k_sor_mp,
// where r32 is the float rounding of the double residual at the interval's
// start; then k_mp_refine forms
//   x = phi + e   (double; written to the other phi pair),
//   r = V b - A x (double; summed into the stop-test partials, and rounded to
//                  float as the next interval's r32, into the other r32 pair).
// SOR is a stationary iteration, so these iterates equal the double-precision
// ones up to rounding relative to the correction.  The single-precision
// coefficients are products of the float-rounded 1-D arrays, and 1/d a float
// division.
// ---------------------------------------------------------------------------
struct MpArrays {
    const float *er, *eb;  // e in (unless e_zero)
    float *oer, *oeb;      // e out
    const float *rr, *rb;  // r32 in
};

// Tile t of the float sweeps (S iterations on A e = r32).
__device__ __forceinline__ void mp_tile(const Grid& g, const MpArrays& a, double omega, Ctl* ctl, const TbCheck& chk,
                                        const TbShape& ts, int t, int nsweep, int e_zero,
                                        float (&edge32)[2][kTrSlots][kWave], double* lds, int* s_flag) {
    const int txi = t % ts.ntx, tyi = t / ts.ntx;
    const int X0 = txi * ts.tx, Y0 = tyi * ts.ty;
    const int X1 = min(X0 + ts.tx, g.nx), Y1 = min(Y0 + ts.ty, g.ny);
    const int H = ts.halo;
    const int xa = max(0, X0 - H), xb = min(g.nx, X1 + H);
    const int ya = max(0, Y0 - H), yb = min(g.ny, Y1 + H);
    const int lxh = (xb - xa) >> 1, ly = yb - ya;
    const int m0 = xa >> 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave index, uniform
    const bool col = lane < lxh;
    const int jw = kTbRows * w;
    constexpr int P = 0;  // even tile height: the strip starts on an even row
    const int ic = 2 * (m0 + lane);
    const int ii0 = col ? ic : 0, ii1 = col ? ic + 1 : 0;
    const size_t kg0 = (size_t)(ya + jw) * g.nh + m0 + lane;  // row r of the strip: kg0 + r nh

    int dq[2];  // distance of the lane's cells i = ic + q from the interior
#pragma unroll
    for (int q = 0; q < 2; ++q) dq[q] = col ? max(max(X0 - (ic + q), (ic + q) - (X1 - 1)), 0) : (1 << 20);
    int rdist[kTbRows];
    float e[2][kTbRows], b32[2][kTbRows], wrd[2][kTbRows];
    const float fom = (float)omega;
    float fdx[2] = {(float)g.dx[ii0], (float)g.dx[ii1]};
    float fE[2] = {(float)g.pcE[ii0], (float)g.pcE[ii1]};
    float fW[2] = {(float)g.pcW[ii0], (float)g.pcW[ii1]};
    const float fD[2] = {(float)g.pcD[ii0], (float)g.pcD[ii1]};
    float fdy[kTbRows], fpn[kTbRows], fps[kTbRows];
#pragma unroll
    for (int r = 0; r < kTbRows; ++r) {
        const int jl = jw + r;
        const int j = min(ya + jl, g.ny - 1);
        rdist[r] = jl < ly ? max(max(Y0 - (ya + jl), (ya + jl) - (Y1 - 1)), 0) : (1 << 20);
        fdy[r] = wave_uniform((float)g.dy[j]);
        fpn[r] = wave_uniform((float)g.pcN[j]);
        fps[r] = wave_uniform((float)g.pcS[j]);
#pragma unroll
        for (int c = 0; c < 2; ++c) e[c][r] = b32[c][r] = 0.0f;
        if (jl < ly && col) {
            const size_t k = kg0 + (size_t)r * g.nh;
            if (!e_zero) {
                e[0][r] = a.er[k];
                e[1][r] = a.eb[k];
            }
            b32[0][r] = a.rr[k];
            b32[1][r] = a.rb[k];
        }
        // omega / d in single precision, from the products of the
        // float-rounded coefficients
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int q = (P + r + c) & 1;
            const float f = rb_diag(fdy[r] * fE[q], fdy[r] * fD[q], fdy[r] * fW[q], fdx[q] * fpn[r], fdx[q] * fps[r]);
            wrd[c][r] = (jl < ly && col) ? fom * (1.0f / f) : 0.0f;
        }
    }
    if (tb_begin(ctl, s_flag)) return;
    tbr_edges(e, edge32, w, lane);
    __syncthreads();
    tbr_sweeps<P>(e, b32, wrd, fdx, fE, fW, fdy, fpn, fps, rdist, edge32, w, lane, nsweep, 0, 1.0f - fom);
    tbr_store<P>(e, a.oer, a.oeb, kg0, (size_t)g.nh, dq, rdist);
}

__global__ __launch_bounds__(kTbThreads) void k_sor_mp(
    Grid g, MpArrays a, double omega, Ctl* ctl, TbCheck chk, TbShape ts, int nsweep, int e_zero) {
    __shared__ float edge32[2][kTrSlots][kWave];
    __shared__ double lds[2 * kTbWaves];
    __shared__ int s_flag;
    if (tb_is_check_block(chk, ts)) {
        tb_check_block(ctl, chk, lds, &s_flag);
        return;
    }
    const int t = tb_tile(ts);
    if (t >= ts.ntx * ts.nty) return;
    mp_tile(g, a, omega, ctl, chk, ts, t, nsweep, e_zero, edge32, lds, &s_flag);
}

// Refinement of a mixed-precision interval: x = phi + e (e = 0 with e_zero)
// into ophi, r = V b - A x rounded to float into or32; per-block partials of
// r^2 and (V b)^2 in double.  The work is split into items of one wave: a
// chunk of kMpRefineCols consecutive split positions (lanes 1..62; lanes 0 and
// 63 carry the neighbouring positions) by kMpRefineRows rows.  A wave loads
// x of both colours for its rows and the rows above and below once, takes
// the east/west neighbours from the adjacent lanes (cross-lane moves) and
// the north/south ones from its own registers; positions and rows outside
// the grid hold x = 0, the value of an absent neighbour.
constexpr int kMpRefineThreads = 256;          // four items per block
constexpr int kMpRefineRows = 4;
constexpr int kMpRefineCols = kWave - 2;

__device__ inline double mp_x(const double* __restrict__ ph, const float* __restrict__ e, size_t k, int e_zero) {
    return e_zero ? ph[k] : ph[k] + (double)e[k];
}

// Block blk of nblk: its items' refinement and its partials.
__device__ __forceinline__ void mp_refine_block(const Grid& g, const double* __restrict__ phr,
                                                const double* __restrict__ phb, const float* __restrict__ er,
                                                const float* __restrict__ eb, int e_zero,
                                                const double* __restrict__ vbr, const double* __restrict__ vbb,
                                                double* __restrict__ ophr, double* __restrict__ ophb,
                                                float* __restrict__ orr, float* __restrict__ orb, int blk, int nblk,
                                                const Ctl* __restrict__ ctl, double* partials, double* lds) {
    constexpr int R = kMpRefineRows;
    double acc[2] = {0.0, 0.0};
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int nchunk = (g.nh + kMpRefineCols - 1) / kMpRefineCols;
    const int nstrip = (g.ny + R - 1) / R;
    const int item = blk * (kMpRefineThreads / kWave) + w;
    const bool work = item < nchunk * nstrip;  // wave-uniform
    const int chunk = work ? item % nchunk : 0, strip = work ? item / nchunk : 0;
    const int m = chunk * kMpRefineCols - 1 + lane;  // the lane's split position
    const bool inx = work && m >= 0 && m < g.nh;
    const bool own = inx && lane > 0 && lane < kWave - 1;
    const int j0 = strip * R;
    // x of both colours in rows j0 - 1 .. j0 + R, and V b of the lane's cells:
    // one round trip of loads
    double X[2][R + 2], bv[2][R];
#pragma unroll
    for (int q = 0; q < R + 2; ++q) {
        const int j = j0 - 1 + q;
        X[0][q] = X[1][q] = 0.0;
        if (inx && j >= 0 && j < g.ny) {
            const size_t k = (size_t)j * g.nh + m;
            X[0][q] = mp_x(phr, er, k, e_zero);
            X[1][q] = mp_x(phb, eb, k, e_zero);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        bv[0][r] = bv[1][r] = 0.0;
        if (own && j < g.ny) {
            const size_t k = (size_t)j * g.nh + m;
            bv[0][r] = vbr[k];
            bv[1][r] = vbb[k];
        }
    }
    // a finished solve is seen after the loads are issued (the flag's latency
    // overlaps theirs; a finished solve only wastes them)
    if (ctl->done) return;  // the same for the whole block
    if (work) {
        // x coefficients by position parity q (cell i = 2 m + q)
        const int i0 = inx ? 2 * m : 0;
        const double cdx[2] = {g.dx[i0], g.dx[i0 + 1]}, cE[2] = {g.pcE[i0], g.pcE[i0 + 1]};
        const double cW[2] = {g.pcW[i0], g.pcW[i0 + 1]}, cD[2] = {g.pcD[i0], g.pcD[i0 + 1]};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = j0 + r;
            if (j >= g.ny) break;  // wave-uniform
            const double dyj = g.dy[j], pN = g.pcN[j], pS = g.pcS[j];
            const size_t k = (size_t)j * g.nh + (inx ? m : 0);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int s = (j + c) & 1;  // position parity of colour c in row j
                const double xo = X[1 - c][r + 1];
                const double up = from_upper_lane(xo), dn = from_lower_lane(xo);
                const double xE = s ? up : xo, xW = s ? xo : dn;
                const double xN = X[1 - c][r + 2], xS = X[1 - c][r];
                const double aE = dyj * cE[s], aW = dyj * cW[s], aD = dyj * cD[s];
                const double aN = cdx[s] * pN, aS = cdx[s] * pS;
                const double d = rb_diag(aE, aD, aW, aN, aS);
                const double sum = rb_sum(aE, xE, aW, xW, aN, xN, aS, xS);
                if (own) {
                    const double x = X[c][r + 1];
                    const double res = bv[c][r] - (sum - d * x);
                    (c ? ophb : ophr)[k] = x;
                    (c ? orb : orr)[k] = (float)res;
                    acc[0] += res * res;
                    acc[1] += bv[c][r] * bv[c][r];
                }
            }
        }
    }
    block_partials(acc, partials, nblk, blk, lds);
}

__global__ __launch_bounds__(kMpRefineThreads) void k_mp_refine(Grid g, const double* __restrict__ phr,
                                                           const double* __restrict__ phb,
                                                           const float* __restrict__ er,
                                                           const float* __restrict__ eb, int e_zero,
                                                           const double* __restrict__ vbr,
                                                           const double* __restrict__ vbb,
                                                           double* __restrict__ ophr, double* __restrict__ ophb,
                                                           float* __restrict__ orr, float* __restrict__ orb,
                                                           const Ctl* __restrict__ ctl, double* partials) {
    __shared__ double lds[2 * kRedThreads / kWave];
    mp_refine_block(g, phr, phb, er, eb, e_zero, vbr, vbb, ophr, ophb, orr, orb, blockIdx.x, gridDim.x, ctl, partials,
                    lds);
}

// Many cases of the mixed-precision solve in one launch per step of the
// solve, as the double-precision batch: the float sweeps over a work list of
// all cases' tiles, the refinement over a list of all cases' row blocks (case
// c's nbr blocks from rblk0, the split of its single-grid refinement), and
// the stop tests one block per case.  Pair selectors are global: every case
// advances in lockstep until it finishes, after which its launches return.
struct MpCase {
    Grid g;
    double* ph[2][2];  // phi [pair][colour]
    float* e[2][2];    // corrections [pair][colour]
    float* r[2][2];    // float residuals [pair][colour]
    const double *bred, *bblack;
    double* partials[2];
    Ctl* ctl;
    TbShape ts;
    double omega, tol;
    int tile0, ntiles, rblk0, nbr, max_iter;
    int fixed;  // 1: max_iter is a replayed iteration count (tolerance ignored)
};

template <class CaseT>
__device__ inline int batch_case(const CaseT* __restrict__ cases, int ncase, int item, int CaseT::*start) {
    int lo = 0, hi = ncase - 1;  // last case whose first item is <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cases[mid].*start <= item) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Sweeps: e pair `eflip` in, the other out; float residual pair rsel.
__global__ __launch_bounds__(kTbThreads) void k_sor_mp_batch(
    const MpCase* __restrict__ cases, int ncase, int ntotal, int per, int eflip, int rsel, int nsweep, int e_zero) {
    __shared__ float edge32[2][kTrSlots][kWave];
    __shared__ double lds[2 * kTbWaves];
    __shared__ int s_flag;
    const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (t >= ntotal) return;
    const MpCase& C = cases[batch_case(cases, ncase, t, &MpCase::tile0)];
    MpArrays a;
    a.er = C.e[eflip][0];
    a.eb = C.e[eflip][1];
    a.oer = C.e[eflip ^ 1][0];
    a.oeb = C.e[eflip ^ 1][1];
    a.rr = C.r[rsel][0];
    a.rb = C.r[rsel][1];
    const TbCheck none = {nullptr, 0, 0, 0, 0, 0.0, nullptr};
    mp_tile(C.g, a, C.omega, C.ctl, none, C.ts, t - C.tile0, nsweep, e_zero, edge32, lds, &s_flag);
}

// Refinement: phi pair `pin` plus e pair `ein` into the other phi pair, the
// float residual into pair rout, partials into set pbuf.
__global__ __launch_bounds__(kMpRefineThreads) void k_mp_refine_batch(const MpCase* __restrict__ cases, int ncase,
                                                                 int nblocks, int pin, int ein, int e_zero, int rout,
                                                                 int pbuf) {
    __shared__ double lds[2 * kRedThreads / kWave];
    if ((int)blockIdx.x >= nblocks) return;
    const MpCase& C = cases[batch_case(cases, ncase, (int)blockIdx.x, &MpCase::rblk0)];
    mp_refine_block(C.g, C.ph[pin][0], C.ph[pin][1], C.e[ein][0], C.e[ein][1], e_zero, C.bred, C.bblack,
                    C.ph[pin ^ 1][0], C.ph[pin ^ 1][1], C.r[rout][0], C.r[rout][1], (int)blockIdx.x - C.rblk0, C.nbr,
                    C.ctl, C.partials[pbuf], lds);
}

// Stop tests after a refinement, one block per case: the nbr partials of set
// pbuf (phase 0: the initial residual), summed with the single-grid tests'
// thread count, so in their order.
// Inside a captured stretch the iteration base and snapshot entry come from
// the cursor (cur non-null), as for k_check_batch.
__global__ __launch_bounds__(kTbThreads) void k_check_mp_batch(const MpCase* __restrict__ cases, int phase, int it,
                                                               int pbuf, Slot* slots, const int* __restrict__ cur) {
    __shared__ double lds[2 * kTbWaves];
    if (cur) {
        it += cur[0];
        slots += (size_t)cur[1] * gridDim.x;
    }
    const MpCase& C = cases[blockIdx.x];
    if (C.ctl->done) {
        if (threadIdx.x == 0) publish(C.ctl, slots + blockIdx.x);
        return;
    }
    double acc[2];
    sum_partials(acc, C.partials[pbuf], C.nbr, lds);
    if (threadIdx.x == 0) {
        check_finish(C.ctl, acc[0], acc[1], phase, it, C.max_iter, C.tol, C.fixed, 0);
        publish(C.ctl, slots + blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// Pressure Poisson: Jacobi-preconditioned CG on M = -A, natural layout
// ---------------------------------------------------------------------------
__device__ inline double nat_row(const Grid& g, const double* __restrict__ x, int i, int j, size_t k, double& d) {
    const double dyj = g.dy[j], dxi = g.dx[i];
    const double aE = dyj * g.pcE[i], aW = dyj * g.pcW[i], aD = dyj * g.pcD[i];
    const double aN = dxi * g.pcN[j], aS = dxi * g.pcS[j];
    const size_t W = g.nx, top = (size_t)(g.ny - 1) * g.nx;  // periodic mode wraps
    const double xE = i < g.nx - 1 ? x[k + 1] : (g.per ? x[k + 1 - W] : 0.0);
    const double xW = i > 0 ? x[k - 1] : (g.per ? x[k + W - 1] : 0.0);
    const double xN = j < g.ny - 1 ? x[k + W] : (g.per ? x[k - top] : 0.0);
    const double xS = j > 0 ? x[k - W] : (g.per ? x[k + top] : 0.0);
    d = rb_diag(aE, aD, aW, aN, aS);
    return rb_sum(aE, xE, aW, xW, aN, xN, aS, xS);
}

__device__ inline double nat_diag(const Grid& g, int i, int j) {
    const double dyj = g.dy[j], dxi = g.dx[i];
    return rb_diag(dyj * g.pcE[i], dyj * g.pcD[i], dyj * g.pcW[i], dxi * g.pcN[j], dxi * g.pcS[j]);
}

// Grid-stride walk over the nx*ny cells of the natural layout that keeps the
// cell's (i, j) up to date without an integer division per step.  Blocks go
// to the 8 XCDs round-robin; when the grid is a multiple of 8 blocks the walk
// gives each XCD a contiguous range of block positions, so that the rows
// above and below a block's cells were mostly fetched into the same L2.
struct CellWalk {
    size_t k, n, stride;
    int i, j, si, sj, nx;
    __device__ explicit CellWalk(const Grid& g) {
        nx = g.nx;
        n = (size_t)g.nx * g.ny;
        stride = (size_t)gridDim.x * blockDim.x;
        sj = (int)(stride / nx);
        si = (int)(stride - (size_t)sj * nx);
        const unsigned b = blockIdx.x, nb = gridDim.x;
        const unsigned lb = (nb & 7u) ? b : (b & 7u) * (nb >> 3) + (b >> 3);
        k = (size_t)lb * blockDim.x + threadIdx.x;
        j = (int)(k / nx);
        i = (int)(k - (size_t)j * nx);
    }
    __device__ bool ok() const { return k < n; }
    __device__ void next() {
        k += stride;
        i += si;
        j += sj;
        if (i >= nx) {
            i -= nx;
            ++j;
        }
    }
};

// Diagonal of M = -A in natural layout (fixed by the grid: once per context).
__global__ __launch_bounds__(kBlock) void k_ndiag(Grid g, double* __restrict__ dn) {
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    if (i >= g.nx || j >= g.ny) return;
    dn[(size_t)j * g.nx + i] = nat_diag(g, i, j);
}

// All PCG kernels are grid-stride over the nx*ny cells with at most kRedMax
// blocks of kRedThreads; cross-block sums go through per-block partials.  The
// preconditioned residual z = r / diag(M) is stored wherever r is written, so
// every reader of z (a cell and its neighbours) sees the same value.

// New search direction of one cell, p = z + beta p_old.
__device__ inline double pcg_dir(double z, double pold, double beta) { return __fma_rn(beta, pold, z); }

// r = -V b + A x (residual of M x = -V b), z = r / d; partials of r.r, r.z,
// (V b)^2.
__global__ __launch_bounds__(kRedThreads) void k_pcg_init(Grid g, const double* __restrict__ x,
                                                          const double* __restrict__ vb, double* __restrict__ r,
                                                          double* __restrict__ z, double* partials) {
    __shared__ double lds[3 * kRedThreads / kWave];
    double acc[3] = {0.0, 0.0, 0.0};
    for (CellWalk c(g); c.ok(); c.next()) {
        const size_t k = c.k;
        double d;
        const double sum = nat_row(g, x, c.i, c.j, k, d);
        const double rk = -vb[k] + (sum - d * x[k]);
        const double zk = rk / d;
        r[k] = rk;
        z[k] = zk;
        acc[0] += rk * rk;
        acc[1] += rk * zk;
        acc[2] += vb[k] * vb[k];
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// One block: r.z of iteration 0 and the first stop test.  Partials of every
// r-producing PCG kernel come in the order (r.r, r.z[, b.b]).
__global__ __launch_bounds__(kBlock) void k_pcg_init_check(Ctl* ctl, const double* __restrict__ partials, int nb,
                                                           double tol, Slot* hs) {
    __shared__ double lds[3 * kBlock / kWave];
    double acc[3];
    sum_partials(acc, partials, nb, lds);
    if (threadIdx.x == 0) {
        ctl->rz[0] = acc[1];
        check_finish(ctl, acc[0], acc[2], 0, 0, 0, tol, 0, 0);
        publish(ctl, hs);
    }
}

// Iteration kk, first kernel.  Every block sums the r.r, r.z partials of r_kk
// and takes the same decision: for kk > 0 stop (NaN, the recursive residual
// passed -> kStConfirm, or the iteration limit) or beta = (r.z)_kk /
// (r.z)_{kk-1}; kk = 0 and restarts use beta = 0 (p = z).  Block 0 records the
// decision and publishes it.  Then p_kk = z + beta p_{kk-1} (into pnew,
// recomputed for the four neighbours as well) and q = M p_kk; partials of p.q.
__global__ __launch_bounds__(kRedThreads) void k_pcg_dir_spmv(Grid g, const double* __restrict__ z,
                                                              const double* __restrict__ pold,
                                                              double* __restrict__ pnew, double* __restrict__ q,
                                                              Ctl* ctl, const double* __restrict__ rpart, int nb,
                                                              double* __restrict__ pqpart, int kk, int max_iter,
                                                              double tol, int fixed, int restart, Slot* hs) {
    __shared__ double lds[2 * kRedThreads / kWave];
    __shared__ double s_beta;
    __shared__ int s_stop, s_done;
    // Block 0 of this launch may set ctl->done while other blocks start:
    // read it once per block so every thread of a block takes one branch.
    if (threadIdx.x == 0) s_done = ctl->done;
    __syncthreads();
    if (s_done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) publish(ctl, hs);
        return;
    }
    double acc[2];
    sum_partials(acc, rpart, nb, lds);
    if (threadIdx.x == 0) {
        const double rn = sqrt(acc[0]);
        const bool first = (kk == 0) || restart;
        int stop = 0, status = kStOk;
        if (!first) {
            if (!isfinite(rn)) { stop = 1; status = kStNan; }
            else if (rn <= tol * ctl->bn) { stop = 1; status = kStConfirm; }
            else if (kk >= max_iter) { stop = 1; status = fixed ? kStOk : kStNotConverged; }
        }
        s_stop = stop;
        s_beta = first ? 0.0 : acc[1] / ctl->rz[(kk - 1) & 1];
        if (blockIdx.x == 0) {
            ctl->rn = rn;
            ctl->iters = kk;
            if (stop) {
                ctl->done = kDone;
                ctl->status = status;
            } else {
                ctl->rz[kk & 1] = acc[1];
            }
            publish(ctl, hs);
        }
    }
    __syncthreads();
    if (s_stop) return;
    const double beta = s_beta;
    double pacc[1] = {0.0};
    const size_t nx = g.nx, top = (size_t)(g.ny - 1) * g.nx;
    for (CellWalk c(g); c.ok(); c.next()) {
        const size_t k = c.k;
        const int i = c.i, j = c.j;
        const double dyj = g.dy[j], dxi = g.dx[i];
        const double aE = dyj * g.pcE[i], aW = dyj * g.pcW[i], aD = dyj * g.pcD[i];
        const double aN = dxi * g.pcN[j], aS = dxi * g.pcS[j];
        const double d = rb_diag(aE, aD, aW, aN, aS);
        const double pk = pcg_dir(z[k], pold[k], beta);
        // neighbours (periodic mode wraps; channel mode has none beyond the ends)
        const bool hE = i < g.nx - 1 || g.per, hW = i > 0 || g.per;
        const bool hN = j < g.ny - 1 || g.per, hS = j > 0 || g.per;
        const size_t kE = i < g.nx - 1 ? k + 1 : k + 1 - nx, kW = i > 0 ? k - 1 : k + nx - 1;
        const size_t kN = j < g.ny - 1 ? k + nx : k - top, kS = j > 0 ? k - nx : k + top;
        const double pE = hE ? pcg_dir(z[kE], pold[kE], beta) : 0.0;
        const double pW = hW ? pcg_dir(z[kW], pold[kW], beta) : 0.0;
        const double pN = hN ? pcg_dir(z[kN], pold[kN], beta) : 0.0;
        const double pS = hS ? pcg_dir(z[kS], pold[kS], beta) : 0.0;
        const double sum = rb_sum(aE, pE, aW, pW, aN, pN, aS, pS);
        const double qk = d * pk - sum;  // M p = -A p
        pnew[k] = pk;
        q[k] = qk;
        pacc[0] += pk * qk;
    }
    block_partials(pacc, pqpart, gridDim.x, blockIdx.x, lds);
}

// Iteration kk, second kernel: alpha = (r.z)_kk / p.q (every block sums the
// p.q partials); x += alpha p, r -= alpha q, z = r / d; partials of r.r and
// r.z.
__global__ __launch_bounds__(kRedThreads) void k_pcg_update(Grid g, double* __restrict__ x, double* __restrict__ r,
                                                            double* __restrict__ z, const double* __restrict__ p,
                                                            const double* __restrict__ q,
                                                            const double* __restrict__ dn, const Ctl* ctl,
                                                            const double* __restrict__ pqpart, int nb,
                                                            double* __restrict__ rpart, int kk) {
    __shared__ double lds[2 * kRedThreads / kWave];
    __shared__ double s_alpha;
    if (ctl->done) return;
    {
        double pq[1];
        sum_partials(pq, pqpart, nb, lds);
        if (threadIdx.x == 0) s_alpha = ctl->rz[kk & 1] / pq[0];
        __syncthreads();
    }
    const double alpha = s_alpha;
    double acc[2] = {0.0, 0.0};
    const size_t n = (size_t)g.nx * g.ny;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        x[k] = __fma_rn(alpha, p[k], x[k]);
        const double rk = __fma_rn(-alpha, q[k], r[k]);
        const double zk = rk / dn[k];
        r[k] = rk;
        z[k] = zk;
        acc[0] += rk * rk;
        acc[1] += rk * zk;
    }
    block_partials(acc, rpart, gridDim.x, blockIdx.x, lds);
}

// True residual r = -V b + A x and z = r / d (written to r, z); partials of
// r.r, r.z.
__global__ __launch_bounds__(kRedThreads) void k_pcg_true_residual(Grid g, const double* __restrict__ x,
                                                                   const double* __restrict__ vb,
                                                                   double* __restrict__ r, double* __restrict__ z,
                                                                   double* partials) {
    __shared__ double lds[2 * kRedThreads / kWave];
    double acc[2] = {0.0, 0.0};
    for (CellWalk c(g); c.ok(); c.next()) {
        const size_t k = c.k;
        double d;
        const double sum = nat_row(g, x, c.i, c.j, k, d);
        const double rk = -vb[k] + (sum - d * x[k]);
        const double zk = rk / d;
        r[k] = rk;
        z[k] = zk;
        acc[0] += rk * rk;
        acc[1] += rk * zk;
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// One block: the true residual accepts the solve (status ok, done) or the
// solve resumes (done = 0) and restarts from it; stats_only records rn.
__global__ __launch_bounds__(kBlock) void k_pcg_confirm(Ctl* ctl, const double* __restrict__ partials, int nb,
                                                        double tol, int stats_only, Slot* hs) {
    __shared__ double lds[2 * kBlock / kWave];
    double acc[2];
    sum_partials(acc, partials, nb, lds);
    if (threadIdx.x == 0) {
        const double rn = sqrt(acc[0]);
        ctl->rn = rn;
        if (!stats_only) {
            if (!isfinite(rn)) {
                ctl->status = kStNan;
            } else if (rn <= tol * ctl->bn) {
                ctl->status = kStOk;
            } else {
                ctl->status = kStOk;
                ctl->done = kRunning;
            }
        }
        publish(ctl, hs);
    }
}

// ---------------------------------------------------------------------------
// Jacobi-PCG with one reduction per iteration (Chronopoulos and Gear): on
// M x = -V b with M = -A, u = D^-1 r (D = diag M, applied as a product with
// the stored 1/D), w = M u, and s = M p carried by its own recurrence, so the
// iteration's two inner products gamma = (r, u) and delta = (w, u) come from
// one reduction:
//   beta_i = gamma_i / gamma_{i-1},
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1},
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,
//   w_{i+1} = M u_{i+1}.
// One kernel per iteration: it reads r_i, w_i, s_{i-1} (double-buffered by
// iteration parity), forms u_{i+1} of the cell and of its four neighbours
// from those (each neighbour's value with exactly the operations its own
// thread uses), and writes p, s_i, x, r_{i+1}, w_{i+1} and the partials of
// gamma, delta and (r, r) of iteration i+1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_rdiag(Grid g, const double* __restrict__ dn, double* __restrict__ rdn) {
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    if (i >= g.nx || j >= g.ny) return;
    const size_t k = (size_t)j * g.nx + i;
    rdn[k] = 1.0 / dn[k];
}

// Neighbour indices of cell (i, j) in natural layout and whether each
// neighbour exists (periodic mode wraps; channel mode has none beyond the ends).
struct NatNb {
    size_t kE, kW, kN, kS;
    bool hE, hW, hN, hS;
    __device__ NatNb(const Grid& g, int i, int j, size_t k) {
        const size_t nx = g.nx, top = (size_t)(g.ny - 1) * g.nx;
        hE = i < g.nx - 1 || g.per;
        hW = i > 0 || g.per;
        hN = j < g.ny - 1 || g.per;
        hS = j > 0 || g.per;
        kE = i < g.nx - 1 ? k + 1 : k + 1 - nx;
        kW = i > 0 ? k - 1 : k + nx - 1;
        kN = j < g.ny - 1 ? k + nx : k - top;
        kS = j > 0 ? k - nx : k + top;
    }
};

// w = M u for u = r / D, with the partials of (r, u), (w, u), (r, r): the
// start of a solve and of a restart.
__global__ __launch_bounds__(kRedThreads) void k_cg1_w(Grid g, const double* __restrict__ r,
                                                       const double* __restrict__ rdn, double* __restrict__ w,
                                                       double* partials) {
    __shared__ double lds[3 * kRedThreads / kWave];
    double acc[3] = {0.0, 0.0, 0.0};
    for (CellWalk c(g); c.ok(); c.next()) {
        const size_t k = c.k;
        const int i = c.i, j = c.j;
        const double dyj = g.dy[j], dxi = g.dx[i];
        const double aE = dyj * g.pcE[i], aW = dyj * g.pcW[i], aD = dyj * g.pcD[i];
        const double aN = dxi * g.pcN[j], aS = dxi * g.pcS[j];
        const double d = rb_diag(aE, aD, aW, aN, aS);
        const NatNb nb(g, i, j, k);
        const double rk = r[k], uk = rk * rdn[k];
        const double uE = nb.hE ? r[nb.kE] * rdn[nb.kE] : 0.0;
        const double uW = nb.hW ? r[nb.kW] * rdn[nb.kW] : 0.0;
        const double uN = nb.hN ? r[nb.kN] * rdn[nb.kN] : 0.0;
        const double uS = nb.hS ? r[nb.kS] * rdn[nb.kS] : 0.0;
        const double wk = d * uk - rb_sum(aE, uE, aW, uW, aN, uN, aS, uS);
        w[k] = wk;
        acc[0] += rk * uk;
        acc[1] += wk * uk;
        acc[2] += rk * rk;
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// u_{i+1} of a cell from r_i, w_i, s_{i-1} (s_i = w_i when first).
__device__ inline double cg1_unext(double r, double w, double s, double rd, double alpha, double beta, bool first) {
    const double si = first ? w : __fma_rn(beta, s, w);
    return __fma_rn(-alpha, si, r) * rd;
}

// Iteration kk on 2-D tiles of kCgTx x kCgTy cells, one tile per block.
// Every block first sums the partials (gamma, delta, rho) of r_kk and takes
// the same decision: for kk > 0 (not after a restart) stop on NaN, on the
// recursive residual sqrt(rho) <= tol ||V b|| (kStConfirm: the host confirms
// with the true residual) or at the iteration limit; block 0 records it (and
// gamma, alpha of iteration kk) and publishes it.  Then wave w, lane l own
// the cells (bx kCgTx + l, by kCgTy + kCgRows w + r), r < kCgRows: each
// thread forms u_{kk+1} of its cells (kept in registers and in LDS), the
// first threads also those of the tile's one-cell frame, and after a barrier
// every cell takes its neighbours' u_{kk+1} from LDS: the frame is read once
// per tile instead of once per neighbour.  Blocks past the last tile (the
// XCD banding rounds the grid up) add zero partials.
constexpr int kCgTx = 64, kCgTy = 32, kCgRows = 4;
constexpr int kCgThreads = kCgTx * kCgTy / kCgRows;  // 512: 8 waves of kCgRows rows
constexpr int kCgPitch = kCgTx + 2;

__global__ __launch_bounds__(kCgThreads) void k_cg1_iter(
    Grid g, double* __restrict__ x, double* __restrict__ p, const double* __restrict__ r_in,
    const double* __restrict__ w_in, const double* __restrict__ s_in, double* __restrict__ r_out,
    double* __restrict__ w_out, double* __restrict__ s_out, const double* __restrict__ rdn, Ctl* ctl,
    const double* __restrict__ part_in, int nb, double* __restrict__ part_out, int kk, int max_iter, double tol,
    int fixed, int first, Slot* hs, int ntx, int ntiles, int per) {
    __shared__ double su[(kCgTy + 2) * kCgPitch];  // u_{kk+1} of the tile and its frame
    __shared__ double lds[3 * kCgThreads / kWave];
    __shared__ double s_alpha, s_beta;
    __shared__ int s_stop, s_done;
    // The tile's loads that do not depend on this iteration's alpha and beta
    // are issued first, so that their latency overlaps the control block's
    // and the partial sums' (a finished solve only wastes them).
    const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);  // XCD band of tiles
    const bool tile = t < ntiles;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int X0 = tile ? (t % ntx) * kCgTx : 0, Y0 = tile ? (t / ntx) * kCgTy : 0;
    const int i = X0 + lane;
    const bool col = tile && i < g.nx;
    const bool fst = first != 0;
    double rr[kCgRows], ww[kCgRows], ss[kCgRows], rd[kCgRows], xo[kCgRows], po[kCgRows];
#pragma unroll
    for (int r = 0; r < kCgRows; ++r) {
        const int j = Y0 + kCgRows * w + r;
        rr[r] = ww[r] = ss[r] = rd[r] = xo[r] = po[r] = 0.0;
        if (col && j < g.ny) {
            const size_t k = (size_t)j * g.nx + i;
            rr[r] = r_in[k];
            ww[r] = w_in[k];
            ss[r] = fst ? 0.0 : s_in[k];
            rd[r] = rdn[k];
            xo[r] = x[k];
            po[r] = fst ? 0.0 : p[k];
        }
    }
    // the frame: rows -1 and kCgTy (threads 0..127), columns -1 and kCgTx
    // (threads 128..191); cells outside the domain read as 0 (channel),
    // periodic mode wraps
    const int ft = threadIdx.x;
    const bool frame = tile && ft < 2 * kCgTx + 2 * kCgTy;
    int hx = 0, hy = 0;
    bool fin = false;
    double fr = 0.0, fw = 0.0, fs = 0.0, frd = 0.0;
    if (frame) {
        if (ft < 2 * kCgTx) {
            hx = ft & (kCgTx - 1);
            hy = ft < kCgTx ? -1 : kCgTy;
        } else {
            const int q = ft - 2 * kCgTx;
            hx = q < kCgTy ? -1 : kCgTx;
            hy = q < kCgTy ? q : q - kCgTy;
        }
        int gi = X0 + hx, gj = Y0 + hy;
        fin = gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
        if (g.per && !fin) {
            // only across the domain's ends (a ragged tile's frame past
            // nx or ny inside the grid does not exist there)
            if (gi == -1) gi = g.nx - 1;
            else if (gi == g.nx) gi = 0;
            if (gj == -1) gj = g.ny - 1;
            else if (gj == g.ny) gj = 0;
            fin = gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
        }
        if (fin) {
            const size_t k = (size_t)gj * g.nx + gi;
            fr = r_in[k];
            fw = w_in[k];
            fs = fst ? 0.0 : s_in[k];
            frd = rdn[k];
        }
    }
    if (threadIdx.x == 0) s_done = ctl->done;
    __syncthreads();
    if (s_done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) publish(ctl, hs);
        return;
    }

    double acc[3];
    sum_partials(acc, part_in, nb, lds);
    if (threadIdx.x == 0) {
        const double gamma = acc[0], delta = acc[1], rn = sqrt(acc[2]);
        int stop = 0, status = kStOk;
        if (!first) {
            if (!isfinite(rn)) { stop = 1; status = kStNan; }
            else if (rn <= tol * ctl->bn) { stop = 1; status = kStConfirm; }
            else if (kk >= max_iter) { stop = 1; status = fixed ? kStOk : kStNotConverged; }
        } else if (kk >= max_iter) {
            stop = 1;
            status = fixed ? kStOk : kStNotConverged;
        }
        double beta = 0.0, alpha;
        if (first) {
            alpha = gamma / delta;
        } else {
            beta = gamma / ctl->rz[(kk - 1) & 1];
            alpha = gamma / (delta - beta * gamma / ctl->al[(kk - 1) & 1]);
        }
        s_stop = stop;
        s_alpha = alpha;
        s_beta = beta;
        if (blockIdx.x == 0) {
            ctl->rn = rn;
            ctl->iters = kk;
            if (stop) {
                ctl->done = kDone;
                ctl->status = status;
            } else {
                ctl->rz[kk & 1] = gamma;
                ctl->al[kk & 1] = alpha;
            }
            publish(ctl, hs);
        }
    }
    __syncthreads();
    if (s_stop) return;
    const double alpha = s_alpha, beta = s_beta;
    double pacc[3] = {0.0, 0.0, 0.0};
    if (tile) {
        double un[kCgRows];
#pragma unroll
        for (int r = 0; r < kCgRows; ++r) {
            const int tr = kCgRows * w + r, j = Y0 + tr;
            un[r] = (col && j < g.ny) ? cg1_unext(rr[r], ww[r], ss[r], rd[r], alpha, beta, fst) : 0.0;
            su[(tr + 1) * kCgPitch + lane + 1] = un[r];
        }
        if (frame) su[(hy + 1) * kCgPitch + hx + 1] = fin ? cg1_unext(fr, fw, fs, frd, alpha, beta, fst) : 0.0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kCgRows; ++r) {
            const int tr = kCgRows * w + r, j = Y0 + tr;
            if (!col || j >= g.ny) continue;
            const size_t k = (size_t)j * g.nx + i;
            const double dyj = g.dy[j], dxi = g.dx[i];
            const double aE = dyj * g.pcE[i], aW = dyj * g.pcW[i], aD = dyj * g.pcD[i];
            const double aN = dxi * g.pcN[j], aS = dxi * g.pcS[j];
            const double d = rb_diag(aE, aD, aW, aN, aS);
            const double uk = rr[r] * rd[r];
            const double pk = fst ? uk : __fma_rn(beta, po[r], uk);
            const double sk = fst ? ww[r] : __fma_rn(beta, ss[r], ww[r]);
            x[k] = __fma_rn(alpha, pk, xo[r]);
            const double rnew = __fma_rn(-alpha, sk, rr[r]);
            const double unew = un[r];  // rnew * rd[r], formed as for the neighbours
            const int o = (tr + 1) * kCgPitch + lane + 1;
            double uE = su[o + 1], uN = su[o + kCgPitch];
            if (g.per) {
                // the domain's last column or row inside a ragged tile: the
                // wrapped neighbour is not in the tile's frame
                if (i == g.nx - 1 && lane + 1 < kCgTx) {
                    const size_t kn = (size_t)j * g.nx;
                    uE = cg1_unext(r_in[kn], w_in[kn], fst ? 0.0 : s_in[kn], rdn[kn], alpha, beta, fst);
                }
                if (j == g.ny - 1 && tr + 1 < kCgTy) {
                    const size_t kn = (size_t)i;
                    uN = cg1_unext(r_in[kn], w_in[kn], fst ? 0.0 : s_in[kn], rdn[kn], alpha, beta, fst);
                }
            }
            const double wnew = d * unew - rb_sum(aE, uE, aW, su[o - 1], aN, uN, aS, su[o - kCgPitch]);
            p[k] = pk;
            s_out[k] = sk;
            r_out[k] = rnew;
            w_out[k] = wnew;
            pacc[0] += rnew * unew;
            pacc[1] += wnew * unew;
            pacc[2] += rnew * rnew;
        }
    }
    block_partials(pacc, part_out, gridDim.x, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Periodic (singular) Poisson problem: the right-hand side V b is made to sum
// to zero and the solution to have zero volume-weighted mean.
// k_per_sums: per-block partials of sum a (weighted = 0) or sum V a
// (weighted = 1), and of sum V; k_per_shift: every block sums them and
// subtracts m V (by_volume = 1) or m from every cell, m = (first sum) / (sum V).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRedThreads) void k_per_sums(Grid g, const double* __restrict__ a, int weighted,
                                                          double* partials) {
#pragma clang fp contract(off)
    __shared__ double lds[2 * kRedThreads / kWave];
    double acc[2] = {0.0, 0.0};
    for (CellWalk c(g); c.ok(); c.next()) {
        const double vol = g.dx[c.i] * g.dy[c.j];
        acc[0] += weighted ? vol * a[c.k] : a[c.k];
        acc[1] += vol;
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

__global__ __launch_bounds__(kRedThreads) void k_per_shift(Grid g, double* __restrict__ a,
                                                           const double* __restrict__ partials, int nb,
                                                           int by_volume) {
#pragma clang fp contract(off)
    __shared__ double lds[2 * kRedThreads / kWave];
    __shared__ double s_m;
    double acc[2];
    sum_partials(acc, partials, nb, lds);
    if (threadIdx.x == 0) s_m = acc[0] / acc[1];
    __syncthreads();
    const double m = s_m;
    for (CellWalk c(g); c.ok(); c.next()) a[c.k] -= by_volume ? m * (g.dx[c.i] * g.dy[c.j]) : m;
}

// ---------------------------------------------------------------------------
// Implicit viscous half: (I - beta L) x = rhs by red-black SOR, natural layout
// ---------------------------------------------------------------------------
template <int COLOR>
__global__ __launch_bounds__(kBlock) void k_helm_u_sweep(Grid g, double* __restrict__ u,
                                                         const double* __restrict__ rhs, double beta, double omega,
                                                         const Ctl* ctl) {
#pragma clang fp contract(off)
    if (ctl->done) return;
    const int m = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    const int i = 2 * m + ((j + COLOR) & 1);
    if (j >= g.ny || i < (g.per ? 0 : 1) || i > g.nx - 1) return;
    const int W = g.nx + 1;
    const size_t k = (size_t)j * W + i, top = (size_t)(g.ny - 1) * W;
    const double ce = g.uce[i], cw = g.ucw[i];
    // periodic mode wraps (face nx mirrors face 0; rows ny-1 and 0 are neighbours)
    const double uE = (g.per && i == g.nx - 1) ? u[k + 1 - g.nx] : u[k + 1];
    const double uW = (g.per && i == 0) ? u[k + g.nx - 1] : u[k - 1];
    double s = ce * uE + cw * uW;
    double cs = ce + cw;
    if (j < g.ny - 1 || g.per) {
        const double a = g.ucn[j];
        s += a * u[j < g.ny - 1 ? k + W : k - top];
        cs += a;
    }
    if (j > 0 || g.per) {
        const double a = g.ucs[j];
        s += a * u[j > 0 ? k - W : k + top];
        cs += a;
    }
    const double gs = (rhs[k] + beta * s) / (1.0 + beta * cs);
    u[k] = (1.0 - omega) * u[k] + omega * gs;
}

template <int COLOR>
__global__ __launch_bounds__(kBlock) void k_helm_v_sweep(Grid g, double* __restrict__ v,
                                                         const double* __restrict__ rhs, double beta, double omega,
                                                         const Ctl* ctl) {
#pragma clang fp contract(off)
    if (ctl->done) return;
    const int m = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    const int i = 2 * m + ((j + COLOR) & 1);
    if (j < (g.per ? 0 : 1) || j > g.ny - 1 || i > g.nx - 1) return;
    const int W = g.nx;
    const size_t k = (size_t)j * W + i, top = (size_t)(g.ny - 1) * W;
    const double cn = g.vcn[j], cso = g.vcs[j];
    // periodic mode wraps (face row ny mirrors row 0; columns nx-1 and 0 are neighbours)
    const double vN = (g.per && j == g.ny - 1) ? v[k - top] : v[k + W];
    const double vS = (g.per && j == 0) ? v[k + top] : v[k - W];
    double s = cn * vN + cso * vS;
    double cs = cn + cso;
    if (i < g.nx - 1 || g.per) {
        const double a = g.vce[i];
        s += a * v[i < g.nx - 1 ? k + 1 : k + 1 - W];
        cs += a;
    }
    if (i > 0 || g.per) {
        const double a = g.vcw[i];
        s += a * v[i > 0 ? k - 1 : k + W - 1];
        cs += a;
    } else {
        const double a = g.vcw[0];
        s += a * 0.0;
        cs += a;
    }
    const double gs = (rhs[k] + beta * s) / (1.0 + beta * cs);
    v[k] = (1.0 - omega) * v[k] + omega * gs;
}

__device__ inline double lap_u(const Grid& g, const double* __restrict__ u, int i, int j) {
#pragma clang fp contract(off)
    const int W = g.nx + 1;
    const size_t k = (size_t)j * W + i, top = (size_t)(g.ny - 1) * W;
    const double uP = u[k];
    // periodic mode wraps (face nx mirrors face 0)
    const double uE = (g.per && i == g.nx - 1) ? u[k + 1 - g.nx] : u[k + 1];
    const double uW = (g.per && i == 0) ? u[k + g.nx - 1] : u[k - 1];
    const int im1 = (g.per && i == 0) ? g.nx - 1 : i - 1;
    double L = (uE - uP) / (g.dx[i] * g.dxu[i]) + (uW - uP) / (g.dx[im1] * g.dxu[i]);
    if (j < g.ny - 1 || g.per) L += (u[j < g.ny - 1 ? k + W : k - top] - uP) / (g.dyv[j + 1] * g.dy[j]);
    if (j > 0 || g.per) L += (u[j > 0 ? k - W : k + top] - uP) / (g.dyv[j] * g.dy[j]);
    return L;
}

__device__ inline double lap_v(const Grid& g, const double* __restrict__ v, int i, int j) {
#pragma clang fp contract(off)
    const int W = g.nx;
    const size_t k = (size_t)j * W + i, top = (size_t)(g.ny - 1) * W;
    const double vP = v[k];
    // periodic mode wraps (face row ny mirrors row 0)
    const double vN = (g.per && j == g.ny - 1) ? v[k - top] : v[k + W];
    const double vS = (g.per && j == 0) ? v[k + top] : v[k - W];
    const int jm1 = (g.per && j == 0) ? g.ny - 1 : j - 1;
    double L = (vN - vP) / (g.dy[j] * g.dyv[j]) + (vS - vP) / (g.dy[jm1] * g.dyv[j]);
    if (i < g.nx - 1 || g.per) L += (v[i < g.nx - 1 ? k + 1 : k + 1 - W] - vP) / (g.dxu[i + 1] * g.dx[i]);
    if (i > 0 || g.per) L += (v[i > 0 ? k - 1 : k + W - 1] - vP) / (g.dxu[i] * g.dx[i]);
    else L += (0.0 - vP) / (g.dxu[0] * g.dx[0]);
    return L;
}

// Residual of the implicit viscous equation, r = rhs - (x - beta L x), over
// the unknowns of component comp (0: u faces 1..nx-1, 1: v faces 1..ny-1):
// per-block partials of r^2 and rhs^2 (grid-stride, at most kRedMax blocks).
__global__ __launch_bounds__(kRedThreads) void k_helm_residual(Grid g, int comp, const double* __restrict__ x,
                                                               const double* __restrict__ rhs, double beta,
                                                               const Ctl* ctl, double* partials) {
#pragma clang fp contract(off)
    __shared__ double lds[2 * kRedThreads / kWave];
    if (ctl->done) return;
    const int i0 = (comp == 0 && !g.per) ? 1 : 0;  // first unknown face in x
    const int j0 = (comp == 1 && !g.per) ? 1 : 0;  // first unknown row
    const int w = comp == 0 ? g.nx - i0 : g.nx;   // unknowns per row
    const int h = comp == 0 ? g.ny : g.ny - j0;   // rows of unknowns
    const size_t n = (size_t)w * h;
    double acc[2] = {0.0, 0.0};
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const int jr = (int)(q / w), ir = (int)(q - (size_t)jr * w);
        if (comp == 0) {
            const int i = ir + i0, j = jr;
            const size_t k = (size_t)j * (g.nx + 1) + i;
            const double r = rhs[k] - (x[k] - beta * lap_u(g, x, i, j));
            acc[0] += r * r;
            acc[1] += rhs[k] * rhs[k];
        } else {
            const int i = ir, j = jr + j0;
            const size_t k = (size_t)j * g.nx + i;
            const double r = rhs[k] - (x[k] - beta * lap_v(g, x, i, j));
            acc[0] += r * r;
            acc[1] += rhs[k] * rhs[k];
        }
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Momentum predictor (Adams-Bashforth convection, Crank-Nicolson diffusion)
//   R = u^n + dt [-(3/2 N^n - 1/2 N^{n-1}) - G p^n + 1/(2Re) L u^n]
// N in divergence form with arithmetic averages; N^{-1} := N^0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_momentum_u(Grid g, const double* __restrict__ u,
                                                       const double* __restrict__ v, const double* __restrict__ p,
                                                       double* __restrict__ nu, double* __restrict__ ru, double dt,
                                                       double re, double uinf, int have_hist) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    // unknown faces: 1..nx-1 and the outlet nx (channel); 0..nx-1 (periodic)
    if (i < (g.per ? 0 : 1) || i > (g.per ? g.nx - 1 : g.nx) || j >= g.ny) return;
    const int nx = g.nx, ny = g.ny, W = nx + 1;
    const size_t k = (size_t)j * W + i;
    if (i == nx) {  // convective outlet, kept in the R array until committed
        const double uo = u[k], ui = u[k - 1];
        ru[k] = uo - dt * uinf * (uo - ui) / g.dx[nx - 1];
        return;
    }
    // neighbours; periodic mode wraps (face nx mirrors face 0, row ny row 0)
    const int im1 = (g.per && i == 0) ? nx - 1 : i - 1;
    const int jp1 = j < ny - 1 ? j + 1 : 0, jm1 = j > 0 ? j - 1 : ny - 1;
    const double uP = u[k];
    const double uE = (g.per && i == nx - 1) ? u[k + 1 - nx] : u[k + 1];
    const double uW = u[(size_t)j * W + im1];
    const double ue = 0.5 * (uP + uE);
    const double uw = 0.5 * (uW + uP);
    const double nxp = (ue * ue - uw * uw) / g.dxu[i];
    double fn = 0.0, fs = 0.0;
    if (j < ny - 1 || g.per) {
        const double vc = 0.5 * (v[(size_t)jp1 * nx + im1] + v[(size_t)jp1 * nx + i]);
        const double uc = 0.5 * (uP + u[(size_t)jp1 * W + i]);
        fn = vc * uc;
    }
    if (j > 0 || g.per) {
        const double vc = 0.5 * (v[(size_t)j * nx + im1] + v[(size_t)j * nx + i]);
        const double uc = 0.5 * (u[(size_t)jm1 * W + i] + uP);
        fs = vc * uc;
    }
    const double N = nxp + (fn - fs) / g.dy[j];
    const double L = lap_u(g, u, i, j);
    const double G = (p[(size_t)j * nx + i] - p[(size_t)j * nx + im1]) / g.dxu[i];
    const double Nold = have_hist ? nu[k] : N;
    ru[k] = uP + dt * (-(1.5 * N - 0.5 * Nold) - G + (0.5 / re) * L);
    nu[k] = N;
}

__global__ __launch_bounds__(kBlock) void k_momentum_v(Grid g, const double* __restrict__ u,
                                                       const double* __restrict__ v, const double* __restrict__ p,
                                                       double* __restrict__ nv, double* __restrict__ rv, double dt,
                                                       double re, int have_hist) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    // unknown rows: 1..ny-1 (channel); 0..ny-1 (periodic)
    if (i >= g.nx || j < (g.per ? 0 : 1) || j > g.ny - 1) return;
    const int nx = g.nx, ny = g.ny, W = nx + 1;
    const size_t k = (size_t)j * nx + i;
    // neighbours; periodic mode wraps (row ny mirrors row 0, face nx face 0)
    const int jm1 = (g.per && j == 0) ? ny - 1 : j - 1;
    const int ip1 = (g.per && i == nx - 1) ? 0 : i + 1;
    const double vP = v[k];
    const double vNv = (g.per && j == ny - 1) ? v[i] : v[k + nx];
    const double vSv = v[(size_t)jm1 * nx + i];
    const double vn = 0.5 * (vP + vNv);
    const double vs = 0.5 * (vSv + vP);
    const double nyp = (vn * vn - vs * vs) / g.dyv[j];
    const double ue = 0.5 * (u[(size_t)jm1 * W + ip1] + u[(size_t)j * W + ip1]);
    const double ve = (i < nx - 1 || g.per) ? 0.5 * (vP + v[(size_t)j * nx + ip1]) : vP;
    const double uw = 0.5 * (u[(size_t)jm1 * W + i] + u[(size_t)j * W + i]);
    const double vw = (i > 0 || g.per) ? 0.5 * (v[i > 0 ? k - 1 : k + nx - 1] + vP) : 0.0;
    const double N = (ue * ve - uw * vw) / g.dx[i] + nyp;
    const double L = lap_v(g, v, i, j);
    const double G = (p[(size_t)j * nx + i] - p[(size_t)jm1 * nx + i]) / g.dyv[j];
    const double Nold = have_hist ? nv[k] : N;
    rv[k] = vP + dt * (-(1.5 * N - 0.5 * Nold) - G + (0.5 / re) * L);
    nv[k] = N;
}

// Move the convective-outlet value from R into u before the implicit solve.
__global__ void k_outlet_commit(int nx, int ny, double* __restrict__ u, const double* __restrict__ ru) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ny) return;
    const size_t k = (size_t)j * (nx + 1) + nx;
    u[k] = ru[k];
}

// ---------------------------------------------------------------------------
// Immersed boundary: classification (one block over the body's motion box)
// ---------------------------------------------------------------------------
// Box in cell indices [bi0, bi1) x [bj0, bj1): u faces i in [bi0, bi1],
// v faces j in [bj0, bj1]; every node that can be inside the body during the
// run lies in it.  flu/flv = 0 fluid, 1 forcing, 2 deep; msrc = 1 for cells
// with a forced face.  Forced nodes are listed in row-major order.
struct Box {
    int bi0, bi1, bj0, bj1;
};

__device__ inline int node_type_u(const Grid& g, const Body& B, int i, int j) {
    if (!inside(g.xf[i], g.yc[j], B)) return 0;
    const bool all = inside(g.xf[i + 1], g.yc[j], B) && inside(g.xf[i - 1], g.yc[j], B) &&
                     inside(g.xf[i], g.yc[j + 1], B) && inside(g.xf[i], g.yc[j - 1], B);
    return all ? 2 : 1;
}
__device__ inline int node_type_v(const Grid& g, const Body& B, int i, int j) {
    if (!inside(g.xc[i], g.yf[j], B)) return 0;
    const bool all = inside(g.xc[i + 1], g.yf[j], B) && inside(g.xc[i - 1], g.yf[j], B) &&
                     inside(g.xc[i], g.yf[j + 1], B) && inside(g.xc[i], g.yf[j - 1], B);
    return all ? 2 : 1;
}

// Block-wide ordered compaction: append the flagged items of this chunk
// (one per thread, in thread order) at list[base...].  Returns the count.
__device__ inline int block_append(bool flag, int value, int* list, int base, int* lds_w) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const unsigned long long mask = __ballot(flag);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) lds_w[w] = __popcll(mask);
    __syncthreads();
    int off = 0, tot = 0;
    for (int q = 0; q < nw; ++q) {
        if (q < w) off += lds_w[q];
        tot += lds_w[q];
    }
    if (flag) list[base + off + before] = value;
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(1024) void k_classify(Grid g, Body B, Box bx, uint8_t* __restrict__ flu,
                                                   uint8_t* __restrict__ flv, uint8_t* __restrict__ msrc,
                                                   int* __restrict__ list_u, int* __restrict__ list_v,
                                                   int* __restrict__ counts) {
    __shared__ int lds_w[1024 / kWave];
    const int nx = g.nx;
    const int wu = bx.bi1 - bx.bi0 + 1, hu = bx.bj1 - bx.bj0;
    const int wv = bx.bi1 - bx.bi0, hv = bx.bj1 - bx.bj0 + 1;
    const int nu = wu * hu, nvv = wv * hv;
    // u nodes
    int base = 0;
    for (int c0 = 0; c0 < nu; c0 += blockDim.x) {
        const int c = c0 + threadIdx.x;
        int t = 0, k = 0;
        if (c < nu) {
            const int i = bx.bi0 + c % wu, j = bx.bj0 + c / wu;
            t = B.present ? node_type_u(g, B, i, j) : 0;
            k = j * (nx + 1) + i;
            flu[k] = (uint8_t)t;
        }
        base += block_append(t != 0, k, list_u, base, lds_w);
    }
    const int cu = base;
    base = 0;
    for (int c0 = 0; c0 < nvv; c0 += blockDim.x) {
        const int c = c0 + threadIdx.x;
        int t = 0, k = 0;
        if (c < nvv) {
            const int i = bx.bi0 + c % wv, j = bx.bj0 + c / wv;
            t = B.present ? node_type_v(g, B, i, j) : 0;
            k = j * nx + i;
            flv[k] = (uint8_t)t;
        }
        base += block_append(t != 0, k, list_v, base, lds_w);
    }
    const int cv = base;
    __syncthreads();
    // cells with at least one forced face (flags written above by this block)
    const int wc = bx.bi1 - bx.bi0, hc = bx.bj1 - bx.bj0, nc = wc * hc;
    int cm = 0;
    for (int c0 = 0; c0 < nc; c0 += blockDim.x) {
        const int c = c0 + threadIdx.x;
        bool f = false;
        if (c < nc) {
            const int i = bx.bi0 + c % wc, j = bx.bj0 + c / wc;
            const int nf = (flu[j * (nx + 1) + i] != 0) + (flu[j * (nx + 1) + i + 1] != 0) +
                           (flv[j * nx + i] != 0) + (flv[(j + 1) * nx + i] != 0);
            f = nf > 0;
            msrc[j * nx + i] = f ? 1 : 0;
        }
        const unsigned long long mask = __ballot(f);
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        if (lane == 0) lds_w[w] = __popcll(mask);
        __syncthreads();
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) cm += lds_w[q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[0] = cu;
        counts[1] = cv;
        counts[2] = cm;
    }
}

// ---------------------------------------------------------------------------
// Immersed boundary: forcing at the listed nodes, and the force coefficients
// ---------------------------------------------------------------------------
__device__ inline double alpha_of(double df, double dout, double amax) {
#pragma clang fp contract(off)
    double al = dout > 0.0 ? df / dout : amax;
    if (al > amax) al = amax;
    if (al < 0.0) al = 0.0;
    return al;
}

// explicit predictor u~ = R + dt/(2Re) L u^n at u node (i, j)
__device__ inline double pred_u(const Grid& g, const double* u, const double* ru, int i, int j, double beta) {
#pragma clang fp contract(off)
    return ru[(size_t)j * (g.nx + 1) + i] + beta * lap_u(g, u, i, j);
}
__device__ inline double pred_v(const Grid& g, const double* v, const double* rv, int i, int j, double beta) {
#pragma clang fp contract(off)
    return rv[(size_t)j * g.nx + i] + beta * lap_v(g, v, i, j);
}

__device__ inline double target_u(const Grid& g, const Body& B, const double* u, const double* ru, int i, int j,
                                  double beta, double amax) {
#pragma clang fp contract(off)
    const double ub = 0.0;
    double sum = 0.0;
    int cnt = 0;
    double sy = 1.0 - ((g.yc[j] - B.yb) / B.b) * ((g.yc[j] - B.yb) / B.b);
    if (sy < 0.0) sy = 0.0;
    double sx = 1.0 - ((g.xf[i] - B.xb) / B.a) * ((g.xf[i] - B.xb) / B.a);
    if (sx < 0.0) sx = 0.0;
    if (!inside(g.xf[i + 1], g.yc[j], B)) {
        const double xbd = B.xb + B.a * sqrt(sy);
        const double al = alpha_of(xbd - g.xf[i], g.xf[i + 1] - xbd, amax);
        sum += ub + (ub - pred_u(g, u, ru, i + 1, j, beta)) * al;
        ++cnt;
    }
    if (!inside(g.xf[i - 1], g.yc[j], B)) {
        const double xbd = B.xb - B.a * sqrt(sy);
        const double al = alpha_of(g.xf[i] - xbd, xbd - g.xf[i - 1], amax);
        sum += ub + (ub - pred_u(g, u, ru, i - 1, j, beta)) * al;
        ++cnt;
    }
    if (!inside(g.xf[i], g.yc[j + 1], B)) {
        const double ybd = B.yb + B.b * sqrt(sx);
        const double al = alpha_of(ybd - g.yc[j], g.yc[j + 1] - ybd, amax);
        sum += ub + (ub - pred_u(g, u, ru, i, j + 1, beta)) * al;
        ++cnt;
    }
    if (!inside(g.xf[i], g.yc[j - 1], B)) {
        const double ybd = B.yb - B.b * sqrt(sx);
        const double al = alpha_of(g.yc[j] - ybd, ybd - g.yc[j - 1], amax);
        sum += ub + (ub - pred_u(g, u, ru, i, j - 1, beta)) * al;
        ++cnt;
    }
    return sum / cnt;
}

__device__ inline double target_v(const Grid& g, const Body& B, const double* v, const double* rv, int i, int j,
                                  double beta, double amax) {
#pragma clang fp contract(off)
    const double vbd = B.vb;
    double sum = 0.0;
    int cnt = 0;
    double sy = 1.0 - ((g.yf[j] - B.yb) / B.b) * ((g.yf[j] - B.yb) / B.b);
    if (sy < 0.0) sy = 0.0;
    double sx = 1.0 - ((g.xc[i] - B.xb) / B.a) * ((g.xc[i] - B.xb) / B.a);
    if (sx < 0.0) sx = 0.0;
    if (!inside(g.xc[i + 1], g.yf[j], B)) {
        const double xbd = B.xb + B.a * sqrt(sy);
        const double al = alpha_of(xbd - g.xc[i], g.xc[i + 1] - xbd, amax);
        sum += vbd + (vbd - pred_v(g, v, rv, i + 1, j, beta)) * al;
        ++cnt;
    }
    if (!inside(g.xc[i - 1], g.yf[j], B)) {
        const double xbd = B.xb - B.a * sqrt(sy);
        const double al = alpha_of(g.xc[i] - xbd, xbd - g.xc[i - 1], amax);
        sum += vbd + (vbd - pred_v(g, v, rv, i - 1, j, beta)) * al;
        ++cnt;
    }
    if (!inside(g.xc[i], g.yf[j + 1], B)) {
        const double ybd = B.yb + B.b * sqrt(sx);
        const double al = alpha_of(ybd - g.yf[j], g.yf[j + 1] - ybd, amax);
        sum += vbd + (vbd - pred_v(g, v, rv, i, j + 1, beta)) * al;
        ++cnt;
    }
    if (!inside(g.xc[i], g.yf[j - 1], B)) {
        const double ybd = B.yb - B.b * sqrt(sx);
        const double al = alpha_of(g.yf[j] - ybd, ybd - g.yf[j - 1], amax);
        sum += vbd + (vbd - pred_v(g, v, rv, i, j - 1, beta)) * al;
        ++cnt;
    }
    return sum / cnt;
}

// One block: f = (target - u~)/dt at every listed node, R += dt f; then the
// force F = -sum f dV + pi a b (0, a_body) summed in list (row-major) order
// and the coefficients C = F / (u_ref^2 chord / 2), u_ref = u_inf or 1.
__global__ __launch_bounds__(1024) void k_forcing(Grid g, Body B, const double* __restrict__ u,
                                                  const double* __restrict__ v, double* __restrict__ ru,
                                                  double* __restrict__ rv, const uint8_t* __restrict__ flu,
                                                  const uint8_t* __restrict__ flv, const int* __restrict__ list_u,
                                                  const int* __restrict__ list_v, const int* __restrict__ counts,
                                                  double* __restrict__ f_u, double* __restrict__ f_v, double dt,
                                                  double beta, double amax, double qn, double* __restrict__ coef) {
#pragma clang fp contract(off)
    const int nx = g.nx;
    const int cu = counts[0], cv = counts[1];
    for (int n = threadIdx.x; n < cu; n += blockDim.x) {
        const int k = list_u[n];
        const int j = k / (nx + 1), i = k - j * (nx + 1);
        const double ut = pred_u(g, u, ru, i, j, beta);
        const double V = flu[k] == 2 ? 0.0 : target_u(g, B, u, ru, i, j, beta, amax);
        const double f = (V - ut) / dt;
        f_u[n] = f;
    }
    for (int n = threadIdx.x; n < cv; n += blockDim.x) {
        const int k = list_v[n];
        const int j = k / nx, i = k - j * nx;
        const double vt = pred_v(g, v, rv, i, j, beta);
        const double V = flv[k] == 2 ? B.vb : target_v(g, B, v, rv, i, j, beta, amax);
        const double f = (V - vt) / dt;
        f_v[n] = f;
    }
    __syncthreads();
    // R is updated only after every target has read the predictor of its
    // (fluid) neighbours.
    for (int n = threadIdx.x; n < cu; n += blockDim.x) ru[list_u[n]] += dt * f_u[n];
    for (int n = threadIdx.x; n < cv; n += blockDim.x) rv[list_v[n]] += dt * f_v[n];
    if (threadIdx.x == 0) {
        double fx = 0.0, fy = 0.0;
        for (int n = 0; n < cu; ++n) {
            const int k = list_u[n];
            const int j = k / (nx + 1), i = k - j * (nx + 1);
            fx -= f_u[n] * (g.dxu[i] * g.dy[j]);
        }
        for (int n = 0; n < cv; ++n) {
            const int k = list_v[n];
            const int j = k / nx, i = k - j * nx;
            fy -= f_v[n] * (g.dx[i] * g.dyv[j]);
        }
        if (B.present) {
            const double pi = 3.14159265358979323846;
            fy += pi * B.a * B.b * B.ab;
        }
        coef[0] = qn > 0.0 ? fx / qn : 0.0;
        coef[1] = qn > 0.0 ? fy / qn : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Poisson source, projection and pressure update
// ---------------------------------------------------------------------------
// V b = V (D(u^) - q) / dt; q = divergence of (u^ - body velocity) over the
// forced faces of the cell (mass source), 0 when q_mode = 0.
__global__ __launch_bounds__(kBlock) void k_poisson_rhs(Grid g, const double* __restrict__ u,
                                                        const double* __restrict__ v,
                                                        const uint8_t* __restrict__ flu,
                                                        const uint8_t* __restrict__ flv,
                                                        const uint8_t* __restrict__ msrc, double vbody, double dt,
                                                        int q_mode, double* __restrict__ vb) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    if (i >= g.nx || j >= g.ny) return;
    const int nx = g.nx, W = nx + 1;
    const size_t ku = (size_t)j * W + i, kv = (size_t)j * nx + i;
    // periodic mode wraps (face nx mirrors face 0, row ny row 0)
    const double uE = (g.per && i == nx - 1) ? u[ku + 1 - nx] : u[ku + 1];
    const double vN = (g.per && j == g.ny - 1) ? v[i] : v[kv + nx];
    const double d = (uE - u[ku]) / g.dx[i] + (vN - v[kv]) / g.dy[j];
    double q = 0.0;
    if (q_mode && msrc[kv]) {
        const double fe = flu[ku + 1] ? u[ku + 1] - 0.0 : 0.0;
        const double fw = flu[ku] ? u[ku] - 0.0 : 0.0;
        const double fn = flv[kv + nx] ? v[kv + nx] - vbody : 0.0;
        const double fs = flv[kv] ? v[kv] - vbody : 0.0;
        q = (fe - fw) / g.dx[i] + (fn - fs) / g.dy[j];
    }
    vb[kv] = (g.dx[i] * g.dy[j]) * ((d - q) / dt);
}

// u^{n+1} = u^ - dt G phi on the interior faces and the outlet face (phi = 0
// on the outlet face, half a cell from the last centre).
__global__ __launch_bounds__(kBlock) void k_project_u(Grid g, double* __restrict__ u, const double* __restrict__ phi,
                                                      double dt) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    // faces 1..nx (channel, nx the outlet); 0..nx-1 (periodic)
    if (i < (g.per ? 0 : 1) || i > (g.per ? g.nx - 1 : g.nx) || j >= g.ny) return;
    const int nx = g.nx;
    const size_t k = (size_t)j * (nx + 1) + i;
    if (i < nx) {
        const int im1 = (g.per && i == 0) ? nx - 1 : i - 1;
        u[k] -= dt * ((phi[(size_t)j * nx + i] - phi[(size_t)j * nx + im1]) / g.dxu[i]);
    } else {
        u[k] -= dt * (0.0 - phi[(size_t)j * nx + nx - 1]) / g.dxu[nx];
    }
}

__global__ __launch_bounds__(kBlock) void k_project_v(Grid g, double* __restrict__ v, const double* __restrict__ phi,
                                                      double dt) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    // rows 1..ny-1 (channel); 0..ny-1 (periodic)
    if (i >= g.nx || j < (g.per ? 0 : 1) || j > g.ny - 1) return;
    const int nx = g.nx;
    const size_t k = (size_t)j * nx + i;
    const size_t ks = j > 0 ? k - nx : k + (size_t)(g.ny - 1) * nx;
    v[k] -= dt * ((phi[k] - phi[ks]) / g.dyv[j]);
}

// Periodic mode: u face nx and v face row ny mirror face 0 / row 0.
__global__ void k_sync_periodic(int nx, int ny, double* __restrict__ u, double* __restrict__ v) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ny) u[(size_t)t * (nx + 1) + nx] = u[(size_t)t * (nx + 1)];
    if (t < nx) v[(size_t)ny * nx + t] = v[t];
}

// p^{n+1} = p^n + phi - dt/(2Re) (A phi)/V, A evaluated as a plain
// finite-volume sum (coefficients by division).
__global__ __launch_bounds__(kBlock) void k_update_p(Grid g, double* __restrict__ p, const double* __restrict__ phi,
                                                     double beta) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
    const int j = blockIdx.y * kBlockRows + threadIdx.x / kWave;
    if (i >= g.nx || j >= g.ny) return;
    const int nx = g.nx, ny = g.ny;
    const size_t k = (size_t)j * nx + i, top = (size_t)(ny - 1) * nx;
    double s = 0.0, d = 0.0, a;
    // periodic mode wraps; channel mode: Neumann, phi = 0 on the outlet face
    if (i < nx - 1 || g.per) {
        a = g.dy[j] / g.dxu[i + 1];
        s += a * phi[i < nx - 1 ? k + 1 : k + 1 - nx];
        d += a;
    } else {
        d += g.dy[j] / g.dxu[nx];
    }
    if (i > 0 || g.per) {
        a = g.dy[j] / g.dxu[i];
        s += a * phi[i > 0 ? k - 1 : k + nx - 1];
        d += a;
    }
    if (j < ny - 1 || g.per) {
        a = g.dx[i] / g.dyv[j + 1];
        s += a * phi[j < ny - 1 ? k + nx : k - top];
        d += a;
    }
    if (j > 0 || g.per) {
        a = g.dx[i] / g.dyv[j];
        s += a * phi[j > 0 ? k - nx : k + top];
        d += a;
    }
    const double Aphi = s - d * phi[k];
    p[k] += phi[k] - beta * (Aphi / (g.dx[i] * g.dy[j]));
}

// Scatter the listed forcing values into full-size arrays (diagnostics).
__global__ void k_scatter_forcing(const int* __restrict__ list, const int* __restrict__ counts, int which,
                                  const double* __restrict__ f, double* __restrict__ full) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < counts[which]) full[list[n]] = f[n];
}

// ---------------------------------------------------------------------------
// Learned guess and correction of the pressure solve (an extension of the
// method).  The network works on a grid coarsened by a factor F in both
// directions (F = 1: the grid itself): coarse cell (I, J) averages the fine
// cells i in [F I, F I + F), j in [F J, F J + F).  It sees r = V b - A phi (the
// residual of the current phi), phi and the body mask, each averaged and
// scaled to unit RMS over the coarse grid, and predicts the coarse average of
// the remaining change of phi in units of s_r = RMS(coarse r); the fine cells
// of a coarse cell all receive its value.
// ---------------------------------------------------------------------------
struct Coarse {
    int f, ncx, ncy;
};

__device__ inline double cell_resid(const Grid& g, const double* __restrict__ phi, const double* __restrict__ vb,
                                    int i, int j) {
    const size_t k = (size_t)j * g.nx + i;
    double d;
    const double sum = nat_row(g, phi, i, j, k, d);
    return vb[k] - (sum - d * phi[k]);
}

// Unscaled coarse maps, one fine cell per thread: the F^2 fine cells of a
// coarse cell are F^2 consecutive threads of a block of kWsThreads (F <= 16),
// summed by a tree reduction in LDS.  raw: (3, ncy, ncx) float averages of r,
// phi and the inside indicator; partials of sum r_c^2 and sum phi_c^2.
constexpr int kWsThreads = 256;
__global__ __launch_bounds__(kWsThreads) void k_ws_coarse(Grid g, Coarse cg, Body B, const double* __restrict__ phi,
                                                         const double* __restrict__ vb, float* __restrict__ raw,
                                                         double* partials) {
    __shared__ double sr[kWsThreads], sp[kWsThreads];
    __shared__ int sm[kWsThreads];
    __shared__ double lds[2 * kWsThreads / kWave];
    const int f2 = cg.f * cg.f;
    const int per = kWsThreads / f2;  // coarse cells per block
    const int t = threadIdx.x, l = t % f2;
    const size_t nc = (size_t)cg.ncx * cg.ncy;
    const size_t q = (size_t)blockIdx.x * per + t / f2;
    double r = 0.0, p = 0.0;
    int in = 0;
    if (q < nc) {
        const int I = (int)(q % cg.ncx), J = (int)(q / cg.ncx);
        const int i = I * cg.f + l % cg.f, j = J * cg.f + l / cg.f;
        const size_t k = (size_t)j * g.nx + i;
        double d;
        const double sum = nat_row(g, phi, i, j, k, d);
        r = vb[k] - (sum - d * phi[k]);
        p = phi[k];
        in = (B.present && inside(g.xc[i], g.yc[j], B)) ? 1 : 0;
    }
    sr[t] = r;
    sp[t] = p;
    sm[t] = in;
    __syncthreads();
    for (int o = f2 / 2; o > 0; o >>= 1) {
        if (l < o) {
            sr[t] += sr[t + o];
            sp[t] += sp[t + o];
            sm[t] += sm[t + o];
        }
        __syncthreads();
    }
    double acc[2] = {0.0, 0.0};
    if (l == 0 && q < nc) {
        const double w = 1.0 / (double)f2;
        const double rc = sr[t] * w, pc = sp[t] * w;
        raw[q] = (float)rc;
        raw[nc + q] = (float)pc;
        raw[2 * nc + q] = (float)sm[t] / (float)f2;
        acc[0] = rc * rc;
        acc[1] = pc * pc;
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// Scale maps 0 and 1 to unit RMS in place (every block sums the partials;
// block 0 stores (s_r, s_phi) in scale, a zero RMS replaced by 1) and zero
// the maps whose bit is clear in `maps`.
__global__ __launch_bounds__(kRedThreads) void k_ws_normalize(Coarse cg, const double* __restrict__ partials, int nb,
                                                              int maps, double* __restrict__ scale,
                                                              float* __restrict__ feat) {
    __shared__ double lds[2 * kRedThreads / kWave];
    __shared__ float s_inv[2];
    double acc[2];
    sum_partials(acc, partials, nb, lds);
    const size_t nc = (size_t)cg.ncx * cg.ncy;
    if (threadIdx.x == 0) {
        const double sr = sqrt(acc[0] / (double)nc), sp = sqrt(acc[1] / (double)nc);
        const double a = sr > 0.0 ? sr : 1.0, b = sp > 0.0 ? sp : 1.0;
        s_inv[0] = (maps & 1) ? (float)(1.0 / a) : 0.0f;
        s_inv[1] = (maps & 2) ? (float)(1.0 / b) : 0.0f;
        if (blockIdx.x == 0) {
            scale[0] = a;
            scale[1] = b;
        }
    }
    __syncthreads();
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nc; q += (size_t)gridDim.x * blockDim.x) {
        feat[q] *= s_inv[0];
        feat[nc + q] *= s_inv[1];
        if (!(maps & 4)) feat[2 * nc + q] = 0.0f;
    }
}

// One pass of the binomial filter [1 2 1] / 4 in x, then in y, over the coarse
// map (edge values mirrored): damps the shortest coarse wavelengths of the
// network output (a wavelength of 2 coarse cells vanishes, 4 halves) while
// leaving the smooth part it predicts nearly unchanged.  One thread per
// coarse cell; tmp holds the x pass.
__global__ void k_ws_smooth_x(Coarse cg, const float* __restrict__ y, float* __restrict__ tmp) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cg.ncx * cg.ncy) return;
    const int I = q % cg.ncx;
    const float c = y[q], w = I > 0 ? y[q - 1] : c, e = I < cg.ncx - 1 ? y[q + 1] : c;
    tmp[q] = 0.25f * (w + e) + 0.5f * c;
}
__global__ void k_ws_smooth_y(Coarse cg, const float* __restrict__ tmp, float* __restrict__ y) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cg.ncx * cg.ncy) return;
    const int J = q / cg.ncx;
    const float c = tmp[q], s = J > 0 ? tmp[q - cg.ncx] : c, n = J < cg.ncy - 1 ? tmp[q + cg.ncx] : c;
    y[q] = 0.25f * (s + n) + 0.5f * c;
}

// Bilinear interpolation of the coarse map y (cell centres of the coarse
// grid) at the centre of fine cell (i, j), in index space; constant beyond the
// outermost coarse centres.
__device__ inline double coarse_interp(const Coarse& cg, const float* __restrict__ y, int i, int j) {
    const double fx = ((double)i - 0.5 * (cg.f - 1)) / cg.f, fy = ((double)j - 0.5 * (cg.f - 1)) / cg.f;
    const double cx = fmin(fmax(fx, 0.0), (double)(cg.ncx - 1)), cy = fmin(fmax(fy, 0.0), (double)(cg.ncy - 1));
    const int I0 = min((int)cx, max(cg.ncx - 2, 0)), J0 = min((int)cy, max(cg.ncy - 2, 0));
    const int I1 = min(I0 + 1, cg.ncx - 1), J1 = min(J0 + 1, cg.ncy - 1);
    const double wx = cx - I0, wy = cy - J0;
    const double y00 = y[(size_t)J0 * cg.ncx + I0], y10 = y[(size_t)J0 * cg.ncx + I1];
    const double y01 = y[(size_t)J1 * cg.ncx + I0], y11 = y[(size_t)J1 * cg.ncx + I1];
    return (1.0 - wy) * ((1.0 - wx) * y00 + wx * y10) + wy * ((1.0 - wx) * y01 + wx * y11);
}

// The network's correction on the fine grid: e = out_scale s_r P y, P the
// bilinear interpolation (y: the network output, (ncy, ncx) float).
__global__ __launch_bounds__(kRedThreads) void k_ws_expand(Grid g, Coarse cg, const float* __restrict__ y,
                                                           const double* __restrict__ scale, double out_scale,
                                                           double* __restrict__ e) {
    const double f = out_scale * scale[0];
    for (CellWalk c(g); c.ok(); c.next()) e[c.k] = f * coarse_interp(cg, y, c.i, c.j);
}

// Partials of e.r and e.(A e), r = V b - A phi: the step alpha = e.r / e.A e
// minimises the energy norm (the norm of -A) of the error of phi + alpha e,
// and every step in [0, 2 alpha] leaves that norm no larger than at 0.
__global__ __launch_bounds__(kRedThreads) void k_ws_dots(Grid g, const double* __restrict__ phi,
                                                         const double* __restrict__ vb,
                                                         const double* __restrict__ e, double* partials) {
    __shared__ double lds[2 * kRedThreads / kWave];
    double acc[2] = {0.0, 0.0};
    for (CellWalk c(g); c.ok(); c.next()) {
        double d;
        const double sp = nat_row(g, phi, c.i, c.j, c.k, d);
        const double r = vb[c.k] - (sp - d * phi[c.k]);
        const double se = nat_row(g, e, c.i, c.j, c.k, d);
        const double ae = se - d * e[c.k];
        acc[0] += e[c.k] * r;
        acc[1] += e[c.k] * ae;
    }
    block_partials(acc, partials, gridDim.x, blockIdx.x, lds);
}

// phi += a e.  With step < 0: a = min(1, 2 alpha), alpha the energy-optimal
// step from the partials (every block sums them): the full correction
// whenever it does not increase the error's energy norm, else the largest
// step that does not (a = 0 when the denominator is not negative or alpha is
// not finite); SOR itself never increases that norm, so such corrections
// cannot make the iteration diverge.  With step >= 0: a = step.  Block 0
// records a in scale[2] and adds it to scale[3].
__global__ __launch_bounds__(kRedThreads) void k_ws_apply(Grid g, const double* __restrict__ e,
                                                          const double* __restrict__ partials, int nb, double step,
                                                          double* __restrict__ scale, double* __restrict__ phi) {
    __shared__ double lds[2 * kRedThreads / kWave];
    __shared__ double s_alpha;
    double acc[2] = {0.0, 0.0};
    if (step < 0.0) sum_partials(acc, partials, nb, lds);
    if (threadIdx.x == 0) {
        const double opt = acc[1] < 0.0 ? acc[0] / acc[1] : 0.0;
        s_alpha = step >= 0.0 ? step : (isfinite(opt) ? fmin(1.0, fmax(0.0, 2.0 * opt)) : 0.0);
        if (blockIdx.x == 0) {
            scale[2] = s_alpha;
            scale[3] += s_alpha;
        }
    }
    __syncthreads();
    const double a = s_alpha;
    for (CellWalk c(g); c.ok(); c.next()) phi[c.k] += a * e[c.k];
}

// Training target: coarse average of (phi_new - phi_old) / (out_scale s_r).
__global__ __launch_bounds__(kRedThreads) void k_ws_target(Grid g, Coarse cg, const double* __restrict__ phi,
                                                           const double* __restrict__ phi_old,
                                                           const double* __restrict__ scale, double out_scale,
                                                           float* __restrict__ t) {
    const double f = 1.0 / (out_scale * scale[0] * (double)cg.f * cg.f);
    const size_t nc = (size_t)cg.ncx * cg.ncy;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nc; q += (size_t)gridDim.x * blockDim.x) {
        const int I = (int)(q % cg.ncx), J = (int)(q / cg.ncx);
        double s = 0.0;
        for (int dj = 0; dj < cg.f; ++dj)
            for (int di = 0; di < cg.f; ++di) {
                const size_t k = (size_t)(J * cg.f + dj) * g.nx + I * cg.f + di;
                s += phi[k] - phi_old[k];
            }
        t[q] = (float)(s * f);
    }
}

}  // namespace ibm
