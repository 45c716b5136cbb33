// ibm_lib.hip -- host side of the gfx950 immersed-boundary fractional-step
// solver (arXiv 2402.17337): workspace layout, the per-step pipeline, the
// device-driven iterative solves and the C ABI declared in include/ibm.h.
//
// Every array lives in the caller's workspace; the library allocates only a
// small pinned host block through which the convergence checks report to the
// host, and HIP events.  Iterative solves run ahead of the host: the host
// enqueues iterations in chunks, each chunk ending with a residual check that
// writes the solve's state to device memory (read by every later kernel of
// the solve, which returns at once when the solve has finished) and to the
// pinned block.  The host waits on the check of an older chunk only, so the
// GPU queue never drains while the solve runs.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ibm.h"
#include "ibm_kernels.hpp"
#include "unet_internal.hpp"

using namespace ibm;

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free Poisson solve
// (ibm_poisson_solve_noalloc): the working arrays of its red-black SOR solve
// live in this fixed array of the library's own device memory, one copy per
// device, held until the process ends.  Layout, in doubles: six split
// half-arrays of up to kNoAllocCells / 2 cells each (phi, its second pair,
// V b), the residual partials, then the control blocks.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): it uses the address hipGetSymbolAddress returns for the
// current device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocCells = (size_t)1024 * 768;  // at most nx * ny cells
constexpr size_t kNoAllocTiles = 8192;                // at most this many blocked-sweep tiles
constexpr size_t kNoAllocHalf = ((kNoAllocCells / 2 + 31) / 32) * 32;  // doubles per split array (256-byte multiple)
constexpr size_t kNoAllocPartials = 4 * (size_t)kRedMax + 4 * kNoAllocTiles;
constexpr size_t kNoAllocCtlDoubles = 4 * sizeof(Ctl) / sizeof(double);
constexpr size_t kNoAllocDoubles = 6 * kNoAllocHalf + kNoAllocPartials + kNoAllocCtlDoubles;
}  // namespace
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

constexpr int kSlots = 256;       // host-mapped check slots (ring)
constexpr int kAheadSor = 24;     // SOR chunks in flight before the host waits
constexpr int kFoldMax = 512;     // blocked launches carry the stop test up to this many tiles (every
                                  // block reads all tile partials); beyond it a k_check runs instead
constexpr int kAheadHelm = 3;     // implicit velocity iterations in flight
constexpr int kAheadPcg = 48;     // PCG iterations in flight
constexpr int kMaxSamples = 8192; // event pairs kept per timed kernel
constexpr uint32_t kStateMagic = 0x49424d31u;  // "IBM1"

enum { CTL_U = 0, CTL_V = 1, CTL_P = 2, CTL_N = 4 };

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace layout: one 256-byte aligned array after the other.
struct Layout {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        size_t o = align_up(off, 256);
        off = o + count * sizeof(T);
        return o;
    }
};

struct Offsets {
    size_t xf, yf, dx, dy, xc, yc, dxu, dyv, pcE, pcW, pcD, pcN, pcS, uce, ucw, ucn, ucs, vce, vcw, vcn, vcs;
    size_t u, nu, ru, fufull, v, nv, rv, fvfull, p, phi, vb, pr, pp, pp2, pq, phr, phb, vbr, vbb, pz, dn, phr2, phb2, mpf, phi0, wsf, wscale;
    size_t cgw, cgs, rdn;
    size_t f_u, f_v, coef, partials, ctl, list_u, list_v, counts, flu, flv, msrc;
    size_t total;
    int max_blocks;
};

inline int blocks_for(int cols, int rows) {
    return ((cols + kWave - 1) / kWave) * ((rows + kBlockRows - 1) / kBlockRows);
}

Offsets layout_for(int nx, int ny) {
    Offsets o;
    Layout L;
    const size_t NU = (size_t)(nx + 1) * ny, NV = (size_t)nx * (ny + 1), NC = (size_t)nx * ny;
    const size_t NH = (size_t)(nx / 2) * ny;
    o.xf = L.take<double>(nx + 1); o.yf = L.take<double>(ny + 1);
    o.dx = L.take<double>(nx); o.dy = L.take<double>(ny);
    o.xc = L.take<double>(nx); o.yc = L.take<double>(ny);
    o.dxu = L.take<double>(nx + 1); o.dyv = L.take<double>(ny + 1);
    o.pcE = L.take<double>(nx); o.pcW = L.take<double>(nx); o.pcD = L.take<double>(nx);
    o.pcN = L.take<double>(ny); o.pcS = L.take<double>(ny);
    o.uce = L.take<double>(nx + 1); o.ucw = L.take<double>(nx + 1);
    o.ucn = L.take<double>(ny); o.ucs = L.take<double>(ny);
    o.vce = L.take<double>(nx); o.vcw = L.take<double>(nx);
    o.vcn = L.take<double>(ny + 1); o.vcs = L.take<double>(ny + 1);
    o.u = L.take<double>(NU); o.nu = L.take<double>(NU); o.ru = L.take<double>(NU); o.fufull = L.take<double>(NU);
    o.v = L.take<double>(NV); o.nv = L.take<double>(NV); o.rv = L.take<double>(NV); o.fvfull = L.take<double>(NV);
    o.p = L.take<double>(NC); o.phi = L.take<double>(NC); o.vb = L.take<double>(NC);
    o.pr = L.take<double>(NC); o.pp = L.take<double>(NC); o.pp2 = L.take<double>(NC); o.pq = L.take<double>(NC);
    o.phr = L.take<double>(NH); o.phb = L.take<double>(NH); o.vbr = L.take<double>(NH); o.vbb = L.take<double>(NH);
    o.pz = L.take<double>(NC); o.dn = L.take<double>(NC);
    o.cgw = L.take<double>(NC); o.cgs = L.take<double>(NC); o.rdn = L.take<double>(NC);  // one-reduction CG
    o.phr2 = L.take<double>(NH); o.phb2 = L.take<double>(NH);
    o.mpf = L.take<float>(8 * NH);  // mixed-precision SOR: e and r32, two pairs each
    o.phi0 = L.take<double>(NC);    // learned warm start: phi of the previous step; the network's
    o.wsf = L.take<float>(5 * NC);  // maps, output and smoothing buffer (3 + 1 + 1 coarse maps, at
                                    // most fine-grid size each); RMS scales
    o.wscale = L.take<double>(4);  // s_r, s_phi, alpha of the last correction
    o.f_u = L.take<double>(NU); o.f_v = L.take<double>(NV);
    o.coef = L.take<double>(4);
    // per-block partials: three sums of up to kRedMax blocks, p.q of PCG, and
    // two sums per tile of the blocked sweep (tiles of at least 2x1 cells)
    o.max_blocks = kRedMax;
    o.partials = L.take<double>(std::max((size_t)9 * kRedMax, (size_t)4 * kRedMax + (size_t)2 * (nx / 2) * ny));
    o.ctl = L.take<Ctl>(CTL_N);
    o.list_u = L.take<int>(NU); o.list_v = L.take<int>(NV); o.counts = L.take<int>(4);
    o.flu = L.take<uint8_t>(NU); o.flv = L.take<uint8_t>(NV); o.msrc = L.take<uint8_t>(NC);
    o.total = align_up(L.off, 256);
    return o;
}

// Plunge kinematics (Eqs. 1-2), k = 2 pi freq, evaluated without contraction.
void kinematics(const ibm_params& P, double t, double* yb, double* vb, double* ab) {
#pragma clang fp contract(off)
    const double pi = 3.14159265358979323846;
    double om = 2.0 * pi * P.freq, ph = om * t + P.phase;
    *yb = P.y0 + P.amp * std::sin(ph);
    *vb = om * P.amp * std::cos(ph);
    *ab = -om * om * P.amp * std::sin(ph);
}

const char* validate(const ibm_params* P, const double* xf, const double* yf) {
    if (!P) return "params is NULL";
    if (P->nx < 8 || P->ny < 8 || (P->nx & 1) || (P->ny & 1)) return "nx and ny must be even and >= 8";
    if ((int64_t)(P->nx + 1) * (P->ny + 1) > (int64_t)1 << 30) return "grid too large";
    if (P->bc_mode != IBM_BC_CHANNEL && P->bc_mode != IBM_BC_PERIODIC) return "unknown bc_mode";
    if (P->bc_mode == IBM_BC_PERIODIC &&
        (P->body || P->p_method == IBM_SOLVER_RBSOR_MP || P->p_init == IBM_INIT_LEARNED))
        return "periodic mode takes no body, no mixed-precision sweeps and no learned guess";
    if (P->precision != IBM_PREC_FP64 || P->reserved != 0) return "unsupported precision";
    if (!(P->dt > 0.0) || !(P->re > 0.0) || !std::isfinite(P->u_inf)) return "dt and re must be > 0";
    if (P->p_method != IBM_SOLVER_RBSOR && P->p_method != IBM_SOLVER_PCG && P->p_method != IBM_SOLVER_RBSOR_MP &&
        P->p_method != IBM_SOLVER_CG1)
        return "unknown p_method";
    if (!(P->p_omega > 0.0 && P->p_omega < 2.0) || !(P->uv_omega > 0.0 && P->uv_omega < 2.0))
        return "relaxation factors must lie in (0, 2)";
    if (P->p_max_iter < 1 || P->p_check_every < 1 || P->uv_max_iter < 1) return "iteration limits must be >= 1";
    if (P->p_init != IBM_INIT_ZERO && P->p_init != IBM_INIT_PREVIOUS && P->p_init != IBM_INIT_LEARNED)
        return "unknown p_init";
    if (!(P->alpha_max >= 0.0) || !std::isfinite(P->p_tol) || !std::isfinite(P->uv_tol)) return "invalid tolerances";
    if (!xf || !yf) return "face arrays are NULL";
    for (int i = 0; i < P->nx; ++i)
        if (!(xf[i + 1] > xf[i])) return "xf must be strictly increasing";
    for (int j = 0; j < P->ny; ++j)
        if (!(yf[j + 1] > yf[j])) return "yf must be strictly increasing";
    if (P->body) {
        const double a = 0.5 * P->chord, b = 0.5 * P->thickness * P->chord, amp = std::fabs(P->amp);
        if (!(a > 0.0) || !(b > 0.0)) return "chord and thickness must be > 0";
        const int nx = P->nx, ny = P->ny;
        if (!(P->x0 - a > xf[2]) || !(P->x0 + a < xf[nx - 2]) || !(P->y0 - amp - b > yf[2]) ||
            !(P->y0 + amp + b < yf[ny - 2]))
            return "the body's range of motion must stay two cells clear of the boundary";
    }
    return nullptr;
}

struct Sample {
    hipEvent_t a, b;
    long solve;
    int it;
};

}  // namespace

struct ibm_ctx {
    ibm_params P;
    int nx = 0, ny = 0, nh = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Offsets off;
    Grid g;
    // device arrays
    double *u, *nu, *ru, *fufull, *v, *nv, *rv, *fvfull, *p, *phi, *vb, *pr, *pp, *pp2, *pq, *phr, *phb, *vbr, *vbb;
    double *pz, *dn;    // PCG: z = r / diag(M), and diag(M) (natural layout)
    double *cgw, *cgs, *rdn;  // one-reduction CG: second w and s buffers, 1 / diag(M)
    double *phr2, *phb2;  // second pair of split phi arrays (blocked sweeps alternate)
    float* mpf;           // mixed-precision SOR: e pairs (4 NH), then r32 pairs (4 NH)
    double *phi0, *wscale;  // learned warm start: phi before the solve, (s_r, s_phi)
    float* wsf;             // its maps (3), network output (1) and smoothing buffer (1)
    ibm_unet* net = nullptr;  // warm-start network (borrowed) and its output scale
    double net_scale = 1.0;
    float *snap_feat = nullptr, *snap_target = nullptr;  // training snapshots (borrowed)
    double snap_scale = 1.0;
    int net_f = 1;       // coarsening factor of the network's grid
    int net_every = 0;   // SOR iterations between network corrections (0: none)
    int snap_iter = 0;   // SOR iterations before the snapshot is taken
    int net_smooth = 4;  // binomial passes over the network output
    int net_maps = 7;    // maps given to the network (bit k: map k)
    int net_rule = IBM_NET_STEP_ENERGY;
    double net_step = 1.0;  // IBM_NET_STEP_BACKTRACK: current step
    double *f_u, *f_v, *coef, *partials;
    Ctl* ctl;
    int *list_u, *list_v, *counts;
    uint8_t *flu, *flv, *msrc;
    Box box;
    // host-mapped check slots and staging
    Slot* hslots = nullptr;
    Slot* dslots = nullptr;
    long slot_seq = 0;
    hipEvent_t ev[kSlots];
    double* hstage = nullptr;  // pinned: coef[2], counts[3], sum of the network steps
    int n_net = 0;             // network guesses and corrections of the current step
    int rhs_held = 0;          // vb holds the last time step's V b
    // time stepping
    int have_hist = 0;
    long step = 0;
    double t = 0.0, cd = 0.0, cl = 0.0;
    std::vector<int> schedule;
    size_t sched_pos = 0;
    int batch_fixed = -1;  // replayed iteration count of this step's batched solve (-1: none)
    // profiling
    int prof_every = 0;
    long launches[IBM_KERNEL_COUNT] = {};
    std::vector<Sample> samples[IBM_KERNEL_COUNT];
    std::vector<hipEvent_t> ev_pool;
    long solve_id = 0;
    std::string err;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    // red-black SOR launch shape
    int sor_kernel = IBM_SOR_TEMPORAL;
    int tb_sweeps = 10;
    int tb_tx = 76, tb_ty = 44;
    // device address of this device's static scratch array (the
    // allocation-free solve), resolved at ibm_init; nullptr if unavailable
    double* noalloc = nullptr;
    // phase timing of ibm_step (on while kernel timing is on): events at the
    // phase boundaries of each step, accumulated GPU milliseconds per phase
    bool phase_on = false;
    bool in_batch = false;  // steps of a batch are not phase-timed
    hipEvent_t pev[IBM_PHASE_COUNT + 1] = {};
    double phase_ms[IBM_PHASE_COUNT] = {};
    long phase_steps = 0;
};

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                        \
            return IBM_ERR_HIP;                                                                \
        }                                                                                      \
    } while (0)

#define LAUNCH_CHECK()                                                                         \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess) {                                                                \
            c->err = std::string("kernel launch: ") + hipGetErrorString(e_);                   \
            return IBM_ERR_HIP;                                                                \
        }                                                                                      \
    } while (0)

inline dim3 grid2(int cols, int rows) {
    return dim3((cols + kWave - 1) / kWave, (rows + kBlockRows - 1) / kBlockRows);
}

int next_slot(ibm_ctx* c) { return (int)(c->slot_seq++ % kSlots); }

Slot read_slot(ibm_ctx* c, int s) {
    volatile Slot* hs = c->hslots + s;
    Slot r;
    r.done = hs->done;
    r.status = hs->status;
    r.iters = hs->iters;
    r.zero_rhs = hs->zero_rhs;
    r.bn = hs->bn;
    r.r0 = hs->r0;
    r.rn = hs->rn;
    return r;
}

hipEvent_t pool_event(ibm_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through f(start, stop): sampled launches of kernel kid get a pair
// of events that the runtime records at the dispatch's own start and end
// (hipExtLaunchKernelGGL), so the sampled duration is the kernel's, without
// the dispatch overhead; other launches get null events.
template <class F>
void timed(ibm_ctx* c, int kid, int it, F&& f) {
    const bool take = c->prof_every > 0 && (c->launches[kid] % c->prof_every) == 0 &&
                      (int)c->samples[kid].size() < kMaxSamples;
    c->launches[kid]++;
    if (!take) {
        f(nullptr, nullptr);
        return;
    }
    hipEvent_t a = pool_event(c), b = pool_event(c);
    if (!a || !b) {
        f(nullptr, nullptr);
        return;
    }
    f(a, b);
    c->samples[kid].push_back(Sample{a, b, c->solve_id, it});
}

// Launch with optional dispatch-timing events (see timed()).
#define LAUNCH_EV(ea, eb, kernel, grid, block, shmem, ...)                                              \
    do {                                                                                                \
        if (ea) hipExtLaunchKernelGGL(kernel, grid, block, shmem, c->stream, ea, eb, 0, __VA_ARGS__);  \
        else hipLaunchKernelGGL(kernel, grid, block, shmem, c->stream, __VA_ARGS__);                    \
    } while (0)

// Drop samples of the current solve taken after it had finished.
void prune_samples(ibm_ctx* c, int last_it) {
    for (int k = 0; k < IBM_KERNEL_COUNT; ++k) {
        auto& v = c->samples[k];
        size_t w = 0;
        for (size_t r = 0; r < v.size(); ++r) {
            if (v[r].solve == c->solve_id && v[r].it > last_it) {
                c->ev_pool.push_back(v[r].a);
                c->ev_pool.push_back(v[r].b);
            } else {
                v[w++] = v[r];
            }
        }
        v.resize(w);
    }
}

// Device address of the static scratch on the device that holds
// device_ptr, resolved once per device with that device current (every
// device holds its own copy of the array at its own address); nullptr if the
// runtime cannot resolve it.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

double* noalloc_scratch(const void* device_ptr) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, device_ptr) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    const int dev = attr.device;
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[dev]) return g_noalloc_ptr[dev];
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (cur != dev && hipSetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_noalloc_ptr[dev] = (double*)ptr;
    return g_noalloc_ptr[dev];
}

int32_t reset_ctl(ibm_ctx* c, int which) {
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, c->stream, c->ctl + which, 1);
    LAUNCH_CHECK();
    return IBM_OK;
}

int32_t fill(ibm_ctx* c, double* a, size_t n, double val) {
    if (n == 0) return IBM_OK;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, a, n, val);
    LAUNCH_CHECK();
    return IBM_OK;
}

int32_t fill_u8(ibm_ctx* c, uint8_t* a, size_t n) {
    if (n == 0) return IBM_OK;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, a, n);
    LAUNCH_CHECK();
    return IBM_OK;
}

struct LoopOut {
    int status = kStOk;
    int iters = 0;
    double bn = 0.0, r0 = 0.0, rn = 0.0;
    int zero_rhs = 0;
};

int32_t map_status(int s) {
    if (s == kStNan) return IBM_ERR_NAN;
    if (s == kStNotConverged) return IBM_NOT_CONVERGED;
    return IBM_OK;
}

// Wait for the check written to slot s and return its snapshot.
int32_t wait_slot(ibm_ctx* c, int s, Slot* out) {
    HIP_TRY(hipEventSynchronize(c->ev[s]));
    *out = read_slot(c, s);
    return IBM_OK;
}

// Checks enqueued ahead of the host.  Each entry names the host-mapped slot
// its check writes and a tag (the launch or refinement count behind it).
// Only every kEventEvery-th entry gets an event recorded behind it on the
// stream (an event record leaves the GPU idle for a few microseconds between
// two launches); the host waits on the first event at or after the entry it
// needs, and the entries before that event are complete with it.
constexpr int kEventEvery = 6;
struct PendingCheck {
    int slot;
    long tag;
    bool ev, ready;
};
struct CheckQueue {
    std::deque<PendingCheck> q;
    long count = 0;
    bool empty() const { return q.empty(); }
    size_t size() const { return q.size(); }
    void clear() { q.clear(); }
};

int32_t pend_push(ibm_ctx* c, CheckQueue& cq, int s, long tag) {
    const bool ev = (cq.count++ % kEventEvery) == 0;
    if (ev) HIP_TRY(hipEventRecord(c->ev[s], c->stream));
    cq.q.push_back(PendingCheck{s, tag, ev, false});
    return IBM_OK;
}

// The oldest entry's snapshot, once its check has run; pops it.
int32_t pend_pop(ibm_ctx* c, CheckQueue& cq, Slot* out, long* tag) {
    std::deque<PendingCheck>& q = cq.q;
    if (!q.front().ready) {
        size_t k = 0;
        while (k < q.size() && !q[k].ev) ++k;
        if (k == q.size()) {  // no event behind any entry yet: one behind the newest
            k = q.size() - 1;
            HIP_TRY(hipEventRecord(c->ev[q[k].slot], c->stream));
            q[k].ev = true;
        }
        HIP_TRY(hipEventSynchronize(c->ev[q[k].slot]));
        for (size_t m = 0; m <= k; ++m) q[m].ready = true;
    }
    *out = read_slot(c, q.front().slot);
    if (tag) *tag = q.front().tag;
    q.pop_front();
    return IBM_OK;
}

// Blocks of the mixed-precision refinement of a grid with nh_ny split
// positions (the same split for the single-grid and the batched refinement).
// Blocks of the refinement of an nx x ny grid (nh = nx / 2): items of
// kMpRefineCols split positions by kMpRefineRows rows, four per block.
inline int mp_refine_blocks(int nh, int ny) {
    const long items = (long)((nh + kMpRefineCols - 1) / kMpRefineCols) * ((ny + kMpRefineRows - 1) / kMpRefineRows);
    return (int)((items + kMpRefineThreads / kWave - 1) / (kMpRefineThreads / kWave));
}

inline int red_blocks(size_t n) {
    return (int)std::max<size_t>(1, std::min<size_t>(kRedMax, (n + kRedThreads - 1) / kRedThreads));
}

// Tile shape of the temporally blocked sweep for S iterations per launch:
// halo H = 2S + 2 (even, one ring more for the fused residual).  Returns false
// when the loaded tile would not fit the LDS budget or the per-thread
// position registers.
bool tb_shape(const ibm_ctx* c, int S, int tx, int ty, TbShape* ts) {
    if (S < 1 || S > 12 || tx < 2 || (tx & 1) || ty < 2 || (ty & 1)) return false;
    const int H = 2 * S + 2;
    const int lx = std::min(c->nx, tx + 2 * H), ly = std::min(c->ny, ty + 2 * H);
    // one lane per split column, kTbRows rows per wave
    if (lx / 2 > kTbCols || ly > kTbWaves * kTbRows) return false;
    ts->tx = tx;
    ts->ty = ty;
    ts->halo = H;
    ts->ntx = (c->nx + tx - 1) / tx;
    ts->nty = (c->ny + ty - 1) / ty;
    ts->per = (ts->ntx * ts->nty + 7) / 8;
    // two sets of per-tile residual partials (r^2, b^2) must fit the partials area
    if (4 * (size_t)ts->ntx * ts->nty > 4 * (size_t)kRedMax + (size_t)c->nx * c->ny) return false;
    return true;
}

// ---------------------------------------------------------------------------
// Red-black SOR on A x = vb, both in split storage (phr/phb, vbr/vbb).
// The residual is tested before the first iteration and after iterations
// K, 2K, ...  fixed >= 0: exactly `fixed` iterations (tolerance ignored).
// Blocked launches: the residual of each interval is summed by its last
// launch (per-tile partials, two alternating sets) and tested by the first
// launch of the next interval; the last interval's test is a k_check.  They
// read one pair of phi arrays and write the other; the launches enqueued
// after the finishing test do nothing, so the pair that holds the result
// follows from the number of blocked launches enqueued before that test.  On
// return phr/phb hold the result.
// ---------------------------------------------------------------------------
int32_t sor_loop(ibm_ctx* c, double omega, double tol, int max_iter, int K, int fixed, LoopOut* out) {
    Ctl* ctl = c->ctl + CTL_P;
    const dim3 bl(kBlock);
    const bool fixed_mode = fixed >= 0;
    const double tol_e = fixed_mode ? -1.0 : tol;
    const int max_e = fixed_mode ? fixed : max_iter;
    const int nbr = red_blocks((size_t)c->nh * c->ny);
    TbShape ts;
    // the blocked sweeps treat the domain edge as the end of the grid: periodic
    // mode sweeps colour by colour
    const bool use_tb = !c->g.per && c->sor_kernel != IBM_SOR_PER_COLOUR &&
                        tb_shape(c, c->tb_sweeps, c->tb_tx, c->tb_ty, &ts);
    auto* tb_kernel = c->sor_kernel == IBM_SOR_TEMPORAL_LDS ? k_sor_tb : k_sor_tbr;
    const int S = c->tb_sweeps;
    const int ntiles = use_tb ? ts.ntx * ts.nty : 0;
    const int tb_blocks = use_tb ? 8 * ts.per : 0;
    double* tb_part[2] = {c->partials, c->partials + 2 * (size_t)ntiles};
    int32_t rc = reset_ctl(c, CTL_P);
    if (rc) return rc;
    ++c->solve_id;
    CheckQueue pending;  // tags: blocked launches before the test
    double* cur[2] = {c->phr, c->phb};
    double* alt[2] = {c->phr2, c->phb2};
    long nlaunch = 0;
    int nint = 0;  // intervals enqueued
    // test of the last interval not yet enqueued (blocked launches)
    TbCheck carry = {nullptr, 0, 0, max_e, (int)fixed_mode, tol_e, nullptr};
    long carry_nl = 0;
    auto check = [&](int phase, int it, int nb, const double* part, long nl) -> int32_t {
        const int s = next_slot(c);
        hipLaunchKernelGGL(k_check, dim3(1), dim3(kRedThreads), 0, c->stream, ctl, part, nb, phase, it, max_e, tol_e,
                           (int)fixed_mode, 0, c->dslots + s);
        LAUNCH_CHECK();
        return pend_push(c, pending, s, nl);
    };
    timed(c, IBM_KERNEL_SOR_RESIDUAL, 0, [&](hipEvent_t ea, hipEvent_t eb) {
        LAUNCH_EV(ea, eb, k_sor_residual, dim3(nbr), dim3(kRedThreads), 0, c->g, (const double*)c->phr,
                  (const double*)c->phb, (const double*)c->vbr, (const double*)c->vbb, (const Ctl*)ctl, c->partials);
    });
    rc = check(0, 0, nbr, c->partials, 0);
    if (rc) return rc;
    Slot sn;
    bool first = true;
    int it = 0;
    long done_launches = 0;
    for (;;) {
        if (it < max_e) {
            const int next = std::min(it + K, max_e);
            double* part = tb_part[nint & 1];
            while (it < next) {
                if (use_tb) {
                    const int n = std::min(S, next - it);
                    const int resid = (it + n == next) ? 1 : 0;
                    TbCheck chk = carry;
                    int cs = -1;
                    if (chk.nb > 0) {
                        cs = next_slot(c);
                        chk.slot = c->dslots + cs;
                    }
                    auto launch = [&](hipEvent_t ea, hipEvent_t eb) {
                        // one more block takes the carried test (past the tiles)
                        LAUNCH_EV(ea, eb, tb_kernel, dim3(tb_blocks + (chk.nb > 0 ? 1 : 0)), dim3(kTbThreads), 0, c->g,
                                  (const double*)cur[0], (const double*)cur[1], alt[0], alt[1],
                                  (const double*)c->vbr, (const double*)c->vbb, omega, ctl, chk, ts, n, resid,
                                  part);
                    };
                    if (n == S) timed(c, IBM_KERNEL_SOR_TB, it + n, launch);
                    else launch(nullptr, nullptr);
                    if (cs >= 0) {
                        rc = pend_push(c, pending, cs, carry_nl);
                        if (rc) return rc;
                        carry.nb = 0;
                    }
                    std::swap(cur, alt);
                    ++nlaunch;
                    it += n;
                    if (resid) {
                        if (ntiles <= kFoldMax) {
                            carry.partials = part;
                            carry.nb = ntiles;
                            carry.it = it;
                            carry_nl = nlaunch;
                        } else {
                            rc = check(1, it, ntiles, part, nlaunch);
                            if (rc) return rc;
                        }
                    }
                } else {
                    const int itk = it + 1;
                    const dim3 grs((unsigned)((c->nh + kWave - 1) / kWave),
                                   (unsigned)((c->ny + kBlockRows * kSwRows - 1) / (kBlockRows * kSwRows)));
                    timed(c, IBM_KERNEL_SOR_SWEEP, itk, [&](hipEvent_t ea, hipEvent_t eb) {
                        LAUNCH_EV(ea, eb, k_sor_sweep<0>, grs, bl, 0, c->g, cur[0], (const double*)cur[1],
                                  (const double*)c->vbr, omega, (const Ctl*)ctl);
                    });
                    timed(c, IBM_KERNEL_SOR_SWEEP, itk, [&](hipEvent_t ea, hipEvent_t eb) {
                        LAUNCH_EV(ea, eb, k_sor_sweep<1>, grs, bl, 0, c->g, cur[1], (const double*)cur[0],
                                  (const double*)c->vbb, omega, (const Ctl*)ctl);
                    });
                    it = itk;
                }
            }
            LAUNCH_CHECK();
            ++nint;
            if (!use_tb) {
                timed(c, IBM_KERNEL_SOR_RESIDUAL, it, [&](hipEvent_t ea, hipEvent_t eb) {
                    LAUNCH_EV(ea, eb, k_sor_residual, dim3(nbr), dim3(kRedThreads), 0, c->g, (const double*)cur[0],
                              (const double*)cur[1], (const double*)c->vbr, (const double*)c->vbb, (const Ctl*)ctl,
                              c->partials);
                });
                rc = check(1, it, nbr, c->partials, nlaunch);
                if (rc) return rc;
            }
            if ((int)pending.size() < kAheadSor && it < max_e) continue;
        }
        if (it >= max_e && carry.nb > 0) {  // the last interval's test
            rc = check(1, carry.it, carry.nb, carry.partials, carry_nl);
            if (rc) return rc;
            carry.nb = 0;
        }
        if (pending.empty()) {
            c->err = "SOR loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        rc = pend_pop(c, pending, &sn, &done_launches);
        if (rc) return rc;
        if (first) {
            out->bn = sn.bn;
            out->r0 = sn.r0;
            out->zero_rhs = sn.zero_rhs;
            first = false;
        }
        if (sn.done) break;
        if (it >= max_e && pending.empty()) break;  // max_e == 0: only the first check
    }
    if (done_launches & 1) {  // the result is in the second pair
        std::swap(c->phr, c->phr2);
        std::swap(c->phb, c->phb2);
    }
    out->status = sn.status;
    out->iters = sn.iters;
    out->rn = sn.rn;
    prune_samples(c, sn.iters);
    return IBM_OK;
}

// ---------------------------------------------------------------------------
// Mixed-precision red-black SOR on A x = vb (split storage).  A refinement
// without a correction forms the residual of the initial phi (tested by a
// k_check, phase 0); each check interval then runs k_sor_mp launches on the
// correction from e = 0 and a k_mp_refine; the first launch of the next
// interval tests that refinement (the last one, a k_check).  phi and r32
// pairs alternate per refinement, e pairs per sweep launch; the phi pair that
// holds the result follows from the number of refinements enqueued before the
// finishing test.  On return phr/phb hold the result.
// ---------------------------------------------------------------------------
int32_t mp_loop(ibm_ctx* c, double omega, double tol, int max_iter, int K, int fixed, LoopOut* out) {
    Ctl* ctl = c->ctl + CTL_P;
    const bool fixed_mode = fixed >= 0;
    const double tol_e = fixed_mode ? -1.0 : tol;
    const int max_e = fixed_mode ? fixed : max_iter;
    TbShape ts;
    if (!tb_shape(c, c->tb_sweeps, c->tb_tx, c->tb_ty, &ts)) {
        c->err = "the blocked-sweep tile shape does not fit this grid";
        return IBM_ERR_INVALID;
    }
    const int S = c->tb_sweeps;
    const int tb_blocks = 8 * ts.per;
    const size_t NH = (size_t)c->nh * c->ny;
    const int nbr = mp_refine_blocks(c->nh, c->ny);
    double* part[2] = {c->partials, c->partials + 2 * (size_t)nbr};
    double* cur[2] = {c->phr, c->phb};
    double* alt[2] = {c->phr2, c->phb2};
    float* ecur[2] = {c->mpf, c->mpf + NH};
    float* ealt[2] = {c->mpf + 2 * NH, c->mpf + 3 * NH};
    float* rcur[2] = {c->mpf + 4 * NH, c->mpf + 5 * NH};
    float* ralt[2] = {c->mpf + 6 * NH, c->mpf + 7 * NH};
    int32_t rc = reset_ctl(c, CTL_P);
    if (rc) return rc;
    ++c->solve_id;
    CheckQueue pending;  // tags: refinements before the test
    long nref = 0;
    TbCheck carry = {nullptr, 0, 0, max_e, (int)fixed_mode, tol_e, nullptr};
    long carry_nl = 0;
    auto check = [&](int phase, int it, const double* prt, long nl) -> int32_t {
        const int s = next_slot(c);
        hipLaunchKernelGGL(k_check, dim3(1), dim3(kRedThreads), 0, c->stream, ctl, prt, nbr, phase, it, max_e, tol_e,
                           (int)fixed_mode, 0, c->dslots + s);
        LAUNCH_CHECK();
        return pend_push(c, pending, s, nl);
    };
    // phi + e and its residual into the other pairs
    auto refine = [&](int e_zero, int it_after) -> int32_t {
        double* prt = part[nref & 1];
        timed(c, IBM_KERNEL_SOR_MP_REFINE, it_after, [&](hipEvent_t ea, hipEvent_t eb) {
            LAUNCH_EV(ea, eb, k_mp_refine, dim3(nbr), dim3(kMpRefineThreads), 0, c->g, (const double*)cur[0],
                      (const double*)cur[1], (const float*)ecur[0], (const float*)ecur[1], e_zero,
                      (const double*)c->vbr, (const double*)c->vbb, alt[0], alt[1], ralt[0], ralt[1],
                      (const Ctl*)ctl, prt);
        });
        LAUNCH_CHECK();
        std::swap(cur, alt);
        std::swap(rcur, ralt);
        ++nref;
        carry.partials = prt;
        carry.nb = nbr;
        carry.it = it_after;
        carry_nl = nref;
        return IBM_OK;
    };
    // one sweep launch (carrying the pending test, if any)
    auto sweep = [&](int n, int e_zero, int it_after) -> int32_t {
        TbCheck chk = carry;
        int cs = -1;
        if (chk.nb > 0) {
            cs = next_slot(c);
            chk.slot = c->dslots + cs;
        }
        MpArrays a;
        a.er = ecur[0]; a.eb = ecur[1]; a.oer = ealt[0]; a.oeb = ealt[1];
        a.rr = rcur[0]; a.rb = rcur[1];
        auto go = [&](hipEvent_t ea, hipEvent_t eb) {
            LAUNCH_EV(ea, eb, k_sor_mp, dim3(tb_blocks + (chk.nb > 0 ? 1 : 0)), dim3(kTbThreads), 0, c->g, a, omega,
                      ctl, chk, ts, n,
                      e_zero);
        };
        if (n == S) timed(c, IBM_KERNEL_SOR_MP, it_after, go);
        else go(nullptr, nullptr);
        LAUNCH_CHECK();
        if (cs >= 0) {
            const int32_t r2 = pend_push(c, pending, cs, carry_nl);
            if (r2) return r2;
            carry.nb = 0;
        }
        std::swap(ecur, ealt);
        return IBM_OK;
    };
    // residual of the initial guess (phase-0 test)
    rc = refine(1, 0);
    if (rc) return rc;
    carry.nb = 0;
    rc = check(0, 0, part[0], nref);
    if (rc) return rc;
    Slot sn;
    bool first = true;
    int it = 0;
    long done_refs = 0;
    for (;;) {
        if (it < max_e) {
            const int next = std::min(it + K, max_e);
            bool start = true;
            while (it < next) {
                const int n = std::min(S, next - it);
                rc = sweep(n, start ? 1 : 0, it + n);
                if (rc) return rc;
                start = false;
                it += n;
            }
            rc = refine(0, it);
            if (rc) return rc;
            if ((int)pending.size() < kAheadSor && it < max_e) continue;
        }
        if (it >= max_e && carry.nb > 0) {  // the last refinement's test
            rc = check(1, carry.it, carry.partials, carry_nl);
            if (rc) return rc;
            carry.nb = 0;
        }
        if (pending.empty()) {
            c->err = "mixed-precision SOR loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        rc = pend_pop(c, pending, &sn, &done_refs);
        if (rc) return rc;
        if (first) {
            out->bn = sn.bn;
            out->r0 = sn.r0;
            out->zero_rhs = sn.zero_rhs;
            first = false;
        }
        if (sn.done) break;
        if (it >= max_e && pending.empty()) break;
    }
    if (done_refs & 1) {  // the result is in the second pair
        std::swap(c->phr, c->phr2);
        std::swap(c->phb, c->phb2);
    }
    out->status = sn.status;
    out->iters = sn.iters;
    out->rn = sn.rn;
    prune_samples(c, sn.iters);
    return IBM_OK;
}

// ---------------------------------------------------------------------------
// Jacobi-PCG on M x = -vb (natural layout).  fixed >= 0: exactly that many.
// Iteration kk: k_pcg_dir_spmv (stop test of r_kk, new direction, q = M p)
// then k_pcg_update (x, r); the direction is double-buffered in pp / pq2.
// ---------------------------------------------------------------------------
int32_t pcg_loop(ibm_ctx* c, double* x, const double* vb, double tol, int max_iter, int fixed, LoopOut* out) {
    Ctl* ctl = c->ctl + CTL_P;
    const dim3 bl(kBlock), rb(kRedThreads);
    const bool fixed_mode = fixed >= 0;
    const double tol_e = fixed_mode ? -1.0 : tol;
    const int max_e = fixed_mode ? fixed : max_iter;
    const size_t n = (size_t)c->nx * c->ny;
    const int nb = red_blocks(n);
    double* part_r = c->partials;                          // r.r, r.z (and b.b at the start)
    double* part_pq = c->partials + 3 * (size_t)kRedMax;  // p.q
    double* pbuf[2] = {c->pp, c->pp2};
    int32_t rc = reset_ctl(c, CTL_P);
    if (rc) return rc;
    rc = fill(c, c->pp, n, 0.0);
    if (!rc) rc = fill(c, c->pp2, n, 0.0);
    if (rc) return rc;
    ++c->solve_id;
    CheckQueue pending;
    hipLaunchKernelGGL(k_pcg_init, dim3(nb), rb, 0, c->stream, c->g, (const double*)x, vb, c->pr, c->pz, part_r);
    const int s0 = next_slot(c);
    hipLaunchKernelGGL(k_pcg_init_check, dim3(1), bl, 0, c->stream, ctl, (const double*)part_r, nb, tol_e,
                       c->dslots + s0);
    LAUNCH_CHECK();
    rc = pend_push(c, pending, s0, 0);
    if (rc) return rc;
    Slot sn;
    bool first = true;
    int kk = 0;          // next iteration to enqueue
    int restart = 0;
    for (;;) {
        if (kk <= max_e) {
            const int s = next_slot(c);
            const int k0 = kk, rs = restart;
            timed(c, IBM_KERNEL_PCG_DIR_SPMV, k0 + 1, [&](hipEvent_t ea, hipEvent_t eb) {
                LAUNCH_EV(ea, eb, k_pcg_dir_spmv, dim3(nb), rb, 0, c->g, (const double*)c->pz,
                          (const double*)pbuf[(k0 + 1) & 1], pbuf[k0 & 1], c->pq, ctl, (const double*)part_r, nb,
                          part_pq, k0, max_e, tol_e, (int)fixed_mode, rs, c->dslots + s);
            });
            restart = 0;
            if (k0 < max_e) {
                timed(c, IBM_KERNEL_PCG_UPDATE, k0 + 1, [&](hipEvent_t ea, hipEvent_t eb) {
                    LAUNCH_EV(ea, eb, k_pcg_update, dim3(nb), rb, 0, c->g, x, c->pr, c->pz, (const double*)pbuf[k0 & 1],
                              (const double*)c->pq, (const double*)c->dn, (const Ctl*)ctl, (const double*)part_pq, nb, part_r, k0);
                });
            }
            LAUNCH_CHECK();
            rc = pend_push(c, pending, s, k0);
            if (rc) return rc;
            ++kk;
            if ((int)pending.size() < kAheadPcg && kk <= max_e) continue;
        }
        if (pending.empty()) {
            c->err = "PCG loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        rc = pend_pop(c, pending, &sn, nullptr);
        if (rc) return rc;
        if (first) {
            out->bn = sn.bn;
            out->r0 = sn.r0;
            out->zero_rhs = sn.zero_rhs;
            first = false;
        }
        if (!sn.done) continue;
        if (sn.status != kStConfirm) break;
        // the recursive residual passed: confirm with the true residual
        pending.clear();
        hipLaunchKernelGGL(k_pcg_true_residual, dim3(nb), rb, 0, c->stream, c->g, (const double*)x, vb, c->pr,
                           c->pz, part_r);
        const int sc = next_slot(c);
        hipLaunchKernelGGL(k_pcg_confirm, dim3(1), bl, 0, c->stream, ctl, (const double*)part_r, nb, tol_e, 0,
                           c->dslots + sc);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(c->ev[sc], c->stream));
        rc = wait_slot(c, sc, &sn);
        if (rc) return rc;
        if (sn.done) break;
        // resume from the true residual: iteration sn.iters again with p = z
        kk = sn.iters;
        restart = 1;
    }
    if (fixed_mode && sn.status == kStOk && sn.iters > 0) {
        hipLaunchKernelGGL(k_pcg_true_residual, dim3(nb), rb, 0, c->stream, c->g, (const double*)x, vb, c->pr,
                           c->pz, part_r);
        const int s = next_slot(c);
        hipLaunchKernelGGL(k_pcg_confirm, dim3(1), bl, 0, c->stream, ctl, (const double*)part_r, nb, tol_e, 1,
                           c->dslots + s);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(c->ev[s], c->stream));
        Slot f;
        rc = wait_slot(c, s, &f);
        if (rc) return rc;
        sn.rn = f.rn;
    }
    out->status = sn.status;
    out->iters = sn.iters;
    out->rn = sn.rn;
    prune_samples(c, sn.iters);
    return IBM_OK;
}

// ---------------------------------------------------------------------------
// One-reduction Jacobi-PCG on M x = -vb (natural layout).  r = -vb + A x and
// the phase-0 test (k_pcg_init, k_pcg_init_check), w = M u (k_cg1_w), then
// one k_cg1_iter per iteration; r, w and s alternate between two buffers by
// iteration parity (r: pr / pz, w: pq / cgw, s: pp2 / cgs; p in pp), the
// partials between two sets.  A recursive residual that passes is confirmed
// with the true residual; on failure the recurrences restart from it.
// ---------------------------------------------------------------------------
int32_t cg1_loop(ibm_ctx* c, double* x, const double* vb, double tol, int max_iter, int fixed, LoopOut* out) {
    Ctl* ctl = c->ctl + CTL_P;
    const dim3 bl(kBlock), rb(kRedThreads);
    const bool fixed_mode = fixed >= 0;
    const double tol_e = fixed_mode ? -1.0 : tol;
    const int max_e = fixed_mode ? fixed : max_iter;
    const size_t n = (size_t)c->nx * c->ny;
    const int nb = red_blocks(n);  // blocks of the start kernels
    // the iteration kernel: one tile of kCgTx x kCgTy cells per block, tiles
    // banded over the XCDs as the blocked sweeps' are
    const int ntx = (c->nx + kCgTx - 1) / kCgTx, nty = (c->ny + kCgTy - 1) / kCgTy;
    const int ntiles = ntx * nty, tper = (ntiles + 7) / 8, nbt = 8 * tper;
    const size_t pstride = 3 * (size_t)std::max(nbt, kRedMax);
    double* part[2] = {c->partials, c->partials + pstride};
    double* part_b = c->partials + 2 * pstride;  // r.r, r.z, b.b of the start
    double* R[2] = {c->pr, c->pz};
    double* Wb[2] = {c->pq, c->cgw};
    double* S[2] = {c->pp2, c->cgs};
    int32_t rc = reset_ctl(c, CTL_P);
    if (rc) return rc;
    ++c->solve_id;
    CheckQueue pending;
    hipLaunchKernelGGL(k_pcg_init, dim3(nb), rb, 0, c->stream, c->g, (const double*)x, vb, R[0], Wb[1], part_b);
    const int s0 = next_slot(c);
    hipLaunchKernelGGL(k_pcg_init_check, dim3(1), bl, 0, c->stream, ctl, (const double*)part_b, nb, tol_e,
                       c->dslots + s0);
    hipLaunchKernelGGL(k_cg1_w, dim3(nb), rb, 0, c->stream, c->g, (const double*)R[0], (const double*)c->rdn, Wb[0],
                       part[0]);
    LAUNCH_CHECK();
    rc = pend_push(c, pending, s0, 0);
    if (rc) return rc;
    Slot sn;
    bool first = true;
    int kk = 0;  // next iteration to enqueue
    int restart = 1;
    for (;;) {
        if (kk <= max_e) {
            const int s = next_slot(c);
            const int k0 = kk, fr = restart;
            timed(c, IBM_KERNEL_CG1_ITER, k0 + 1, [&](hipEvent_t ea, hipEvent_t eb) {
                // the partials it reads come from k_cg1_w after a (re)start
                LAUNCH_EV(ea, eb, k_cg1_iter, dim3(nbt), dim3(kCgThreads), 0, c->g, x, c->pp,
                          (const double*)R[k0 & 1], (const double*)Wb[k0 & 1], (const double*)S[(k0 + 1) & 1],
                          R[(k0 + 1) & 1], Wb[(k0 + 1) & 1], S[k0 & 1], (const double*)c->rdn, ctl,
                          (const double*)part[k0 & 1], fr ? nb : nbt, part[(k0 + 1) & 1], k0, max_e, tol_e,
                          (int)fixed_mode, fr, c->dslots + s, ntx, ntiles, tper);
            });
            restart = 0;
            LAUNCH_CHECK();
            rc = pend_push(c, pending, s, k0);
            if (rc) return rc;
            ++kk;
            if ((int)pending.size() < kAheadPcg && kk <= max_e) continue;
        }
        if (pending.empty()) {
            c->err = "one-reduction CG loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        rc = pend_pop(c, pending, &sn, nullptr);
        if (rc) return rc;
        if (first) {
            out->bn = sn.bn;
            out->r0 = sn.r0;
            out->zero_rhs = sn.zero_rhs;
            first = false;
        }
        if (!sn.done) continue;
        if (sn.status != kStConfirm) break;
        // the recursive residual passed: confirm with the true residual of x
        // (into the r buffer of iteration sn.iters, for a restart)
        pending.clear();
        const int k1 = sn.iters;
        hipLaunchKernelGGL(k_pcg_true_residual, dim3(nb), rb, 0, c->stream, c->g, (const double*)x, vb, R[k1 & 1],
                           Wb[(k1 + 1) & 1], part_b);
        const int sc = next_slot(c);
        hipLaunchKernelGGL(k_pcg_confirm, dim3(1), bl, 0, c->stream, ctl, (const double*)part_b, nb, tol_e, 0,
                           c->dslots + sc);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(c->ev[sc], c->stream));
        rc = wait_slot(c, sc, &sn);
        if (rc) return rc;
        if (sn.done) break;
        // resume from the true residual: w = M u, then iteration k1 afresh
        hipLaunchKernelGGL(k_cg1_w, dim3(nb), rb, 0, c->stream, c->g, (const double*)R[k1 & 1],
                           (const double*)c->rdn, Wb[k1 & 1], part[k1 & 1]);
        LAUNCH_CHECK();
        kk = k1;
        restart = 1;
    }
    if (fixed_mode && sn.status == kStOk && sn.iters > 0) {
        hipLaunchKernelGGL(k_pcg_true_residual, dim3(nb), rb, 0, c->stream, c->g, (const double*)x, vb, R[0], R[1],
                           part_b);
        const int s = next_slot(c);
        hipLaunchKernelGGL(k_pcg_confirm, dim3(1), bl, 0, c->stream, ctl, (const double*)part_b, nb, tol_e, 1,
                           c->dslots + s);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(c->ev[s], c->stream));
        Slot f;
        rc = wait_slot(c, s, &f);
        if (rc) return rc;
        sn.rn = f.rn;
    }
    out->status = sn.status;
    out->iters = sn.iters;
    out->rn = sn.rn;
    prune_samples(c, sn.iters);
    return IBM_OK;
}

// ---------------------------------------------------------------------------
// Implicit viscous solve of one component, in place on u (comp 0) or v.
// ---------------------------------------------------------------------------
int32_t helm_loop(ibm_ctx* c, int comp, double beta, LoopOut* out) {
    const int which = comp == 0 ? CTL_U : CTL_V;
    Ctl* ctl = c->ctl + which;
    double* x = comp == 0 ? c->u : c->v;
    const double* rhs = comp == 0 ? c->ru : c->rv;
    const dim3 gs = grid2(c->nh, c->ny + 1), bl(kBlock);
    const size_t nunk = c->g.per ? (size_t)c->nx * c->ny
                                 : comp == 0 ? (size_t)(c->nx - 1) * c->ny : (size_t)c->nx * (c->ny - 1);
    const int nb = red_blocks(nunk);
    const double omega = c->P.uv_omega, tol = c->P.uv_tol;
    const int max_e = c->P.uv_max_iter;
    int32_t rc = reset_ctl(c, which);
    if (rc) return rc;
    std::deque<int> pending;
    auto check = [&](int phase, int it) -> int32_t {
        hipLaunchKernelGGL(k_helm_residual, dim3(nb), dim3(kRedThreads), 0, c->stream, c->g, comp, (const double*)x,
                           rhs, beta, (const Ctl*)ctl, c->partials);
        const int s = next_slot(c);
        hipLaunchKernelGGL(k_check, dim3(1), dim3(kRedThreads), 0, c->stream, ctl, (const double*)c->partials, nb, phase, it, max_e,
                           tol, 0, 1, c->dslots + s);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(c->ev[s], c->stream));
        pending.push_back(s);
        return IBM_OK;
    };
    rc = check(0, 0);
    if (rc) return rc;
    Slot sn;
    bool first = true;
    int it = 0;
    for (;;) {
        if (it < max_e) {
            if (comp == 0) {
                hipLaunchKernelGGL(k_helm_u_sweep<0>, gs, bl, 0, c->stream, c->g, x, rhs, beta, omega, (const Ctl*)ctl);
                hipLaunchKernelGGL(k_helm_u_sweep<1>, gs, bl, 0, c->stream, c->g, x, rhs, beta, omega, (const Ctl*)ctl);
            } else {
                hipLaunchKernelGGL(k_helm_v_sweep<0>, gs, bl, 0, c->stream, c->g, x, rhs, beta, omega, (const Ctl*)ctl);
                hipLaunchKernelGGL(k_helm_v_sweep<1>, gs, bl, 0, c->stream, c->g, x, rhs, beta, omega, (const Ctl*)ctl);
            }
            ++it;
            rc = check(1, it);
            if (rc) return rc;
            if ((int)pending.size() < kAheadHelm && it < max_e) continue;
        }
        if (pending.empty()) {
            c->err = "viscous loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        const int s = pending.front();
        pending.pop_front();
        rc = wait_slot(c, s, &sn);
        if (rc) return rc;
        if (first) {
            out->bn = sn.bn;
            out->r0 = sn.r0;
            first = false;
        }
        if (sn.done) break;
    }
    out->status = sn.status;
    out->iters = sn.iters;
    out->rn = sn.rn;
    return IBM_OK;
}

int worst(int a, int b) {
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

Body body_at(const ibm_ctx* c, double t) {
    Body B;
    double yb, vb, ab;
    kinematics(c->P, t, &yb, &vb, &ab);
    B.xb = c->P.x0;
    B.yb = yb;
    B.a = 0.5 * c->P.chord;
    B.b = 0.5 * c->P.thickness * c->P.chord;
    B.vb = vb;
    B.ab = ab;
    B.present = c->P.body ? 1 : 0;
    return B;
}

Coarse coarse_of(const ibm_ctx* c) { return Coarse{c->net_f, c->nx / c->net_f, c->ny / c->net_f}; }

// The network's maps of the current phi (natural layout) into wsf, and the
// RMS scales into wscale.
int32_t net_maps(ibm_ctx* c, const Body& B) {
    const Coarse cg = coarse_of(c);
    const size_t nc = (size_t)cg.ncx * cg.ncy;
    const int per = kWsThreads / (cg.f * cg.f);
    const int nb = (int)((nc + per - 1) / per);
    hipLaunchKernelGGL(k_ws_coarse, dim3(nb), dim3(kWsThreads), 0, c->stream, c->g, cg, B, (const double*)c->phi,
                       (const double*)c->vb, c->wsf, c->partials);
    hipLaunchKernelGGL(k_ws_normalize, dim3(red_blocks(nc)), dim3(kRedThreads), 0, c->stream, cg,
                       (const double*)c->partials, nb, c->net_maps, c->wscale, c->wsf);
    LAUNCH_CHECK();
    return IBM_OK;
}

// phi += a e: e the network's prediction from the maps in wsf, smoothed on
// the coarse grid and interpolated to the fine grid (into pr, free outside
// PCG), a the step of the context's rule.
int32_t net_apply(ibm_ctx* c) {
    const Coarse cg = coarse_of(c);
    const size_t nc = (size_t)cg.ncx * cg.ncy, n = (size_t)c->nx * c->ny;
    const int32_t rc = ibm_unet_forward(c->net, c->wsf, c->wsf + 3 * nc, 1);
    if (rc) {
        c->err = std::string("warm-start network: ") + ibm_unet_last_error(c->net);
        return rc;
    }
    float* y = c->wsf + 3 * nc;
    for (int k = 0; k < c->net_smooth; ++k) {
        const unsigned gb = (unsigned)((nc + 255) / 256);
        hipLaunchKernelGGL(k_ws_smooth_x, dim3(gb), dim3(256), 0, c->stream, cg, (const float*)y, y + nc);
        hipLaunchKernelGGL(k_ws_smooth_y, dim3(gb), dim3(256), 0, c->stream, cg, (const float*)(y + nc), y);
    }
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_ws_expand, dim3(nb), dim3(kRedThreads), 0, c->stream, c->g, cg, (const float*)y,
                       (const double*)c->wscale, c->net_scale, c->pr);
    const bool energy = c->net_rule == IBM_NET_STEP_ENERGY;
    if (energy)
        hipLaunchKernelGGL(k_ws_dots, dim3(nb), dim3(kRedThreads), 0, c->stream, c->g, (const double*)c->phi,
                           (const double*)c->vb, (const double*)c->pr, c->partials);
    hipLaunchKernelGGL(k_ws_apply, dim3(nb), dim3(kRedThreads), 0, c->stream, c->g, (const double*)c->pr,
                       (const double*)c->partials, nb, energy ? -1.0 : c->net_step, c->wscale, c->phi);
    LAUNCH_CHECK();
    c->n_net += 1;
    return IBM_OK;
}

// Record the maps of the current phi as the snapshot and keep phi for its
// target.
int32_t snapshot_maps(ibm_ctx* c, const Body& B) {
    int32_t rc = net_maps(c, B);
    if (rc) return rc;
    const Coarse cg = coarse_of(c);
    const size_t nc = (size_t)cg.ncx * cg.ncy, n = (size_t)c->nx * c->ny;
    HIP_TRY(hipMemcpyAsync(c->snap_feat, c->wsf, 3 * nc * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->phi0, c->phi, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return IBM_OK;
}

bool snapshot_mid_solve(const ibm_ctx* c) {
    return c->snap_feat && c->snap_iter > 0 && c->P.p_method != IBM_SOLVER_PCG;
}

// Initial guess of the step's pressure solve from phi^n (natural layout):
// zero, phi^n itself, or phi^n plus the network's prediction.  Snapshots taken
// at the start of the solve describe phi^n, whatever the initial guess.
int32_t warm_start(ibm_ctx* c, const Body& B) {
    const ibm_params& P = c->P;
    const size_t n = (size_t)c->nx * c->ny;
    if (P.p_init == IBM_INIT_LEARNED && !c->net) {
        c->err = "p_init is IBM_INIT_LEARNED but no network is attached (ibm_set_warm_start)";
        return IBM_ERR_STATE;
    }
    int32_t rc;
    if (c->snap_feat && !snapshot_mid_solve(c)) {
        rc = snapshot_maps(c, B);
        if (rc) return rc;
    }
    if (P.p_init == IBM_INIT_ZERO) return fill(c, c->phi, n, 0.0);
    if (P.p_init == IBM_INIT_LEARNED) {
        if (!c->snap_feat || snapshot_mid_solve(c)) {
            rc = net_maps(c, B);
            if (rc) return rc;
        }
        return net_apply(c);
    }
    return IBM_OK;
}

// Pressure solve of the time step on phi (natural) with vb (natural, V b).
// SOR runs in segments when a network corrects phi every net_every
// iterations, or when the snapshot is taken snap_iter iterations into the
// solve (then PCG finishes the solve for the snapshot's target).  Every
// segment ends on SOR's own stop test, so the last one decides convergence.
// Periodic (singular) mode: with rhs = 1, V b (natural layout) is made to
// sum to zero; with rhs = 0, x is shifted to zero volume-weighted mean.
// Nothing in channel mode.
int32_t per_project(ibm_ctx* c, double* a, int rhs) {
    if (!c->g.per) return IBM_OK;
    const int nb = red_blocks((size_t)c->nx * c->ny);
    hipLaunchKernelGGL(k_per_sums, dim3(nb), dim3(kRedThreads), 0, c->stream, c->g, (const double*)a, rhs ? 0 : 1,
                       c->partials);
    hipLaunchKernelGGL(k_per_shift, dim3(nb), dim3(kRedThreads), 0, c->stream, c->g, a, (const double*)c->partials,
                       nb, rhs);
    LAUNCH_CHECK();
    return IBM_OK;
}

// Periodic mode: u face nx and v row ny take the values of face 0 and row 0.
int32_t sync_periodic(ibm_ctx* c) {
    if (!c->g.per) return IBM_OK;
    const int n = std::max(c->nx, c->ny);
    hipLaunchKernelGGL(k_sync_periodic, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->nx, c->ny, c->u, c->v);
    LAUNCH_CHECK();
    return IBM_OK;
}

int32_t pressure_solve_body(ibm_ctx* c, const Body& B, int fixed, LoopOut* out);

// The pressure solve of a step; periodic mode solves the singular problem on
// the zero-sum part of V b and returns the zero-mean solution.
int32_t pressure_solve(ibm_ctx* c, const Body& B, int fixed, LoopOut* out) {
    int32_t rc = per_project(c, c->vb, 1);
    if (rc) return rc;
    rc = pressure_solve_body(c, B, fixed, out);
    if (rc) return rc;
    return out->status == kStNan ? IBM_OK : per_project(c, c->phi, 0);
}

int32_t pressure_solve_body(ibm_ctx* c, const Body& B, int fixed, LoopOut* out) {
    const ibm_params& P = c->P;
    if (P.p_method == IBM_SOLVER_PCG || P.p_method == IBM_SOLVER_CG1) {
        int32_t rc = P.p_method == IBM_SOLVER_PCG ? pcg_loop(c, c->phi, c->vb, P.p_tol, P.p_max_iter, fixed, out)
                                                  : cg1_loop(c, c->phi, c->vb, P.p_tol, P.p_max_iter, fixed, out);
        if (rc) return rc;
        if (out->zero_rhs) return fill(c, c->phi, (size_t)c->nx * c->ny, 0.0);
        return IBM_OK;
    }
    const dim3 gr = grid2(c->nh, c->ny), bl(kBlock);
    auto split_phi = [&]() {
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->phi, c->phr, c->phb, 0);
    };
    auto merge_phi = [&]() {
        hipLaunchKernelGGL(k_merge, gr, bl, 0, c->stream, c->g, (const double*)c->phr, (const double*)c->phb,
                           c->phi);
    };
    auto run = [&](int max_iter, int fx, LoopOut* o) {
        return P.p_method == IBM_SOLVER_RBSOR_MP ? mp_loop(c, P.p_omega, P.p_tol, max_iter, P.p_check_every, fx, o)
                                                 : sor_loop(c, P.p_omega, P.p_tol, max_iter, P.p_check_every, fx, o);
    };
    split_phi();
    hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->vb, c->vbr, c->vbb, 0);
    LAUNCH_CHECK();
    const bool snap_mid = fixed < 0 && snapshot_mid_solve(c);
    const bool correct = fixed < 0 && c->net && c->net_every > 0;
    int32_t rc;
    if (!snap_mid && !correct) {
        rc = run(P.p_max_iter, fixed, out);
        if (rc) return rc;
    } else {
        int done = 0;
        double rn_prev = -1.0;  // residual at the end of the previous segment
        bool corrections = correct;
        for (int seg = 0;; ++seg) {
            int lim = P.p_max_iter - done;
            if (corrections) lim = std::min(lim, c->net_every);
            if (snap_mid) lim = std::min(lim, c->snap_iter - done);
            LoopOut so;
            rc = run(lim, -1, &so);
            if (rc) return rc;
            if (seg == 0) {
                out->bn = so.bn;
                out->r0 = so.r0;
                out->zero_rhs = so.zero_rhs;
            }
            done += so.iters;
            out->iters = done;
            out->rn = so.rn;
            out->status = so.status;
            if (so.zero_rhs) break;
            const bool finished = so.status != kStNotConverged || done >= P.p_max_iter;
            merge_phi();
            LAUNCH_CHECK();
            if (snap_mid && (finished || done >= c->snap_iter)) {
                rc = snapshot_maps(c, B);
                if (rc) return rc;
                if (finished) return IBM_OK;
                LoopOut po;
                rc = pcg_loop(c, c->phi, c->vb, P.p_tol, P.p_max_iter, -1, &po);
                if (rc) return rc;
                out->iters = done + po.iters;
                out->rn = po.rn;
                out->status = po.status;
                return IBM_OK;
            }
            if (finished) return IBM_OK;
            if (corrections && c->net_rule == IBM_NET_STEP_BACKTRACK) {
                // the last correction left a larger residual after a whole
                // segment of SOR than the segment before it ended with: halve;
                // below 1/64 the rest of the solve is plain SOR
                if (rn_prev >= 0.0 && so.rn > rn_prev) c->net_step *= 0.5;
                rn_prev = so.rn;
                if (c->net_step < 1.0 / 64) corrections = false;
            }
            if (corrections) {
                rc = net_maps(c, B);
                if (rc) return rc;
                rc = net_apply(c);
                if (rc) return rc;
                split_phi();
                LAUNCH_CHECK();
            }
        }
    }
    if (out->zero_rhs) return fill(c, c->phi, (size_t)c->nx * c->ny, 0.0);
    merge_phi();
    LAUNCH_CHECK();
    return IBM_OK;
}

// Phase boundary k of the current step (phase k starts here).
int32_t phase_mark(ibm_ctx* c, int k) {
    if (!c->phase_on || c->in_batch) return IBM_OK;
    HIP_TRY(hipEventRecord(c->pev[k], c->stream));
    return IBM_OK;
}

// After the step's final synchronisation: add the phases' durations.
int32_t phase_accumulate(ibm_ctx* c) {
    if (!c->phase_on || c->in_batch) return IBM_OK;
    for (int k = 0; k < IBM_PHASE_COUNT; ++k) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, c->pev[k], c->pev[k + 1]));
        c->phase_ms[k] += ms;
    }
    c->phase_steps += 1;
    return IBM_OK;
}

// A time step is step_pre (everything up to the initial guess of the
// pressure solve), the pressure solve, and step_post (projection, pressure
// update, statistics).  A batch of contexts runs step_pre and step_post per
// context around one batched pressure solve.
int32_t step_pre(ibm_ctx* c, ibm_step_stats* st, Body* Bout, int* status_out) {
    const ibm_params& P = c->P;
    const int nx = c->nx, ny = c->ny;
    const double dt = P.dt, re = P.re, beta = dt / (2.0 * re);
    const double t1 = (double)(c->step + 1) * dt;
    std::memset(st, 0, sizeof(*st));
    const Body B = body_at(c, t1);
    *Bout = B;
    const dim3 bl(kBlock);

    // flags and forced-node lists for the body at t^{n+1}
    int32_t rc = phase_mark(c, IBM_PHASE_FLAGGING);
    if (rc) return rc;
    hipLaunchKernelGGL(k_classify, dim3(1), dim3(1024), 0, c->stream, c->g, B, c->box, c->flu, c->flv, c->msrc,
                       c->list_u, c->list_v, c->counts);
    // explicit momentum predictor
    rc = phase_mark(c, IBM_PHASE_MOMENTUM);
    if (rc) return rc;
    hipLaunchKernelGGL(k_momentum_u, grid2(nx + 1, ny), bl, 0, c->stream, c->g, (const double*)c->u,
                       (const double*)c->v, (const double*)c->p, c->nu, c->ru, dt, re, P.u_inf, c->have_hist);
    hipLaunchKernelGGL(k_momentum_v, grid2(nx, ny + 1), bl, 0, c->stream, c->g, (const double*)c->u,
                       (const double*)c->v, (const double*)c->p, c->nv, c->rv, dt, re, c->have_hist);
    // discrete forcing and forces
    rc = phase_mark(c, IBM_PHASE_FORCING);
    if (rc) return rc;
    const double uref = P.u_inf != 0.0 ? P.u_inf : 1.0;
    const double qn = 0.5 * uref * uref * P.chord;
    hipLaunchKernelGGL(k_forcing, dim3(1), dim3(1024), 0, c->stream, c->g, B, (const double*)c->u,
                       (const double*)c->v, c->ru, c->rv, (const uint8_t*)c->flu, (const uint8_t*)c->flv,
                       (const int*)c->list_u, (const int*)c->list_v, (const int*)c->counts, c->f_u, c->f_v, dt, beta,
                       P.alpha_max, qn, c->coef);
    if (!c->g.per)
        hipLaunchKernelGGL(k_outlet_commit, dim3((ny + 255) / 256), dim3(256), 0, c->stream, nx, ny, c->u,
                           (const double*)c->ru);
    LAUNCH_CHECK();
    c->have_hist = 1;

    // implicit viscous half
    rc = phase_mark(c, IBM_PHASE_UV_SOLVE);
    if (rc) return rc;
    LoopOut hu, hv;
    rc = helm_loop(c, 0, beta, &hu);
    if (rc) return rc;
    rc = helm_loop(c, 1, beta, &hv);
    if (rc) return rc;
    rc = sync_periodic(c);
    if (rc) return rc;
    st->u_iters = hu.iters;
    st->v_iters = hv.iters;
    int status = worst(map_status(hu.status), map_status(hv.status));
    if (status < 0) {
        st->status = status;
        return status;
    }

    // pressure correction
    rc = phase_mark(c, IBM_PHASE_POISSON_RHS);
    if (rc) return rc;
    hipLaunchKernelGGL(k_poisson_rhs, grid2(nx, ny), bl, 0, c->stream, c->g, (const double*)c->u,
                       (const double*)c->v, (const uint8_t*)c->flu, (const uint8_t*)c->flv,
                       (const uint8_t*)c->msrc, B.vb, dt, P.q_mode, c->vb);
    LAUNCH_CHECK();
    c->rhs_held = 1;
    c->n_net = 0;
    c->net_step = 1.0;
    if (c->net) HIP_TRY(hipMemsetAsync(c->wscale + 3, 0, sizeof(double), c->stream));
    rc = warm_start(c, B);
    if (rc) return rc;
    rc = phase_mark(c, IBM_PHASE_P_SOLVE);
    if (rc) return rc;
    *status_out = status;
    return IBM_OK;
}

int32_t step_post(ibm_ctx* c, ibm_step_stats* st, const LoopOut& po, int status) {
    const ibm_params& P = c->P;
    const int nx = c->nx, ny = c->ny;
    const double dt = P.dt, beta = dt / (2.0 * P.re);
    const double t1 = (double)(c->step + 1) * dt;
    const dim3 bl(kBlock);
    int32_t rc = phase_mark(c, IBM_PHASE_PROJECTION);
    if (rc) return rc;
    if (c->snap_target) {
        const Coarse cg = coarse_of(c);
        hipLaunchKernelGGL(k_ws_target, dim3(red_blocks((size_t)cg.ncx * cg.ncy)), dim3(kRedThreads), 0, c->stream,
                           c->g, cg, (const double*)c->phi, (const double*)c->phi0, (const double*)c->wscale,
                           c->snap_scale, c->snap_target);
        LAUNCH_CHECK();
    }
    st->p_iters = po.iters;
    st->p_r0 = po.bn > 0.0 ? po.r0 / po.bn : 0.0;
    st->p_rel = po.bn > 0.0 ? po.rn / po.bn : 0.0;
    status = worst(status, map_status(po.status));
    if (status < 0) {
        st->status = status;
        return status;
    }

    // projection and pressure update
    hipLaunchKernelGGL(k_project_u, grid2(nx + 1, ny), bl, 0, c->stream, c->g, c->u, (const double*)c->phi, dt);
    hipLaunchKernelGGL(k_project_v, grid2(nx, ny + 1), bl, 0, c->stream, c->g, c->v, (const double*)c->phi, dt);
    hipLaunchKernelGGL(k_update_p, grid2(nx, ny), bl, 0, c->stream, c->g, c->p, (const double*)c->phi, beta);
    LAUNCH_CHECK();
    rc = sync_periodic(c);
    if (rc) return rc;

    // statistics of the step
    HIP_TRY(hipMemcpyAsync(c->hstage, c->coef, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync((int*)(c->hstage + 2), c->counts, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if (c->n_net) HIP_TRY(hipMemcpyAsync(c->hstage + 4, c->wscale + 3, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    rc = phase_mark(c, IBM_PHASE_COUNT);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    rc = phase_accumulate(c);
    if (rc) return rc;
    c->cd = c->hstage[0];
    c->cl = c->hstage[1];
    const int* cnt = (const int*)(c->hstage + 2);
    st->n_forced_u = cnt[0];
    st->n_forced_v = cnt[1];
    st->n_msrc = cnt[2];
    st->n_net = c->n_net;
    st->net_step = c->n_net ? c->hstage[4] / c->n_net : 0.0;
    c->step += 1;
    c->t = t1;
    st->cd = c->cd;
    st->cl = c->cl;
    st->t = c->t;
    st->status = status;
    return status;
}

int32_t step_once(ibm_ctx* c, ibm_step_stats* st) {
    Body B;
    int status = IBM_OK;
    int32_t rc = step_pre(c, st, &B, &status);
    if (rc) return rc;
    if (status < 0) return status;
    int fixed = -1;
    if (c->sched_pos < c->schedule.size()) fixed = c->schedule[c->sched_pos++];
    LoopOut po;
    rc = pressure_solve(c, B, fixed, &po);
    if (rc) return rc;
    return step_post(c, st, po, status);
}

// Face metrics and operator coefficients, computed on the host.
void host_metrics(const ibm_params& P, const double* xf, const double* yf, std::vector<std::vector<double>>& A) {
    const int nx = P.nx, ny = P.ny;
    std::vector<double> dx(nx), dy(ny), xc(nx), yc(ny), dxu(nx + 1), dyv(ny + 1);
    for (int i = 0; i < nx; ++i) { dx[i] = xf[i + 1] - xf[i]; xc[i] = 0.5 * (xf[i] + xf[i + 1]); }
    for (int j = 0; j < ny; ++j) { dy[j] = yf[j + 1] - yf[j]; yc[j] = 0.5 * (yf[j] + yf[j + 1]); }
    for (int i = 1; i < nx; ++i) dxu[i] = xc[i] - xc[i - 1];
    for (int j = 1; j < ny; ++j) dyv[j] = yc[j] - yc[j - 1];
    const bool per = P.bc_mode == IBM_BC_PERIODIC;
    if (per) {  // the two ends are neighbours
        dxu[0] = dxu[nx] = 0.5 * (dx[nx - 1] + dx[0]);
        dyv[0] = dyv[ny] = 0.5 * (dy[ny - 1] + dy[0]);
    } else {    // half cells at the ends
        dxu[0] = 0.5 * dx[0];
        dxu[nx] = 0.5 * dx[nx - 1];
        dyv[0] = 0.5 * dy[0];
        dyv[ny] = 0.5 * dy[ny - 1];
    }
    std::vector<double> pcE(nx, 0.0), pcW(nx, 0.0), pcD(nx, 0.0), pcN(ny, 0.0), pcS(ny, 0.0);
    for (int i = 0; i < nx; ++i) {
        if (per || i < nx - 1) pcE[i] = 1.0 / dxu[i + 1];
        if (per || i > 0) pcW[i] = 1.0 / dxu[i];
        if (!per && i == nx - 1) pcD[i] = 1.0 / dxu[nx];
    }
    for (int j = 0; j < ny; ++j) {
        if (per || j < ny - 1) pcN[j] = 1.0 / dyv[j + 1];
        if (per || j > 0) pcS[j] = 1.0 / dyv[j];
    }
    std::vector<double> uce(nx + 1, 0.0), ucw(nx + 1, 0.0), ucn(ny, 0.0), ucs(ny, 0.0);
    for (int i = per ? 0 : 1; i < nx; ++i) {
        uce[i] = 1.0 / (dx[i] * dxu[i]);
        ucw[i] = 1.0 / (dx[i > 0 ? i - 1 : nx - 1] * dxu[i]);
    }
    for (int j = 0; j < ny; ++j) {
        if (per || j < ny - 1) ucn[j] = 1.0 / (dyv[j + 1] * dy[j]);
        if (per || j > 0) ucs[j] = 1.0 / (dyv[j] * dy[j]);
    }
    std::vector<double> vce(nx, 0.0), vcw(nx, 0.0), vcn(ny + 1, 0.0), vcs(ny + 1, 0.0);
    for (int i = 0; i < nx; ++i) {
        if (per || i < nx - 1) vce[i] = 1.0 / (dxu[i + 1] * dx[i]);
        vcw[i] = 1.0 / (dxu[i] * dx[i]);
    }
    for (int j = per ? 0 : 1; j < ny; ++j) {
        vcn[j] = 1.0 / (dy[j] * dyv[j]);
        vcs[j] = 1.0 / (dy[j > 0 ? j - 1 : ny - 1] * dyv[j]);
    }
    A = {std::vector<double>(xf, xf + nx + 1), std::vector<double>(yf, yf + ny + 1), dx, dy, xc, yc, dxu, dyv,
         pcE, pcW, pcD, pcN, pcS, uce, ucw, ucn, ucs, vce, vcw, vcn, vcs};
}

// Motion box: cells that any forced node of the run can touch, with margin.
Box motion_box(const ibm_params& P, const double* xf, const double* yf) {
    Box b;
    const int nx = P.nx, ny = P.ny;
    if (!P.body) {
        b.bi0 = 1; b.bi1 = 1; b.bj0 = 1; b.bj1 = 1;
        return b;
    }
    const double a = 0.5 * P.chord, bb = 0.5 * P.thickness * P.chord, amp = std::fabs(P.amp);
    const double xlo = P.x0 - a, xhi = P.x0 + a, ylo = P.y0 - amp - bb, yhi = P.y0 + amp + bb;
    int i0 = 0, i1 = nx, j0 = 0, j1 = ny;
    while (i0 < nx && xf[i0 + 1] < xlo) ++i0;
    while (i1 > 0 && xf[i1 - 1] > xhi) --i1;
    while (j0 < ny && yf[j0 + 1] < ylo) ++j0;
    while (j1 > 0 && yf[j1 - 1] > yhi) --j1;
    b.bi0 = std::max(1, i0 - 3);
    b.bi1 = std::min(nx - 1, i1 + 3);
    b.bj0 = std::max(1, j0 - 3);
    b.bj1 = std::min(ny - 1, j1 + 3);
    return b;
}

// ---------------------------------------------------------------------------
// Batches: many contexts whose red-black SOR pressure solves run as one
// blocked launch per S iterations over a work list of all their tiles.
// ---------------------------------------------------------------------------
constexpr int kBatchRing = kAheadSor + 2;  // check entries in flight
constexpr int kMaxGraphIntervals = 1000;   // check intervals in one captured stretch

}  // namespace

struct ibm_batch {
    std::vector<ibm_ctx*> cs;
    hipStream_t stream = nullptr;
    int S = 0, K = 0, ntotal = 0, per = 0, max_iter = 0;
    TbCase* dcases = nullptr;  // device descriptors
    TbCase* hcases = nullptr;  // pinned staging of the descriptors
    Slot* hslots = nullptr;    // kBatchRing x n host-mapped snapshots
    Slot* dslots = nullptr;
    hipEvent_t ev[kBatchRing] = {};
    long seq = 0;
    // captured stretches: graph_iv check intervals of launches in one HIP graph
    int graph_iv = 0;                // 0: every launch from the host
    hipStream_t cap = nullptr;       // private stream the graph is captured on
    hipGraphExec_t gexec = nullptr;  // instantiated for (g_ntotal, g_per, g_iv)
    int g_ntotal = -1, g_per = -1, g_iv = 0;
    int* dcur = nullptr;             // {iteration base, slot entry} read by the captured checks
    // mixed-precision batches (every context IBM_SOLVER_RBSOR_MP)
    bool mp = false;
    MpCase* dmp = nullptr;  // device descriptors
    MpCase* hmp = nullptr;  // pinned staging
    int nrblk = 0;          // refinement blocks of all cases
    int g_nrblk = -1;       // refinement blocks the captured graph was made for
    std::string err;
};

namespace {

#define BATCH_TRY(expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            b->err = std::string(#expr) + ": " + hipGetErrorString(e_);                        \
            return IBM_ERR_HIP;                                                                \
        }                                                                                      \
    } while (0)

// The descriptors of the current split phi pairs (they swap between solves).
int32_t batch_upload(ibm_batch* b) {
    const int n = (int)b->cs.size();
    int tile0 = 0;
    b->max_iter = 0;
    for (int k = 0; k < n; ++k) {
        ibm_ctx* c = b->cs[k];
        TbCase& d = b->hcases[k];
        if (!tb_shape(c, b->S, c->tb_tx, c->tb_ty, &d.ts) || d.ts.ntx * d.ts.nty > kFoldMax) {
            b->err = "case " + std::to_string(k) + ": its tile shape no longer fits the batched sweep";
            return IBM_ERR_STATE;
        }
        d.g = c->g;
        d.ph[0][0] = c->phr;
        d.ph[0][1] = c->phb;
        d.ph[1][0] = c->phr2;
        d.ph[1][1] = c->phb2;
        d.bred = c->vbr;
        d.bblack = c->vbb;
        d.ntiles = d.ts.ntx * d.ts.nty;
        d.partials[0] = c->partials;
        d.partials[1] = c->partials + 2 * (size_t)d.ntiles;
        d.ctl = c->ctl + CTL_P;
        d.omega = c->P.p_omega;
        d.tol = c->batch_fixed >= 0 ? -1.0 : c->P.p_tol;
        d.max_iter = c->batch_fixed >= 0 ? c->batch_fixed : c->P.p_max_iter;
        d.fixed = c->batch_fixed >= 0 ? 1 : 0;
        b->max_iter = std::max(b->max_iter, d.max_iter);
        d.tile0 = tile0;
        d.nb0 = red_blocks((size_t)c->nh * c->ny);
        tile0 += d.ntiles;
    }
    b->ntotal = tile0;
    b->per = (tile0 + 7) / 8;
    BATCH_TRY(hipMemcpyAsync(b->dcases, b->hcases, n * sizeof(TbCase), hipMemcpyHostToDevice, b->stream));
    return IBM_OK;
}

// Blocked launches of the batched sweep before the check after `it`
// iterations: check intervals of K iterations (the last one of a solve may be
// shorter), each split into launches of at most S iterations.
long batch_launches_at(const ibm_batch* b, int it) {
    const long per_iv = (b->K + b->S - 1) / b->S;
    return (long)(it / b->K) * per_iv + ((it % b->K) + b->S - 1) / b->S;
}

// Captures graph_iv check intervals of the batched loop (starting after an
// even number of intervals and launches, so that the pair flips and partial
// sets repeat from one stretch to the next) into one HIP graph.  The checks
// take their iteration base and snapshot entry from the cursor.
int32_t batch_capture(ibm_batch* b) {
    if (b->gexec && b->g_ntotal == b->ntotal && b->g_per == b->per && b->g_iv == b->graph_iv) return IBM_OK;
    if (b->gexec) {
        BATCH_TRY(hipStreamSynchronize(b->stream));  // a replay of the old graph may still run
        BATCH_TRY(hipGraphExecDestroy(b->gexec));
        b->gexec = nullptr;
    }
    const int n = (int)b->cs.size();
    BATCH_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    long nl = 0;
    for (int j = 0; j < b->graph_iv; ++j) {
        for (int i = 0; i < b->K;) {
            const int ns = std::min(b->S, b->K - i);
            const int resid = (i + ns == b->K) ? 1 : 0;
            hipLaunchKernelGGL(k_sor_tbr_batch, dim3(8 * b->per), dim3(kTbThreads), 0, b->cap,
                               (const TbCase*)b->dcases, n, b->ntotal, b->per, (int)(nl & 1), ns, resid, j & 1);
            ++nl;
            i += ns;
        }
        hipLaunchKernelGGL(k_check_batch, dim3(n), dim3(kTbThreads), 0, b->cap, (const TbCase*)b->dcases, 1,
                           (j + 1) * b->K, j & 1, b->dslots, (const int*)b->dcur);
    }
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        b->err = std::string("capture of the batched sweep failed: ") +
                 hipGetErrorString(le != hipSuccess ? le : ce);
        return IBM_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiateWithFlags(&b->gexec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        b->gexec = nullptr;
        b->err = std::string("hipGraphInstantiateWithFlags: ") + hipGetErrorString(ie);
        return IBM_ERR_HIP;
    }
    b->g_ntotal = b->ntotal;
    b->g_per = b->per;
    b->g_iv = b->graph_iv;
    return IBM_OK;
}

// The descriptors of the mixed-precision cases (current phi pairs).
int32_t batch_upload_mp(ibm_batch* b) {
    const int n = (int)b->cs.size();
    b->max_iter = 0;
    int tile0 = 0, rblk0 = 0;
    for (int k = 0; k < n; ++k) {
        ibm_ctx* c = b->cs[k];
        MpCase& d = b->hmp[k];
        if (!tb_shape(c, b->S, c->tb_tx, c->tb_ty, &d.ts)) {
            b->err = "case " + std::to_string(k) + ": its tile shape no longer fits the batched sweep";
            return IBM_ERR_STATE;
        }
        const size_t NH = (size_t)c->nh * c->ny;
        d.g = c->g;
        d.ph[0][0] = c->phr;
        d.ph[0][1] = c->phb;
        d.ph[1][0] = c->phr2;
        d.ph[1][1] = c->phb2;
        for (int q = 0; q < 2; ++q)
            for (int col = 0; col < 2; ++col) {
                d.e[q][col] = c->mpf + (2 * q + col) * NH;
                d.r[q][col] = c->mpf + (4 + 2 * q + col) * NH;
            }
        d.bred = c->vbr;
        d.bblack = c->vbb;
        d.nbr = mp_refine_blocks(c->nh, c->ny);
        d.partials[0] = c->partials;
        d.partials[1] = c->partials + 2 * (size_t)d.nbr;
        d.ctl = c->ctl + CTL_P;
        d.omega = c->P.p_omega;
        d.tol = c->batch_fixed >= 0 ? -1.0 : c->P.p_tol;
        d.max_iter = c->batch_fixed >= 0 ? c->batch_fixed : c->P.p_max_iter;
        d.fixed = c->batch_fixed >= 0 ? 1 : 0;
        b->max_iter = std::max(b->max_iter, d.max_iter);
        d.tile0 = tile0;
        d.ntiles = d.ts.ntx * d.ts.nty;
        d.rblk0 = rblk0;
        tile0 += d.ntiles;
        rblk0 += d.nbr;
    }
    b->ntotal = tile0;
    b->per = (tile0 + 7) / 8;
    b->nrblk = rblk0;
    BATCH_TRY(hipMemcpyAsync(b->dmp, b->hmp, n * sizeof(MpCase), hipMemcpyHostToDevice, b->stream));
    return IBM_OK;
}

// Captures graph_iv check intervals of the batched mixed-precision loop
// (float sweeps from e = 0, refinement, stop tests) into one HIP graph.  A
// stretch starts after an even number of intervals, i.e. after an odd number
// of refinements (the initial one included) and an even number of sweep
// launches, so its pair selectors are the same in every stretch; the checks
// take their iteration base and snapshot entry from the cursor.
int32_t batch_capture_mp(ibm_batch* b) {
    if (b->gexec && b->g_ntotal == b->ntotal && b->g_per == b->per && b->g_iv == b->graph_iv &&
        b->g_nrblk == b->nrblk)
        return IBM_OK;
    if (b->gexec) {
        BATCH_TRY(hipStreamSynchronize(b->stream));  // a replay of the old graph may still run
        BATCH_TRY(hipGraphExecDestroy(b->gexec));
        b->gexec = nullptr;
    }
    const int n = (int)b->cs.size();
    BATCH_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    long nsw = 0, nref = 1;
    for (int j = 0; j < b->graph_iv; ++j) {
        int e_zero = 1;
        for (int i = 0; i < b->K;) {
            const int ns = std::min(b->S, b->K - i);
            hipLaunchKernelGGL(k_sor_mp_batch, dim3(8 * b->per), dim3(kTbThreads), 0, b->cap, (const MpCase*)b->dmp,
                               n, b->ntotal, b->per, (int)(nsw & 1), (int)(nref & 1), ns, e_zero);
            ++nsw;
            e_zero = 0;
            i += ns;
        }
        hipLaunchKernelGGL(k_mp_refine_batch, dim3(b->nrblk), dim3(kMpRefineThreads), 0, b->cap, (const MpCase*)b->dmp, n,
                           b->nrblk, (int)(nref & 1), (int)(nsw & 1), 0, (int)((nref + 1) & 1), (int)(nref & 1));
        ++nref;
        hipLaunchKernelGGL(k_check_mp_batch, dim3(n), dim3(kTbThreads), 0, b->cap, (const MpCase*)b->dmp, 1,
                           (j + 1) * b->K, (int)((nref - 1) & 1), b->dslots, (const int*)b->dcur);
    }
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        b->err = std::string("capture of the batched mixed-precision solve failed: ") +
                 hipGetErrorString(le != hipSuccess ? le : ce);
        return IBM_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiateWithFlags(&b->gexec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        b->gexec = nullptr;
        b->err = std::string("hipGraphInstantiateWithFlags: ") + hipGetErrorString(ie);
        return IBM_ERR_HIP;
    }
    b->g_ntotal = b->ntotal;
    b->g_per = b->per;
    b->g_iv = b->graph_iv;
    b->g_nrblk = b->nrblk;
    return IBM_OK;
}

// The mixed-precision pressure solves of all contexts of the batch, in the
// single-grid order: a refinement of the initial phi (phase-0 test), then per
// check interval the float sweeps from e = 0, a refinement and the test.
// Pair selectors advance with the global counts of sweeps and refinements;
// the phi pair holding a case's result follows from the refinements before
// its finishing test.
int32_t batch_sor_mp(ibm_batch* b, std::vector<LoopOut>& outs) {
    const int n = (int)b->cs.size();
    for (ibm_ctx* c : b->cs) {
        const dim3 gr = grid2(c->nh, c->ny), bl(kBlock);
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->phi, c->phr, c->phb, 0);
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->vb, c->vbr, c->vbb, 0);
        int32_t rc = reset_ctl(c, CTL_P);
        if (rc) return rc;
        if (hipGetLastError() != hipSuccess) {
            b->err = "launch failed";
            return IBM_ERR_HIP;
        }
    }
    int32_t rc = batch_upload_mp(b);
    if (rc) return rc;
    if (b->graph_iv > 0) {
        rc = batch_capture_mp(b);
        if (rc) return rc;
    }
    long nref = 0, nsw = 0;
    auto refine = [&](int e_zero) -> int32_t {
        hipLaunchKernelGGL(k_mp_refine_batch, dim3(b->nrblk), dim3(kMpRefineThreads), 0, b->stream, (const MpCase*)b->dmp,
                           n, b->nrblk, (int)(nref & 1), (int)(nsw & 1), e_zero, (int)((nref + 1) & 1),
                           (int)(nref & 1));
        if (hipGetLastError() != hipSuccess) {
            b->err = "k_mp_refine_batch launch failed";
            return IBM_ERR_HIP;
        }
        ++nref;
        return IBM_OK;
    };
    std::deque<std::pair<int, long>> pending;  // (ring entry, refinements before its test)
    auto check = [&](int phase, int it) -> int32_t {
        const int e = (int)(b->seq++ % kBatchRing);
        hipLaunchKernelGGL(k_check_mp_batch, dim3(n), dim3(kTbThreads), 0, b->stream,
                           (const MpCase*)b->dmp, phase, it, (int)((nref - 1) & 1), b->dslots + (size_t)e * n,
                           (const int*)nullptr);
        if (hipGetLastError() != hipSuccess) {
            b->err = "k_check_mp_batch launch failed";
            return IBM_ERR_HIP;
        }
        BATCH_TRY(hipEventRecord(b->ev[e], b->stream));
        pending.emplace_back(e, nref);
        return IBM_OK;
    };
    rc = refine(1);
    if (rc) return rc;
    rc = check(0, 0);
    if (rc) return rc;
    std::vector<char> finished(n, 0);
    std::vector<long> done_refs(n, 0);
    int nfin = 0, it = 0, nint = 0;
    bool first = true;
    const int max_e = b->max_iter;
    const long stretch = (long)b->graph_iv * b->K;
    const long per_iv = (b->K + b->S - 1) / b->S;
    const int ahead = b->graph_iv > 0 ? std::max(2, kAheadSor / b->graph_iv) : kAheadSor;
    for (;;) {
        if (it < max_e && b->gexec && (nint & 1) == 0 && it + stretch <= max_e) {
            // a captured stretch of graph_iv intervals (it starts after an even
            // number of intervals: an odd number of refinements, an even
            // number of sweep launches, as at its capture)
            const int e = (int)(b->seq++ % kBatchRing);
            hipLaunchKernelGGL(k_batch_cursor, dim3(1), dim3(kWave), 0, b->stream, b->dcur, it, e);
            if (hipGetLastError() != hipSuccess) {
                b->err = "k_batch_cursor launch failed";
                return IBM_ERR_HIP;
            }
            BATCH_TRY(hipGraphLaunch(b->gexec, b->stream));
            BATCH_TRY(hipEventRecord(b->ev[e], b->stream));
            pending.emplace_back(e, -1L);
            it += (int)stretch;
            nint += b->graph_iv;
            nsw += per_iv * b->graph_iv;
            nref += b->graph_iv;
            if ((int)pending.size() < ahead && it < max_e) continue;
        } else if (it < max_e) {
            ++nint;
            const int next = std::min(it + b->K, max_e);
            int e_zero = 1;
            while (it < next) {
                const int ns = std::min(b->S, next - it);
                hipLaunchKernelGGL(k_sor_mp_batch, dim3(8 * b->per), dim3(kTbThreads), 0, b->stream,
                                   (const MpCase*)b->dmp, n, b->ntotal, b->per, (int)(nsw & 1), (int)(nref & 1), ns,
                                   e_zero);
                ++nsw;
                e_zero = 0;
                it += ns;
            }
            if (hipGetLastError() != hipSuccess) {
                b->err = "k_sor_mp_batch launch failed";
                return IBM_ERR_HIP;
            }
            rc = refine(0);
            if (rc) return rc;
            rc = check(1, it);
            if (rc) return rc;
            if ((int)pending.size() < kAheadSor && it < max_e) continue;
        }
        if (pending.empty()) {
            b->err = "batched mixed-precision loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        const int e = pending.front().first;
        const long nr = pending.front().second;
        pending.pop_front();
        BATCH_TRY(hipEventSynchronize(b->ev[e]));
        for (int k = 0; k < n; ++k) {
            if (finished[k]) continue;
            volatile Slot* hs = b->hslots + (size_t)e * n + k;
            if (first) {
                outs[k].bn = hs->bn;
                outs[k].r0 = hs->r0;
                outs[k].zero_rhs = hs->zero_rhs;
            }
            if (hs->done) {
                finished[k] = 1;
                ++nfin;
                // inside a captured stretch: the initial refinement and one per
                // interval up to the case's test
                done_refs[k] = nr >= 0 ? nr : 1 + (hs->iters + b->K - 1) / b->K;
                outs[k].status = hs->status;
                outs[k].iters = hs->iters;
                outs[k].rn = hs->rn;
            }
        }
        first = false;
        if (nfin == n) break;
        if (it >= max_e && pending.empty()) {
            b->err = "batched mixed-precision loop: a case neither finished nor reached its iteration limit";
            return IBM_ERR_STATE;
        }
    }
    for (int k = 0; k < n; ++k) {
        if (done_refs[k] & 1) {
            ibm_ctx* c = b->cs[k];
            std::swap(c->phr, c->phr2);
            std::swap(c->phb, c->phb2);
        }
    }
    return IBM_OK;
}

// The pressure solves of all contexts of the batch (phi and V b natural on
// entry; on return the solution is in each context's (phr, phb) pair).
int32_t batch_sor(ibm_batch* b, std::vector<LoopOut>& outs) {
    if (b->mp) return batch_sor_mp(b, outs);
    const int n = (int)b->cs.size();
    for (ibm_ctx* c : b->cs) {
        const dim3 gr = grid2(c->nh, c->ny), bl(kBlock);
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->phi, c->phr, c->phb, 0);
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->vb, c->vbr, c->vbb, 0);
        int32_t rc = reset_ctl(c, CTL_P);
        if (rc) return rc;
        hipLaunchKernelGGL(k_sor_residual, dim3(red_blocks((size_t)c->nh * c->ny)), dim3(kRedThreads), 0,
                           c->stream, c->g, (const double*)c->phr, (const double*)c->phb, (const double*)c->vbr,
                           (const double*)c->vbb, (const Ctl*)(c->ctl + CTL_P), c->partials);
        if (hipGetLastError() != hipSuccess) {
            b->err = "launch failed";
            return IBM_ERR_HIP;
        }
    }
    int32_t rc = batch_upload(b);
    if (rc) return rc;
    if (b->graph_iv > 0) {
        rc = batch_capture(b);
        if (rc) return rc;
    }
    // (ring entry, blocked launches before its test; -1: a captured stretch,
    // whose launch count at a case's finish follows from its iteration count)
    std::deque<std::pair<int, long>> pending;
    auto check = [&](int phase, int it, int pbuf, long nl) -> int32_t {
        const int e = (int)(b->seq++ % kBatchRing);
        // every phase sums its partials with the thread count of the
        // single-grid tests (k_check and the folded test), so in their order
        hipLaunchKernelGGL(k_check_batch, dim3(n), dim3(kTbThreads), 0, b->stream,
                           (const TbCase*)b->dcases, phase, it, pbuf, b->dslots + (size_t)e * n,
                           (const int*)nullptr);
        if (hipGetLastError() != hipSuccess) {
            b->err = "k_check_batch launch failed";
            return IBM_ERR_HIP;
        }
        BATCH_TRY(hipEventRecord(b->ev[e], b->stream));
        pending.emplace_back(e, nl);
        return IBM_OK;
    };
    rc = check(0, 0, 0, 0);
    if (rc) return rc;
    std::vector<char> finished(n, 0);
    std::vector<long> done_launches(n, 0);
    int nfin = 0;
    bool first = true;
    long nlaunch = 0;
    int nint = 0, it = 0;
    const int max_e = b->max_iter;
    const long stretch = (long)b->graph_iv * b->K;
    const int ahead = b->graph_iv > 0 ? std::max(2, kAheadSor / b->graph_iv) : kAheadSor;
    for (;;) {
        if (it < max_e && b->gexec && (nint & 1) == 0 && (nlaunch & 1) == 0 && it + stretch <= max_e) {
            const int e = (int)(b->seq++ % kBatchRing);
            hipLaunchKernelGGL(k_batch_cursor, dim3(1), dim3(kWave), 0, b->stream, b->dcur, it, e);
            if (hipGetLastError() != hipSuccess) {
                b->err = "k_batch_cursor launch failed";
                return IBM_ERR_HIP;
            }
            BATCH_TRY(hipGraphLaunch(b->gexec, b->stream));
            BATCH_TRY(hipEventRecord(b->ev[e], b->stream));
            pending.emplace_back(e, -1L);
            it += (int)stretch;
            nint += b->graph_iv;
            nlaunch += batch_launches_at(b, (int)stretch);
            if ((int)pending.size() < ahead && it < max_e) continue;
        } else if (it < max_e) {
            const int next = std::min(it + b->K, max_e);
            const int pbuf = nint & 1;
            while (it < next) {
                const int ns = std::min(b->S, next - it);
                const int resid = (it + ns == next) ? 1 : 0;
                hipLaunchKernelGGL(k_sor_tbr_batch, dim3(8 * b->per), dim3(kTbThreads), 0, b->stream,
                                   (const TbCase*)b->dcases, n, b->ntotal, b->per, (int)(nlaunch & 1), ns, resid,
                                   pbuf);
                ++nlaunch;
                it += ns;
            }
            if (hipGetLastError() != hipSuccess) {
                b->err = "k_sor_tbr_batch launch failed";
                return IBM_ERR_HIP;
            }
            ++nint;
            rc = check(1, it, pbuf, nlaunch);
            if (rc) return rc;
            if ((int)pending.size() < kAheadSor && it < max_e) continue;
        }
        if (pending.empty()) {
            b->err = "batched SOR loop ended without a finishing check";
            return IBM_ERR_STATE;
        }
        const int e = pending.front().first;
        const long nl = pending.front().second;
        pending.pop_front();
        BATCH_TRY(hipEventSynchronize(b->ev[e]));
        for (int k = 0; k < n; ++k) {
            if (finished[k]) continue;
            volatile Slot* hs = b->hslots + (size_t)e * n + k;
            if (first) {
                outs[k].bn = hs->bn;
                outs[k].r0 = hs->r0;
                outs[k].zero_rhs = hs->zero_rhs;
            }
            if (hs->done) {
                finished[k] = 1;
                ++nfin;
                done_launches[k] = nl >= 0 ? nl : batch_launches_at(b, hs->iters);
                outs[k].status = hs->status;
                outs[k].iters = hs->iters;
                outs[k].rn = hs->rn;
            }
        }
        first = false;
        if (nfin == n) break;
        if (it >= max_e && pending.empty()) {
            b->err = "batched SOR loop: a case neither finished nor reached its iteration limit";
            return IBM_ERR_STATE;
        }
    }
    for (int k = 0; k < n; ++k) {
        if (done_launches[k] & 1) {
            ibm_ctx* c = b->cs[k];
            std::swap(c->phr, c->phr2);
            std::swap(c->phb, c->phb2);
        }
    }
    return IBM_OK;
}

}  // namespace

namespace {

// Red-black SOR solve of a stand-alone right-hand side: x and V rhs into the
// split arrays, the solve, the result back into x (x = 0 for rhs = 0).
int32_t split_sor_solve(ibm_ctx* c, const double* rhs_dev, double* x_dev, const ibm_solve_opts* o, int fixed,
                        LoopOut* lo) {
    const dim3 gr = grid2(c->nh, c->ny), bl(kBlock);
    hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)x_dev, c->phr, c->phb, 0);
    hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, rhs_dev, c->vbr, c->vbb, 1);
    LAUNCH_CHECK();
    int32_t rc;
    if (c->g.per) {  // singular: the zero-sum part of V rhs (natural layout in vb)
        hipLaunchKernelGGL(k_merge, gr, bl, 0, c->stream, c->g, (const double*)c->vbr, (const double*)c->vbb, c->vb);
        LAUNCH_CHECK();
        rc = per_project(c, c->vb, 1);
        if (rc) return rc;
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, (const double*)c->vb, c->vbr, c->vbb, 0);
        LAUNCH_CHECK();
    }
    rc = o->method == IBM_SOLVER_RBSOR_MP ? mp_loop(c, o->omega, o->tol, o->max_iter, o->check_every, fixed, lo)
                                          : sor_loop(c, o->omega, o->tol, o->max_iter, o->check_every, fixed, lo);
    if (rc) return rc;
    if (lo->zero_rhs) return fill(c, x_dev, (size_t)c->nx * c->ny, 0.0);
    hipLaunchKernelGGL(k_merge, gr, bl, 0, c->stream, c->g, (const double*)c->phr, (const double*)c->phb, x_dev);
    LAUNCH_CHECK();
    return lo->status == kStNan ? IBM_OK : per_project(c, x_dev, 0);
}

// Statistics of a stand-alone solve (GPU time between the context's t0 and
// t1 events) and its status.
int32_t solve_stats(ibm_ctx* c, const LoopOut& lo, ibm_solve_stats* st) {
    HIP_TRY(hipEventRecord(c->t1, c->stream));
    HIP_TRY(hipEventSynchronize(c->t1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, c->t0, c->t1));
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->status = map_status(lo.status);
        st->iters = lo.iters;
        st->r0_rel = lo.bn > 0.0 ? lo.r0 / lo.bn : 0.0;
        st->rel = lo.bn > 0.0 ? lo.rn / lo.bn : 0.0;
        st->seconds = 1e-3 * ms;
    }
    return map_status(lo.status);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

size_t ibm_workspace_bytes(const ibm_params* prm) {
    if (!prm || prm->nx < 8 || prm->ny < 8 || (prm->nx & 1) || (prm->ny & 1)) return 0;
    if ((int64_t)(prm->nx + 1) * (prm->ny + 1) > (int64_t)1 << 30) return 0;
    return layout_for(prm->nx, prm->ny).total;
}

int32_t ibm_batch_create(int32_t n, ibm_ctx* const* ctxs, ibm_batch** out) {
    if (!out) return IBM_ERR_INVALID;
    *out = nullptr;
    if (n < 1 || n > 4096 || !ctxs) return IBM_ERR_INVALID;
    for (int k = 0; k < n; ++k) {
        const ibm_ctx* c = ctxs[k];
        if (!c) return IBM_ERR_INVALID;
        for (int q = 0; q < k; ++q)
            if (ctxs[q] == c) return IBM_ERR_INVALID;  // a context appears once
        const bool method_ok = c->P.p_method == ctxs[0]->P.p_method &&
                               ((c->P.p_method == IBM_SOLVER_RBSOR && c->sor_kernel == IBM_SOR_TEMPORAL) ||
                                c->P.p_method == IBM_SOLVER_RBSOR_MP);
        if (c->stream != ctxs[0]->stream || !method_ok ||
            c->tb_sweeps != ctxs[0]->tb_sweeps || c->P.p_check_every != ctxs[0]->P.p_check_every ||
            (c->net && c->net_every > 0) || c->snap_feat || c->g.per)
            return IBM_ERR_INVALID;
        TbShape ts;
        if (!tb_shape(c, c->tb_sweeps, c->tb_tx, c->tb_ty, &ts) || ts.ntx * ts.nty > kFoldMax) return IBM_ERR_INVALID;
    }
    // The batched loop advances every case in whole check intervals; a case
    // stops at its own limit only when that limit falls on an interval's end
    // (or when all cases share it, so the last interval is shortened for all).
    bool same_limit = true, limits_on_checks = true;
    for (int k = 0; k < n; ++k) {
        same_limit = same_limit && ctxs[k]->P.p_max_iter == ctxs[0]->P.p_max_iter;
        limits_on_checks = limits_on_checks && ctxs[k]->P.p_max_iter % ctxs[0]->P.p_check_every == 0;
    }
    if (!same_limit && !limits_on_checks) return IBM_ERR_INVALID;
    ibm_batch* b = new ibm_batch();
    b->cs.assign(ctxs, ctxs + n);
    b->stream = ctxs[0]->stream;
    b->S = ctxs[0]->tb_sweeps;
    b->K = ctxs[0]->P.p_check_every;
    for (int k = 0; k < n; ++k) b->max_iter = std::max(b->max_iter, ctxs[k]->P.p_max_iter);
    auto fail = [&](int32_t rc) {
        ibm_batch_destroy(b);
        return rc;
    };
    b->mp = ctxs[0]->P.p_method == IBM_SOLVER_RBSOR_MP;
    if (b->mp) {
        if (hipMalloc((void**)&b->dmp, n * sizeof(MpCase)) != hipSuccess) return fail(IBM_ERR_HIP);
        if (hipHostMalloc((void**)&b->hmp, n * sizeof(MpCase), hipHostMallocDefault) != hipSuccess)
            return fail(IBM_ERR_HIP);
    } else {
        if (hipMalloc((void**)&b->dcases, n * sizeof(TbCase)) != hipSuccess) return fail(IBM_ERR_HIP);
        if (hipHostMalloc((void**)&b->hcases, n * sizeof(TbCase), hipHostMallocDefault) != hipSuccess)
            return fail(IBM_ERR_HIP);
    }
    if (hipHostMalloc((void**)&b->hslots, sizeof(Slot) * kBatchRing * n,
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return fail(IBM_ERR_HIP);
    if (hipHostGetDevicePointer((void**)&b->dslots, b->hslots, 0) != hipSuccess) return fail(IBM_ERR_HIP);
    for (int e = 0; e < kBatchRing; ++e)
        if (hipEventCreateWithFlags(&b->ev[e], hipEventDisableTiming) != hipSuccess) return fail(IBM_ERR_HIP);
    *out = b;
    return IBM_OK;
}

int32_t ibm_batch_step(ibm_batch* b, int32_t nsteps, ibm_step_stats* last) {
    if (!b || nsteps < 1) return IBM_ERR_INVALID;
    b->err.clear();
    const int n = (int)b->cs.size();
    for (ibm_ctx* c : b->cs) {
        if (c->P.p_init == IBM_INIT_LEARNED && !c->net) {
            b->err = "p_init is IBM_INIT_LEARNED but no network is attached";
            return IBM_ERR_STATE;
        }
    }
    // the steps of a batch are not phase-timed (a case's phases would span
    // the other cases' work)
    struct InBatch {
        std::vector<ibm_ctx*>& cs;
        explicit InBatch(std::vector<ibm_ctx*>& v) : cs(v) { for (ibm_ctx* c : cs) c->in_batch = true; }
        ~InBatch() { for (ibm_ctx* c : cs) c->in_batch = false; }
    } in_batch(b->cs);
    std::vector<ibm_step_stats> st(n);
    std::vector<int> status(n, IBM_OK);
    std::vector<double> wall(n, 0.0);
    int32_t worst_rc = IBM_OK;
    for (int s = 0; s < nsteps; ++s) {
        const auto w0 = std::chrono::steady_clock::now();
        // replayed iteration counts (ibm_set_poisson_schedule) of this step:
        // every case stops at its own count only if the counts fall on check
        // intervals or are all the same (as for the contexts' limits)
        {
            bool any = false, same = true, on_checks = true;
            int first = -1;
            for (int k = 0; k < n; ++k) {
                const ibm_ctx* c = b->cs[k];
                const int lim = c->sched_pos < c->schedule.size() ? c->schedule[c->sched_pos] : c->P.p_max_iter;
                any = any || c->sched_pos < c->schedule.size();
                if (first < 0) first = lim;
                same = same && lim == first;
                on_checks = on_checks && lim % b->K == 0;
            }
            if (any && !same && !on_checks) {
                b->err = "replayed iteration counts of a batch must be multiples of p_check_every or all equal";
                return IBM_ERR_STATE;
            }
            for (ibm_ctx* c : b->cs)
                c->batch_fixed = c->sched_pos < c->schedule.size() ? c->schedule[c->sched_pos++] : -1;
        }
        for (int k = 0; k < n; ++k) {
            Body B;
            int32_t rc = step_pre(b->cs[k], &st[k], &B, &status[k]);
            if (rc < 0) {
                b->err = std::string("case ") + std::to_string(k) + ": " + b->cs[k]->err;
                return rc;
            }
            if (status[k] < 0) {
                b->err = std::string("case ") + std::to_string(k) + ": velocity solve failed";
                return status[k];
            }
        }
        std::vector<LoopOut> outs(n);
        int32_t rc = batch_sor(b, outs);
        if (rc) return rc;
        for (int k = 0; k < n; ++k) {
            ibm_ctx* c = b->cs[k];
            if (outs[k].zero_rhs) {
                rc = fill(c, c->phi, (size_t)c->nx * c->ny, 0.0);
            } else {
                hipLaunchKernelGGL(k_merge, grid2(c->nh, c->ny), dim3(kBlock), 0, c->stream, c->g,
                                   (const double*)c->phr, (const double*)c->phb, c->phi);
                rc = hipGetLastError() == hipSuccess ? IBM_OK : IBM_ERR_HIP;
            }
            if (rc) return rc;
            rc = step_post(c, &st[k], outs[k], status[k]);
            worst_rc = worst(worst_rc, rc);
            if (rc < 0) {
                b->err = std::string("case ") + std::to_string(k) + ": " + c->err;
                return rc;
            }
        }
        const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
        for (int k = 0; k < n; ++k) st[k].seconds = sec;
    }
    if (last)
        for (int k = 0; k < n; ++k) last[k] = st[k];
    return worst_rc;
}

void ibm_batch_destroy(ibm_batch* b) {
    if (!b) return;
    if (b->stream || !b->cs.empty()) (void)hipStreamSynchronize(b->stream);
    for (int e = 0; e < kBatchRing; ++e)
        if (b->ev[e]) (void)hipEventDestroy(b->ev[e]);
    if (b->dcases) (void)hipFree(b->dcases);
    if (b->hcases) (void)hipHostFree(b->hcases);
    if (b->dmp) (void)hipFree(b->dmp);
    if (b->hmp) (void)hipHostFree(b->hmp);
    if (b->hslots) (void)hipHostFree(b->hslots);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->dcur) (void)hipFree(b->dcur);
    delete b;
}

int32_t ibm_batch_set_graph(ibm_batch* b, int32_t intervals) {
    if (!b) return IBM_ERR_INVALID;
    if (intervals != 0 && (intervals < 2 || intervals > kMaxGraphIntervals || (intervals & 1))) return IBM_ERR_INVALID;
    b->err.clear();
    if (intervals > 0) {
        if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
            b->cap = nullptr;
            b->err = "hipStreamCreateWithFlags failed";
            return IBM_ERR_HIP;
        }
        if (!b->dcur && hipMalloc((void**)&b->dcur, 2 * sizeof(int)) != hipSuccess) {
            b->dcur = nullptr;
            b->err = "hipMalloc of the cursor failed";
            return IBM_ERR_HIP;
        }
    }
    b->graph_iv = intervals;
    if (intervals == 0 && b->gexec) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) {
            b->err = "hipStreamSynchronize failed";
            return IBM_ERR_HIP;
        }
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return IBM_OK;
}

const char* ibm_batch_last_error(const ibm_batch* b) { return b ? b->err.c_str() : "null batch"; }

const char* ibm_status_string(int32_t s) {
    switch (s) {
        case IBM_OK: return "ok";
        case IBM_NOT_CONVERGED: return "iteration limit reached before the tolerance";
        case IBM_ERR_INVALID: return "invalid argument";
        case IBM_ERR_HIP: return "HIP runtime error";
        case IBM_ERR_STATE: return "invalid context state";
        case IBM_ERR_NAN: return "residual became NaN or Inf";
        default: return "unknown status";
    }
}

const char* ibm_last_error(const ibm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void ibm_destroy(ibm_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (int s = 0; s < kSlots; ++s)
        if (c->ev[s]) (void)hipEventDestroy(c->ev[s]);
    for (int k = 0; k < IBM_KERNEL_COUNT; ++k)
        for (auto& smp : c->samples[k]) {
            (void)hipEventDestroy(smp.a);
            (void)hipEventDestroy(smp.b);
        }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->t0) (void)hipEventDestroy(c->t0);
    if (c->t1) (void)hipEventDestroy(c->t1);
    for (int k = 0; k <= IBM_PHASE_COUNT; ++k)
        if (c->pev[k]) (void)hipEventDestroy(c->pev[k]);
    if (c->hslots) (void)hipHostFree(c->hslots);
    if (c->hstage) (void)hipHostFree(c->hstage);
    delete c;
}

int32_t ibm_init(const ibm_params* prm, const double* xf, const double* yf, const double* u0, const double* v0,
                 const double* p0, void* workspace, size_t workspace_bytes, void* hip_stream, ibm_ctx** out) {
    if (!out) return IBM_ERR_INVALID;
    *out = nullptr;
    if (validate(prm, xf, yf)) return IBM_ERR_INVALID;
    const Offsets off = layout_for(prm->nx, prm->ny);
    if (!workspace || workspace_bytes < off.total || ((uintptr_t)workspace & 255u)) return IBM_ERR_INVALID;

    ibm_ctx* c = new ibm_ctx();
    for (int s = 0; s < kSlots; ++s) c->ev[s] = nullptr;
    c->P = *prm;
    c->nx = prm->nx;
    c->ny = prm->ny;
    c->nh = prm->nx / 2;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)workspace;
    c->off = off;
    const int nx = c->nx, ny = c->ny;
    char* w = c->ws;
    auto D = [&](size_t o) { return (double*)(w + o); };
    Grid& g = c->g;
    g.nx = nx; g.ny = ny; g.nh = c->nh;
    g.per = prm->bc_mode == IBM_BC_PERIODIC ? 1 : 0;
    g.xf = D(off.xf); g.yf = D(off.yf); g.dx = D(off.dx); g.dy = D(off.dy); g.xc = D(off.xc); g.yc = D(off.yc);
    g.dxu = D(off.dxu); g.dyv = D(off.dyv);
    g.pcE = D(off.pcE); g.pcW = D(off.pcW); g.pcD = D(off.pcD); g.pcN = D(off.pcN); g.pcS = D(off.pcS);
    g.uce = D(off.uce); g.ucw = D(off.ucw); g.ucn = D(off.ucn); g.ucs = D(off.ucs);
    g.vce = D(off.vce); g.vcw = D(off.vcw); g.vcn = D(off.vcn); g.vcs = D(off.vcs);
    c->u = D(off.u); c->nu = D(off.nu); c->ru = D(off.ru); c->fufull = D(off.fufull);
    c->v = D(off.v); c->nv = D(off.nv); c->rv = D(off.rv); c->fvfull = D(off.fvfull);
    c->p = D(off.p); c->phi = D(off.phi); c->vb = D(off.vb); c->pr = D(off.pr); c->pp = D(off.pp);
    c->pp2 = D(off.pp2); c->pq = D(off.pq);
    c->phr = D(off.phr); c->phb = D(off.phb); c->vbr = D(off.vbr); c->vbb = D(off.vbb);
    c->pz = D(off.pz); c->dn = D(off.dn);
    c->cgw = D(off.cgw); c->cgs = D(off.cgs); c->rdn = D(off.rdn);
    c->phr2 = D(off.phr2); c->phb2 = D(off.phb2);
    c->mpf = (float*)(w + off.mpf);
    c->phi0 = D(off.phi0);
    c->wscale = D(off.wscale);
    c->wsf = (float*)(w + off.wsf);
    c->f_u = D(off.f_u); c->f_v = D(off.f_v); c->coef = D(off.coef); c->partials = D(off.partials);
    c->ctl = (Ctl*)(w + off.ctl);
    c->list_u = (int*)(w + off.list_u); c->list_v = (int*)(w + off.list_v); c->counts = (int*)(w + off.counts);
    c->flu = (uint8_t*)(w + off.flu); c->flv = (uint8_t*)(w + off.flv); c->msrc = (uint8_t*)(w + off.msrc);
    c->box = motion_box(*prm, xf, yf);

    auto fail = [&](int32_t rc) {
        ibm_destroy(c);
        return rc;
    };
    if (hipHostMalloc((void**)&c->hslots, sizeof(Slot) * kSlots, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return fail(IBM_ERR_HIP);
    std::memset(c->hslots, 0, sizeof(Slot) * kSlots);
    if (hipHostGetDevicePointer((void**)&c->dslots, c->hslots, 0) != hipSuccess) return fail(IBM_ERR_HIP);
    if (hipHostMalloc((void**)&c->hstage, 64, hipHostMallocDefault) != hipSuccess) return fail(IBM_ERR_HIP);
    for (int s = 0; s < kSlots; ++s)
        if (hipEventCreateWithFlags(&c->ev[s], hipEventDisableTiming) != hipSuccess) return fail(IBM_ERR_HIP);
    if (hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess) return fail(IBM_ERR_HIP);
    c->noalloc = noalloc_scratch(workspace);  // the allocation-free solve reports its absence

    // metrics
    std::vector<std::vector<double>> A;
    host_metrics(*prm, xf, yf, A);
    const size_t dst[] = {off.xf, off.yf, off.dx, off.dy, off.xc, off.yc, off.dxu, off.dyv, off.pcE, off.pcW, off.pcD,
                          off.pcN, off.pcS, off.uce, off.ucw, off.ucn, off.ucs, off.vce, off.vcw, off.vcn, off.vcs};
    for (size_t k = 0; k < A.size(); ++k)
        if (hipMemcpyAsync(w + dst[k], A[k].data(), A[k].size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream) != hipSuccess)
            return fail(IBM_ERR_HIP);
    // initial fields with their boundary values
    const size_t NU = (size_t)(nx + 1) * ny, NV = (size_t)nx * (ny + 1), NC = (size_t)nx * ny;
    std::vector<double> hu(NU), hv(NV), hp(NC);
    for (size_t k = 0; k < NU; ++k) hu[k] = u0 ? u0[k] : prm->u_inf;
    for (size_t k = 0; k < NV; ++k) hv[k] = v0 ? v0[k] : 0.0;
    for (size_t k = 0; k < NC; ++k) hp[k] = p0 ? p0[k] : 0.0;
    if (g.per) {  // face nx and face row ny mirror face 0 and row 0
        for (int j = 0; j < ny; ++j) hu[(size_t)j * (nx + 1) + nx] = hu[(size_t)j * (nx + 1)];
        for (int i = 0; i < nx; ++i) hv[(size_t)ny * nx + i] = hv[i];
    } else {      // inflow u and wall v
        for (int j = 0; j < ny; ++j) hu[(size_t)j * (nx + 1)] = prm->u_inf;
        for (int i = 0; i < nx; ++i) {
            hv[i] = 0.0;
            hv[(size_t)ny * nx + i] = 0.0;
        }
    }
    if (hipMemcpyAsync(c->u, hu.data(), NU * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->v, hv.data(), NV * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->p, hp.data(), NC * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return fail(IBM_ERR_HIP);
    int32_t rc = IBM_OK;
    double* zero_d[] = {c->phi, c->nu, c->nv, c->ru, c->rv, c->coef, c->fufull, c->fvfull};
    size_t zero_n[] = {NC, NU, NV, NU, NV, 4, NU, NV};
    for (int k = 0; k < 8 && !rc; ++k) rc = fill(c, zero_d[k], zero_n[k], 0.0);
    if (!rc) rc = fill_u8(c, c->flu, NU);
    if (!rc) rc = fill_u8(c, c->flv, NV);
    if (!rc) rc = fill_u8(c, c->msrc, NC);
    if (!rc) rc = fill_u8(c, (uint8_t*)c->counts, 4 * sizeof(int));
    if (!rc) {
        hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, c->stream, c->ctl, (int)CTL_N);
        hipLaunchKernelGGL(k_ndiag, grid2(nx, ny), dim3(kBlock), 0, c->stream, c->g, c->dn);
        hipLaunchKernelGGL(k_rdiag, grid2(nx, ny), dim3(kBlock), 0, c->stream, c->g, (const double*)c->dn, c->rdn);
        if (hipGetLastError() != hipSuccess) rc = IBM_ERR_HIP;
    }
    if (rc) return fail(rc);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(IBM_ERR_HIP);
    *out = c;
    return IBM_OK;
}

int32_t ibm_step(ibm_ctx* c, int32_t nsteps, ibm_step_stats* last) {
    if (!c) return IBM_ERR_INVALID;
    if (nsteps < 1) {
        c->err = "nsteps must be >= 1";
        return IBM_ERR_INVALID;
    }
    c->err.clear();
    if (c->P.p_init == IBM_INIT_LEARNED && !c->net) {  // checked before anything is enqueued
        c->err = "p_init is IBM_INIT_LEARNED but no network is attached (ibm_set_warm_start)";
        return IBM_ERR_STATE;
    }
    if (c->net) {
        int mb, h, w;
        ibm::unet::net_shape(c->net, &mb, &h, &w);
        if (h * c->net_f != c->ny || w * c->net_f != c->nx) {
            c->err = "the attached network's shape does not match IBM_OPT_NET_FACTOR";
            return IBM_ERR_STATE;
        }
    }
    const auto w0 = std::chrono::steady_clock::now();
    int32_t status = IBM_OK;
    ibm_step_stats st;
    std::memset(&st, 0, sizeof(st));
    for (int s = 0; s < nsteps; ++s) {
        int32_t rc = step_once(c, &st);
        status = worst(status, rc);
        if (rc < 0) break;
    }
    const auto w1 = std::chrono::steady_clock::now();
    st.seconds = std::chrono::duration<double>(w1 - w0).count();
    if (last) *last = st;
    return status;
}

int32_t ibm_poisson_solve(ibm_ctx* c, const double* rhs_dev, double* x_dev, const ibm_solve_opts* o,
                          ibm_solve_stats* st) {
    if (!c) return IBM_ERR_INVALID;
    if (!rhs_dev || !x_dev || !o || o->max_iter < 1 || o->check_every < 1 || o->fixed_iters < 0 ||
        (o->method != IBM_SOLVER_RBSOR && o->method != IBM_SOLVER_PCG && o->method != IBM_SOLVER_RBSOR_MP &&
         o->method != IBM_SOLVER_CG1) ||
        ((o->method == IBM_SOLVER_RBSOR || o->method == IBM_SOLVER_RBSOR_MP) && !(o->omega > 0.0 && o->omega < 2.0)) ||
        !std::isfinite(o->tol) ||
        (c->g.per && o->method == IBM_SOLVER_RBSOR_MP)) {
        c->err = "invalid solve options";
        return IBM_ERR_INVALID;
    }
    c->err.clear();
    c->rhs_held = 0;
    const dim3 bl(kBlock);
    const int fixed = o->fixed_iters > 0 ? o->fixed_iters : -1;
    LoopOut lo;
    HIP_TRY(hipEventRecord(c->t0, c->stream));
    int32_t rc;
    if (o->method == IBM_SOLVER_PCG || o->method == IBM_SOLVER_CG1) {
        // V b in the natural-layout scratch, x in place
        const dim3 gr = grid2(c->nh, c->ny);
        hipLaunchKernelGGL(k_split, gr, bl, 0, c->stream, c->g, rhs_dev, c->vbr, c->vbb, 1);
        hipLaunchKernelGGL(k_merge, gr, bl, 0, c->stream, c->g, (const double*)c->vbr, (const double*)c->vbb, c->vb);
        LAUNCH_CHECK();
        rc = per_project(c, c->vb, 1);
        if (rc) return rc;
        rc = o->method == IBM_SOLVER_PCG ? pcg_loop(c, x_dev, c->vb, o->tol, o->max_iter, fixed, &lo)
                                         : cg1_loop(c, x_dev, c->vb, o->tol, o->max_iter, fixed, &lo);
        if (rc) return rc;
        if (lo.zero_rhs) {
            rc = fill(c, x_dev, (size_t)c->nx * c->ny, 0.0);
            if (rc) return rc;
        } else if (lo.status != kStNan) {
            rc = per_project(c, x_dev, 0);
            if (rc) return rc;
        }
    } else {
        rc = split_sor_solve(c, rhs_dev, x_dev, o, fixed, &lo);
        if (rc) return rc;
    }
    return solve_stats(c, lo, st);
}

// Allocation-free variant of ibm_poisson_solve (red-black SOR): the solve's
// working arrays come from this device's static scratch instead of the
// context's workspace; the context's own pointers are swapped back before
// returning, whatever the outcome.
int32_t ibm_poisson_solve_noalloc(ibm_ctx* c, const double* rhs_dev, double* x_dev, const ibm_solve_opts* o,
                                  ibm_solve_stats* st) {
    if (!c) return IBM_ERR_INVALID;
    if (!rhs_dev || !x_dev || !o || o->method != IBM_SOLVER_RBSOR || o->max_iter < 1 || o->check_every < 1 ||
        o->fixed_iters < 0 || !(o->omega > 0.0 && o->omega < 2.0) || !std::isfinite(o->tol)) {
        c->err = "invalid solve options (the allocation-free solve takes IBM_SOLVER_RBSOR only)";
        return IBM_ERR_INVALID;
    }
    if ((size_t)c->nx * c->ny > kNoAllocCells) {
        c->err = "grid larger than the static scratch of the allocation-free solve (1024*768 cells)";
        return IBM_ERR_INVALID;
    }
    TbShape ts;
    if (c->sor_kernel != IBM_SOR_PER_COLOUR && tb_shape(c, c->tb_sweeps, c->tb_tx, c->tb_ty, &ts) &&
        (size_t)ts.ntx * ts.nty > kNoAllocTiles) {
        c->err = "more blocked-sweep tiles than the static scratch of the allocation-free solve holds (8192)";
        return IBM_ERR_INVALID;
    }
    if (!c->noalloc) {
        c->err = "the static scratch of this device could not be resolved";
        return IBM_ERR_HIP;
    }
    c->err.clear();
    c->rhs_held = 0;
    double* base = c->noalloc;
    double* saved[] = {c->phr, c->phb, c->phr2, c->phb2, c->vbr, c->vbb, c->partials};
    Ctl* saved_ctl = c->ctl;
    const int saved_prof = c->prof_every;
    c->phr = base;
    c->phb = base + kNoAllocHalf;
    c->phr2 = base + 2 * kNoAllocHalf;
    c->phb2 = base + 3 * kNoAllocHalf;
    c->vbr = base + 4 * kNoAllocHalf;
    c->vbb = base + 5 * kNoAllocHalf;
    c->partials = base + 6 * kNoAllocHalf;
    c->ctl = (Ctl*)(base + 6 * kNoAllocHalf + kNoAllocPartials);
    c->prof_every = 0;  // sampled timing would create events
    const int fixed = o->fixed_iters > 0 ? o->fixed_iters : -1;
    LoopOut lo;
    int32_t rc = IBM_OK;
    if (hipEventRecord(c->t0, c->stream) != hipSuccess) {
        c->err = "hipEventRecord failed";
        rc = IBM_ERR_HIP;
    }
    if (!rc) rc = split_sor_solve(c, rhs_dev, x_dev, o, fixed, &lo);
    c->phr = saved[0];
    c->phb = saved[1];
    c->phr2 = saved[2];
    c->phb2 = saved[3];
    c->vbr = saved[4];
    c->vbb = saved[5];
    c->partials = saved[6];
    c->ctl = saved_ctl;
    c->prof_every = saved_prof;
    if (rc) return rc;
    return solve_stats(c, lo, st);
}

int32_t ibm_forces(ibm_ctx* c, double* cd, double* cl) {
    if (!c || !cd || !cl) return IBM_ERR_INVALID;
    HIP_TRY(hipStreamSynchronize(c->stream));
    *cd = c->cd;
    *cl = c->cl;
    return IBM_OK;
}

int32_t ibm_get_fields(ibm_ctx* c, double* u, double* v, double* p, double* phi) {
    if (!c) return IBM_ERR_INVALID;
    const size_t NU = (size_t)(c->nx + 1) * c->ny, NV = (size_t)c->nx * (c->ny + 1), NC = (size_t)c->nx * c->ny;
    if (u) HIP_TRY(hipMemcpyAsync(u, c->u, NU * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (v) HIP_TRY(hipMemcpyAsync(v, c->v, NV * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (p) HIP_TRY(hipMemcpyAsync(p, c->p, NC * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (phi) HIP_TRY(hipMemcpyAsync(phi, c->phi, NC * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return IBM_OK;
}

int32_t ibm_get_poisson_rhs(ibm_ctx* c, double* vb) {
    if (!c || !vb) return IBM_ERR_INVALID;
    if (!c->rhs_held) {
        c->err = "no time step's right-hand side is held (no step yet, or a stand-alone solve or a restored "
                 "state since the last step)";
        return IBM_ERR_INVALID;
    }
    HIP_TRY(hipMemcpyAsync(vb, c->vb, (size_t)c->nx * c->ny * sizeof(double), hipMemcpyDefault, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return IBM_OK;
}

int32_t ibm_get_ibm(ibm_ctx* c, uint8_t* flu, uint8_t* flv, uint8_t* msrc, double* fu, double* fv) {
    if (!c) return IBM_ERR_INVALID;
    const size_t NU = (size_t)(c->nx + 1) * c->ny, NV = (size_t)c->nx * (c->ny + 1), NC = (size_t)c->nx * c->ny;
    if (flu) HIP_TRY(hipMemcpyAsync(flu, c->flu, NU, hipMemcpyDeviceToHost, c->stream));
    if (flv) HIP_TRY(hipMemcpyAsync(flv, c->flv, NV, hipMemcpyDeviceToHost, c->stream));
    if (msrc) HIP_TRY(hipMemcpyAsync(msrc, c->msrc, NC, hipMemcpyDeviceToHost, c->stream));
    if (fu || fv) {
        int32_t rc = fill(c, c->fufull, NU, 0.0);
        if (!rc) rc = fill(c, c->fvfull, NV, 0.0);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scatter_forcing, dim3((unsigned)((NU + 255) / 256)), dim3(256), 0, c->stream,
                           (const int*)c->list_u, (const int*)c->counts, 0, (const double*)c->f_u, c->fufull);
        hipLaunchKernelGGL(k_scatter_forcing, dim3((unsigned)((NV + 255) / 256)), dim3(256), 0, c->stream,
                           (const int*)c->list_v, (const int*)c->counts, 1, (const double*)c->f_v, c->fvfull);
        LAUNCH_CHECK();
        if (fu) HIP_TRY(hipMemcpyAsync(fu, c->fufull, NU * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (fv) HIP_TRY(hipMemcpyAsync(fv, c->fvfull, NV * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return IBM_OK;
}

// State blob: header then u, v, p, phi, nu, nv.
struct StateHeader {
    uint32_t magic;
    int32_t nx, ny, have_hist;
    int64_t step;
    double t, cd, cl;
};

size_t ibm_state_bytes(const ibm_ctx* c) {
    if (!c) return 0;
    const size_t NU = (size_t)(c->nx + 1) * c->ny, NV = (size_t)c->nx * (c->ny + 1), NC = (size_t)c->nx * c->ny;
    return sizeof(StateHeader) + sizeof(double) * (2 * NU + 2 * NV + 2 * NC);
}

int32_t ibm_get_state(ibm_ctx* c, void* host, size_t bytes) {
    if (!c || !host || bytes < ibm_state_bytes(c)) return IBM_ERR_INVALID;
    const size_t NU = (size_t)(c->nx + 1) * c->ny, NV = (size_t)c->nx * (c->ny + 1), NC = (size_t)c->nx * c->ny;
    StateHeader h{kStateMagic, c->nx, c->ny, c->have_hist, (int64_t)c->step, c->t, c->cd, c->cl};
    std::memcpy(host, &h, sizeof(h));
    double* d = (double*)((char*)host + sizeof(h));
    const double* src[] = {c->u, c->v, c->p, c->phi, c->nu, c->nv};
    const size_t n[] = {NU, NV, NC, NC, NU, NV};
    for (int k = 0; k < 6; ++k) {
        HIP_TRY(hipMemcpyAsync(d, src[k], n[k] * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        d += n[k];
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return IBM_OK;
}

int32_t ibm_set_state(ibm_ctx* c, const void* host, size_t bytes) {
    if (!c || !host || bytes < ibm_state_bytes(c)) return IBM_ERR_INVALID;
    StateHeader h;
    std::memcpy(&h, host, sizeof(h));
    if (h.magic != kStateMagic || h.nx != c->nx || h.ny != c->ny) {
        c->err = "state blob does not match this grid";
        return IBM_ERR_INVALID;
    }
    const size_t NU = (size_t)(c->nx + 1) * c->ny, NV = (size_t)c->nx * (c->ny + 1), NC = (size_t)c->nx * c->ny;
    const double* d = (const double*)((const char*)host + sizeof(h));
    double* dst[] = {c->u, c->v, c->p, c->phi, c->nu, c->nv};
    const size_t n[] = {NU, NV, NC, NC, NU, NV};
    for (int k = 0; k < 6; ++k) {
        HIP_TRY(hipMemcpyAsync(dst[k], d, n[k] * sizeof(double), hipMemcpyHostToDevice, c->stream));
        d += n[k];
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->rhs_held = 0;
    c->have_hist = h.have_hist;
    c->step = h.step;
    c->t = h.t;
    c->cd = h.cd;
    c->cl = h.cl;
    return IBM_OK;
}

int32_t ibm_set_poisson_schedule(ibm_ctx* c, const int32_t* iters, int32_t n) {
    if (!c || n < 0 || (n > 0 && !iters)) return IBM_ERR_INVALID;
    for (int k = 0; k < n; ++k)
        if (iters[k] < 0) return IBM_ERR_INVALID;
    c->schedule.assign(iters, iters + n);
    c->sched_pos = 0;
    return IBM_OK;
}

int32_t ibm_set_warm_start(ibm_ctx* c, ibm_unet* net, double out_scale) {
    if (!c) return IBM_ERR_INVALID;
    if (!net) {
        c->net = nullptr;
        return IBM_OK;
    }
    if (c->g.per) {
        c->err = "periodic mode takes no learned guess or correction";
        return IBM_ERR_INVALID;
    }
    int mb, h, w;
    ibm::unet::net_shape(net, &mb, &h, &w);
    if (h * c->net_f != c->ny || w * c->net_f != c->nx || mb < 1) {
        c->err = "the network's image shape must be (ny, nx) / IBM_OPT_NET_FACTOR";
        return IBM_ERR_INVALID;
    }
    if (ibm::unet::net_stream(net) != c->stream) {
        c->err = "the network must run on the context's stream";
        return IBM_ERR_INVALID;
    }
    if (!(out_scale > 0.0) || !std::isfinite(out_scale)) {
        c->err = "out_scale must be finite and > 0";
        return IBM_ERR_INVALID;
    }
    c->net = net;
    c->net_scale = out_scale;
    return IBM_OK;
}

int32_t ibm_set_snapshot(ibm_ctx* c, float* feat_dev, float* target_dev, double out_scale) {
    if (!c) return IBM_ERR_INVALID;
    if ((feat_dev == nullptr) != (target_dev == nullptr) || !(out_scale > 0.0) || !std::isfinite(out_scale)) {
        c->err = "feat_dev and target_dev must both be set or both be NULL; out_scale > 0";
        return IBM_ERR_INVALID;
    }
    c->snap_feat = feat_dev;
    c->snap_target = target_dev;
    c->snap_scale = out_scale;
    return IBM_OK;
}

int32_t ibm_set_option(ibm_ctx* c, int32_t option, int64_t value) {
    if (!c) return IBM_ERR_INVALID;
    int kern = c->sor_kernel, S = c->tb_sweeps, tx = c->tb_tx, ty = c->tb_ty;
    switch (option) {
        case IBM_OPT_SOR_KERNEL:
            if (value != IBM_SOR_TEMPORAL && value != IBM_SOR_PER_COLOUR && value != IBM_SOR_TEMPORAL_LDS)
                return IBM_ERR_INVALID;
            kern = (int)value;
            break;
        case IBM_OPT_TB_SWEEPS: S = (int)value; break;
        case IBM_OPT_TB_TILE_X: tx = (int)value; break;
        case IBM_OPT_TB_TILE_Y: ty = (int)value; break;
        case IBM_OPT_NET_FACTOR:
            if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16) return IBM_ERR_INVALID;
            if (c->nx % value || c->ny % value) {
                c->err = "the network's coarsening factor must divide nx and ny";
                return IBM_ERR_INVALID;
            }
            c->net_f = (int)value;
            return IBM_OK;
        case IBM_OPT_NET_MAPS:
            if (value < 1 || value > 7) return IBM_ERR_INVALID;
            c->net_maps = (int)value;
            return IBM_OK;
        case IBM_OPT_NET_SMOOTH:
            if (value < 0 || value > 16) return IBM_ERR_INVALID;
            c->net_smooth = (int)value;
            return IBM_OK;
        case IBM_OPT_NET_STEP:
            if (value != IBM_NET_STEP_ENERGY && value != IBM_NET_STEP_BACKTRACK) return IBM_ERR_INVALID;
            c->net_rule = (int)value;
            return IBM_OK;
        case IBM_OPT_NET_EVERY:
        case IBM_OPT_SNAPSHOT_ITER:
            if (value < 0 || value > (1 << 30) || value % c->P.p_check_every) {
                c->err = "the interval must be >= 0 and a multiple of p_check_every";
                return IBM_ERR_INVALID;
            }
            (option == IBM_OPT_NET_EVERY ? c->net_every : c->snap_iter) = (int)value;
            return IBM_OK;
        default: return IBM_ERR_INVALID;
    }
    if (value < 0 || value > (1 << 20)) return IBM_ERR_INVALID;
    TbShape ts;
    if (!tb_shape(c, S, tx, ty, &ts)) {
        c->err = "tile shape does not fit the blocked sweep";
        return IBM_ERR_INVALID;
    }
    c->sor_kernel = kern;
    c->tb_sweeps = S;
    c->tb_tx = tx;
    c->tb_ty = ty;
    return IBM_OK;
}

int32_t ibm_profile(ibm_ctx* c, int32_t sample_every) {
    if (!c || sample_every < 0) return IBM_ERR_INVALID;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < IBM_KERNEL_COUNT; ++k) {
        for (auto& s : c->samples[k]) {
            c->ev_pool.push_back(s.a);
            c->ev_pool.push_back(s.b);
        }
        c->samples[k].clear();
        c->launches[k] = 0;
    }
    c->prof_every = sample_every;
    for (int k = 0; k < IBM_PHASE_COUNT; ++k) c->phase_ms[k] = 0.0;
    c->phase_steps = 0;
    c->phase_on = false;
    if (sample_every > 0) {
        for (int k = 0; k <= IBM_PHASE_COUNT; ++k)
            if (!c->pev[k]) HIP_TRY(hipEventCreate(&c->pev[k]));
        c->phase_on = true;
    }
    return IBM_OK;
}

int32_t ibm_profile_phases(ibm_ctx* c, double* ms, int32_t n, int64_t* steps) {
    if (!c || n < 0 || (n > 0 && !ms)) return IBM_ERR_INVALID;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) ms[k] = k < IBM_PHASE_COUNT ? c->phase_ms[k] : 0.0;
    if (steps) *steps = c->phase_steps;
    return IBM_OK;
}

int32_t ibm_profile_query(ibm_ctx* c, int32_t kernel, double* avg_ms, int64_t* samples, int64_t* launches,
                          double* bytes_per_launch) {
    if (!c || kernel < 0 || kernel >= IBM_KERNEL_COUNT) return IBM_ERR_INVALID;
    HIP_TRY(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (auto& s : c->samples[kernel]) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, s.a, s.b));
        tot += ms;
    }
    const size_t n = c->samples[kernel].size();
    const double cells = (double)c->nx * c->ny;
    const double S = c->tb_sweeps;
    const double bytes[IBM_KERNEL_COUNT] = {24.0 * cells / 2.0, 16.0 * cells, 32.0 * cells, 64.0 * cells,
                                            24.0 * cells * S, 12.0 * cells * S, 32.0 * cells, 88.0 * cells};
    if (avg_ms) *avg_ms = n ? tot / n : 0.0;
    if (samples) *samples = (int64_t)n;
    if (launches) *launches = c->launches[kernel];
    if (bytes_per_launch) *bytes_per_launch = bytes[kernel];
    return IBM_OK;
}

}  // extern "C"
