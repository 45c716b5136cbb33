"""Thin ctypes binding of the gfx950 immersed-boundary solver library.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libibm_hip.so`` (declared in ``include/ibm.h``).  PyTorch provides the
device workspace and the HIP stream.  There is no CPU fallback: if the library
is not built or no GPU is visible, construction raises.

Array conventions (float64, row-major, x fastest):
    u (ny, nx+1) x-faces, v (ny+1, nx) y-faces, p and phi (ny, nx) centres.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibm_hip.so")

OK, NOT_CONVERGED, ERR_INVALID, ERR_HIP, ERR_STATE, ERR_NAN = 0, 1, -1, -2, -3, -5
BC_CHANNEL, BC_PERIODIC = 0, 1
RBSOR, PCG, RBSOR_MP = 0, 1, 2   # RBSOR_MP: float sweeps on the correction, double refinement
CG1 = 3                          # Jacobi-PCG with one reduction per iteration
INIT_ZERO, INIT_PREVIOUS, INIT_LEARNED = 0, 1, 2
(KERNEL_SOR_SWEEP, KERNEL_SOR_RESIDUAL, KERNEL_PCG_DIR_SPMV, KERNEL_PCG_UPDATE, KERNEL_SOR_TB, KERNEL_SOR_MP,
 KERNEL_SOR_MP_REFINE, KERNEL_CG1_ITER) = range(8)
# KERNEL_SOR_TB times whichever blocked sweep runs; named for the default one
# (k_sor_tb is the LDS-tile variant).
KERNEL_NAMES = {KERNEL_SOR_SWEEP: "k_sor_sweep", KERNEL_SOR_RESIDUAL: "k_sor_residual",
                KERNEL_PCG_DIR_SPMV: "k_pcg_dir_spmv", KERNEL_PCG_UPDATE: "k_pcg_update",
                KERNEL_SOR_TB: "k_sor_tbr", KERNEL_SOR_MP: "k_sor_mp", KERNEL_SOR_MP_REFINE: "k_mp_refine",
                KERNEL_CG1_ITER: "k_cg1_iter"}
(OPT_SOR_KERNEL, OPT_TB_SWEEPS, OPT_TB_TILE_X, OPT_TB_TILE_Y, OPT_NET_FACTOR, OPT_NET_EVERY, OPT_SNAPSHOT_ITER,
 OPT_NET_SMOOTH, OPT_NET_STEP, OPT_NET_MAPS) = range(10)
NET_STEP_ENERGY, NET_STEP_BACKTRACK = 0, 1
# phases of ibm_step timed while kernel timing is on (ibm_profile_phases)
PHASES = ("flagging", "momentum", "forcing", "uv_solve", "poisson_rhs", "p_solve", "projection")
SOR_TEMPORAL, SOR_PER_COLOUR, SOR_TEMPORAL_LDS = 0, 1, 2

EXPORTED = ("ibm_workspace_bytes", "ibm_init", "ibm_step", "ibm_poisson_solve", "ibm_poisson_solve_noalloc",
            "ibm_forces",
            "ibm_get_fields", "ibm_get_poisson_rhs", "ibm_get_ibm", "ibm_state_bytes", "ibm_get_state", "ibm_set_state",
            "ibm_set_poisson_schedule", "ibm_set_option", "ibm_set_warm_start", "ibm_set_snapshot",
            "ibm_batch_create", "ibm_batch_step", "ibm_batch_set_graph", "ibm_batch_destroy", "ibm_batch_last_error",
            "ibm_profile", "ibm_profile_query", "ibm_profile_phases", "ibm_destroy",
            "ibm_status_string", "ibm_last_error")


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc_mode", C.c_int32), ("body", C.c_int32),
        ("re", C.c_double), ("dt", C.c_double), ("u_inf", C.c_double),
        ("chord", C.c_double), ("thickness", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double),
        ("p_method", C.c_int32), ("p_max_iter", C.c_int32), ("p_check_every", C.c_int32),
        ("p_init", C.c_int32),
        ("p_omega", C.c_double), ("p_tol", C.c_double),
        ("uv_omega", C.c_double), ("uv_tol", C.c_double),
        ("uv_max_iter", C.c_int32), ("q_mode", C.c_int32),
        ("alpha_max", C.c_double),
        ("precision", C.c_int32), ("reserved", C.c_int32),
    ]


class StepStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("p_iters", C.c_int32), ("u_iters", C.c_int32),
                ("v_iters", C.c_int32), ("n_forced_u", C.c_int32), ("n_forced_v", C.c_int32),
                ("n_msrc", C.c_int32), ("n_net", C.c_int32),
                ("p_r0", C.c_double), ("p_rel", C.c_double), ("cd", C.c_double), ("cl", C.c_double),
                ("t", C.c_double), ("seconds", C.c_double), ("net_step", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("fixed_iters", C.c_int32), ("omega", C.c_double), ("tol", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("reserved0", C.c_int32),
                ("reserved1", C.c_int32), ("r0_rel", C.c_double), ("rel", C.c_double),
                ("seconds", C.c_double)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        u8 = C.POINTER(C.c_uint8)
        L.ibm_workspace_bytes.argtypes = [C.POINTER(Params)]
        L.ibm_workspace_bytes.restype = C.c_size_t
        L.ibm_init.argtypes = [C.POINTER(Params), dp, dp, dp, dp, dp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.ibm_init.restype = C.c_int32
        L.ibm_step.argtypes = [vp, C.c_int32, C.POINTER(StepStats)]
        L.ibm_step.restype = C.c_int32
        L.ibm_poisson_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats)]
        L.ibm_poisson_solve.restype = C.c_int32
        L.ibm_poisson_solve_noalloc.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats)]
        L.ibm_poisson_solve_noalloc.restype = C.c_int32
        L.ibm_forces.argtypes = [vp, dp, dp]
        L.ibm_forces.restype = C.c_int32
        L.ibm_get_fields.argtypes = [vp, dp, dp, dp, dp]
        L.ibm_get_fields.restype = C.c_int32
        L.ibm_get_poisson_rhs.argtypes = [vp, vp]
        L.ibm_get_poisson_rhs.restype = C.c_int32
        L.ibm_get_ibm.argtypes = [vp, u8, u8, u8, dp, dp]
        L.ibm_get_ibm.restype = C.c_int32
        L.ibm_state_bytes.argtypes = [vp]
        L.ibm_state_bytes.restype = C.c_size_t
        L.ibm_get_state.argtypes = [vp, vp, C.c_size_t]
        L.ibm_get_state.restype = C.c_int32
        L.ibm_set_state.argtypes = [vp, vp, C.c_size_t]
        L.ibm_set_state.restype = C.c_int32
        L.ibm_set_poisson_schedule.argtypes = [vp, ip, C.c_int32]
        L.ibm_set_poisson_schedule.restype = C.c_int32
        L.ibm_set_warm_start.argtypes = [vp, vp, C.c_double]
        L.ibm_set_warm_start.restype = C.c_int32
        L.ibm_set_snapshot.argtypes = [vp, vp, vp, C.c_double]
        L.ibm_set_snapshot.restype = C.c_int32
        L.ibm_batch_create.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp)]
        L.ibm_batch_create.restype = C.c_int32
        L.ibm_batch_step.argtypes = [vp, C.c_int32, C.POINTER(StepStats)]
        L.ibm_batch_step.restype = C.c_int32
        L.ibm_batch_set_graph.argtypes = [vp, C.c_int32]
        L.ibm_batch_set_graph.restype = C.c_int32
        L.ibm_batch_destroy.argtypes = [vp]
        L.ibm_batch_destroy.restype = None
        L.ibm_batch_last_error.argtypes = [vp]
        L.ibm_batch_last_error.restype = C.c_char_p
        L.ibm_set_option.argtypes = [vp, C.c_int32, C.c_int64]
        L.ibm_set_option.restype = C.c_int32
        L.ibm_profile.argtypes = [vp, C.c_int32]
        L.ibm_profile.restype = C.c_int32
        L.ibm_profile_query.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), dp]
        L.ibm_profile_query.restype = C.c_int32
        L.ibm_profile_phases.argtypes = [vp, dp, C.c_int32, C.POINTER(C.c_int64)]
        L.ibm_profile_phases.restype = C.c_int32
        L.ibm_destroy.argtypes = [vp]
        L.ibm_destroy.restype = None
        L.ibm_status_string.argtypes = [C.c_int32]
        L.ibm_status_string.restype = C.c_char_p
        L.ibm_last_error.argtypes = [vp]
        L.ibm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


# Parameter names shared with the workload presets -> ibm_params fields.
_MAP = dict(bc="bc_mode", body="body", re="re", dt="dt", uinf="u_inf", chord="chord",
            thick="thickness", x0="x0", y0="y0", amp="amp", freq="freq", phase="phase",
            p_method="p_method", p_max_iter="p_max_iter", p_check="p_check_every",
            p_init_prev="p_init", p_omega="p_omega", p_tol="p_tol", uv_omega="uv_omega",
            uv_tol="uv_tol", uv_max_iter="uv_max_iter", q_mode="q_mode", alpha_max="alpha_max")

DEFAULTS = dict(bc=0, body=1, re=100.0, dt=1e-3, uinf=1.0, chord=1.0, thick=0.12, x0=4.0, y0=6.0,
                amp=0.0, freq=0.0, phase=0.0, p_method=RBSOR, p_max_iter=2_000_000, p_check=10,
                p_init_prev=1, p_omega=1.8, p_tol=1e-8, uv_omega=1.0, uv_tol=1e-10,
                uv_max_iter=200, q_mode=1, alpha_max=1.0)


def make_params(nx: int, ny: int, **kw) -> Params:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown parameter {k!r}")
        d[k] = v
    P = Params()
    P.nx, P.ny = nx, ny
    for k, v in d.items():
        setattr(P, _MAP[k], v)
    P.precision = 0
    P.reserved = 0
    return P


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def status_string(s: int) -> str:
    return lib().ibm_status_string(s).decode()


class IbmError(RuntimeError):
    pass


class Solver:
    """One solver context on a CUDA/HIP device; workspace is a torch tensor."""

    def __init__(self, nx, ny, xf, yf, u0=None, v0=None, p0=None, device="cuda:0", stream=None,
                 **params):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the solver runs only on the HIP device")
        L = lib()
        self.torch = torch
        self.nx, self.ny = nx, ny
        self.device = torch.device(device)
        self.P = make_params(nx, ny, **params)
        nbytes = L.ibm_workspace_bytes(C.byref(self.P))
        if nbytes == 0:
            raise ValueError("invalid grid size")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        yf = np.ascontiguousarray(yf, dtype=np.float64)
        arrs = []
        for a, shp in ((u0, (ny, nx + 1)), (v0, (ny + 1, nx)), (p0, (ny, nx))):
            if a is None:
                arrs.append(None)
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != shp:
                    raise ValueError(f"initial field shape {a.shape}, expected {shp}")
                arrs.append(a)
        h = C.c_void_p()
        rc = L.ibm_init(C.byref(self.P), _dp(xf), _dp(yf), _dp(arrs[0]), _dp(arrs[1]), _dp(arrs[2]),
                        C.c_void_p(self.ws.data_ptr()), nbytes, C.c_void_p(self.stream.cuda_stream),
                        C.byref(h))
        if rc != OK:
            raise IbmError(f"ibm_init failed: {status_string(rc)}")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ibm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, what, rc):
        msg = lib().ibm_last_error(self._h).decode()
        raise IbmError(f"{what} failed: {status_string(rc)} {msg}")

    # -- time stepping -------------------------------------------------------
    def step(self, n: int = 1):
        st = StepStats()
        rc = lib().ibm_step(self._h, n, C.byref(st))
        if rc < 0 and rc != ERR_NAN:
            self._err("ibm_step", rc)
        d = {k: getattr(st, k) for k, _ in StepStats._fields_ if k != "reserved"}
        d["rc"] = rc
        return d

    def forces(self):
        cd, cl = C.c_double(), C.c_double()
        rc = lib().ibm_forces(self._h, C.byref(cd), C.byref(cl))
        if rc != OK:
            self._err("ibm_forces", rc)
        return cd.value, cl.value

    def fields(self):
        nx, ny = self.nx, self.ny
        u = np.empty((ny, nx + 1)); v = np.empty((ny + 1, nx))
        p = np.empty((ny, nx)); phi = np.empty((ny, nx))
        rc = lib().ibm_get_fields(self._h, _dp(u), _dp(v), _dp(p), _dp(phi))
        if rc != OK:
            self._err("ibm_get_fields", rc)
        return u, v, p, phi

    def poisson_rhs(self, out=None):
        """V b of the last time step's pressure equation A phi = V b, (ny, nx)
        float64: into `out` (a contiguous float64 tensor on this device) when
        given, else a new host array."""
        if out is None:
            out = np.empty((self.ny, self.nx))
            ptr = out.ctypes.data_as(C.c_void_p)
        else:
            if out.dtype != self.torch.float64 or not out.is_contiguous() or out.device != self.device \
                    or out.numel() != self.nx * self.ny:
                raise ValueError("out must be a contiguous float64 device tensor of nx*ny")
            ptr = C.c_void_p(out.data_ptr())
        rc = lib().ibm_get_poisson_rhs(self._h, ptr)
        if rc != OK:
            self._err("ibm_get_poisson_rhs", rc)
        return out

    def ibm(self):
        nx, ny = self.nx, self.ny
        flu = np.zeros((ny, nx + 1), np.uint8); flv = np.zeros((ny + 1, nx), np.uint8)
        ms = np.zeros((ny, nx), np.uint8)
        fu = np.zeros((ny, nx + 1)); fv = np.zeros((ny + 1, nx))
        u8 = C.POINTER(C.c_uint8)
        rc = lib().ibm_get_ibm(self._h, flu.ctypes.data_as(u8), flv.ctypes.data_as(u8),
                               ms.ctypes.data_as(u8), _dp(fu), _dp(fv))
        if rc != OK:
            self._err("ibm_get_ibm", rc)
        return dict(flu=flu, flv=flv, msrc=ms, fu=fu, fv=fv)

    def get_state(self) -> bytes:
        n = lib().ibm_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        rc = lib().ibm_get_state(self._h, buf, n)
        if rc != OK:
            self._err("ibm_get_state", rc)
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        rc = lib().ibm_set_state(self._h, buf, len(blob))
        if rc != OK:
            self._err("ibm_set_state", rc)

    def set_poisson_schedule(self, iters):
        a = (C.c_int32 * len(iters))(*[int(x) for x in iters])
        rc = lib().ibm_set_poisson_schedule(self._h, a, len(iters))
        if rc != OK:
            self._err("ibm_set_poisson_schedule", rc)

    def set_warm_start(self, net, out_scale: float):
        """Attach a warm-start network (paper_2402_17337_amd.unet.UNet of shape
        (ny, nx) on this solver's stream), or detach with net=None."""
        self._ws_net = net  # keep it alive while attached
        rc = lib().ibm_set_warm_start(self._h, net.handle if net is not None else None, out_scale)
        if rc:
            self._err("ibm_set_warm_start", rc)

    def set_snapshot(self, feat=None, target=None, out_scale: float = 1.0):
        """Record each step's network maps into feat (3, ny/F, nx/F) and its
        target into target (ny/F, nx/F), float32 device tensors (F: the
        network's coarsening factor); None clears."""
        ptrs = []
        f = getattr(self, "net_f", 1)
        ny, nx = self.ny // f, self.nx // f
        for t, shp in ((feat, (3, ny, nx)), (target, (ny, nx))):
            if t is None:
                ptrs.append(None)
                continue
            if t.dtype != self.torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError(f"snapshot buffers: contiguous float32 device tensors of shape {shp}")
            ptrs.append(C.c_void_p(t.data_ptr()))
        self._snap = (feat, target)
        rc = lib().ibm_set_snapshot(self._h, ptrs[0], ptrs[1], out_scale)
        if rc:
            self._err("ibm_set_snapshot", rc)

    def set_option(self, option: int, value: int) -> int:
        """Tuning option (launch shape of the SOR sweeps, the network's grid and
        correction interval); returns the status."""
        rc = lib().ibm_set_option(self._h, option, int(value))
        if rc == OK and option == OPT_NET_FACTOR:
            self.net_f = int(value)
        return rc

    def autotune_tiles(self, candidates=((76, 44), (84, 52), (64, 40), (48, 32), (48, 16), (32, 16)), iters: int = 200,
                       seed: int = 0):
        """Time `iters` fixed SOR iterations of a stand-alone solve (random
        right-hand side) with each candidate tile shape of the blocked sweep,
        keep the fastest and return it with the timings (seconds, GPU events).
        Every shape gives the same iterates; only the speed differs."""
        torch = self.torch
        g = torch.Generator(device="cpu").manual_seed(seed)
        rhs = (torch.rand(self.ny, self.nx, generator=g, dtype=torch.float64) - 0.5).to(self.device)
        times = {}
        for tx, ty in candidates:
            if self.set_option(OPT_TB_TILE_X, tx) != OK or self.set_option(OPT_TB_TILE_Y, ty) != OK:
                continue
            x = torch.zeros_like(rhs)
            self.poisson_solve(rhs, x, fixed_iters=iters)          # warm-up
            x.zero_()
            st = self.poisson_solve(rhs, x, fixed_iters=iters)
            times[(tx, ty)] = st["seconds"]
        best = min(times, key=times.get)
        self.set_option(OPT_TB_TILE_X, best[0])
        self.set_option(OPT_TB_TILE_Y, best[1])
        return best, times

    # -- stand-alone Poisson solve ------------------------------------------
    def poisson_solve(self, rhs, x, method=RBSOR, omega=1.8, tol=1e-8, max_iter=2_000_000,
                      check_every=10, fixed_iters=0, noalloc=False):
        """Solve (D G) x = rhs in place on device tensors (float64, (ny, nx)).
        noalloc=True calls ibm_poisson_solve_noalloc (red-black SOR with the
        library's static scratch instead of the context's workspace)."""
        torch = self.torch
        for t in (rhs, x):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device \
                    or t.numel() != self.nx * self.ny:
                raise ValueError("rhs and x must be contiguous float64 device tensors of nx*ny")
        o = SolveOpts(method, max_iter, check_every, fixed_iters, omega, tol)
        st = SolveStats()
        name = "ibm_poisson_solve_noalloc" if noalloc else "ibm_poisson_solve"
        rc = getattr(lib(), name)(self._h, C.c_void_p(rhs.data_ptr()), C.c_void_p(x.data_ptr()),
                                  C.byref(o), C.byref(st))
        if rc < 0 and rc != ERR_NAN:
            self._err(name, rc)
        d = {k: getattr(st, k) for k, _ in SolveStats._fields_ if not k.startswith("reserved")}
        d["rc"] = rc
        return d

    # -- kernel timing --------------------------------------------------------
    def profile(self, sample_every: int):
        rc = lib().ibm_profile(self._h, sample_every)
        if rc != OK:
            self._err("ibm_profile", rc)

    def profile_phases(self):
        """Accumulated GPU ms per phase of ibm_step since profile(n > 0), and
        the number of steps summed."""
        ms = (C.c_double * len(PHASES))()
        n = C.c_int64()
        rc = lib().ibm_profile_phases(self._h, ms, len(PHASES), C.byref(n))
        if rc != OK:
            self._err("ibm_profile_phases", rc)
        return dict(zip(PHASES, list(ms))), n.value

    def profile_query(self, kernel: int):
        avg, ns, nl, by = C.c_double(), C.c_int64(), C.c_int64(), C.c_double()
        rc = lib().ibm_profile_query(self._h, kernel, C.byref(avg), C.byref(ns), C.byref(nl), C.byref(by))
        if rc != OK:
            self._err("ibm_profile_query", rc)
        return dict(avg_ms=avg.value, samples=ns.value, launches=nl.value, bytes_per_launch=by.value)


def workspace_bytes(nx, ny, **params) -> int:
    P = make_params(nx, ny, **params)
    return lib().ibm_workspace_bytes(C.byref(P))


def init_status(nx, ny, xf, yf, workspace_ptr=0, workspace_bytes_=None, **params) -> int:
    """Call ibm_init with a given (possibly bogus) workspace; for argument
    validation, which happens before any GPU call.  Returns the status."""
    P = make_params(nx, ny, **params)
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    yf = np.ascontiguousarray(yf, dtype=np.float64)
    h = C.c_void_p()
    nb = workspace_bytes_ if workspace_bytes_ is not None else lib().ibm_workspace_bytes(C.byref(P))
    return lib().ibm_init(C.byref(P), _dp(xf), _dp(yf), None, None, None, C.c_void_p(workspace_ptr),
                          nb, None, C.byref(h))


class Batch:
    """The pressure solves of several solvers advanced by one batched launch
    per blocked sweep (see ibm_batch_create); the solvers stay usable alone."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s._h.value for s in self.solvers])
        h = C.c_void_p()
        rc = lib().ibm_batch_create(len(self.solvers), arr, C.byref(h))
        if rc != OK:
            raise IbmError(f"ibm_batch_create failed: {status_string(rc)}")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ibm_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, intervals: int):
        """Replay the batched solve from a HIP graph of `intervals` check
        intervals (even; 0 switches the graph off)."""
        rc = lib().ibm_batch_set_graph(self._h, intervals)
        if rc != OK:
            raise IbmError(f"ibm_batch_set_graph({intervals}) failed: {status_string(rc)}")

    def autotune_tiles(self, candidates=((76, 44), (84, 52), (80, 48), (64, 40), (48, 16)),
                       iters: int = 400):
        """Time one batched step of every case with its pressure solve replayed
        for `iters` iterations (ibm_set_poisson_schedule), from the current
        state (restored after each trial), with each candidate tile shape set
        on every case, and keep the fastest shape for the whole batch.  The
        tile shape never changes a case's iterates.  Returns the chosen shape
        and the timings (s)."""
        import time
        import torch
        blobs = [s.get_state() for s in self.solvers]
        times = {}
        for tx, ty in candidates:
            if any(s.set_option(OPT_TB_TILE_X, tx) != OK or s.set_option(OPT_TB_TILE_Y, ty) != OK
                   for s in self.solvers):
                continue
            try:
                for s in self.solvers:
                    s.set_poisson_schedule([iters])
                self.step(1)  # warm-up (descriptor upload, first touch)
                for s, blob in zip(self.solvers, blobs):
                    s.set_state(blob)
                    s.set_poisson_schedule([iters])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                self.step(1)
                torch.cuda.synchronize()
                times[(tx, ty)] = time.perf_counter() - t0
            except IbmError:
                pass  # a shape with more tiles than the batched sweep takes
            for s, blob in zip(self.solvers, blobs):
                s.set_state(blob)
                s.set_poisson_schedule([])
        best = min(times, key=times.get)
        for s in self.solvers:
            s.set_option(OPT_TB_TILE_X, best[0])
            s.set_option(OPT_TB_TILE_Y, best[1])
        return best, times

    def step(self, n: int = 1):
        """n time steps of every case; returns the last step's statistics per case."""
        st = (StepStats * len(self.solvers))()
        rc = lib().ibm_batch_step(self._h, n, st)
        if rc < 0:
            raise IbmError(f"ibm_batch_step failed: {status_string(rc)} {lib().ibm_batch_last_error(self._h).decode()}")
        out = []
        for x in st:
            d = {k: getattr(x, k) for k, _ in StepStats._fields_}
            d["rc"] = rc
            out.append(d)
        return out
