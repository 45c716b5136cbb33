"""ctypes wrapper of the plain FP64 CPU oracle (``ibm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The GPU product path never imports
this module.

The oracle follows the solver of arXiv 2402.17337 (Sec. 2.1-2.3, Eqs. 1-4):
fractional-step staggered finite volumes, AB2/CN time stepping, discrete-forcing
immersed boundary, red-black SOR (or Jacobi-PCG) pressure correction.  Every
array here is float64 numpy, row-major with x fastest:

    u   : (ny, nx+1)   x-face velocity
    v   : (ny+1, nx)   y-face velocity
    p   : (ny, nx)     cell-centred pressure (also phi, b)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibm_oracle.c")
_LIB = os.path.join(_HERE, "libibm_oracle.so")

CHANNEL, PERIODIC = 0, 1
SOR, PCG, SOR_MP = 0, 1, 2   # SOR_MP: single-precision sweeps, double-precision refinement
CG1, PCG_MP = 3, 4           # CG1: one reduction per iteration; PCG_MP: float CG, double reliable updates
OK, NOT_CONVERGED, ERR_INVALID, ERR_NAN = 0, 1, -1, -5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32), ("body", C.c_int32),
        ("re", C.c_double), ("dt", C.c_double), ("uinf", C.c_double),
        ("chord", C.c_double), ("thick", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double),
        ("p_method", C.c_int32), ("p_max_iter", C.c_int32), ("p_check", C.c_int32),
        ("p_init_prev", C.c_int32),
        ("p_omega", C.c_double), ("p_tol", C.c_double),
        ("uv_omega", C.c_double), ("uv_tol", C.c_double),
        ("uv_max_iter", C.c_int32), ("q_mode", C.c_int32),
        ("alpha_max", C.c_double),
    ]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("pad0", C.c_int32),
                ("pad1", C.c_int32), ("r0_rel", C.c_double), ("rel", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("p_iters", C.c_int32), ("u_iters", C.c_int32),
                ("v_iters", C.c_int32), ("n_forced_u", C.c_int32), ("n_forced_v", C.c_int32),
                ("n_msrc", C.c_int32), ("pad", C.c_int32),
                ("p_r0", C.c_double), ("p_rel", C.c_double), ("cd", C.c_double),
                ("cl", C.c_double), ("t", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_create.argtypes = [C.POINTER(Params), dp, dp, dp, dp, dp, C.POINTER(C.c_void_p)]
        L.orc_create.restype = C.c_int
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(StepStats)]
        L.orc_step.restype = C.c_int
        L.orc_get_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_set_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_get_rhs.argtypes = [C.c_void_p, dp]
        L.orc_apply_A.argtypes = [C.c_void_p, dp, dp]
        L.orc_poisson_solve.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_double, C.c_double,
                                        C.c_int, C.c_int, C.c_int, C.POINTER(SolveStats)]
        L.orc_poisson_solve.restype = C.c_int
        L.orc_poisson_sor_f32.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int, C.POINTER(SolveStats)]
        L.orc_poisson_sor_f32.restype = C.c_int
        L.orc_poisson_pcg_f32.argtypes = [C.c_void_p, dp, dp, C.c_int, C.POINTER(SolveStats)]
        L.orc_poisson_pcg_f32.restype = C.c_int
        L.orc_momentum_terms.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp]
        L.orc_divergence.argtypes = [C.c_void_p, dp]
        ub = C.POINTER(C.c_ubyte)
        L.orc_get_ibm.argtypes = [C.c_void_p, ub, ub, ub, dp, dp]
        L.orc_classify_at.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_int32)]
        L.orc_targets_at.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, dp]
        L.orc_forces.argtypes = [C.c_void_p, dp, dp]
        L.orc_helm_solve.argtypes = [C.c_void_p, C.c_int, dp, C.c_double, C.POINTER(C.c_int)]
        L.orc_helm_solve.restype = C.c_int
        L.orc_outlet_predictor.argtypes = [C.c_void_p, dp]
        L.orc_outlet_predictor.restype = C.c_int
        L.orc_kinematics.argtypes = [C.c_void_p, C.c_double, dp, dp, dp]
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_double
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_step_count.restype = C.c_long
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        assert L.orc_sizeof_params() == C.sizeof(Params)
        assert L.orc_sizeof_step_stats() == C.sizeof(StepStats)
        assert L.orc_sizeof_solve_stats() == C.sizeof(SolveStats)
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ub(a):
    return a.ctypes.data_as(C.POINTER(C.c_ubyte))


# Defaults follow the plain FP64 configuration: red-black SOR (omega 1.8),
# residual tolerance 1e-8 checked every 10 iterations, previous phi as the
# initial guess, Gauss-Seidel (omega 1) viscous solves to 1e-10.
DEFAULTS = dict(bc=CHANNEL, body=1, re=100.0, dt=1e-3, uinf=1.0, chord=1.0, thick=0.12,
                x0=4.0, y0=6.0, amp=0.0, freq=0.0, phase=0.0,
                p_method=SOR, p_max_iter=2_000_000, p_check=10, p_init_prev=1,
                p_omega=1.8, p_tol=1e-8, uv_omega=1.0, uv_tol=1e-10, uv_max_iter=200,
                q_mode=1, alpha_max=1.0)


def make_params(nx: int, ny: int, **kw) -> Params:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown oracle parameter {k!r}")
        d[k] = v
    P = Params()
    P.nx, P.ny = nx, ny
    for k, v in d.items():
        setattr(P, k, v)
    return P


class Oracle:
    """One oracle solver instance (a C context)."""

    def __init__(self, nx, ny, xf, yf, u0=None, v0=None, p0=None, **params):
        self.nx, self.ny = nx, ny
        self.P = make_params(nx, ny, **params)
        self.xf = np.ascontiguousarray(xf, dtype=np.float64)
        self.yf = np.ascontiguousarray(yf, dtype=np.float64)
        assert self.xf.shape == (nx + 1,) and self.yf.shape == (ny + 1,)
        arrs = []
        for a, shp in ((u0, (ny, nx + 1)), (v0, (ny + 1, nx)), (p0, (ny, nx))):
            if a is None:
                arrs.append(None)
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
                assert a.shape == shp, (a.shape, shp)
                arrs.append(a)
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(self.P), _dp(self.xf), _dp(self.yf), _dp(arrs[0]),
                              _dp(arrs[1]), _dp(arrs[2]), C.byref(h))
        if rc != OK:
            raise ValueError(f"oracle rejected the parameters (status {rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # -- time stepping -------------------------------------------------------
    def step(self, n: int = 1):
        st = (StepStats * n)()
        rc = lib().orc_step(self._h, n, st)
        out = []
        for s in st[:n]:
            out.append({k: getattr(s, k) for k, _ in StepStats._fields_ if not k.startswith("pad")})
        return rc, out

    def fields(self):
        nx, ny = self.nx, self.ny
        u = np.empty((ny, nx + 1)); v = np.empty((ny + 1, nx))
        p = np.empty((ny, nx)); phi = np.empty((ny, nx))
        lib().orc_get_fields(self._h, _dp(u), _dp(v), _dp(p), _dp(phi))
        return u, v, p, phi

    def poisson_rhs(self):
        """V b of the last pressure solve (A phi = V b; a time step's, or
        poisson_solve's), shape (ny, nx)."""
        vb = np.empty((self.ny, self.nx))
        lib().orc_get_rhs(self._h, _dp(vb))
        return vb

    def set_fields(self, u=None, v=None, p=None):
        f = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (u, v, p)]
        lib().orc_set_fields(self._h, _dp(f[0]), _dp(f[1]), _dp(f[2]))

    def forces(self):
        cd, cl = C.c_double(), C.c_double()
        lib().orc_forces(self._h, C.byref(cd), C.byref(cl))
        return cd.value, cl.value

    def kinematics(self, t):
        y, v, a = C.c_double(), C.c_double(), C.c_double()
        lib().orc_kinematics(self._h, t, C.byref(y), C.byref(v), C.byref(a))
        return y.value, v.value, a.value

    @property
    def time(self):
        return lib().orc_time(self._h)

    # -- operators -----------------------------------------------------------
    def apply_A(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.ny, self.nx)
        y = np.empty_like(x)
        lib().orc_apply_A(self._h, _dp(x), _dp(y))
        return y

    def poisson_solve(self, b, x0=None, method=SOR, omega=1.8, tol=1e-8, max_iter=2_000_000,
                      check=10, fixed=0):
        """Solve (D G) x = b (b per unit volume); returns (x, stats dict, status)."""
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(self.ny, self.nx)
        x = (np.zeros_like(b) if x0 is None
             else np.array(x0, dtype=np.float64, copy=True).reshape(self.ny, self.nx))
        st = SolveStats()
        rc = lib().orc_poisson_solve(self._h, _dp(b), _dp(x), method, omega, tol, max_iter,
                                     check, fixed, C.byref(st))
        return x, {"iters": st.iters, "r0_rel": st.r0_rel, "rel": st.rel, "status": st.status}, rc

    def poisson_sor_f32(self, b, x0=None, omega=1.8, iters=1000):
        """Single-precision SOR on the correction of x without refinement
        (iters float iterations, then x += e); returns (x, stats dict, status)."""
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(self.ny, self.nx)
        x = (np.zeros_like(b) if x0 is None
             else np.array(x0, dtype=np.float64, copy=True).reshape(self.ny, self.nx))
        st = SolveStats()
        rc = lib().orc_poisson_sor_f32(self._h, _dp(b), _dp(x), omega, iters, C.byref(st))
        return x, {"iters": st.iters, "r0_rel": st.r0_rel, "rel": st.rel, "status": st.status}, rc

    def poisson_pcg_f32(self, b, x0=None, iters=1000):
        """Single-precision one-reduction CG on the correction of x without
        refinement (iters float iterations, then x += e); returns (x, stats
        dict, status)."""
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(self.ny, self.nx)
        x = (np.zeros_like(b) if x0 is None
             else np.array(x0, dtype=np.float64, copy=True).reshape(self.ny, self.nx))
        st = SolveStats()
        rc = lib().orc_poisson_pcg_f32(self._h, _dp(b), _dp(x), iters, C.byref(st))
        return x, {"iters": st.iters, "r0_rel": st.r0_rel, "rel": st.rel, "status": st.status}, rc

    def momentum_terms(self):
        nx, ny = self.nx, self.ny
        a = [np.zeros((ny, nx + 1)) for _ in range(3)] + [np.zeros((ny + 1, nx)) for _ in range(3)]
        lib().orc_momentum_terms(self._h, *[_dp(x) for x in a])
        return dict(Nu=a[0], Gu=a[1], Lu=a[2], Nv=a[3], Gv=a[4], Lv=a[5])

    def helm_solve(self, comp, rhs, beta):
        """(I - beta L) x = rhs for component comp (0: u, 1: v) by the step's
        red-black SOR, from the current field; returns (x, iters, status)."""
        shp = (self.ny, self.nx + 1) if comp == 0 else (self.ny + 1, self.nx)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        assert rhs.shape == shp
        it = C.c_int()
        rc = lib().orc_helm_solve(self._h, comp, _dp(rhs), beta, C.byref(it))
        u, v, _, _ = self.fields()
        return (u if comp == 0 else v), it.value, rc

    def outlet_predictor(self):
        """Convective-outlet predictor u* of every row for the current fields."""
        out = np.empty(self.ny)
        rc = lib().orc_outlet_predictor(self._h, _dp(out))
        assert rc == OK
        return out

    def divergence(self):
        d = np.empty((self.ny, self.nx))
        lib().orc_divergence(self._h, _dp(d))
        return d

    def ibm(self):
        nx, ny = self.nx, self.ny
        flu = np.zeros((ny, nx + 1), np.uint8); flv = np.zeros((ny + 1, nx), np.uint8)
        ms = np.zeros((ny, nx), np.uint8)
        fu = np.zeros((ny, nx + 1)); fv = np.zeros((ny + 1, nx))
        lib().orc_get_ibm(self._h, _ub(flu), _ub(flv), _ub(ms), _dp(fu), _dp(fv))
        return dict(flu=flu, flv=flv, msrc=ms, fu=fu, fv=fv)

    def classify_at(self, t):
        cnt = (C.c_int32 * 3)()
        lib().orc_classify_at(self._h, t, cnt)
        d = self.ibm()
        d["counts"] = tuple(cnt)
        return d

    def targets_at(self, t, ut, vt):
        ut = np.ascontiguousarray(ut, dtype=np.float64)
        vt = np.ascontiguousarray(vt, dtype=np.float64)
        Vu = np.full_like(ut, np.nan); Vv = np.full_like(vt, np.nan)
        lib().orc_targets_at(self._h, t, _dp(ut), _dp(vt), _dp(Vu), _dp(Vv))
        return Vu, Vv


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(n)
