"""Seeded synthetic inputs for the plunging-ellipse workloads.

This module only builds inputs: face coordinates of uniform and stretched
Cartesian grids, seeded noise, and the parameter sets of the standard
workloads.  It contains none of the solver's arithmetic and is shared by the
tests, the benchmark and the smoke check.

Paper context (arXiv 2402.17337, Sec. 2.1 and 2.3): a 2-D ellipse of
thickness/chord 0.12 in a uniform stream, plunging as y = h sin(k t); the mesh
is uniform around the body's path and stretched geometrically towards the
outer boundaries.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` outputs of SplitMix64 (Steele, Lea & Flood 2014) from `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm(seed: int, count: int, amplitude: float) -> np.ndarray:
    """`count` values uniform in [-amplitude, amplitude) from 53-bit mantissas."""
    z = splitmix64(seed, count)
    u01 = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (2.0 * u01 - 1.0) * amplitude


def uniform_faces(n: int, length: float, origin: float = 0.0) -> np.ndarray:
    return origin + length * (np.arange(n + 1, dtype=np.float64) / n)


def _geometric_ratio(h: float, m: int, length: float) -> float:
    """Ratio r > 1 with sum_{k=1..m} h r^k = length (bisection)."""
    if m * h >= length:
        raise ValueError("side too short for the requested cell count")

    def total(r):
        e = min(m * np.log(r), 700.0)
        return h * r * np.expm1(e) / (r - 1.0)

    lo, hi = 1.0 + 1e-14, 1.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < length:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def stretched_faces(n: int, length: float, core_lo: float, core_hi: float, h: float):
    """Faces of an n-cell grid on [0, length]: uniform spacing h on
    [core_lo, core_hi], geometric growth outward on both sides.  The split of
    the remaining cells between the two sides is the one whose two growth
    ratios are closest.  Returns (faces, info)."""
    ncore = int(round((core_hi - core_lo) / h))
    if abs(ncore * h - (core_hi - core_lo)) > 1e-9 * length:
        raise ValueError("core length must be a multiple of h")
    rest = n - ncore
    left, right = core_lo, length - core_hi
    best = None
    for nl in range(1, rest):
        nr = rest - nl
        if nl * h >= left or nr * h >= right:
            continue
        rl = _geometric_ratio(h, nl, left)
        rr = _geometric_ratio(h, nr, right)
        if best is None or abs(rl - rr) < best[0]:
            best = (abs(rl - rr), nl, nr, rl, rr)
    _, nl, nr, rl, rr = best
    lf = core_lo - np.cumsum(h * rl ** np.arange(1, nl + 1))
    lf[-1] = 0.0
    core = core_lo + h * np.arange(ncore + 1)
    core[-1] = core_hi
    rf = core_hi + np.cumsum(h * rr ** np.arange(1, nr + 1))
    rf[-1] = length
    faces = np.concatenate([lf[::-1], core, rf])
    assert faces.shape == (n + 1,)
    assert np.all(np.diff(faces) > 0)
    info = dict(n_left=nl, n_core=ncore, n_right=nr, r_left=rl, r_right=rr,
                h_max=float(np.max(np.diff(faces))))
    return faces, info


def initial_fields(nx: int, ny: int, uinf: float, noise: float = 0.0, seed: int = 0):
    """u = uinf, v = 0, p = 0, plus seeded noise uniform in [-noise, noise) on
    the non-Dirichlet velocity nodes: u faces 1..nx of every row, then v faces
    of rows 1..ny-1, in row-major order from one SplitMix64 stream."""
    u = np.full((ny, nx + 1), float(uinf))
    v = np.zeros((ny + 1, nx))
    p = np.zeros((ny, nx))
    if noise > 0.0:
        nu = ny * nx
        nv = (ny - 1) * nx
        r = uniform_pm(seed, nu + nv, noise)
        u[:, 1:] += r[:nu].reshape(ny, nx)
        v[1:ny, :] += r[nu:].reshape(ny - 1, nx)
    return u, v, p


# --------------------------------------------------------------------------
# Standard workloads.  Parameter names are shared by the oracle and the GPU
# binding; each maps them onto its own parameter block.
# --------------------------------------------------------------------------
COMMON = dict(bc=0, body=1, uinf=1.0, chord=1.0, thick=0.12, x0=4.0, y0=6.0, phase=0.0,
              p_method=0, p_omega=1.8, p_tol=1e-8, p_check=10, p_max_iter=20_000_000,
              p_init_prev=1, uv_omega=1.0, uv_tol=1e-10, uv_max_iter=200, q_mode=1,
              alpha_max=1.0)


def _pack(name, nx, ny, xf, yf, u0, v0, p0, steps, grid_info=None, **params):
    prm = dict(COMMON)
    prm.update(params)
    return dict(name=name, nx=nx, ny=ny, xf=xf, yf=yf, u0=u0, v0=v0, p0=p0, steps=steps,
                params=prm, grid=grid_info or {})


def stationary_128x96():
    """Plain FP64, stationary ellipse, uniform 128x96 grid on 16c x 12c, foil at
    (4c, 6c), Re 100, dt 1e-3, 100 steps, red-black SOR (omega 1.8) to 1e-8,
    u = 1 and v = 0 plus seeded noise of amplitude 1e-3 (seed 0)."""
    nx, ny = 128, 96
    xf, yf = uniform_faces(nx, 16.0), uniform_faces(ny, 12.0)
    u0, v0, p0 = initial_fields(nx, ny, 1.0, noise=1e-3, seed=0)
    return _pack("stationary ellipse 128x96, Re 100", nx, ny, xf, yf, u0, v0, p0, 100,
                 re=100.0, dt=1e-3, amp=0.0, freq=0.0)


def plunging_1024x768():
    """Plain FP64, plunging ellipse h = 0.5, f = 0.4, Re 500, dt 5e-4, 2000
    steps, 1024x768 grid uniform (0.01c) on the core [3, 5.5] x [5.2, 6.8] and
    stretched geometrically outward on 16c x 12c."""
    nx, ny = 1024, 768
    xf, ix = stretched_faces(nx, 16.0, 3.0, 5.5, 0.01)
    yf, iy = stretched_faces(ny, 12.0, 5.2, 6.8, 0.01)
    u0, v0, p0 = initial_fields(nx, ny, 1.0)
    return _pack("plunging ellipse 1024x768, Re 500", nx, ny, xf, yf, u0, v0, p0, 2000,
                 grid_info=dict(x=ix, y=iy), re=500.0, dt=5e-4, amp=0.5, freq=0.4)


def plunging_2048x1536():
    """Plunging ellipse h = 0.6, f = 0.5, Re 1000, dt 5e-4 on a 2048x1536 grid
    (core 0.005c on [3, 5.5] x [5.1, 6.9], stretched outward)."""
    nx, ny = 2048, 1536
    xf, ix = stretched_faces(nx, 16.0, 3.0, 5.5, 0.005)
    yf, iy = stretched_faces(ny, 12.0, 5.1, 6.9, 0.005)
    u0, v0, p0 = initial_fields(nx, ny, 1.0)
    return _pack("plunging ellipse 2048x1536, Re 1000", nx, ny, xf, yf, u0, v0, p0, 2000,
                 grid_info=dict(x=ix, y=iy), re=1000.0, dt=5e-4, amp=0.6, freq=0.5)


def plunging_stretched(nx: int, ny: int, core_h: float):
    """The 1024x768 plunging case (h = 0.5, f = 0.4, Re 500, dt 5e-4) on another
    grid of the same construction: uniform spacing core_h on the core
    [3, 5.5] x [5.2, 6.8], stretched geometrically outward."""
    xf, ix = stretched_faces(nx, 16.0, 3.0, 5.5, core_h)
    yf, iy = stretched_faces(ny, 12.0, 5.2, 6.8, core_h)
    u0, v0, p0 = initial_fields(nx, ny, 1.0)
    return _pack(f"plunging ellipse {nx}x{ny}, Re 500", nx, ny, xf, yf, u0, v0, p0, 2000,
                 grid_info=dict(x=ix, y=iy), re=500.0, dt=5e-4, amp=0.5, freq=0.4)


def plunging_scaled(nx: int, ny: int):
    """The 1024x768 plunging case (h = 0.5, f = 0.4, Re 500, dt 5e-4) on an
    nx x ny grid of the same construction, its core spacing 0.01 * 1024 / nx
    rounded so that the core [3, 5.5] x [5.2, 6.8] holds a whole number of
    cells in each direction (the input-scaling series)."""
    h0 = 0.01 * 1024 / nx
    xf, ix = stretched_faces(nx, 16.0, 3.0, 5.5, 2.5 / round(2.5 / h0))
    yf, iy = stretched_faces(ny, 12.0, 5.2, 6.8, 1.6 / round(1.6 / h0))
    u0, v0, p0 = initial_fields(nx, ny, 1.0)
    return _pack(f"plunging ellipse {nx}x{ny}, Re 500", nx, ny, xf, yf, u0, v0, p0, 2000,
                 grid_info=dict(x=ix, y=iy), re=500.0, dt=5e-4, amp=0.5, freq=0.4)


def batched_plunging(n: int = 64, seed: int = 0):
    """The many-case workload: n plunging-ellipse cases from a seeded
    generator, nx uniform on the multiples of 32 in [256, 1024], ny = 3 nx / 4,
    core spacing 0.01 * 1024 / nx rounded so that the core [3, 5.5] x
    [5.2, 6.8] holds a whole number of cells in each direction, h uniform in
    [0.2, 0.8], f uniform in [0.2, 0.6], Re in {100, 300, 500}; dt 5e-4."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = 32 * int(rng.integers(8, 33))
        ny = 3 * nx // 4
        h0 = 0.01 * 1024 / nx
        hx = 2.5 / round(2.5 / h0)
        hy = 1.6 / round(1.6 / h0)
        amp = float(rng.uniform(0.2, 0.8))
        freq = float(rng.uniform(0.2, 0.6))
        re = float(rng.choice([100.0, 300.0, 500.0]))
        xf, ix = stretched_faces(nx, 16.0, 3.0, 5.5, hx)
        yf, iy = stretched_faces(ny, 12.0, 5.2, 6.8, hy)
        u0, v0, p0 = initial_fields(nx, ny, 1.0)
        out.append(_pack(f"plunging ellipse {nx}x{ny}, h {amp:.3f}, f {freq:.3f}, Re {re:g}", nx, ny, xf, yf,
                         u0, v0, p0, 1, grid_info=dict(x=ix, y=iy), re=re, dt=5e-4, amp=amp, freq=freq))
    return out


def small_plunging(nx=64, ny=48, seed=0):
    """A small plunging case (uniform grid, visible body) for quick checks."""
    xf, yf = uniform_faces(nx, 8.0), uniform_faces(ny, 6.0)
    u0, v0, p0 = initial_fields(nx, ny, 1.0, noise=1e-3, seed=seed)
    return _pack(f"plunging ellipse {nx}x{ny}", nx, ny, xf, yf, u0, v0, p0, 20,
                 re=200.0, dt=2e-3, amp=0.4, freq=0.5, x0=2.5, y0=3.0, chord=1.0)
