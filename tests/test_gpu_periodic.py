"""GPU parity of the periodic boundary mode against the FP64 oracle, through
the C ABI: the singular Poisson problem (zero-sum right-hand side, zero-mean
solution) and the Taylor-Green vortex stepped by the fractional-step method
of Sec. 2.2 with no body.

The oracle pins this mode on its own (tests/test_oracle_flow.py: the vortex
decays as exp(-2t/Re) with second order in space and time, energy at the
exact rate); here the GPU library must reproduce the oracle's fields to a
relative L2 of 1e-10."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_17337_amd import ibm
from paper_2402_17337_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _faces(nx, ny, stretched):
    xf = W.uniform_faces(nx, 2 * np.pi)
    yf = W.uniform_faces(ny, 1.5 * np.pi)
    if stretched:
        s = W.uniform_faces(nx, 1.0)
        xf = 2 * np.pi * (s - 0.1 * np.sin(2 * np.pi * s) / (2 * np.pi))
        s = W.uniform_faces(ny, 1.0)
        yf = 1.5 * np.pi * (s - 0.08 * np.sin(2 * np.pi * s) / (2 * np.pi))
    return xf, yf


@pytest.mark.parametrize("nx,ny,stretched", [(64, 48, False), (200, 150, True)])
def test_singular_poisson_sor_fixed_iterations(torch, nx, ny, stretched):
    xf, yf = _faces(nx, ny, stretched)
    o = O.Oracle(nx, ny, xf, yf, bc=O.PERIODIC, body=0)
    g = ibm.Solver(nx, ny, xf, yf, bc=ibm.BC_PERIODIC, body=0)
    rng = np.random.default_rng(nx)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    xo, so, rc = o.poisson_solve(b, x0=x0, omega=1.8, fixed=37, check=10)
    x = _dev(torch, x0)
    st = g.poisson_solve(_dev(torch, b), x, omega=1.8, fixed_iters=37, check_every=10)
    assert st["rc"] == ibm.OK and st["iters"] == 37
    xg = x.cpu().numpy()
    assert rel_l2(xg, xo) <= TOL
    # the solution has zero volume-weighted mean on both sides
    vol = np.outer(np.diff(yf), np.diff(xf))
    assert abs(np.sum(vol * xg)) <= 1e-12 * np.sum(vol * np.abs(xg))


def test_singular_poisson_to_tolerance(torch):
    nx, ny = 96, 64
    xf, yf = _faces(nx, ny, False)
    o = O.Oracle(nx, ny, xf, yf, bc=O.PERIODIC, body=0)
    g = ibm.Solver(nx, ny, xf, yf, bc=ibm.BC_PERIODIC, body=0)
    X, Y = np.meshgrid(0.5 * (xf[1:] + xf[:-1]), 0.5 * (yf[1:] + yf[:-1]))
    b = np.cos(X) * np.sin(2 * Y / 1.5) + 0.3  # a nonzero mean the solve projects away
    # SOR: the same iteration sequence as the oracle
    xo, so, _ = o.poisson_solve(b, omega=1.8, tol=1e-10, check=10)
    x = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    st = g.poisson_solve(_dev(torch, b), x, omega=1.8, tol=1e-10, check_every=10)
    assert st["rc"] == ibm.OK and abs(st["iters"] - so["iters"]) <= 10
    # the oracle's iteration count replayed: the same iterate
    x.zero_()
    st = g.poisson_solve(_dev(torch, b), x, omega=1.8, fixed_iters=so["iters"], check_every=10)
    assert rel_l2(x.cpu().numpy(), xo) <= TOL
    # PCG: both near the exact discrete solution
    xo, so, _ = o.poisson_solve(b, method=O.PCG, tol=1e-13)
    x.zero_()
    st = g.poisson_solve(_dev(torch, b), x, method=ibm.PCG, tol=1e-13)
    assert st["rc"] == ibm.OK and st["rel"] <= 1e-13
    assert rel_l2(x.cpu().numpy(), xo) <= TOL


def _tg(nx, ny, **kw):
    L, H = 2 * np.pi, 2 * np.pi
    xf, yf = W.uniform_faces(nx, L), W.uniform_faces(ny, H)
    xc, yc = 0.5 * (xf[1:] + xf[:-1]), 0.5 * (yf[1:] + yf[:-1])
    Xu, Yu = np.meshgrid(xf, yc)
    Xv, Yv = np.meshgrid(xc, yf)
    Xc, Yc = np.meshgrid(xc, yc)
    u0 = np.sin(Xu) * np.cos(Yu)
    v0 = -np.cos(Xv) * np.sin(Yv)
    p0 = 0.25 * (np.cos(2 * Xc) + np.cos(2 * Yc))
    prm = dict(bc=O.PERIODIC, body=0, re=10.0, dt=2.5e-3, uinf=0.0, uv_tol=1e-13)
    prm.update(kw)
    o = O.Oracle(nx, ny, xf, yf, u0, v0, p0, **prm)
    g = ibm.Solver(nx, ny, xf, yf, u0, v0, p0, **prm)
    return o, g


def test_taylor_green_pcg_steps_match_oracle(torch):
    # 48 x 32 cells: x and y differ, so a transposed index would show
    o, g = _tg(48, 32, p_method=O.PCG, p_tol=1e-12, p_max_iter=20000)
    n = 40
    rc, so = o.step(n)
    assert rc == O.OK
    for k in range(n):
        st = g.step(1)
        assert st["rc"] == ibm.OK, st
    for a, b, name in zip(g.fields()[:3], o.fields()[:3], "uvp"):
        assert rel_l2(a, b) <= TOL, (name, rel_l2(a, b))
    # the last step's right-hand side V b, after its zero-sum projection (the
    # singular periodic problem), on both sides.  V b = (dy (u_E - u_W) +
    # dx (v_N - v_S)) / dt of the predicted velocity is a small difference of
    # O(1) face fluxes, so the fields' relative bar carries over to it through
    # the largest flux, not through V b's own size
    vb, vo = g.poisson_rhs(), o.poisson_rhs()
    u, v = o.fields()[:2]
    dx, dy = 2 * np.pi / 48, 2 * np.pi / 32
    flux = dy * (np.abs(u[:, 1:]) + np.abs(u[:, :-1])) + dx * (np.abs(v[1:, :]) + np.abs(v[:-1, :]))
    bar = TOL * np.max(flux) / 2.5e-3
    assert np.max(np.abs(vb - vo)) <= bar, (np.max(np.abs(vb - vo)), bar)
    assert bar < 1e-2 * np.max(np.abs(vo))  # the bar still resolves V b
    assert abs(vb.sum()) <= 1e-12 * np.abs(vb).sum() and abs(vo.sum()) <= 1e-12 * np.abs(vo).sum()
    # the vortex decayed as the exact solution does (the oracle's own pin, to
    # the discretisation error at this resolution)
    u = g.fields()[0]
    F = np.exp(-2.0 * n * 2.5e-3 / 10.0)
    xf = W.uniform_faces(48, 2 * np.pi)
    yc = 0.5 * (W.uniform_faces(32, 2 * np.pi)[1:] + W.uniform_faces(32, 2 * np.pi)[:-1])
    Xu, Yu = np.meshgrid(xf, yc)
    assert np.max(np.abs(u - F * np.sin(Xu) * np.cos(Yu))) < 1e-2
    assert np.array_equal(u[:, -1], u[:, 0])  # face nx mirrors face 0


def test_taylor_green_sor_steps_replay_oracle_counts(torch):
    o, g = _tg(32, 32, p_method=O.SOR, p_tol=1e-10, p_check=10)
    n = 20
    rc, so = o.step(n)
    assert rc == O.OK
    g.set_poisson_schedule([s["p_iters"] for s in so])
    for k in range(n):
        st = g.step(1)
        assert st["rc"] == ibm.OK and st["p_iters"] == so[k]["p_iters"], (k, st, so[k])
        assert abs(st["u_iters"] - so[k]["u_iters"]) <= 1 and abs(st["v_iters"] - so[k]["v_iters"]) <= 1
    for a, b, name in zip(g.fields()[:3], o.fields()[:3], "uvp"):
        assert rel_l2(a, b) <= TOL, (name, rel_l2(a, b))


def test_periodic_mode_rejections(torch):
    xf, yf = _faces(64, 48, False)
    g = ibm.Solver(64, 48, xf, yf, bc=ibm.BC_PERIODIC, body=0)
    z = torch.zeros(48, 64, dtype=torch.float64, device="cuda")
    with pytest.raises(ibm.IbmError):
        g.poisson_solve(z, z.clone(), method=ibm.RBSOR_MP)
    with pytest.raises(ibm.IbmError):
        ibm.Batch([g])


@pytest.mark.parametrize("nx,ny", [(96, 64), (200, 150)])
def test_singular_poisson_one_reduction_cg(torch, nx, ny):
    """The one-reduction CG (tiled kernel; 200x150 leaves ragged tiles whose
    wrapped neighbours lie outside the tile's frame) to 1e-13 against the
    oracle's, and fixed iteration counts against the GPU's textbook PCG."""
    xf, yf = _faces(nx, ny, nx == 200)
    o = O.Oracle(nx, ny, xf, yf, bc=O.PERIODIC, body=0)
    g = ibm.Solver(nx, ny, xf, yf, bc=ibm.BC_PERIODIC, body=0)
    rng = np.random.default_rng(ny)
    b = rng.standard_normal((ny, nx))
    xo, so, _ = o.poisson_solve(b, method=O.CG1, tol=1e-13, max_iter=50000)
    x = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    st = g.poisson_solve(_dev(torch, b), x, method=ibm.CG1, tol=1e-13, max_iter=50000)
    assert st["rc"] == ibm.OK and st["rel"] <= 1e-13
    assert rel_l2(x.cpu().numpy(), xo) <= TOL
    xa = torch.zeros_like(x)
    xb = torch.zeros_like(x)
    g.poisson_solve(_dev(torch, b), xa, method=ibm.CG1, fixed_iters=40)
    g.poisson_solve(_dev(torch, b), xb, method=ibm.PCG, fixed_iters=40)
    assert rel_l2(xa.cpu().numpy(), xb.cpu().numpy()) <= TOL


def test_taylor_green_one_reduction_cg_steps_match_oracle(torch):
    o, g = _tg(48, 32, p_method=O.CG1, p_tol=1e-12, p_max_iter=20000)
    rc, so = o.step(20)
    assert rc == O.OK
    for k in range(20):
        assert g.step(1)["rc"] == ibm.OK
    for a, b, name in zip(g.fields()[:3], o.fields()[:3], "uvp"):
        assert rel_l2(a, b) <= TOL, (name, rel_l2(a, b))
