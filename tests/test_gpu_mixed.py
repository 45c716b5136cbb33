"""GPU mixed-precision red-black SOR (single-precision sweeps on the
correction equation, double-precision refinement) against the oracle's
mixed-precision and double-precision solves, through the C ABI.

The method accelerates the paper's red-black SOR pressure solve (Sec. 2.2,
3.1).  The float sweeps round differently on the two sides (fused
multiply-adds and float-rounded 1-D coefficient arrays on the GPU, plain float
operations on the oracle's coefficients), so the bar is derived from the
arithmetic rather than 1e-10:
  - after one check interval of K iterations from the same start, the
    correction agrees to single-precision rounding:
    |x_gpu - x_oracle| <= max(1e-5, 10 K u) |x_oracle - x0|, u = 2^-24 (the
    sweeps are contractive, so rounding errors of the K float iterations add
    at most linearly; K = 10 and the benchmark's K = 100);
  - to tolerance, both stop within one check interval of each other and of
    double SOR, and the GPU result meets the double-precision stop test when
    its residual is recomputed by the oracle's operator;
  - the tile shape never changes the iterates (bitwise).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_17337_amd import ibm
from test_gpu_poisson import _dev, _grid, _pair, rel_l2, torch  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _vb(o, b):
    return b * np.diff(o.xf)[None, :] * np.diff(o.yf)[:, None]


@pytest.mark.parametrize("nx,ny,stretched,check", [(128, 96, False, 10), (200, 150, True, 10), (16, 8, False, 10),
                                                   (128, 96, False, 100), (200, 150, True, 100)])
def test_one_interval_matches_oracle_to_float_rounding(torch, nx, ny, stretched, check):
    o, g = _pair(torch, nx, ny, stretched)
    rng = np.random.default_rng(nx * 3 + ny)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    bar = max(1e-5, 10 * check * 2.0 ** -24)
    for fixed in (check, 2 * check + 3):
        xo, so, rco = o.poisson_solve(b, x0=x0, method=O.SOR_MP, omega=1.8, fixed=fixed, check=check)
        x64, _, _ = o.poisson_solve(b, x0=x0, method=O.SOR, omega=1.8, fixed=fixed, check=check)
        xd = _dev(torch, x0)
        st = g.poisson_solve(_dev(torch, b), xd, method=ibm.RBSOR_MP, omega=1.8, fixed_iters=fixed,
                             check_every=check)
        xg = xd.cpu().numpy()
        corr = np.linalg.norm(xo - x0)
        d_or = np.linalg.norm(xg - xo) / corr
        d_64 = np.linalg.norm(xg - x64) / corr
        print(f"{nx}x{ny} fixed={fixed}: |gpu-oracle_mp|/|corr| {d_or:.3e}  |gpu-oracle_f64|/|corr| {d_64:.3e} "
              f"rel {st['rel']:.3e} vs {so['rel']:.3e}", flush=True)
        assert rco == O.OK and st["rc"] == ibm.OK and st["iters"] == fixed
        assert d_or <= bar and d_64 <= bar
        assert abs(st["rel"] - so["rel"]) <= 1e-4 * so["rel"]


@pytest.mark.parametrize("nx,ny,stretched,check", [(128, 96, False, 10), (200, 150, True, 10), (200, 150, True, 100)])
def test_to_tolerance_meets_the_double_stop_test(torch, nx, ny, stretched, check):
    o, g = _pair(torch, nx, ny, stretched)
    rng = np.random.default_rng(nx + 5)
    b = rng.standard_normal((ny, nx))
    _, s64, _ = o.poisson_solve(b, method=O.SOR, omega=1.8, tol=1e-8, check=check)
    xo, smp, _ = o.poisson_solve(b, method=O.SOR_MP, omega=1.8, tol=1e-8, check=check)
    xd = _dev(torch, np.zeros((ny, nx)))
    st = g.poisson_solve(_dev(torch, b), xd, method=ibm.RBSOR_MP, omega=1.8, tol=1e-8, check_every=check)
    xg = xd.cpu().numpy()
    vb = _vb(o, b)
    r = vb - o.apply_A(xg)
    true_rel = np.linalg.norm(r) / np.linalg.norm(vb)
    print(f"{nx}x{ny}: iters gpu {st['iters']} oracle_mp {smp['iters']} oracle_f64 {s64['iters']}; "
          f"true rel {true_rel:.3e}; |gpu-oracle_mp| {rel_l2(xg, xo):.3e}", flush=True)
    assert st["rc"] == ibm.OK
    assert abs(st["iters"] - smp["iters"]) <= check and abs(st["iters"] - s64["iters"]) <= check
    assert true_rel <= 1e-8 * (1 + 1e-6)
    assert abs(true_rel - st["rel"]) <= 1e-6 * true_rel + 1e-16


@pytest.mark.parametrize("sweeps,tiles", [(5, [(104, 32), (16, 12), (64, 40)]), (3, [(32, 24), (112, 48)])])
def test_tile_shape_does_not_change_iterates(torch, sweeps, tiles):
    nx, ny = 200, 150
    o, g = _pair(torch, nx, ny, True)
    rng = np.random.default_rng(sweeps)
    b = _dev(torch, rng.standard_normal((ny, nx)))
    x0 = rng.standard_normal((ny, nx))
    out = []
    for tx, ty in tiles:
        assert g.set_option(ibm.OPT_TB_SWEEPS, 1) == ibm.OK
        assert g.set_option(ibm.OPT_TB_TILE_X, tx) == ibm.OK
        assert g.set_option(ibm.OPT_TB_TILE_Y, ty) == ibm.OK
        assert g.set_option(ibm.OPT_TB_SWEEPS, sweeps) == ibm.OK
        xd = _dev(torch, x0)
        st = g.poisson_solve(b, xd, method=ibm.RBSOR_MP, omega=1.8, fixed_iters=27, check_every=10)
        out.append((xd.cpu().numpy(), st))
    for x, st in out[1:]:
        assert np.array_equal(x, out[0][0])
        # the residual norm is summed per tile: equal up to summation order
        assert abs(st["rel"] - out[0][1]["rel"]) <= 1e-12 * out[0][1]["rel"]


def test_status_paths(torch):
    nx, ny = 64, 48
    o, g = _pair(torch, nx, ny, False)
    zero = _dev(torch, np.zeros((ny, nx)))
    xd = _dev(torch, np.ones((ny, nx)))
    st = g.poisson_solve(zero, xd, method=ibm.RBSOR_MP)
    assert st["rc"] == ibm.OK and st["iters"] == 0
    assert np.all(xd.cpu().numpy() == 0.0)
    rng = np.random.default_rng(1)
    b = _dev(torch, rng.standard_normal((ny, nx)))
    xd = _dev(torch, np.zeros((ny, nx)))
    st = g.poisson_solve(b, xd, method=ibm.RBSOR_MP, tol=1e-14, max_iter=40)
    assert st["rc"] == ibm.NOT_CONVERGED and st["iters"] == 40
    bad = rng.standard_normal((ny, nx))
    bad[5, 7] = np.nan
    st = g.poisson_solve(_dev(torch, bad), _dev(torch, np.zeros((ny, nx))), method=ibm.RBSOR_MP)
    assert st["rc"] == ibm.ERR_NAN


def test_time_steps_match_the_oracle(torch):
    """Small plunging case, pressure by mixed-precision SOR on both sides (the
    GPU replays the oracle's iteration counts).  The fields agree to the
    single-precision rounding of the corrections, far below the 1e-8 stop
    test; the distance to the double-precision oracle run is printed."""
    from paper_2402_17337_amd import workloads as W
    from test_gpu_step import _oracle, _solver
    c = W.small_plunging()
    nsteps = 6
    o = _oracle(c, p_method=O.SOR_MP)
    rc, so = o.step(nsteps)
    assert rc == O.OK
    iters = [s["p_iters"] for s in so]
    o64 = _oracle(c)
    assert o64.step(nsteps)[0] == O.OK
    g = _solver(c, p_method=ibm.RBSOR_MP)
    g.set_poisson_schedule(iters)
    for k in range(nsteps):
        sg = g.step(1)
        assert sg["rc"] == ibm.OK and sg["p_iters"] == iters[k]
    ug, vg, pg, _ = g.fields()
    uo, vo, po, _ = o.fields()
    u6, v6, p6, _ = o64.fields()
    du, dv, dp = rel_l2(ug, uo), rel_l2(vg, vo), rel_l2(pg, po)
    e64 = (rel_l2(ug, u6), rel_l2(vg, v6), rel_l2(pg, p6))
    print(f"mixed steps: iters {iters}; gpu vs oracle_mp u {du:.3e} v {dv:.3e} p {dp:.3e}; "
          f"vs oracle_f64 u {e64[0]:.3e} v {e64[1]:.3e} p {e64[2]:.3e}", flush=True)
    assert du <= 1e-8 and dv <= 1e-8 and dp <= 1e-6


def test_many_tiles_test_the_residual_outside_the_sweep(torch):
    """With more tiles than a blocked launch sums itself (1024 here), the stop
    test runs as a separate kernel: same iterates and stop decision as the
    default tiling."""
    nx, ny = 512, 384
    o, g = _pair(torch, nx, ny, True)
    rng = np.random.default_rng(9)
    b = _dev(torch, rng.standard_normal((ny, nx)))
    res = []
    for tx, ty in ((104, 32), (16, 12)):
        assert g.set_option(ibm.OPT_TB_SWEEPS, 1) == ibm.OK
        assert g.set_option(ibm.OPT_TB_TILE_X, tx) == ibm.OK
        assert g.set_option(ibm.OPT_TB_TILE_Y, ty) == ibm.OK
        assert g.set_option(ibm.OPT_TB_SWEEPS, 5 if tx > 16 else 2) == ibm.OK
        xf = _dev(torch, np.zeros((ny, nx)))
        sf = g.poisson_solve(b, xf, method=ibm.RBSOR_MP, fixed_iters=33, check_every=10)
        xt = _dev(torch, np.zeros((ny, nx)))
        st = g.poisson_solve(b, xt, method=ibm.RBSOR_MP, tol=1e-3, check_every=10)
        res.append((xf.cpu().numpy(), sf, xt.cpu().numpy(), st))
    a, c = res
    print(f"many tiles: iters {a[3]['iters']} {c[3]['iters']}", flush=True)
    assert np.array_equal(a[0], c[0])
    assert a[3]["iters"] == c[3]["iters"] and np.array_equal(a[2], c[2])


@pytest.mark.parametrize("which", ["plunging_1024x768", "plunging_2048x1536"])
def test_full_size_grids_in_the_benchmark_configuration(torch, which):
    """The stretched grids of the 1024x768 and 2048x1536 workloads with the
    benchmark's refinement interval (100 iterations): one full interval and a
    partial one (130 iterations) from the same start against the oracle's
    mixed and double-precision solves, to the one-interval bar."""
    from paper_2402_17337_amd import workloads as W
    c = getattr(W, which)()
    nx, ny = c["nx"], c["ny"]
    o, g = _pair(torch, nx, ny, faces=(c["xf"], c["yf"]))
    rng = np.random.default_rng(nx + 17)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    check, fixed = 100, 130
    xo, so, rco = o.poisson_solve(b, x0=x0, method=O.SOR_MP, omega=1.8, fixed=fixed, check=check)
    x64, _, _ = o.poisson_solve(b, x0=x0, method=O.SOR, omega=1.8, fixed=fixed, check=check)
    xd = _dev(torch, x0)
    st = g.poisson_solve(_dev(torch, b), xd, method=ibm.RBSOR_MP, omega=1.8, fixed_iters=fixed, check_every=check)
    xg = xd.cpu().numpy()
    corr = np.linalg.norm(xo - x0)
    d_or, d_64 = np.linalg.norm(xg - xo) / corr, np.linalg.norm(xg - x64) / corr
    print(f"{which}: |gpu-oracle_mp|/|corr| {d_or:.3e} |gpu-oracle_f64|/|corr| {d_64:.3e}", flush=True)
    bar = 10 * check * 2.0 ** -24
    assert rco == O.OK and st["rc"] == ibm.OK and st["iters"] == fixed
    assert d_or <= bar and d_64 <= bar
    assert abs(st["rel"] - so["rel"]) <= 1e-4 * so["rel"]


def test_full_size_mixed_step_to_tolerance_leaves_the_residual_as_divergence(torch):
    """The 2048x1536 workload, one step with FP32 sweeps refined every 100
    iterations to the 1e-8 tolerance, as the benchmark runs it: the FP64
    refinement leaves a residual that meets the double stop test, and the
    projection turns it into the divergence, V D(u^{n+1}) = dt (V b - A phi),
    in every cell without a mass source (a property that holds at any size;
    A is the oracle's operator)."""
    from paper_2402_17337_amd import workloads as W
    from projection_identity import divergence_identity
    c = W.plunging_2048x1536()
    g = ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"],
                   **dict(c["params"], p_method=ibm.RBSOR_MP, p_check=100))
    st = g.step(1)
    print("2048x1536 mixed step: iterations", st["p_iters"], "p_rel", st["p_rel"], flush=True)
    assert st["rc"] == ibm.OK and st["p_rel"] <= c["params"]["p_tol"]
    u, v, _, phi = g.fields()
    A = O.Oracle(c["nx"], c["ny"], c["xf"], c["yf"], **c["params"]).apply_A
    d = divergence_identity(u, v, g.poisson_rhs(), phi, g.ibm()["msrc"], c["xf"], c["yf"], c["params"]["dt"], A)
    print("divergence identity", d, flush=True)
    assert d["rel"] <= c["params"]["p_tol"] and abs(d["rel"] - st["p_rel"]) <= 1e-3 * d["rel"]
    assert d["scale"] > 100 * d["bar"] and d["err"] <= d["bar"]
    g.close()
