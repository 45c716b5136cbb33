"""GPU parity of the pressure Poisson solvers (red-black SOR, Jacobi-PCG)
against the FP64 oracle, through the C ABI.

Paper: the pressure-correction equation, solved by red-black Gauss-Seidel SOR,
is the dominant cost of a step (Table 1, Sec. 3.4.1).  Bar: relative L2
difference <= 1e-10 in FP64 (and equal iteration counts for SOR, which runs
the same iteration sequence as the oracle)."""
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


def _grid(nx, ny, stretched):
    if not stretched:
        return W.uniform_faces(nx, 16.0), W.uniform_faces(ny, 12.0)
    s = W.uniform_faces(nx, 1.0)
    xf = 16.0 * (s - 0.12 * np.sin(2 * np.pi * s) / (2 * np.pi))
    s = W.uniform_faces(ny, 1.0)
    yf = 12.0 * (s - 0.10 * np.sin(2 * np.pi * s) / (2 * np.pi))
    return xf, yf


def _pair(torch, nx, ny, stretched=False, faces=None):
    xf, yf = faces if faces is not None else _grid(nx, ny, stretched)
    o = O.Oracle(nx, ny, xf, yf, body=0)
    g = ibm.Solver(nx, ny, xf, yf, body=0)
    return o, g


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


# (nx, ny): several 64-wide tiles with ragged tails in x (nx/2 = 100) and y
@pytest.mark.parametrize("nx,ny,stretched", [(128, 96, False), (200, 150, True), (16, 8, False)])
def test_sor_fixed_iterations_match_oracle(torch, nx, ny, stretched):
    o, g = _pair(torch, nx, ny, stretched)
    rng = np.random.default_rng(nx + ny)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    xo, so, rc = o.poisson_solve(b, x0=x0, omega=1.8, fixed=37, check=10)
    xd = _dev(torch, x0)
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.RBSOR, omega=1.8, fixed_iters=37, check_every=10)
    xg = xd.cpu().numpy()
    print(f"case nx={nx} ny={ny} rel={rel_l2(xg, xo):.3e}", flush=True)
    assert sg["iters"] == so["iters"] == 37
    assert rel_l2(xg, xo) <= 1e-12
    assert np.max(np.abs(xg - xo)) <= 1e-12 * np.max(np.abs(xo))
    assert abs(sg["rel"] - so["rel"]) <= 1e-9 * so["rel"]


@pytest.mark.parametrize("stretched", [False, True])
def test_sor_to_tolerance_same_iterations(torch, stretched):
    nx, ny = 128, 96
    o, g = _pair(torch, nx, ny, stretched)
    xf, yf = _grid(nx, ny, stretched)
    xc, yc = 0.5 * (xf[1:] + xf[:-1]), 0.5 * (yf[1:] + yf[:-1])
    X, Y = np.meshgrid(xc, yc)
    b = np.cos(np.pi * X / 32.0) * np.cos(np.pi * Y / 12.0) + 0.3 * np.sin(3 * X) * np.cos(2 * Y)
    xo, so, rc = o.poisson_solve(b, omega=1.8, tol=1e-8, check=10)
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.RBSOR, omega=1.8, tol=1e-8, check_every=10)
    xg = xd.cpu().numpy()
    print(f"iters gpu {sg['iters']} oracle {so['iters']} rel {rel_l2(xg, xo):.3e}", flush=True)
    assert rc == O.OK and sg["rc"] == ibm.OK
    assert sg["iters"] == so["iters"]
    assert sg["rel"] <= 1e-8
    assert rel_l2(xg, xo) <= TOL


@pytest.mark.parametrize("nx,ny,stretched", [(128, 96, False), (200, 150, True)])
def test_pcg_fixed_iterations_match_oracle(torch, nx, ny, stretched):
    o, g = _pair(torch, nx, ny, stretched)
    rng = np.random.default_rng(7)
    b = rng.standard_normal((ny, nx))
    xo, so, rc = o.poisson_solve(b, method=O.PCG, fixed=60)
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.PCG, fixed_iters=60)
    xg = xd.cpu().numpy()
    print(f"pcg rel {rel_l2(xg, xo):.3e}", flush=True)
    assert sg["iters"] == so["iters"] == 60
    assert rel_l2(xg, xo) <= TOL


def test_pcg_to_tolerance_agrees_with_oracle(torch):
    nx, ny = 96, 64
    o, g = _pair(torch, nx, ny, True)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((ny, nx))
    xo, so, rc = o.poisson_solve(b, method=O.PCG, tol=1e-12, max_iter=20000)
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.PCG, tol=1e-12, max_iter=20000)
    xg = xd.cpu().numpy()
    print(f"pcg iters gpu {sg['iters']} oracle {so['iters']} rel {rel_l2(xg, xo):.3e}", flush=True)
    assert rc == O.OK and sg["rc"] == ibm.OK
    assert abs(sg["iters"] - so["iters"]) <= 3
    assert sg["rel"] <= 1e-12
    assert rel_l2(xg, xo) <= TOL
    # the GPU solution's true residual measured by the oracle's own operator
    V = np.outer(np.diff(o.yf), np.diff(o.xf))
    r = V * b - o.apply_A(xg)
    assert np.linalg.norm(r) <= 1.01e-12 * np.linalg.norm(V * b)


@pytest.mark.parametrize("method", [ibm.RBSOR, ibm.PCG])
def test_zero_rhs_gives_zero(torch, method):
    nx, ny = 64, 48
    _, g = _pair(torch, nx, ny)
    xd = torch.ones((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(torch.zeros_like(xd), xd, method=method)
    assert sg["iters"] == 0 and sg["rc"] == ibm.OK
    assert float(xd.abs().max()) == 0.0


def test_iteration_limit_is_soft(torch):
    nx, ny = 64, 48
    _, g = _pair(torch, nx, ny)
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    b = torch.ones_like(xd)
    sg = g.poisson_solve(b, xd, method=ibm.RBSOR, tol=1e-14, max_iter=25, check_every=10)
    assert sg["rc"] == ibm.NOT_CONVERGED and sg["iters"] == 25


def test_nan_rhs_reports_nan(torch):
    nx, ny = 64, 48
    _, g = _pair(torch, nx, ny)
    b = torch.ones((ny, nx), dtype=torch.float64, device="cuda")
    b[5, 7] = float("nan")
    xd = torch.zeros_like(b)
    sg = g.poisson_solve(b, xd, method=ibm.RBSOR)
    assert sg["rc"] == ibm.ERR_NAN


def test_full_size_grid_fixed_iterations(torch):
    """The 1024x768 stretched grid of the plunging workload, in the launch
    configuration the benchmark times: 40 SOR iterations and 20 PCG
    iterations against the oracle."""
    c = W.plunging_1024x768()
    nx, ny = c["nx"], c["ny"]
    o, g = _pair(torch, nx, ny, faces=(c["xf"], c["yf"]))
    rng = np.random.default_rng(11)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    xo, so, _ = o.poisson_solve(b, x0=x0, omega=1.8, fixed=40, check=10)
    xd = _dev(torch, x0)
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.RBSOR, omega=1.8, fixed_iters=40, check_every=10)
    xg = xd.cpu().numpy()
    print(f"full SOR rel {rel_l2(xg, xo):.3e}", flush=True)
    assert rel_l2(xg, xo) <= 1e-12
    xo, so, _ = o.poisson_solve(b, method=O.PCG, fixed=20)
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    g.poisson_solve(_dev(torch, b), xd, method=ibm.PCG, fixed_iters=20)
    xg = xd.cpu().numpy()
    print(f"full PCG rel {rel_l2(xg, xo):.3e}", flush=True)
    assert rel_l2(xg, xo) <= TOL


@pytest.mark.parametrize("nx,ny,sweeps,tile", [
    (128, 96, 5, (64, 40)),      # 2x3 tiles
    (200, 150, 10, (76, 44)),    # the default shape; ragged tiles in x and y, stretched
    (200, 150, 5, (104, 32)),    # ragged tiles in x and y, stretched
    (200, 150, 1, (32, 24)),
    (200, 150, 3, (16, 8)),      # many small tiles
    (256, 192, 2, (16, 12)),     # 256 tiles in the XCD-banded order
    (64, 48, 8, (64, 48)),       # one tile, deep halo clipped by the domain
    (64, 48, 12, (64, 48)),      # the deepest halo (S = 12)
    (1024, 768, 10, (76, 44)),   # the plunging-workload grid in the default shape, 252 tiles
    (1024, 768, 5, (104, 32)),   # the same grid, 240 tiles of 5 iterations
    (1024, 768, 5, (104, 28)),   # 280 tiles: more blocks than compute units
    (512, 384, 2, (16, 12)),     # 1024 small tiles, several blocks per compute unit in turn
])
def test_blocked_sweep_is_bitwise_the_per_colour_sweep(torch, nx, ny, sweeps, tile):
    """The temporally blocked launch performs the same cell updates with the
    same neighbour values as one launch per colour: identical iterates, for
    fixed iteration counts that are not multiples of the sweep count, and the
    same stop decision in tolerance mode.  Grids with more tiles than compute
    units check that no tile reads a halo another tile of the same launch has
    already rewritten."""
    xf, yf = _grid(nx, ny, stretched=(nx != 128))
    g = ibm.Solver(nx, ny, xf, yf, body=0)
    rng = np.random.default_rng(nx * 7 + sweeps)
    b = _dev(torch, rng.standard_normal((ny, nx)))
    x0 = rng.standard_normal((ny, nx))
    out = {}
    kernels = (ibm.SOR_PER_COLOUR, ibm.SOR_TEMPORAL, ibm.SOR_TEMPORAL_LDS)
    for kern in kernels:
        assert g.set_option(ibm.OPT_SOR_KERNEL, kern) == ibm.OK
        assert g.set_option(ibm.OPT_TB_SWEEPS, sweeps) == ibm.OK
        assert g.set_option(ibm.OPT_TB_TILE_X, tile[0]) == ibm.OK
        assert g.set_option(ibm.OPT_TB_TILE_Y, tile[1]) == ibm.OK
        xd = _dev(torch, x0)
        st = g.poisson_solve(b, xd, method=ibm.RBSOR, omega=1.8, fixed_iters=23, check_every=10)
        xt = _dev(torch, np.zeros((ny, nx)))
        st2 = g.poisson_solve(b, xt, method=ibm.RBSOR, omega=1.7, tol=1e-3, check_every=10)
        out[kern] = (xd.cpu().numpy(), st, xt.cpu().numpy(), st2)
    a = out[ibm.SOR_PER_COLOUR]
    for kern in kernels[1:]:
        bb_ = out[kern]
        print(f"kernel {kern} nx={nx} S={sweeps} tile={tile} maxdiff={np.max(np.abs(a[0] - bb_[0])):.3e} "
              f"iters {a[3]['iters']} {bb_[3]['iters']}", flush=True)
        assert np.array_equal(a[0], bb_[0])
        assert a[1]["iters"] == bb_[1]["iters"] == 23
        assert abs(a[1]["rel"] - bb_[1]["rel"]) <= 1e-12 * a[1]["rel"]
        assert a[3]["iters"] == bb_[3]["iters"]
        assert np.array_equal(a[2], bb_[2])


def test_blocked_sweep_rejects_shapes_that_do_not_fit(torch):
    xf, yf = _grid(256, 192, False)
    g = ibm.Solver(256, 192, xf, yf, body=0)
    assert g.set_option(ibm.OPT_TB_TILE_X, 63) == ibm.ERR_INVALID      # odd width
    assert g.set_option(ibm.OPT_TB_SWEEPS, 13) == ibm.ERR_INVALID      # too deep
    assert g.set_option(ibm.OPT_TB_TILE_X, 100) == ibm.ERR_INVALID     # 100 + 2 x 22 > 128 at S = 10
    assert g.set_option(ibm.OPT_TB_TILE_X, 256) == ibm.ERR_INVALID     # halo tile > LDS
    assert g.set_option(99, 1) == ibm.ERR_INVALID
    assert g.set_option(ibm.OPT_TB_SWEEPS, 4) == ibm.OK


# --- one-reduction Jacobi-PCG (IBM_SOLVER_CG1) -------------------------------

@pytest.mark.parametrize("nx,ny,stretched", [(128, 96, False), (200, 150, True), (16, 8, False)])
def test_cg1_fixed_iterations_match_oracle(torch, nx, ny, stretched):
    """The GPU's one-reduction CG against the oracle's (the same recurrences;
    sums in another order), and against textbook PCG on the GPU."""
    o, g = _pair(torch, nx, ny, stretched)
    rng = np.random.default_rng(17)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    k = 60 if nx > 16 else 20
    xo, so, rc = o.poisson_solve(b, x0=x0, method=O.CG1, fixed=k)
    xd = _dev(torch, x0)
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.CG1, fixed_iters=k)
    xg = xd.cpu().numpy()
    xp = _dev(torch, x0)
    g.poisson_solve(_dev(torch, b), xp, method=ibm.PCG, fixed_iters=k)
    print(f"cg1 rel {rel_l2(xg, xo):.3e} vs gpu pcg {rel_l2(xg, xp.cpu().numpy()):.3e}", flush=True)
    assert sg["iters"] == so["iters"] == k
    assert rel_l2(xg, xo) <= TOL
    assert rel_l2(xg, xp.cpu().numpy()) <= TOL
    assert abs(sg["rel"] - so["rel"]) <= 1e-8 * so["rel"]


def test_cg1_to_tolerance_agrees_with_oracle(torch):
    nx, ny = 96, 64
    o, g = _pair(torch, nx, ny, True)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((ny, nx))
    xo, so, rc = o.poisson_solve(b, method=O.CG1, tol=1e-12, max_iter=20000)
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.CG1, tol=1e-12, max_iter=20000)
    xg = xd.cpu().numpy()
    print(f"cg1 iters gpu {sg['iters']} oracle {so['iters']} rel {rel_l2(xg, xo):.3e}", flush=True)
    assert rc == O.OK and sg["rc"] == ibm.OK
    assert abs(sg["iters"] - so["iters"]) <= 3
    assert sg["rel"] <= 1e-12
    assert rel_l2(xg, xo) <= TOL
    V = np.outer(np.diff(o.yf), np.diff(o.xf))
    r = V * b - o.apply_A(xg)
    assert np.linalg.norm(r) <= 1.01e-12 * np.linalg.norm(V * b)


def test_cg1_zero_rhs_limit_and_nan(torch):
    nx, ny = 64, 48
    _, g = _pair(torch, nx, ny)
    xd = torch.ones((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(torch.zeros_like(xd), xd, method=ibm.CG1)
    assert sg["iters"] == 0 and sg["rc"] == ibm.OK and float(xd.abs().max()) == 0.0
    b = torch.ones_like(xd)
    xd.zero_()
    sg = g.poisson_solve(b, xd, method=ibm.CG1, tol=1e-15, max_iter=25)
    assert sg["rc"] == ibm.NOT_CONVERGED and sg["iters"] == 25
    b[5, 7] = float("nan")
    xd.zero_()
    sg = g.poisson_solve(b, xd, method=ibm.CG1)
    assert sg["rc"] == ibm.ERR_NAN


def test_cg1_full_size_grid_to_tolerance(torch):
    """The 1024x768 stretched grid in the benchmark's launch configuration, to
    1e-10: the result meets the stop test by the oracle's operator and lies
    within the solver tolerance of the oracle's textbook PCG."""
    c = W.plunging_1024x768()
    nx, ny = c["nx"], c["ny"]
    o, g = _pair(torch, nx, ny, faces=(c["xf"], c["yf"]))
    X, Y = np.meshgrid(0.5 * (c["xf"][1:] + c["xf"][:-1]), 0.5 * (c["yf"][1:] + c["yf"][:-1]))
    b = np.exp(-((X - 4.0) ** 2 + (Y - 6.0) ** 2)) - np.exp(-((X - 9.0) ** 2 + (Y - 4.0) ** 2))
    xd = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    sg = g.poisson_solve(_dev(torch, b), xd, method=ibm.CG1, tol=1e-10, max_iter=200000)
    xg = xd.cpu().numpy()
    V = np.outer(np.diff(o.yf), np.diff(o.xf))
    r = V * b - o.apply_A(xg)
    print(f"cg1 1024x768 iters {sg['iters']} rel {np.linalg.norm(r) / np.linalg.norm(V * b):.3e}", flush=True)
    assert sg["rc"] == ibm.OK
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(V * b)
    xo, so, _ = o.poisson_solve(b, method=O.PCG, tol=1e-10, max_iter=200000)
    assert abs(sg["iters"] - so["iters"]) <= max(10, so["iters"] // 100)
    assert rel_l2(xg, xo) <= 1e-6  # both within the tolerance of the exact solution (cond ~ 1e4)
