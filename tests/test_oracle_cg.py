"""Pins of the oracle's one-reduction CG and its mixed-precision form against
facts fixed by mathematics.

The paper solves the pressure-correction equation (Sec. 2.2) with red-black
SOR; Jacobi-preconditioned CG is this build's second plain solver.  The
one-reduction form (Chronopoulos and Gear, 1989) carries s = M p by its own
recurrence so that both inner products of an iteration are taken together;
in exact arithmetic its iterates are those of textbook Jacobi-PCG.  The
mixed-precision form refines in double precision around an inner
single-precision CG on the correction equation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_17337_amd import workloads as W


def _grid(nx, ny, stretched=False, Lx=4.0, Ly=3.0):
    xf, yf = W.uniform_faces(nx, Lx), W.uniform_faces(ny, Ly)
    if stretched:
        s = xf / Lx
        xf = Lx * (s - 0.12 * np.sin(2 * np.pi * s) / (2 * np.pi))
        s = yf / Ly
        yf = Ly * (s - 0.10 * np.sin(2 * np.pi * s) / (2 * np.pi))
    return xf, yf


def _dense_M(o):
    """M = -A assembled column by column from the oracle's operator (itself
    pinned in test_oracle_poisson.py)."""
    n = o.nx * o.ny
    M = np.empty((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[:] = 0.0
        e[k] = 1.0
        M[:, k] = -o.apply_A(e).ravel()
    return M


@pytest.mark.parametrize("stretched", [False, True])
def test_one_reduction_iterates_equal_textbook_pcg(stretched):
    nx, ny = 40, 30
    xf, yf = _grid(nx, ny, stretched)
    o = O.Oracle(nx, ny, xf, yf, body=0)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    for k in (1, 2, 7, 25, 60):
        xa, sa, _ = o.poisson_solve(b, x0=x0, method=O.PCG, fixed=k)
        xb, sb, _ = o.poisson_solve(b, x0=x0, method=O.CG1, fixed=k)
        assert np.linalg.norm(xa - xb) <= 1e-11 * np.linalg.norm(xa), k
        assert abs(sa["rel"] - sb["rel"]) <= 1e-9 * sa["rel"]


def test_one_reduction_first_iterate_in_closed_form():
    """x1 = x0 + alpha0 u0, u0 = D^-1 r0, alpha0 = (r0, u0) / (u0, M u0),
    written out with the dense matrix."""
    nx, ny = 12, 10
    xf, yf = _grid(nx, ny, True)
    o = O.Oracle(nx, ny, xf, yf, body=0)
    M = _dense_M(o)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    vb = (np.outer(np.diff(yf), np.diff(xf)) * b).ravel()
    r0 = -vb - M @ x0.ravel()
    u0 = r0 / np.diag(M)
    x1 = x0.ravel() + (r0 @ u0) / (u0 @ (M @ u0)) * u0
    xg, _, _ = o.poisson_solve(b, x0=x0, method=O.CG1, fixed=1)
    assert np.allclose(xg.ravel(), x1, rtol=0, atol=1e-13 * np.abs(x1).max())


@pytest.mark.parametrize("method", [O.CG1, O.PCG_MP])
def test_cg_forms_match_dense_direct_solve(method):
    nx, ny = 16, 12
    xf, yf = _grid(nx, ny, True)
    o = O.Oracle(nx, ny, xf, yf, body=0)
    M = _dense_M(o)
    rng = np.random.default_rng(1)
    b = rng.standard_normal((ny, nx))
    vb = (np.outer(np.diff(yf), np.diff(xf)) * b).ravel()
    exact = np.linalg.solve(-M, vb)
    tol = 1e-12
    x, st, rc = o.poisson_solve(b, method=method, tol=tol, max_iter=20000, check=1000)
    assert rc == O.OK and st["rel"] <= tol
    cond = np.linalg.cond(M)
    assert np.linalg.norm(x.ravel() - exact) <= 2 * cond * tol * np.linalg.norm(exact)


def test_mixed_cg_meets_the_double_stop_test_and_single_alone_stalls():
    """The refined solve reaches a double-precision residual of 1e-12, which
    single-precision CG alone cannot: it stalls near float rounding times the
    condition number."""
    c = W.plunging_scaled(128, 96)
    o = O.Oracle(128, 96, c["xf"], c["yf"], body=0)
    rng = np.random.default_rng(2)
    b = rng.standard_normal((96, 128))
    x, st, rc = o.poisson_solve(b, method=O.PCG_MP, tol=1e-12, max_iter=200000, check=100000)
    assert rc == O.OK and st["rel"] <= 1e-12
    # the residual recomputed with the (pinned) operator
    vb = np.outer(np.diff(c["yf"]), np.diff(c["xf"])) * b
    r = vb - o.apply_A(x)
    assert np.linalg.norm(r) <= 1.0001e-12 * np.linalg.norm(vb)
    xs, ss, _ = o.poisson_pcg_f32(b, iters=st["iters"])
    assert ss["rel"] > 1e-7
    assert ss["rel"] > 1e4 * st["rel"]


def test_mixed_cg_rejects_periodic_mode_and_fixed_counts():
    xf, yf = W.uniform_faces(16, 2 * np.pi), W.uniform_faces(16, 2 * np.pi)
    o = O.Oracle(16, 16, xf, yf, bc=O.PERIODIC, body=0)
    _, _, rc = o.poisson_solve(np.ones((16, 16)), method=O.PCG_MP)
    assert rc == O.ERR_INVALID
    xf, yf = _grid(16, 12)
    o = O.Oracle(16, 12, xf, yf, body=0)
    _, _, rc = o.poisson_solve(np.ones((12, 16)), method=O.PCG_MP, fixed=5)
    assert rc == O.ERR_INVALID
