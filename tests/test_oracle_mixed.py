"""Pins of the oracle's mixed-precision SOR (single-precision sweeps on the
correction equation, double-precision residual, update and stop test) against
facts fixed by mathematics.

The method it speeds up is the paper's red-black SOR pressure solve (Sec. 2.2
and 3.1); the precision split is an extension of it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from test_oracle_poisson import _dense_A, _oracle


def _rhs(o, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((o.ny, o.nx))


@pytest.mark.parametrize("stretched", [False, True])
def test_mixed_solution_within_the_condition_bound_of_the_dense_solve(stretched):
    """A stop at relative residual tol bounds the relative error by cond(A) tol."""
    o, _, _ = _oracle(16, 12, stretched)
    b = _rhs(o, 3)
    A = _dense_A(o)
    x, st, rc = o.poisson_solve(b, method=O.SOR_MP, omega=1.8, tol=1e-9)
    assert rc == O.OK and st["rel"] <= 1e-9
    # V b from the operator's own scaling: A x* = V b with V the cell volumes
    dx = np.diff(o.xf)[None, :]
    dy = np.diff(o.yf)[:, None]
    vb = (b * dx * dy).ravel()
    xs = np.linalg.solve(A, vb)
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(x.ravel() - xs) / np.linalg.norm(xs)
    assert err <= kappa * 1e-9
    # and the residual reported is the true double-precision residual
    r = vb - A @ x.ravel()
    assert np.linalg.norm(r) <= 1.0000001e-9 * np.linalg.norm(vb)


@pytest.mark.parametrize("stretched,check", [(False, 10), (True, 10), (True, 100)])
def test_refinement_reproduces_double_sor_iteration_counts(stretched, check):
    """SOR is stationary: restarting it on the correction equation every check
    interval gives the double-precision iterates in exact arithmetic, so the
    mixed solve stops within one check interval of plain SOR (with the same
    interval: the same iteration count up to rounding at the threshold)."""
    o, _, _ = _oracle(48, 36, stretched)
    b = _rhs(o, 5)
    _, s64, rc64 = o.poisson_solve(b, method=O.SOR, omega=1.8, tol=1e-8, check=10)
    _, s64k, _ = o.poisson_solve(b, method=O.SOR, omega=1.8, tol=1e-8, check=check)
    x, smp, rcmp = o.poisson_solve(b, method=O.SOR_MP, omega=1.8, tol=1e-8, check=check)
    assert rc64 == O.OK and rcmp == O.OK
    assert abs(smp["iters"] - s64["iters"]) <= check, (smp["iters"], s64["iters"])
    assert abs(smp["iters"] - s64k["iters"]) <= check and smp["iters"] % check == 0


@pytest.mark.parametrize("check", [10, 100])
def test_first_interval_matches_double_sor_to_single_precision(check):
    """One interval from the same start: the mixed iterate equals the double
    SOR iterate up to single-precision rounding of the correction (rounding
    over K contractive float sweeps grows at most linearly in K)."""
    o, _, _ = _oracle(40, 30, True)
    b = _rhs(o, 7)
    rng = np.random.default_rng(8)
    x0 = rng.standard_normal((o.ny, o.nx))
    x64, _, _ = o.poisson_solve(b, x0=x0, method=O.SOR, omega=1.8, fixed=check, check=check)
    xmp, _, _ = o.poisson_solve(b, x0=x0, method=O.SOR_MP, omega=1.8, fixed=check, check=check)
    corr = np.linalg.norm(x64 - x0)
    assert np.linalg.norm(xmp - x64) <= max(1e-5, 10 * check * 2.0 ** -24) * corr
    assert np.linalg.norm(xmp - x64) > 0.0   # the sweeps are not done in double


def test_single_precision_alone_stalls_where_refinement_does_not():
    """Without refinement the float sweep stops improving near its rounding
    floor; with refinement the same number of sweeps reaches double-precision
    tolerances."""
    o, _, _ = _oracle(32, 24, False)
    b = _rhs(o, 11)
    _, s64, _ = o.poisson_solve(b, method=O.SOR, omega=1.8, tol=1e-12)
    n = s64["iters"]
    _, s32, rc32 = o.poisson_sor_f32(b, omega=1.8, iters=n)
    _, smp, rcmp = o.poisson_solve(b, method=O.SOR_MP, omega=1.8, fixed=n)
    assert rc32 == O.OK and rcmp == O.OK
    assert smp["rel"] <= 2e-12
    assert s32["rel"] > 1e-9           # float rounding floor, far above the double result


def test_mixed_rejects_periodic_mode():
    xf = np.linspace(0.0, 2 * np.pi, 9)
    o = O.Oracle(8, 8, xf, xf, bc=O.PERIODIC, body=0)
    _, _, rc = o.poisson_solve(np.zeros((8, 8)), method=O.SOR_MP)
    assert rc == O.ERR_INVALID
