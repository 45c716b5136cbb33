"""The divergence the projection leaves (Sec. 2.2, the projection step of the
fractional-step method): since D G = A / V, every cell without a mass source
has V D(u^{n+1}) = dt (V b - A phi) after a time step, whatever tolerance the
pressure solve reached.  A property of a solver's state that holds at any
size; its bar is the rounding of the few face fluxes dy u, dx v each side sums
(V b is V D(u^) of the predicted velocity u^ = u^{n+1} + dt G phi)."""
import numpy as np


def divergence_identity(u, v, vb, phi, msrc, xf, yf, dt, apply_A):
    """u (ny, nx+1), v (ny+1, nx), V b, phi, the mass-source flags (ny, nx);
    apply_A: the volume-scaled operator.  Returns the worst mismatch over
    the cells without a mass source (err), the rounding bar, the largest
    dt r there (scale), the relative residual ||V b - A phi|| / ||V b|| (rel)
    and the number of cells checked."""
    xf, yf = np.asarray(xf), np.asarray(yf)
    dx, dy = np.diff(xf), np.diff(yf)
    vol = dy[:, None] * dx[None, :]
    r = vb - apply_A(phi)
    div = (u[:, 1:] - u[:, :-1]) / dx + (v[1:, :] - v[:-1, :]) / dy[:, None]
    free = msrc == 0
    flux = dy[:, None] * (np.abs(u[:, 1:]) + np.abs(u[:, :-1])) + dx * (np.abs(v[1:, :]) + np.abs(v[:-1, :]))
    return {"err": float(np.max(np.abs(vol * div - dt * r)[free])),
            "bar": float(64 * np.finfo(float).eps * np.max(flux)),
            "scale": float(np.max(np.abs(dt * r[free]))),
            "rel": float(np.linalg.norm(r) / np.linalg.norm(vb)),
            "cells": int(free.sum())}
