"""Explicit forward-Euler finite-difference solver, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY.

Sec. 2.4.1 provides forward Euler as the base explicit method; Sec. 2.2.2
names the second-order central stencils (the 5-point Laplacian in 2D, the
7-point one in 3D).  Higher powers of the Laplacian are built here by
composing that stencil, and periodic boundaries wrap the grid.  This is a
discretisation independent of the spectral scheme (real space, no
transforms, no exponentials), so the two agree only if the operator
split, the signs and the coefficients of the spectral side are right.
"""
from __future__ import annotations

import numpy as np


def laplacian(f, dx):
    """Second-order central Laplacian with periodic wrap.

    ``f`` is shaped (..., y, x); ``dx`` is (dx, dy[, dz]).  In 2D this is
    the 5-point stencil, in 3D the 7-point stencil.
    """
    out = np.zeros_like(f)
    dxs = tuple(reversed(tuple(dx)))
    for ax, h in enumerate(dxs):
        out += (np.roll(f, 1, axis=ax) - 2.0 * f + np.roll(f, -1, axis=ax)) / (h * h)
    return out


def rhs(model, coef, q, dx):
    """Right-hand sides of the equations of motion in real space."""
    lap = lambda f: laplacian(f, dx)
    c = [float(v) for v in coef]
    if model == "allen_cahn":
        M, kap, c1, c2 = c
        p = q[0]
        return [M * (kap * lap(p) + c1 * p - c2 * p ** 3)]
    if model == "cahn_hilliard":
        M, kap, c1, c2 = c
        p = q[0]
        return [M * lap(c2 * p ** 3 - c1 * p - kap * lap(p))]
    if model == "pfc":
        r, q0, g2, g3 = c
        p = q[0]
        # (r + (q0^2 + lap)^2) p = (r + q0^4) p + 2 q0^2 lap p + lap lap p
        lp = lap(p)
        inner = (r + q0 ** 4) * p + 2.0 * q0 ** 2 * lp + lap(lp) + g2 * p ** 2 + g3 * p ** 3
        return [lap(inner)]
    if model == "gray_scott":
        du, dv, F, kk = c
        u, v = q
        uvv = u * v * v
        return [du * lap(u) - uvv + F * (1.0 - u),
                dv * lap(v) + uvv - (F + kk) * v]
    if model == "model_c":
        c1, c2, c3, c4, c5 = c
        p, m = q
        return [lap(p) + c1 * p - c2 * p ** 3 + 2.0 * c5 * p * m,
                -lap(lap(m)) - lap(c3 * m - c4 * m ** 3 + c5 * p ** 2)]
    raise ValueError("unknown model %r" % (model,))


def euler_n(fields, model, coef, dt, dx, nsteps):
    """``nsteps`` forward-Euler steps q <- q + dt * rhs(q)."""
    q = [np.array(f, dtype=np.float64, copy=True) for f in fields]
    for _ in range(int(nsteps)):
        r = rhs(model, coef, q, dx)
        q = [a + dt * b for a, b in zip(q, r)]
    return q
