"""Explicit forward-Euler finite-difference solver, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY.

Sec. 2.4.1 provides forward Euler as the base explicit method; Sec. 2.2.2
lists the second-order central Laplacian stencils: 5 and 9 points in 2D,
7 and 19 (among others) in 3D.  The 5/7-point stencils are the axis-wise
central differences; the 9- and 19-point ones are the standard
second-order isotropic stencils (their leading error term depends on |k|
only), weights over 6 h^2: 2D 4 per edge neighbour, 1 per corner, -20 in
the centre; 3D 2 per face neighbour, 1 per edge neighbour, -24 in the
centre (equal spacing on every axis).  Also built: the fourth-order
axis-wise stencil of the fourth-order family (9 points in 2D, 13 in 3D:
per axis (-f[-2] + 16 f[-1] - 30 f + 16 f[+1] - f[+2]) / (12 h^2)) and a
27-point second-order isotropic 3D stencil, weights over 30 h^2: 14 per
face neighbour, 3 per edge neighbour, 1 per corner, -128 in the centre
(zero sum, second moment 2 per axis, and an h^2 error term that depends
on |k| only).  Higher powers of the Laplacian are
built by composing the stencil, and periodic boundaries wrap the grid.
This is a discretisation independent of the spectral scheme (real space,
no transforms, no exponentials), so the two agree only if the operator
split, the signs and the coefficients of the spectral side are right.
"""
from __future__ import annotations

import numpy as np


def laplacian(f, dx, stencil=0):
    """Central finite-difference Laplacian with periodic wrap.

    ``f`` is shaped ([z,] y, x); ``dx`` is (dx, dy[, dz]).  stencil 0, 5
    or 7: the second-order axis-wise stencil (5 points in 2D, 7 in 3D);
    9 (2D), 19 or 27 (3D): second-order isotropic stencils, which need
    equal spacings; 4: the fourth-order axis-wise stencil.
    """
    f = np.asarray(f, dtype=np.float64)
    d = f.ndim
    if stencil in (0, 5, 7):
        assert stencil in (0, 5 if d == 2 else 7)
        out = np.zeros_like(f)
        dxs = tuple(reversed(tuple(dx)))
        for ax, h in enumerate(dxs):
            out += (np.roll(f, 1, axis=ax) - 2.0 * f + np.roll(f, -1, axis=ax)) / (h * h)
        return out
    if stencil == 4:
        out = np.zeros_like(f)
        dxs = tuple(reversed(tuple(dx)))
        for ax, h in enumerate(dxs):
            out += (-np.roll(f, 2, axis=ax) + 16.0 * np.roll(f, 1, axis=ax) - 30.0 * f
                    + 16.0 * np.roll(f, -1, axis=ax) - np.roll(f, -2, axis=ax)) / (12.0 * h * h)
        return out
    h = float(dx[0])
    assert all(abs(float(v) - h) <= 1e-12 * h for v in dx), "isotropic stencils need equal spacing"
    if stencil == 9:
        assert d == 2
        edge = sum(np.roll(f, s, axis=a) for a in (0, 1) for s in (1, -1))
        corner = sum(np.roll(np.roll(f, sy, axis=0), sx, axis=1) for sy in (1, -1) for sx in (1, -1))
        return (4.0 * edge + corner - 20.0 * f) / (6.0 * h * h)
    if stencil == 19:
        assert d == 3
        face = sum(np.roll(f, s, axis=a) for a in (0, 1, 2) for s in (1, -1))
        edge = 0.0
        for a, b in ((0, 1), (0, 2), (1, 2)):
            for sa in (1, -1):
                for sb in (1, -1):
                    edge = edge + np.roll(np.roll(f, sa, axis=a), sb, axis=b)
        return (2.0 * face + edge - 24.0 * f) / (6.0 * h * h)
    if stencil == 27:
        assert d == 3
        face = sum(np.roll(f, s, axis=a) for a in (0, 1, 2) for s in (1, -1))
        edge = 0.0
        for a, b in ((0, 1), (0, 2), (1, 2)):
            for sa in (1, -1):
                for sb in (1, -1):
                    edge = edge + np.roll(np.roll(f, sa, axis=a), sb, axis=b)
        corner = 0.0
        for sz in (1, -1):
            for sy in (1, -1):
                for sx in (1, -1):
                    corner = corner + np.roll(np.roll(np.roll(f, sz, axis=0), sy, axis=1), sx, axis=2)
        return (14.0 * face + 3.0 * edge + corner - 128.0 * f) / (30.0 * h * h)
    raise ValueError("unknown stencil %r" % (stencil,))


def rhs(model, coef, q, dx, stencil=0):
    """Right-hand sides of the equations of motion in real space."""
    lap = lambda f: laplacian(f, dx, stencil)
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


def euler_n(fields, model, coef, dt, dx, nsteps, stencil=0):
    """``nsteps`` forward-Euler steps q <- q + dt * rhs(q)."""
    q = [np.array(f, dtype=np.float64, copy=True) for f in fields]
    for _ in range(int(nsteps)):
        r = rhs(model, coef, q, dx, stencil)
        q = [a + dt * b for a, b in zip(q, r)]
    return q
