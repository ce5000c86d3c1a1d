"""Explicit forward-Euler finite-difference solver, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY.

Sec. 2.4.1 provides forward Euler as the base explicit method; Sec. 2.2.2
lists the Laplacian stencils by family: second order, 5 and 9 points in
2D, 7, 15, 19, 21 and 27 in 3D; fourth order (2D only), 9, 17 and 21
points.  It names the point counts and no weights, so the weights here are
derived from the moment conditions that define each family on its point
set (equal spacing h on every axis for all but the axis-wise stencils):
zero sum, a second moment of 2 along each axis, and

  second order: the h^2 error term depends on |k| only (isotropy of the
  fourth moments: sum w x^4 = 3 sum w x^2 y^2), so that it is
  h^2 |k|^4 / 12 for every isotropic stencil of the family;
  fourth order: the fourth moments vanish, and the h^4 error term depends
  on |k| only (sum w x^4 y^2 = sum w x^6 / 5), so that it is
  h^4 |k|^6 / 90.

Second order:
  5 / 7 points   axis-wise, per axis (f[-1] - 2 f + f[+1]) / h_a^2;
  9 points (2D)  (4 edges + corners - 20 f) / (6 h^2);
  15 points (3D) (8 faces + corners - 56 f) / (12 h^2);
  19 points (3D) (2 faces + edges - 24 f) / (6 h^2);
  21 points (3D) (4 edges - corners - 40 f) / (12 h^2);
  27 points (3D) (14 faces + 3 edges + corners - 128 f) / (30 h^2)
(faces: the 6 neighbours at distance 1, edges: the 12 at sqrt 2,
corners: the 8 at sqrt 3; 2D edges and corners the 4 at 1 and sqrt 2).
Fourth order:
  9 points (13 in 3D)  axis-wise, per axis
                 (-f[-2] + 16 f[-1] - 30 f + 16 f[+1] - f[+2]) / (12 h_a^2);
  17 points (2D) (128 A1 + 16 D1 - 8 A2 - D2 - 540 f) / (120 h^2);
  21 points (2D) (52 A1 + 16 D1 - A2 - 2 K - 252 f) / (60 h^2)
(A1, A2: the 4 axis neighbours at distance 1 and 2; D1, D2: the 4
diagonal ones at (+-1, +-1) and (+-2, +-2); K: the 8 at (+-1, +-2) and
(+-2, +-1)).  With those point sets, the conditions fix every weight.
Higher powers of the Laplacian are built by composing the stencil, and
periodic boundaries wrap the grid.
This is a discretisation independent of the spectral scheme (real space,
no transforms, no exponentials), so the two agree only if the operator
split, the signs and the coefficients of the spectral side are right.
"""
from __future__ import annotations

import itertools

import numpy as np


def laplacian(f, dx, stencil=0):
    """Central finite-difference Laplacian with periodic wrap.

    ``f`` is shaped ([z,] y, x); ``dx`` is (dx, dy[, dz]).  stencil 0, 5
    or 7: the second-order axis-wise stencil (5 points in 2D, 7 in 3D);
    9 (2D), 15, 19, 21 or 27 (3D): second-order isotropic stencils; 4: the
    fourth-order axis-wise stencil; 17 or 21 (2D): fourth-order isotropic
    stencils.  The isotropic stencils need equal spacings.
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

    def shift(*offs):
        """f at the offset (dx, dy[, dz]) from each cell."""
        g = f
        for ax_from_x, o in enumerate(offs):
            if o:
                g = np.roll(g, -o, axis=d - 1 - ax_from_x)
        return g

    def ring(*offs):
        """Sum of f over every sign and axis permutation of the offset."""
        pts = set()
        for perm in itertools.permutations(offs):
            for signs in itertools.product((1, -1), repeat=d):
                pts.add(tuple(s * o for s, o in zip(signs, perm)))
        return sum(shift(*p) for p in sorted(pts))

    if stencil == 9 and d == 2:
        return (4.0 * ring(1, 0) + ring(1, 1) - 20.0 * f) / (6.0 * h * h)
    if stencil == 17 and d == 2:
        return (128.0 * ring(1, 0) + 16.0 * ring(1, 1) - 8.0 * ring(2, 0) - ring(2, 2)
                - 540.0 * f) / (120.0 * h * h)
    if stencil == 21 and d == 2:
        return (52.0 * ring(1, 0) + 16.0 * ring(1, 1) - ring(2, 0) - 2.0 * ring(1, 2)
                - 252.0 * f) / (60.0 * h * h)
    if stencil == 15 and d == 3:
        return (8.0 * ring(1, 0, 0) + ring(1, 1, 1) - 56.0 * f) / (12.0 * h * h)
    if stencil == 19 and d == 3:
        return (2.0 * ring(1, 0, 0) + ring(1, 1, 0) - 24.0 * f) / (6.0 * h * h)
    if stencil == 21 and d == 3:
        return (4.0 * ring(1, 1, 0) - ring(1, 1, 1) - 40.0 * f) / (12.0 * h * h)
    if stencil == 27 and d == 3:
        return (14.0 * ring(1, 0, 0) + 3.0 * ring(1, 1, 0) + ring(1, 1, 1) - 128.0 * f) / (30.0 * h * h)
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
