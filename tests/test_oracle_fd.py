"""Pins of the finite-difference Laplacian stencils of the forward-Euler
oracle (Sec. 2.2.2): the Fourier symbol of each stencil on sampled plane
waves, second-order convergence on a smooth field, and the isotropy of the
leading error term that distinguishes the 9- and 19-point stencils from
the axis-wise 5- and 7-point ones."""
import numpy as np
import pytest

from oracle import fd_euler as fd


def plane(shape, m, phase=0.3):
    """cos(2 pi m . r / N + phase) on a grid of unit spacing (numpy order)."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    arg = sum(2 * np.pi * mi * g / n for mi, g, n in zip(m, grids, shape))
    return np.cos(arg + phase)


def symbol(stencil, theta):
    """Eigenvalue of the stencil (unit spacing) for the mode with phases
    theta_a = k_a h: the stencil's weights summed against cos(theta . offset)."""
    c = [np.cos(t) for t in theta]
    if stencil in (5, 7):
        return sum(2 * ci - 2 for ci in c)
    if stencil == 9:
        cx, cy = c
        return (4 * (2 * cx + 2 * cy) + 4 * cx * cy - 20) / 6.0
    if stencil == 19:
        pairs = c[0] * c[1] + c[0] * c[2] + c[1] * c[2]
        return (2 * 2 * sum(c) + 4 * pairs - 24) / 6.0
    if stencil == 27:
        pairs = c[0] * c[1] + c[0] * c[2] + c[1] * c[2]
        return (14 * 2 * sum(c) + 3 * 4 * pairs + 8 * c[0] * c[1] * c[2] - 128) / 30.0
    if stencil == 4:
        return sum((-2 * np.cos(2 * t) + 32 * np.cos(t) - 30) / 12.0 for t in theta)
    raise ValueError(stencil)


@pytest.mark.parametrize("stencil,shape,m", [
    (5, (16, 32), (3, 5)), (9, (16, 32), (3, 5)), (9, (32, 32), (7, 7)),
    (7, (8, 16, 32), (1, 3, 5)), (19, (8, 16, 32), (1, 3, 5)), (19, (16, 16, 16), (4, 4, 4)),
    (27, (8, 16, 32), (1, 3, 5)), (27, (16, 16, 16), (4, 4, 4)), (4, (16, 32), (3, 5)), (4, (8, 16, 32), (1, 3, 5)),
])
def test_stencil_symbol_on_plane_waves(stencil, shape, m):
    f = plane(shape, m)
    theta = [2 * np.pi * mi / n for mi, n in zip(m, shape)]
    got = fd.laplacian(f, (1.0,) * len(shape), stencil)
    np.testing.assert_allclose(got, symbol(stencil, theta) * f, rtol=0, atol=1e-12)


@pytest.mark.parametrize("stencil,d,order", [(5, 2, 2), (9, 2, 2), (7, 3, 2), (19, 3, 2), (27, 3, 2), (4, 2, 4),
                                             (4, 3, 4)])
def test_convergence_order(stencil, d, order):
    errs = []
    for n in (16, 32):
        L = 2 * np.pi
        h = L / n
        x = np.arange(n) * h
        if d == 2:
            Y, X = np.meshgrid(x, x, indexing="ij")
            f = np.sin(X) * np.cos(2 * Y)
            exact = -(1 + 4) * f
        else:
            Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
            f = np.sin(X) * np.cos(2 * Y) * np.sin(Z)
            exact = -(1 + 4 + 1) * f
        got = fd.laplacian(f, (h,) * d, stencil)
        errs.append(np.max(np.abs(got - exact)))
    ratio = errs[0] / errs[1]
    want = 2.0 ** order
    assert 0.95 * want < ratio < 1.05 * want, (stencil, errs)


def test_isotropy_of_the_leading_error():
    """Modes of equal |m| at different angles: the error of the 9- and
    19-point symbols (lambda + |k|^2, order h^2 |k|^4 / 12) is the same for
    all of them; the axis-wise stencils' error (h^2 sum k_a^4 / 12) is not."""
    n = 512
    def err(stencil, m, d):
        shape = (n,) * d
        f = plane(shape, m, phase=0.0)
        k2 = sum((2 * np.pi * mi / n) ** 2 for mi in m)
        idx = (0,) * d
        lam = fd.laplacian(f, (1.0,) * d, stencil)[idx] / f[idx]
        return lam + k2
    a, b = err(9, (7, 1), 2), err(9, (5, 5), 2)
    assert abs(a / b - 1) < 0.02
    a5, b5 = err(5, (7, 1), 2), err(5, (5, 5), 2)
    assert abs(a5 / b5 - 2402 / 1250) < 0.02
    n = 64
    e = [err(19, m, 3) for m in ((7, 1, 0), (5, 5, 0), (3, 4, 5))]
    assert max(e) / min(e) - 1 < 0.05
    e7 = [err(7, m, 3) for m in ((7, 1, 0), (5, 5, 0), (3, 4, 5))]
    assert max(e7) / min(e7) > 1.5
    e27 = [err(27, m, 3) for m in ((7, 1, 0), (5, 5, 0), (3, 4, 5))]
    assert max(e27) / min(e27) - 1 < 0.05


@pytest.mark.parametrize("model,d,stencil,ns", [("allen_cahn", 2, 9, (32, 64)), ("cahn_hilliard", 2, 9, (32, 64)),
                                                ("gray_scott", 2, 9, (32, 64)), ("allen_cahn", 3, 19, (32, 64)),
                                                ("pfc", 3, 19, (64, 128)), ("cahn_hilliard", 3, 27, (32, 64)),
                                                ("allen_cahn", 2, 4, (32, 64)), ("gray_scott", 3, 4, (32, 64))])
def test_isotropic_euler_converges_with_the_axiswise_one(model, d, stencil, ns):
    """One forward-Euler increment with either stencil family, on a smooth
    field at two resolutions: the two agree to second order in h (PFC's
    sixth-order operator needs the finer pair of grids to be asymptotic)."""
    coef = {"allen_cahn": (1.0, 1.0, 1.0, 1.0), "cahn_hilliard": (1.0, 1.0, 1.0, 1.0),
            "gray_scott": (0.16, 0.08, 0.035, 0.065), "pfc": (-0.25, 1.0, 0.3, 1.0)}[model]
    diffs = []
    for n in ns:
        L = 8 * np.pi
        h = L / n
        x = np.arange(n) * h
        grids = np.meshgrid(*([x] * d), indexing="ij")
        base = 0.3 * np.cos(grids[-1] / 4) * np.sin(2 * grids[0] / 4 + 0.2)
        fields = [base] if model != "gray_scott" else [1.0 - base, 0.25 + base]
        a = fd.rhs(model, coef, fields, (h,) * d, stencil)
        b = fd.rhs(model, coef, fields, (h,) * d, 0)
        diffs.append(max(np.max(np.abs(u - v)) for u, v in zip(a, b)))
    assert 3.5 < diffs[0] / diffs[1] < 4.5, diffs
