"""Pins of the finite-difference Laplacian stencils of the forward-Euler
oracle (Sec. 2.2.2): the Fourier symbol of each stencil on sampled plane
waves, the convergence order of each family on a smooth field, and the
leading error term of the isotropic stencils in closed form (h^2 |k|^4 / 12
for the second-order ones, h^4 |k|^6 / 90 for the fourth-order ones, at
every angle), which the axis-wise 5- and 7-point and fourth-order 9-point
stencils miss by direction-dependent factors."""
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
    if stencil == 15:
        return (8 * 2 * sum(c) + 8 * c[0] * c[1] * c[2] - 56) / 12.0
    if stencil == 21 and len(c) == 3:
        pairs = c[0] * c[1] + c[0] * c[2] + c[1] * c[2]
        return (4 * 4 * pairs - 8 * c[0] * c[1] * c[2] - 56 + 16) / 12.0
    c2 = [np.cos(2 * t) for t in theta]
    if stencil == 17:
        return (128 * 2 * sum(c) + 16 * 4 * c[0] * c[1] - 8 * 2 * sum(c2) - 4 * c2[0] * c2[1] - 540) / 120.0
    if stencil == 21:
        knight = 4 * (c[0] * c2[1] + c2[0] * c[1])
        return (52 * 2 * sum(c) + 16 * 4 * c[0] * c[1] - 2 * sum(c2) - 2 * knight - 252) / 60.0
    raise ValueError(stencil)


@pytest.mark.parametrize("stencil,shape,m", [
    (5, (16, 32), (3, 5)), (9, (16, 32), (3, 5)), (9, (32, 32), (7, 7)),
    (7, (8, 16, 32), (1, 3, 5)), (19, (8, 16, 32), (1, 3, 5)), (19, (16, 16, 16), (4, 4, 4)),
    (27, (8, 16, 32), (1, 3, 5)), (27, (16, 16, 16), (4, 4, 4)), (4, (16, 32), (3, 5)), (4, (8, 16, 32), (1, 3, 5)),
    (15, (8, 16, 32), (1, 3, 5)), (15, (16, 16, 16), (4, 4, 4)), (21, (8, 16, 32), (1, 3, 5)),
    (21, (16, 16, 16), (4, 4, 4)), (17, (16, 32), (3, 5)), (17, (32, 32), (7, 7)), (21, (16, 32), (3, 5)),
    (21, (32, 32), (7, 7)),
])
def test_stencil_symbol_on_plane_waves(stencil, shape, m):
    f = plane(shape, m)
    theta = [2 * np.pi * mi / n for mi, n in zip(m, shape)]
    got = fd.laplacian(f, (1.0,) * len(shape), stencil)
    np.testing.assert_allclose(got, symbol(stencil, theta) * f, rtol=0, atol=1e-12)


@pytest.mark.parametrize("stencil,d,order", [(5, 2, 2), (9, 2, 2), (7, 3, 2), (19, 3, 2), (27, 3, 2), (4, 2, 4),
                                             (4, 3, 4), (15, 3, 2), (21, 3, 2), (17, 2, 4), (21, 2, 4)])
def test_convergence_order(stencil, d, order):
    errs = []
    # the wide fourth-order stencils reach their asymptotic rate one grid later
    for n in ((32, 64) if stencil in (17, 21) and d == 2 else (16, 32)):
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


def centre_error(stencil, k, h, phase=0.3):
    """lambda + |k|^2 for the stencil at spacing h and wavevector k (x, y[, z]):
    cos(k . r + phase) sampled on the 5^d points around the origin, so that
    the stencil at the centre sees the wave itself, unwrapped, at any k."""
    d = len(k)
    ax = (np.arange(5) - 2) * h
    g = np.meshgrid(*([ax] * d), indexing="ij")              # (z,) y, x
    f = np.cos(sum(kk * gg for kk, gg in zip(reversed(k), g)) + phase)
    c = (2,) * d
    return fd.laplacian(f, (h,) * d, stencil)[c] / f[c] + sum(kk * kk for kk in k)


def unit_wavevectors(d):
    for a in (0.1, 0.5, np.pi / 4, 1.2):
        yield (np.cos(a), np.sin(a)) if d == 2 else (np.cos(a) * np.cos(0.4), np.sin(a) * np.cos(0.4), np.sin(0.4))


@pytest.mark.parametrize("stencil,d,order", [(9, 2, 2), (15, 3, 2), (19, 3, 2), (21, 3, 2), (27, 3, 2), (17, 2, 4),
                                             (21, 2, 4)])
def test_leading_error_in_closed_form(stencil, d, order):
    """The defining property of each isotropic stencil: at |k| = 1 and any
    angle, lambda + |k|^2 is h^2 / 12 (second order) or h^4 / 90 (fourth
    order) up to the next order in h; a wrong weight breaks the zero sum,
    the second moment, the vanishing fourth moments or their isotropy, and
    the error then has another power of h or depends on the angle."""
    h = 0.05
    want = h ** 2 / 12 if order == 2 else h ** 4 / 90
    for k in unit_wavevectors(d):
        assert abs(centre_error(stencil, k, h) / want - 1) < 1e-3, k


@pytest.mark.parametrize("stencil,d,order", [(5, 2, 2), (7, 3, 2), (4, 2, 4)])
def test_axiswise_stencils_miss_the_isotropic_error(stencil, d, order):
    """The axis-wise stencils' error is h^2 sum k_a^4 / 12 (h^4 sum k_a^6 / 90
    for fourth order): equal to the isotropic form along an axis only."""
    h = 0.05
    p, den = (4, 12) if order == 2 else (6, 90)
    for k in unit_wavevectors(d):
        want = h ** order * sum(kk ** p for kk in k) / den
        assert abs(centre_error(stencil, k, h) / want - 1) < 1e-3, k
    diagonal = list(unit_wavevectors(d))[2]                   # 45 degrees from the x axis
    assert abs(centre_error(stencil, diagonal, h) / (h ** order / den) - 1) > 0.3


@pytest.mark.parametrize("model,d,stencil,ns", [("allen_cahn", 2, 9, (32, 64)), ("cahn_hilliard", 2, 9, (32, 64)),
                                                ("gray_scott", 2, 9, (32, 64)), ("allen_cahn", 3, 19, (32, 64)),
                                                ("pfc", 3, 19, (64, 128)), ("cahn_hilliard", 3, 27, (32, 64)),
                                                ("allen_cahn", 2, 4, (32, 64)), ("gray_scott", 3, 4, (32, 64)),
                                                ("cahn_hilliard", 3, 15, (32, 64)), ("gray_scott", 3, 21, (32, 64)),
                                                ("allen_cahn", 2, 17, (32, 64)), ("pfc", 2, 21, (64, 128))])
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
