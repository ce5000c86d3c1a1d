"""Pins of the oracle adjoint: central finite differences of the forward
map (an independent computation) and checkpoint-interval invariance."""
import numpy as np
import pytest

from oracle import adjoint, spectral
from paper_2109_02598_amd import inputs

COEF = (0.16, 0.08, 0.035, 0.065)


def small_case(n=32, steps=30):
    w = inputs.gray_scott_2d(n=n, npatch=4, patch=6, steps=steps)
    vstar = inputs.gray_scott_target(n=n)
    return w, vstar


def test_dphi1_series_matches_direct_formula_near_switch():
    z = np.array([-1.5e-3, -1.01e-3, 1.01e-3, 2e-3])
    direct = (z * np.exp(z) - np.expm1(z)) / z ** 2
    assert np.allclose(adjoint.dphi1(z), direct, rtol=1e-9, atol=0)
    zs = np.array([-9.9e-4, 9.9e-4])
    # the series and the closed form agree on either side of the switch
    direct = (zs * np.exp(zs) - np.expm1(zs)) / zs ** 2
    assert np.allclose(adjoint.dphi1(zs), direct, rtol=1e-9, atol=0)
    assert adjoint.dphi1(np.array([0.0]))[0] == 0.5


# the workload's dt = 1 and dx = 1 hide mistakes in powers of dt or in the
# spacings: the pins also run with dt != 1 and unequal spacings
@pytest.mark.parametrize("dt,dx", [(None, None), (0.4, (1.0, 0.8)), (1.7, (0.9, 1.2))])
def test_adjoint_coefficients_vs_central_fd(dt, dx):
    w, vstar = small_case()
    dt = w.dt if dt is None else dt
    dx = w.dx if dx is None else dx
    u0, v0 = w.fields
    res = adjoint.gray_scott_misfit_grad(u0, v0, COEF, dt, dx, w.steps, vstar, K=7)
    for i in range(4):
        h = 1e-6 * COEF[i]
        cp = list(COEF); cp[i] += h
        cm = list(COEF); cm[i] -= h
        jp = adjoint.gray_scott_misfit(u0, v0, cp, dt, dx, w.steps, vstar)
        jm = adjoint.gray_scott_misfit(u0, v0, cm, dt, dx, w.steps, vstar)
        fd = (jp - jm) / (2 * h)
        assert abs(res["dcoef"][i] - fd) <= 1e-5 * abs(fd), (i, dt, dx, res["dcoef"][i], fd)


def test_adjoint_initial_field_vs_central_fd():
    w, vstar = small_case()
    u0, v0 = w.fields
    res = adjoint.gray_scott_misfit_grad(u0, v0, COEF, w.dt, w.dx, w.steps, vstar, K=4)
    d = inputs.uniform_field(7, u0.shape, -1.0, 1.0)
    for which in ("u", "v"):
        h = 1e-6
        if which == "u":
            jp = adjoint.gray_scott_misfit(u0 + h * d, v0, COEF, w.dt, w.dx, w.steps, vstar)
            jm = adjoint.gray_scott_misfit(u0 - h * d, v0, COEF, w.dt, w.dx, w.steps, vstar)
            g = res["du0"]
        else:
            jp = adjoint.gray_scott_misfit(u0, v0 + h * d, COEF, w.dt, w.dx, w.steps, vstar)
            jm = adjoint.gray_scott_misfit(u0, v0 - h * d, COEF, w.dt, w.dx, w.steps, vstar)
            g = res["dv0"]
        fd = (jp - jm) / (2 * h)
        ad = float(np.sum(g * d))
        assert abs(ad - fd) <= 1e-5 * abs(fd), (which, ad, fd)


def test_checkpoint_interval_does_not_change_gradient():
    w, vstar = small_case(steps=20)
    u0, v0 = w.fields
    a = adjoint.gray_scott_misfit_grad(u0, v0, COEF, w.dt, w.dx, w.steps, vstar, K=1)
    b = adjoint.gray_scott_misfit_grad(u0, v0, COEF, w.dt, w.dx, w.steps, vstar, K=20)
    c = adjoint.gray_scott_misfit_grad(u0, v0, COEF, w.dt, w.dx, w.steps, vstar, K=6)
    for r in (b, c):
        assert np.array_equal(a["dv0"], r["dv0"])
        assert np.array_equal(a["du0"], r["du0"])
        assert np.array_equal(a["dcoef"], r["dcoef"])
        assert a["J"] == r["J"]


def test_misfit_matches_forward_map():
    w, vstar = small_case(steps=10)
    u0, v0 = w.fields
    res = adjoint.gray_scott_misfit_grad(u0, v0, COEF, w.dt, w.dx, w.steps, vstar, K=3)
    uT, vT = spectral.step_n([u0, v0], "gray_scott", COEF, w.dt, w.dx, w.steps)
    assert np.array_equal(res["vT"], vT)
    assert res["J"] == 0.5 * float(np.sum((vT - vstar) ** 2))
