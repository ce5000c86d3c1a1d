"""Pins of the generic operator-split oracle (Sec. 2.4.2, the procedure
that builds the scheme from any equation of motion, and its update rule).

Each pin ties the oracle to something outside it: Python's own evaluation
of constant expressions; the hand-written fixed-model oracle (itself pinned
by closed forms); a direct evaluation of the right-hand side with Python's
parser and numpy (first-order consistency of the increment); textbook
scalar recurrences on uniform fields; exact single-mode solutions of
linear equations; the split sets of the procedure worked out by hand."""
import math

import numpy as np
import pytest

from oracle import operator_split as osp
from oracle import spectral
from tests import _equations as eqs
from tests._common import COEF


def const_of(text, coefs=None):
    p = osp._Parser(osp._tokens(text), ["x"], dict(coefs or {}))
    e = p.expr()
    assert p.i == len(p.t)
    assert e.is_const()
    return e.const_value()


@pytest.mark.parametrize("text", ["2*3^2 - -1", "1 - 2 - 3", "2/4*3", "(1+2)^3/9", "-2^2", "+3 - +2",
                                  "2**3*a - b/4", "1.5e-1*(a + 2)^2 - .5", "((a))^0 + 7/(b - 1)"])
def test_parser_agrees_with_python_on_constants(text):
    env = {"a": 0.7, "b": 3.0}
    want = eval(text.replace("^", "**"), {"__builtins__": {}}, dict(env))
    assert const_of(text, env) == pytest.approx(want, rel=1e-15, abs=1e-15)


def rand_fields(nf, shape, seed):
    rng = np.random.default_rng(seed)
    return [0.1 * rng.standard_normal(shape) for _ in range(nf)]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("model,shape,dx,dt", [
    ("allen_cahn", (16, 32), (1.0, 1.0), 0.2), ("cahn_hilliard", (32, 16), (1.0, 0.5), 0.05),
    ("pfc", (16, 16), (math.pi / 4,) * 2, 0.1), ("gray_scott", (16, 32), (1.0, 1.0), 0.5),
    ("model_c", (16, 16), (1.0, 1.0), 0.02), ("cahn_hilliard", (8, 8, 16), (1.0, 1.0, 1.0), 0.05),
    ("pfc", (8, 16, 8), (math.pi / 4,) * 3, 0.1),
])
def test_reduces_to_the_fixed_model_oracle(model, shape, dx, dt):
    text, coefs = eqs.fixed(model, COEF[model] if model != "pfc" else (-0.25, 1.0, 0.3, 1.0))
    nf = spectral.NFIELDS[model]
    q0 = rand_fields(nf, shape, 11)
    if model == "gray_scott":
        q0 = [1.0 + q0[0], 0.25 + q0[1]]
    got = osp.step_n(q0, osp.parse(text, coefs), dt, dx, 10)
    want = spectral.step_n(q0, model, tuple(coefs.values()), dt, dx, 10)
    for a, b in zip(got, want):
        assert rel(a, b) < 1e-13


# --- first-order consistency against a direct evaluation of the text -------

def smooth_fields(nf, shape, seed):
    """Sum of a few low modes (|m| <= 2), amplitude ~0.3, plus offsets."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    out = []
    for f in range(nf):
        q = np.full(shape, 0.1 * (f + 1))
        for _ in range(4):
            m = rng.integers(-2, 3, size=len(shape))
            ph = rng.uniform(0, 2 * np.pi)
            q = q + 0.08 * np.cos(2 * np.pi * sum(mi * g for mi, g in zip(m, grids)) + ph)
        out.append(q)
    return out


def direct_rhs(text, coefs, q, dx):
    """Right-hand sides evaluated by Python's parser on numpy arrays, with a
    spectral Laplacian (multiplication by -|k|^2 on the FFT grid)."""
    shape = q[0].shape
    k2 = sum(np.meshgrid(*[(2 * np.pi * np.fft.fftfreq(n, d=h)) ** 2
                           for n, h in zip(shape, reversed(dx))], indexing="ij"))

    def lap(f):
        f = np.broadcast_to(np.asarray(f, dtype=float), shape)
        return np.fft.ifftn(-k2 * np.fft.fftn(f)).real

    env = dict(coefs)
    env.update(lap=lap, bilap=lambda f: lap(lap(f)))
    lines = [s for s in text.replace(";", "\n").split("\n") if s.strip()]
    names = [s.split("'")[0].strip() for s in lines]
    env.update(zip(names, q))
    return [np.broadcast_to(eval(s.split("=", 1)[1].replace("^", "**"), {"__builtins__": {}}, env), shape)
            for s in lines]


CONSISTENCY = [
    eqs.SWIFT_HOHENBERG, eqs.FITZHUGH_NAGUMO, eqs.CONSERVED_QUARTIC,
    ("psi' = lap(psi) - psi^3 + 0.5*lap(psi^2) + 0.1 - 0.3*psi^2", {}),       # two derivatives (D_1, D_3)
    ("a' = -a + lap(b) + 0.2*b^2; b' = 0.5*lap(b) - a*b + 0.05", {}),          # L_* under lap (D_2)
    eqs.fixed("model_c", (1.0, 1.0, 1.0, 1.0, 1.0)),
]


@pytest.mark.parametrize("scheme", ["etd1", "implicit"])
@pytest.mark.parametrize("case", range(len(CONSISTENCY)))
def test_increment_is_first_order_consistent_with_the_equation(case, scheme):
    text, coefs = CONSISTENCY[case]
    sp = osp.parse(text, coefs)
    shape, dx = (16, 32), (0.9, 1.1)
    q0 = smooth_fields(len(sp.fields), shape, 5 + case)
    R = direct_rhs(text, coefs, q0, dx)
    errs = []
    for dt in (2e-4, 1e-4):
        q1 = osp.step_n(q0, sp, dt, dx, 1, scheme)
        errs.append(max(rel((a - b) / dt, r) for a, b, r in zip(q1, q0, R)))
    assert errs[0] < 5e-3, errs
    assert 1.8 < errs[0] / errs[1] < 2.2, errs


# --- uniform fields: textbook scalar recurrences ---------------------------

def test_uniform_swift_hohenberg_is_the_scalar_etd1_and_implicit_recurrence():
    text, c = eqs.SWIFT_HOHENBERG
    L0 = c["r"] - c["q0"] ** 4
    dt, n, v = 0.3, 20, 0.4
    for scheme in ("etd1", "implicit"):
        q = osp.step_n([np.full((8, 8), v)], osp.parse(text, c), dt, (1.0, 1.0), n, scheme)[0]
        x = v
        for _ in range(n):
            if scheme == "etd1":
                x = math.exp(L0 * dt) * x + math.expm1(L0 * dt) / L0 * (-x ** 3)
            else:
                x = (x + dt * (-x ** 3)) / (1 - L0 * dt)
        assert np.max(np.abs(q - x)) < 1e-14 * abs(x) + 1e-300


def test_uniform_fitzhugh_nagumo_is_the_two_variable_recurrence():
    text, c = eqs.FITZHUGH_NAGUMO
    dt, n = 0.1, 30
    u0, v0 = 0.5, -0.2
    q = osp.step_n([np.full((8, 16), u0), np.full((8, 16), v0)], osp.parse(text, c), dt, (1.0, 1.0), n)
    u, v = u0, v0
    Lu, Lv = 1.0, -c["eps"] * c["a1"]
    for _ in range(n):
        u, v = (math.exp(Lu * dt) * u + math.expm1(Lu * dt) / Lu * (-v - u ** 3),
                math.exp(Lv * dt) * v + math.expm1(Lv * dt) / Lv * (c["eps"] * u - c["eps"] * c["a0"]))
    assert np.max(np.abs(q[0] - u)) < 1e-14
    assert np.max(np.abs(q[1] - v)) < 1e-14


# --- linear equations: exact single-mode solutions -------------------------

@pytest.mark.parametrize("scheme", ["etd1", "implicit"])
def test_single_mode_of_a_linear_equation(scheme):
    a, b, c = 0.5, -0.1, 0.2
    text = "psi' = a*lap(psi) + b*bilap(psi) + c*psi"
    shape, dx, dt, n = (16, 32), (1.0, 0.5), 0.05, 7
    y, x = np.meshgrid(np.arange(16) * dx[1], np.arange(32) * dx[0], indexing="ij")
    kx, ky = 2 * np.pi * 3 / (32 * dx[0]), 2 * np.pi * 2 / (16 * dx[1])
    q0 = 1e-3 * np.cos(kx * x + ky * y)
    k2 = kx * kx + ky * ky
    L = -a * k2 + b * k2 * k2 + c
    g = math.exp(L * dt) if scheme == "etd1" else 1.0 / (1.0 - L * dt)
    q = osp.step_n([q0], osp.parse(text, {"a": a, "b": b, "c": c}), dt, dx, n, scheme)[0]
    np.testing.assert_allclose(q, g ** n * q0, rtol=0, atol=1e-15)


def test_conserved_form_keeps_the_mean():
    text, c = eqs.CONSERVED_QUARTIC
    q0 = rand_fields(1, (32, 32), 3)[0] + 0.2
    q = osp.step_n([q0], osp.parse(text, c), 0.05, (1.0, 1.0), 200)[0]
    assert abs(q.mean() - q0.mean()) < 1e-15


# --- the procedure's sets, worked out by hand -------------------------------

def test_split_sets_of_the_procedure():
    text = "psi' = lap(psi) + 3*m - psi^3 + lap(m^2) + 2*lap(psi^2) - 2*bilap(m) + 0.5"
    with pytest.raises(osp.SplitError):
        osp.parse(text, {})          # m has no equation: an unknown name
    s = osp.parse(text + "; m' = -m", {})
    # L_psi: lap psi -> {1: 1}
    assert s.L[0] == {1: 1.0}
    ch = {p: (e0, e1) for p, e0, e1 in s.channels[0]}
    assert sorted(ch) == [0, 1, 2]
    # D_1 at d = 1: L_* = 3 m + 0.5 paired with N = -psi^3
    assert ch[0] == ({(0, 1): 3.0, (0, 0): 0.5}, {(3, 0): -1.0})
    # D_3 at d = lap: only N terms (m^2 + 2 psi^2)
    assert ch[1] == ({}, {(0, 2): 1.0, (2, 0): 2.0})
    # D_2 at d = bilap: only the L_* term -2 m
    assert ch[2] == ({(0, 1): -2.0}, {})
    assert s.L[1] == {0: -1.0} and s.channels[1] == []


def test_laplacian_of_a_constant_is_zero():
    """lap and bilap of constants vanish (step 3: lap -> -|k|^2 acts on the
    mean only through k = 0, where the symbol is 0): no channel, no term."""
    s = osp.parse("psi' = lap(psi + 3) - 2*psi + bilap(5) + lap(c)", {"c": 0.7})
    assert s.L[0] == {1: 1.0, 0: -2.0}
    assert s.channels[0] == []


@pytest.mark.parametrize("text", [
    "psi' = psi*lap(psi)", "psi' = psi/psi", "psi' = psi^2.5", "psi' = foo", "psi' = 2 psi",
    "psi' = psi^2^2", "psi = psi", "psi' = lap psi", "psi' = psi; psi' = -psi", "psi' = (psi",
    "psi' = psi/0",
])
def test_rejected_texts(text):
    with pytest.raises(osp.SplitError):
        osp.parse(text, {})


def test_implicit_scheme_needs_a_positive_denominator():
    sp = osp.parse("psi' = 5*psi", {})
    with pytest.raises(osp.SplitError):
        osp.step_n([np.zeros((8, 8))], sp, 0.5, (1.0, 1.0), 1, "implicit")


# --- the forward-Euler form of the split ------------------------------------

from oracle import fd_euler  # noqa: E402


@pytest.mark.parametrize("model,stencil,shape", [
    ("allen_cahn", 0, (16, 32)), ("cahn_hilliard", 9, (32, 32)), ("pfc", 0, (16, 16)),
    ("gray_scott", 4, (16, 32)), ("model_c", 0, (16, 16)), ("cahn_hilliard", 19, (8, 8, 8)),
])
def test_euler_form_reduces_to_the_fixed_model_euler_oracle(model, stencil, shape):
    coef = COEF[model] if model != "pfc" else (-0.25, 1.0, 0.3, 1.0)
    text, coefs = eqs.fixed(model, coef)
    nf = spectral.NFIELDS[model]
    q0 = rand_fields(nf, shape, 13)
    if model == "gray_scott":
        q0 = [1.0 + q0[0], 0.25 + q0[1]]
    dx = (1.0,) * len(shape)
    dt = {"pfc": 5e-4}.get(model, 0.01)
    got = osp.euler_n(q0, osp.parse(text, coefs), dt, dx, 10, stencil)
    want = fd_euler.euler_n(q0, model, coef, dt, dx, 10, stencil)
    for a, b in zip(got, want):
        assert rel(a, b) < 1e-12


@pytest.mark.parametrize("case", range(len(CONSISTENCY)))
@pytest.mark.parametrize("stencil", [0, 9])
def test_euler_increment_is_the_directly_evaluated_right_hand_side(case, stencil):
    """One Euler step's increment over dt is the right-hand side itself,
    evaluated by Python's parser with the same finite-difference Laplacian
    (equal up to rounding)."""
    text, coefs = CONSISTENCY[case]
    sp = osp.parse(text, coefs)
    shape, dx = (16, 32), (1.0, 1.0)
    q0 = smooth_fields(len(sp.fields), shape, 9 + case)
    dt = 1e-3
    q1 = osp.euler_n(q0, sp, dt, dx, 1, stencil)
    env = dict(coefs)
    lap = lambda f: fd_euler.laplacian(np.broadcast_to(np.asarray(f, dtype=float), shape), dx, stencil)
    env.update(lap=lap, bilap=lambda f: lap(lap(f)))
    lines = [s for s in text.replace(";", "\n").split("\n") if s.strip()]
    env.update(zip([s.split("'")[0].strip() for s in lines], q0))
    for a, b, s in zip(q1, q0, lines):
        r = np.broadcast_to(eval(s.split("=", 1)[1].replace("^", "**"), {"__builtins__": {}}, env), shape)
        assert rel((a - b) / dt, r) < 1e-11
