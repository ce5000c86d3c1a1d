"""Equations read at run time (Sec. 2.4.2: the scheme built from any
equation of motion) on the GPU, element by element against the oracle's
generic split on the same seeded inputs, with the ETD1 and the linearly
implicit factors, in 2D and 3D, FP64 and FP32."""
import math

import numpy as np
import pytest

from oracle import operator_split as osp
from tests import _equations as eqs
from tests._common import COEF, TOL, as_input, assert_parity, need_gpu, rel_l2, run_gpu, say, synth_fields

pytestmark = pytest.mark.gpu

DT = {"allen_cahn": 0.5, "cahn_hilliard": 0.1, "pfc": 0.5, "gray_scott": 1.0, "model_c": 0.05}
COEF_EQ = dict(COEF)
COEF_EQ["pfc"] = (-0.25, 1.0, 0.3, 1.0)


def gpu_equations(text, coefs, n, dx, dt, steps, fields, dtype, scheme="etd1", mass_capacity=0, tune=False):
    torch, specstep = need_gpu()
    g = specstep.Grid(n, dx, dtype=dtype, equations=text, coefs=coefs, dt=dt, scheme=scheme)
    assert g.nfields == len(fields)
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
    if tune:
        g.autotune(2)
    if mass_capacity:
        g.enable_mass_log(mass_capacity)
    g.step(steps)
    out = [g.get_field(i).double().cpu().numpy() for i in range(len(fields))]
    mass = g.mass_log() if mass_capacity else None
    g.close()
    return out, mass


def check(got, want, dtype, what):
    assert_parity(got, want, dtype, what)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc", "gray_scott", "model_c"])
@pytest.mark.parametrize("n", [(64, 32), (16, 16, 32)])
def test_fixed_models_written_as_equations(model, n, dtype):
    h = math.pi / 4 if model == "pfc" else 1.0
    dx = tuple(h * (1.0 + 0.1 * i) for i in range(len(n)))
    text, coefs = eqs.fixed(model, COEF_EQ[model])
    f0 = as_input(synth_fields(model, n, dx, 21), dtype)
    got, _ = gpu_equations(text, coefs, n, dx, DT[model], 50, f0, dtype)
    want = osp.step_n(f0, osp.parse(text, coefs), DT[model], dx, 50)
    check(got, want, dtype, (model, n))
    if dtype == "f64":
        # the fixed-model kernels on the same input: the same scheme, rounding aside
        fixed, _ = run_gpu(model, n, dx, DT[model], 50, f0, dtype, coef=COEF_EQ[model])
        for a, b in zip(got, fixed):
            assert rel_l2(a, b) <= 1e-12


def smooth_fields(nf, shape, seed, amp=0.1, offsets=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    return [offsets[f] + amp * (rng.random(shape) - 0.5) for f in range(nf)]


NEW = {
    "swift_hohenberg": (eqs.SWIFT_HOHENBERG, 0.2, (0.0, 0.0)),
    "fitzhugh_nagumo": (eqs.FITZHUGH_NAGUMO, 0.05, (0.1, -0.05)),
    "conserved_quartic": (eqs.CONSERVED_QUARTIC, 0.02, (0.1, 0.0)),
    "paired_under_lap": (("a' = -a + lap(b + 0.2*b^2); b' = 0.5*lap(b) - a*b + 0.05", {}), 0.05, (0.2, 0.3)),
    "constant_source": (("c' = 0.3*lap(c) - 0.1*c + 0.02 - c^2*0.5 + c^3/7", {}), 0.2, (0.3, 0.0)),
}


@pytest.mark.parametrize("scheme", ["etd1", "implicit"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(NEW))
@pytest.mark.parametrize("n", [(128, 64), (32, 16, 16)])
def test_equations_outside_the_fixed_set(name, n, dtype, scheme):
    (text, coefs), dt, off = NEW[name]
    sp = osp.parse(text, coefs)
    dx = tuple(1.0 + 0.05 * i for i in range(len(n)))
    shape = tuple(reversed(n))
    f0 = as_input(smooth_fields(len(sp.fields), shape, 31, offsets=off), dtype)
    got, _ = gpu_equations(text, coefs, n, dx, dt, 50, f0, dtype, scheme)
    want = osp.step_n(f0, sp, dt, dx, 50, scheme)
    check(got, want, dtype, (name, n, scheme))


# equations whose explicit terms sit under two derivatives in one field: an
# identity channel and a Laplacian-power channel (two B_i of Eq. 8)
TWO_CHANNELS = {
    "ac_plus_conserved_cubic": (("psi' = lap(psi) - psi^3 + 0.5*lap(psi^3)", {}), 0.05, (0.1, 0.0)),
    "gray_scott_cross_diffusion": (("u' = 0.2*lap(u) - u*v^2 + 0.03*(1 - u) + 0.01*lap(u^2*v)\n"
                                    "v' = 0.1*lap(v) + u*v^2 - 0.09*v", {}), 0.5, (0.8, 0.25)),
    "coupled_lap_and_bilap": (("a' = -a + lap(b + 0.2*b^2) + 0.5*a*b; b' = 0.5*lap(b) - a*b + 0.05 - 0.005*bilap(a^2)", {}),
                              0.05, (0.2, 0.3)),
    "conserved_with_a_source": (("m' = -bilap(m) - lap(0.2*m - m^3) - 0.1*m^3 + 0.05", {}), 0.05, (0.1, 0.0)),
}


@pytest.mark.parametrize("scheme", ["etd1", "implicit"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(TWO_CHANNELS))
@pytest.mark.parametrize("n", [(128, 64), (32, 16, 16), (8, 256)])
def test_two_explicit_channels(name, n, dtype, scheme):
    (text, coefs), dt, off = TWO_CHANNELS[name]
    sp = osp.parse(text, coefs)
    assert max(len(c) for c in sp.channels) == 2, "the text must need two channels"
    assert any(p == 0 for p, _, _ in sp.channels[0]), "one channel without a derivative"
    dx = tuple(1.0 + 0.05 * i for i in range(len(n)))
    shape = tuple(reversed(n))
    f0 = as_input(smooth_fields(len(sp.fields), shape, 37, offsets=off), dtype)
    got, _ = gpu_equations(text, coefs, n, dx, dt, 50, f0, dtype, scheme)
    want = osp.step_n(f0, sp, dt, dx, 50, scheme)
    check(got, want, dtype, (name, n, scheme))


def test_two_channels_are_refused_by_the_finite_difference_solver():
    torch, specstep = need_gpu()
    (text, coefs), _, _ = TWO_CHANNELS["ac_plus_conserved_cubic"]
    g = specstep.Grid((32, 32), (1.0, 1.0), equations=text, coefs=coefs, dt=0.01)
    with pytest.raises(specstep.SpecStepError) as e:
        specstep.ss_set_solver(g.h, 1, 0)
    assert e.value.code == specstep.SS_ERR_UNSUPPORTED
    g.close()
    h = specstep.Grid((32, 32), (1.0, 1.0), equations="psi' = lap(psi) - psi^3", coefs={}, dt=0.01,
                      solver="euler")
    with pytest.raises(specstep.SpecStepError) as e:
        specstep.ss_set_equations(h.h, text, coefs, 0.01)
    assert e.value.code == specstep.SS_ERR_UNSUPPORTED
    h.close()


def test_two_channels_keep_the_mass_of_a_conserved_pair():
    """Both channels under lap: nothing enters the k = 0 mode."""
    text = "c' = lap(c^3 - c) - 0.5*bilap(c) + 0.1*bilap(c^2)"
    sp = osp.parse(text, {})
    assert [p for p, _, _ in sp.channels[0]] == [1, 2]
    n = (128, 128)
    f0 = smooth_fields(1, (128, 128), 5, offsets=(0.1,))
    got, mass = gpu_equations(text, {}, n, (1.0, 1.0), 0.02, 200, f0, "f64", mass_capacity=200)
    m0 = float(np.mean(f0[0]))
    drift = float(np.max(np.abs(mass[:, 0] - m0)))
    say("two-channel conserved mass drift", drift)
    assert drift < 1e-15
    check(got, osp.step_n(f0, sp, 0.02, (1.0, 1.0), 200), "f64", "two-channel conserved")


def test_autotuned_tiles_keep_parity():
    text, coefs = eqs.FITZHUGH_NAGUMO
    n, dx = (256, 128), (1.0, 1.0)
    f0 = smooth_fields(2, (128, 256), 7, offsets=(0.1, -0.05))
    got, _ = gpu_equations(text, coefs, n, dx, 0.05, 30, f0, "f64", tune=True)
    want = osp.step_n(f0, osp.parse(text, coefs), 0.05, dx, 30)
    check(got, want, "f64", "fhn tuned")


def test_conserved_equation_keeps_the_mass():
    text, coefs = eqs.CONSERVED_QUARTIC
    n = (256, 256)
    f0 = smooth_fields(1, (256, 256), 3, offsets=(0.1,))
    got, mass = gpu_equations(text, coefs, n, (1.0, 1.0), 0.02, 200, f0, "f64", mass_capacity=200)
    m0 = float(np.mean(f0[0]))
    drift = float(np.max(np.abs(mass[:, 0] - m0)))
    say("conserved quartic mass drift", drift)
    assert mass.shape == (200, 1)
    assert drift < 1e-15
    assert abs(float(np.mean(got[0])) - m0) < 1e-15


def test_replacing_equations_and_errors():
    torch, specstep = need_gpu()
    g = specstep.Grid((32, 32), (1.0, 1.0), equations="psi' = lap(psi) - psi^3", coefs={}, dt=0.1)
    g.set_field(0, np.zeros((32, 32)))
    E = specstep.SpecStepError
    for text, code in (("psi' = lap(psi) - psi^3 + lap(psi^2) + bilap(psi^2)", 2), ("psi' = bilap(bilap(psi^3))", 2),
                       ("psi' = psi*lap(psi)", 2), ("psi' = foo", 1), ("a' = a; b' = b; c' = c", 2)):
        with pytest.raises(E) as e:
            specstep.ss_set_equations(g.h, text, {}, 0.1)
        assert e.value.code == code
    with pytest.raises(E):                                   # 1 - L dt <= 0 at k = 0
        specstep.ss_set_equations(g.h, "psi' = 5*psi", {}, 0.5, "implicit")
    with pytest.raises(E):                                   # 1 - L dt <= 0 at the largest k
        specstep.ss_set_equations(g.h, "psi' = -psi + 0.1*bilap(psi)", {}, 0.5, "implicit")
    with pytest.raises(E):
        specstep.ss_set_equations(g.h, "psi' = -psi", {}, 0.0)
    specstep.ss_set_equations(g.h, "psi' = lap(psi) - psi^3", {}, 0.1, "implicit")
    with pytest.raises(E):
        specstep.ss_set_solver(g.h, 1, 0)                    # the implicit factors are spectral
    with pytest.raises(E):
        specstep.ss_set_model(g.h, specstep.SS_EQUATIONS, [1.0], 0.1)
    with pytest.raises(E):
        specstep.Batch([g])                                  # batches take the fixed models
    # same field count: the workspace and the field stay bound
    specstep.ss_set_equations(g.h, "psi' = -psi", {}, 0.1)
    g.step(3)
    out = g.get_field(0).cpu().numpy()
    assert np.all(out == 0.0)
    # a two-field system on the same grid
    g.set_equations("u' = lap(u) - v; v' = u", {}, 0.1)
    assert g.nfields == 2
    g.close()


# the table's extremes: degree 7 in either field, eight monomials, no
# explicit term at all, L up to lap^3; long and short lines
EDGE = {
    "no_explicit_terms": ("psi' = 0.3*lap(psi) - 0.01*bilap(psi) - 0.2*psi", {}, 1),
    "degree_7_eight_monomials": ("x' = lap(x) - 0.1*x + 0.01*(1 + x^2 + x^3 - x^4 + x^5/5 - x^6/6 + x^7/7) - 0.02*x^3",
                                 {}, 1),
    "lap_cubed": ("p' = 0.05*lap(lap(lap(p))) + 0.1*lap(p) - 0.3*p - p^3 + 0.2*p^2", {}, 1),
    "two_fields_degree_7": ("a' = lap(a) - a + 0.01*b^7 - 0.02*a^3*b^2 + 0.03*a^7\n"
                            "b' = 0.5*lap(b) - 0.1*b + 0.05*a^2*b^3 - 0.01*a^7*b^7", {}, 2),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("n", [(4096, 8), (8, 1024), (16, 8, 8)])
def test_table_extremes_and_ragged_shapes(name, n, dtype):
    text, coefs, nf = EDGE[name]
    sp = osp.parse(text, coefs)
    assert len(sp.fields) == nf
    dx = tuple(1.0 + 0.03 * i for i in range(len(n)))
    shape = tuple(reversed(n))
    f0 = as_input(smooth_fields(nf, shape, 41, amp=0.6, offsets=(0.2, -0.3)), dtype)
    got, _ = gpu_equations(text, coefs, n, dx, 0.02, 30, f0, dtype)
    want = osp.step_n(f0, sp, 0.02, dx, 30)
    check(got, want, dtype, (name, n))


def test_the_library_split_of_the_extremes_is_the_oracles():
    _, specstep = need_gpu()
    for name, (text, coefs, nf) in EDGE.items():
        got = specstep.ss_split_equations(text, coefs)
        sp = osp.parse(text, coefs)
        assert len(got) == nf
        for j in range(nf):
            merged = {}
            for _, e0, e1 in sp.channels[j]:
                for ex, c in list(e0.items()) + list(e1.items()):
                    key = tuple(ex) + (0,) * (2 - len(ex))
                    merged[key] = merged.get(key, 0.0) + c
            lib = {(e0, e1): c for ch in got[j]["channels"] for c, e0, e1 in ch["terms"]}
            assert set(lib) == set(merged), name
            for k in lib:
                assert lib[k] == pytest.approx(merged[k], rel=1e-14), (name, k)
