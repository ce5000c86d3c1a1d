"""Calls between steps leave the run intact: ss_step_n_profiled gives the
bits of ss_step_n and counts the launches of each pass kind (per step: one
x and one k-space launch for all fields, one y launch of each kind per
field in 3D); ss_time_pass and ss_autotune on a grid whose fields are
stored do not change them (the bench relies on this); new coefficients
and dt through ss_set_model keep the fields and continue as the oracle
does."""
import numpy as np
import pytest

from tests._common import COEF, need_gpu, synth_fields

pytestmark = pytest.mark.gpu

CASES = [("cahn_hilliard", (256, 128), 0.1, "f64"), ("gray_scott", (128, 64), 1.0, "f32"),
         ("pfc", (32, 32, 16), 0.5, "f64"), ("model_c", (16, 32, 8), 0.05, "f32")]


def grid(specstep, model, n, dt, dtype, seed):
    dx = (1.0,) * len(n)
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=dt)
    for i, f in enumerate(synth_fields(model, n, dx, seed)):
        g.set_field(i, f)
    return g


def fields(g):
    return [g.get_field(i).cpu().numpy() for i in range(g.nfields)]


@pytest.mark.parametrize("model,n,dt,dtype", CASES)
def test_profiled_steps_are_the_plain_steps(model, n, dt, dtype):
    torch, specstep = need_gpu()
    a = grid(specstep, model, n, dt, dtype, 120)
    a.step(12)
    want = fields(a)
    a.close()
    b = grid(specstep, model, n, dt, dtype, 120)
    prof = b.step_profiled(12)
    got = fields(b)
    nf = b.nfields
    b.close()
    for x, y in zip(got, want):
        assert np.array_equal(x, y)
    kinds = {"xpass", "kpass"} | ({"ypass_inv", "ypass_fwd"} if len(n) == 3 else set())
    assert set(prof) == kinds, prof
    for name, (ms, launches) in prof.items():
        # the x and k-space launches cover every field; the 3D y passes
        # run once per field
        assert launches == (12 * nf if name.startswith("ypass") else 12), (name, launches)
        assert ms > 0.0, name


@pytest.mark.parametrize("model,n,dt,dtype", CASES)
def test_pass_timing_leaves_stored_fields_alone(model, n, dt, dtype):
    torch, specstep = need_gpu()
    a = grid(specstep, model, n, dt, dtype, 121)
    a.step(6)
    want = fields(a)
    a.close()
    b = grid(specstep, model, n, dt, dtype, 121)
    passes = ["xpass", "kpass"] + (["ypass_inv", "ypass_fwd"] if len(n) == 3 else [])
    for p in passes:
        assert b.time_pass(p, 3) > 0.0, p
    b.step(3)
    for p in passes:
        b.time_pass(p, 2)
    b.step(3)
    got = fields(b)
    b.close()
    for x, y in zip(got, want):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("model,n,dt,dtype", CASES)
def test_autotune_leaves_stored_fields_alone(model, n, dt, dtype):
    """ss_autotune on a grid whose fields are stored (mid-run) keeps them and
    the carried spectrum: the run continues with the bits of an untuned run
    (results do not depend on the tiling)."""
    torch, specstep = need_gpu()
    a = grid(specstep, model, n, dt, dtype, 122)
    a.step(8)
    want = fields(a)
    a.close()
    b = grid(specstep, model, n, dt, dtype, 122)
    b.step(3)
    b.autotune(1)
    b.step(5)
    got = fields(b)
    b.close()
    for x, y in zip(got, want):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("model,n,dt,dtype", CASES)
def test_new_coefficients_and_dt_mid_run(model, n, dt, dtype):
    """ss_set_model with the same model and new coefficients and dt keeps
    the fields: 5 steps with the first set, 5 with the second, as the oracle
    takes them."""
    from oracle import spectral
    from tests._common import as_input, assert_parity
    torch, specstep = need_gpu()
    dx = (1.0,) * len(n)
    f0 = as_input(synth_fields(model, n, dx, 123), dtype)
    c2 = tuple(c * s for c, s in zip(COEF[model], (1.1, 0.9, 1.05, 0.95, 1.2)))
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=dt)
    for i, f in enumerate(f0):
        g.set_field(i, f)
    g.step(5)
    g.set_model(model, c2, 0.7 * dt)
    g.step(5)
    got = fields(g)
    g.close()
    mid = spectral.step_n(f0, model, COEF[model], dt, dx, 5)
    want = spectral.step_n(mid, model, c2, 0.7 * dt, dx, 5)
    assert_parity(got, want, dtype, ("coefficients changed mid-run", model, n))
