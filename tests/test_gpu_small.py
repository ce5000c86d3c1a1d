"""The one-workgroup step for small square 2D grids (ss_set_step_kernel 1):
the whole run of a call stays in one workgroup's registers and LDS.  It must
match the oracle to the parity bars, agree with the pass kernels to
rounding, continue exactly across calls, log the mass, and be refused for
grids it does not take."""
import numpy as np
import pytest

from oracle import spectral
from paper_2109_02598_amd import inputs
from tests._common import COEF, TOL, as_input, assert_parity, need_gpu, rel_l2, say, synth_fields

pytestmark = pytest.mark.gpu

DT = {"allen_cahn": 0.5, "cahn_hilliard": 0.1, "pfc": 0.5}


def run(specstep, torch, model, n, dx, dt, fields, dtype, chunks, kind, mass=0, coef=None):
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model] if coef is None else coef, dt=dt)
    specstep.ss_set_step_kernel(g.h, kind)
    assert specstep.ss_get_step_kernel(g.h) == kind
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
    if mass:
        g.enable_mass_log(mass)
    for c in chunks:
        g.step(c)
    out = g.get_field(0).double().cpu().numpy()
    log = g.mass_log() if mass else None
    g.close()
    return out, log


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_allen_cahn_128_workload(dtype):
    """The Allen-Cahn 128^2 workload (dt 0.5, 100 steps) in one call."""
    torch, specstep = need_gpu()
    w = inputs.allen_cahn_2d(n=128, seed=1)
    f0 = as_input(w.fields, dtype)
    got, _ = run(specstep, torch, w.model, w.n, w.dx, w.dt, f0, dtype, [100], 1, coef=w.coef)
    want = spectral.step_n(f0, w.model, w.coef, w.dt, w.dx, 100)
    assert_parity(got, want[0], dtype, ("one workgroup, allen_cahn 128^2", 100))
    passes, _ = run(specstep, torch, w.model, w.n, w.dx, w.dt, f0, dtype, [100], 0, coef=w.coef)
    e = rel_l2(got, passes)
    say("one workgroup vs pass kernels rel_l2 %.3e" % e)
    assert e <= (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [16, 32, 64, 128])
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc"])
def test_models_and_sizes_vs_oracle(model, n, dtype):
    torch, specstep = need_gpu()
    h = np.pi / 4 if model == "pfc" else 1.0
    dx = (h, h)
    f0 = as_input(synth_fields(model, (n, n), dx, 61), dtype)
    got, _ = run(specstep, torch, model, (n, n), dx, DT[model], f0, dtype, [50], 1)
    want = spectral.step_n(f0, model, COEF[model], DT[model], dx, 50)
    assert_parity(got, want[0], dtype, ("one workgroup", model, n))


def test_runs_continue_exactly_across_calls():
    """The carried spectrum is written at the end of a call and read at the
    start of the next: 30 + 20 steps give the bits of 50 in one call."""
    torch, specstep = need_gpu()
    n, dx = (128, 128), (1.0, 1.0)
    f0 = synth_fields("cahn_hilliard", n, dx, 62)
    one, _ = run(specstep, torch, "cahn_hilliard", n, dx, 0.1, f0, "f64", [50], 1)
    two, _ = run(specstep, torch, "cahn_hilliard", n, dx, 0.1, f0, "f64", [30, 20], 1)
    many, _ = run(specstep, torch, "cahn_hilliard", n, dx, 0.1, f0, "f64", [1] * 50, 1)
    assert np.array_equal(one, two)
    assert np.array_equal(one, many)


def test_switching_kernels_mid_run():
    torch, specstep = need_gpu()
    n, dx = (64, 64), (1.0, 1.0)
    f0 = synth_fields("allen_cahn", n, dx, 63)[0]
    g = specstep.Grid(n, dx, dtype="f64", model="allen_cahn", coef=COEF["allen_cahn"], dt=0.5)
    g.set_field(0, torch.from_numpy(f0).to("cuda:0"))
    for kind in (1, 0, 1, 0):
        specstep.ss_set_step_kernel(g.h, kind)
        g.step(10)
    got = g.get_field(0).cpu().numpy()
    g.close()
    assert_parity(got, spectral.step_n([f0], "allen_cahn", COEF["allen_cahn"], 0.5, dx, 40)[0], "f64",
                  "kernels switched every 10 steps")


def test_mass_log_of_the_conserved_model():
    torch, specstep = need_gpu()
    n, dx = (128, 128), (1.0, 1.0)
    f0 = synth_fields("cahn_hilliard", n, dx, 64)
    got, log = run(specstep, torch, "cahn_hilliard", n, dx, 0.1, f0, "f64", [120, 80], 1, mass=250)
    assert log.shape == (200, 1)
    drift = float(np.max(np.abs(log[:, 0] - np.mean(f0))))
    say("one workgroup mass drift over 200 steps %.3e" % drift)
    assert drift <= 1e-15
    assert abs(float(np.mean(got)) - float(log[-1, 0])) <= 1e-15


def test_zero_steps_and_refusals():
    torch, specstep = need_gpu()
    E = specstep.SpecStepError
    n, dx = (32, 32), (1.0, 1.0)
    f0 = synth_fields("allen_cahn", n, dx, 65)[0]
    got, _ = run(specstep, torch, "allen_cahn", n, dx, 0.5, [f0], "f64", [0], 1)
    assert np.allclose(got, f0, rtol=0, atol=1e-15)
    for kw in (dict(n=(64, 32), model="allen_cahn"), dict(n=(256, 256), model="allen_cahn"),
               dict(n=(64, 64), model="gray_scott"), dict(n=(16, 16, 16), model="allen_cahn")):
        g = specstep.Grid(kw["n"], (1.0,) * len(kw["n"]), dtype="f64", model=kw["model"],
                          coef=COEF[kw["model"]], dt=0.1)
        with pytest.raises(E) as e:
            specstep.ss_set_step_kernel(g.h, 1)
        assert e.value.code == specstep.SS_ERR_UNSUPPORTED
        assert specstep.ss_get_step_kernel(g.h) == 0
        g.close()
    g = specstep.Grid((64, 64), (1.0, 1.0), dtype="f64", equations="psi' = lap(psi) - psi^3", coefs={}, dt=0.1)
    with pytest.raises(E):
        specstep.ss_set_step_kernel(g.h, 1)
    g.close()
    g = specstep.Grid((64, 64), (1.0, 1.0), dtype="f64", model="allen_cahn", coef=COEF["allen_cahn"], dt=0.1,
                      solver="euler")
    with pytest.raises(E):
        specstep.ss_set_step_kernel(g.h, 1)
    with pytest.raises(E):
        specstep.ss_set_step_kernel(g.h, 2)
    g.close()


def test_the_tuner_chooses_a_kernel():
    torch, specstep = need_gpu()
    w = inputs.allen_cahn_2d(n=128, seed=1)
    g = specstep.Grid(w.n, w.dx, dtype="f64", model=w.model, coef=w.coef, dt=w.dt)
    g.autotune(2)
    kind = specstep.ss_get_step_kernel(g.h)
    say("tuned step kernel for allen_cahn 128^2 f64:", kind)
    g.set_field(0, torch.from_numpy(w.fields[0]).to("cuda:0"))
    g.step(100)
    got = g.get_field(0).cpu().numpy()
    g.close()
    assert kind in (0, 1)
    assert_parity(got, spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, 100)[0], "f64", "tuned")


# distinct coefficients, none equal to 1, and unequal spacings
DISTINCT = {"allen_cahn": (1.3, 0.7, 0.6, 1.4), "cahn_hilliard": (0.8, 1.3, 0.7, 1.6),
            "pfc": (-0.2, 0.9, 0.4, 1.3)}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [16, 64, 128])
@pytest.mark.parametrize("model", sorted(DISTINCT))
def test_distinct_coefficients_and_spacings_vs_oracle(model, n, dtype):
    torch, specstep = need_gpu()
    h = np.pi / 4 if model == "pfc" else 1.0
    dx = (h, 1.15 * h)
    dt = {"allen_cahn": 0.3, "cahn_hilliard": 0.05, "pfc": 0.4}[model]
    f0 = as_input(synth_fields(model, (n, n), dx, 68), dtype)
    got, _ = run(specstep, torch, model, (n, n), dx, dt, f0, dtype, [20, 30], 1, coef=DISTINCT[model])
    want = spectral.step_n(f0, model, DISTINCT[model], dt, dx, 50)
    assert_parity(got, want[0], dtype, ("one workgroup, distinct coefficients", model, n))
