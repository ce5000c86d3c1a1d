"""Forward-Euler finite-difference solver on the GPU (Sec. 2.4.1, stencils of
Sec. 2.2.2) against the oracle's forward-Euler solver with the same stencil,
element by element, for every model in 2D and 3D, with every Laplacian
stencil: second order (5, 9; 7, 15, 19, 21, 27 points) and fourth order
(axis-wise; 17 and 21 points in 2D)."""
import numpy as np
import pytest

from oracle import fd_euler
from tests._common import COEF, TOL, as_input, assert_parity, need_gpu, rel_l2, say, synth_fields

pytestmark = pytest.mark.gpu

# explicit time steps inside each model's stability limit at dx = 1
DT = {"allen_cahn": 0.05, "cahn_hilliard": 0.01, "pfc": 0.0005, "gray_scott": 0.1, "model_c": 0.01}
COEF_FD = dict(COEF)
COEF_FD["pfc"] = (-0.25, 1.0, 0.3, 1.0)


def gpu_euler(model, n, dx, dt, steps, fields, dtype, stencil):
    torch, specstep = need_gpu()
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF_FD[model], dt=dt,
                      solver="euler", stencil=stencil)
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
    g.step(steps)
    out = [g.get_field(i).double().cpu().numpy() for i in range(len(fields))]
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc", "gray_scott", "model_c"])
@pytest.mark.parametrize("n,stencil", [((64, 32), 0), ((32, 64), 9), ((16, 8, 32), 0), ((16, 16, 16), 19),
                                       ((16, 16, 16), 27), ((32, 64), 4), ((16, 8, 32), 4),
                                       ((64, 8, 32), 19), ((128, 8, 16), 27), ((64, 16, 16), 0), ((64, 8, 32), 4),
                                       ((256, 16), 9), ((512, 8), 4), ((256, 32), 0),
                                       ((32, 64), 17), ((32, 64), 21), ((16, 16, 16), 15), ((16, 16, 16), 21),
                                       ((256, 16), 17), ((512, 8), 21), ((64, 8, 32), 15), ((128, 8, 16), 21)])
def test_euler_vs_oracle(model, n, stencil, dtype):
    dx = (1.0,) * len(n)
    steps = 20
    # the largest eigenvalue of the fourth-order axis-wise and 17-point
    # stencils is above that of the second-order axis-wise one
    dt = DT[model] * (0.5 if stencil in (4, 17) else 1.0)
    fields = synth_fields(model, n, dx, 500 + len(n))
    got = gpu_euler(model, n, dx, dt, steps, [f.astype(np.float32) if dtype == "f32" else f for f in fields],
                    dtype, stencil)
    ref = fd_euler.euler_n(as_input(fields, dtype), model, COEF_FD[model], dt, dx, steps, stencil)
    assert_parity(list(got), list(ref), dtype, (model, n, stencil))


@pytest.mark.parametrize("stencil,n", [(0, (128, 64)), (9, (64, 64)), (19, (32, 32, 32)), (27, (32, 32, 32)),
                                       (4, (64, 128)), (17, (256, 64)), (21, (64, 64)), (15, (32, 32, 32)),
                                       (21, (64, 16, 32))])
def test_euler_cahn_hilliard_conserves_mass(stencil, n):
    """The update is dt M L(mu), and every stencil's weights sum to zero on a
    periodic grid: the field's sum is conserved to rounding."""
    dx = (1.0,) * len(n)
    f0 = synth_fields("cahn_hilliard", n, dx, 77)[0]
    out = gpu_euler("cahn_hilliard", n, dx, 0.01, 200, [f0], "f64", stencil)[0]
    drift = abs(out.sum() - f0.sum()) / f0.size
    say("CH mass drift per cell", stencil, drift)
    assert drift < 1e-14


def test_solver_choice_errors():
    torch, specstep = need_gpu()
    g = specstep.Grid((32, 32), (1.0, 1.0), dtype="f64", model="allen_cahn", coef=COEF["allen_cahn"], dt=0.1)
    with pytest.raises(specstep.SpecStepError):
        specstep.ss_set_solver(g.h, 1, 19)       # 19 points is 3D
    with pytest.raises(specstep.SpecStepError):
        specstep.ss_set_solver(g.h, 1, 27)       # 27 points is 3D
    with pytest.raises(specstep.SpecStepError):
        specstep.ss_set_solver(g.h, 1, 15)       # 15 points is 3D
    specstep.ss_set_solver(g.h, 1, 21)           # 21 points: fourth order in 2D
    specstep.ss_set_solver(g.h, 1, 17)
    specstep.ss_set_solver(g.h, 0, 0)
    with pytest.raises(specstep.SpecStepError):
        specstep.ss_set_solver(g.h, 2, 0)        # unknown solver
    with pytest.raises(specstep.SpecStepError):
        specstep.ss_set_solver(g.h, 0, 9)        # the spectral solver takes no stencil
    g.close()
    for st in (9, 17, 21):                          # isotropic stencils, unequal spacing
        with pytest.raises(specstep.SpecStepError):
            specstep.Grid((32, 32), (1.0, 2.0), model="allen_cahn", coef=COEF["allen_cahn"], dt=0.1,
                          solver="euler", stencil=st)
    g = specstep.Grid((16, 16, 16), (1.0, 1.0, 1.0), model="allen_cahn", coef=COEF["allen_cahn"], dt=0.1)
    for st in (17, 9, 5):                           # 2D stencils
        with pytest.raises(specstep.SpecStepError):
            specstep.ss_set_solver(g.h, 1, st)
    for st in (15, 21, 7):
        specstep.ss_set_solver(g.h, 1, st)
    g.close()
    g = specstep.Grid((32, 32), (1.0, 1.0), model="allen_cahn", coef=COEF["allen_cahn"], dt=0.1, solver="euler")
    g.set_field(0, np.zeros((32, 32)))
    for call in (lambda: g.autotune(1), lambda: g.structure_factor(0), lambda: g.time_pass("xpass", 2)):
        with pytest.raises(specstep.SpecStepError):
            call()
    g.close()


# distinct coefficients, none equal to 1: a coefficient read in place of
# another, or a missing power of one, cannot hide behind the value 1
DISTINCT = {
    "allen_cahn": (1.3, 0.7, 0.6, 1.4),
    "cahn_hilliard": (0.8, 1.3, 0.7, 1.6),
    "pfc": (-0.2, 0.9, 0.4, 1.3),
    "gray_scott": (0.14, 0.07, 0.04, 0.06),
    "model_c": (0.8, 1.2, 0.7, 1.3, 0.9),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", sorted(DISTINCT))
@pytest.mark.parametrize("n,stencil", [((64, 32), 0), ((32, 64), 9), ((32, 64), 17), ((16, 8, 32), 19),
                                       ((64, 8, 32), 4), ((256, 16), 0)])
def test_euler_distinct_coefficients_vs_oracle(model, n, stencil, dtype):
    dx = (0.9,) * len(n)
    steps = 20
    dt = 0.5 * DT[model] * (0.5 if stencil in (4, 17) else 1.0)
    fields = synth_fields(model, n, dx, 600 + len(n))
    torch, specstep = need_gpu()
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=DISTINCT[model], dt=dt, solver="euler",
                      stencil=stencil)
    for i, f in enumerate(fields):
        g.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
    g.step(steps)
    got = [g.get_field(i).double().cpu().numpy() for i in range(len(fields))]
    g.close()
    ref = fd_euler.euler_n(as_input(fields, dtype), model, DISTINCT[model], dt, dx, steps, stencil)
    assert_parity(got, list(ref), dtype, ("distinct coefficients", model, n, stencil))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc", "gray_scott", "model_c"])
@pytest.mark.parametrize("n,dx,stencil", [((64, 32), (1.0, 0.8), 0), ((32, 64), (0.8, 1.25), 4),
                                          ((16, 8, 32), (1.0, 0.8, 1.3), 0), ((64, 8, 32), (1.3, 1.0, 0.8), 4),
                                          ((256, 16), (0.9, 1.2), 0), ((64, 16, 16), (1.2, 0.9, 1.0), 0)])
def test_euler_unequal_spacings_vs_oracle(model, n, dx, stencil, dtype):
    """The axis-wise stencils take a spacing per axis: with unequal ones a
    spacing applied to the wrong axis shows (the other tests use 1)."""
    steps = 20
    hmin = min(dx)
    dt = DT[model] * (0.5 if stencil == 4 else 1.0) * hmin ** (6 if model == "pfc" else 4 if model in
                                                                ("cahn_hilliard", "model_c") else 2)
    fields = synth_fields(model, n, dx, 700 + len(n))
    got = gpu_euler(model, n, dx, dt, steps, [f.astype(np.float32) if dtype == "f32" else f for f in fields],
                    dtype, stencil)
    ref = fd_euler.euler_n(as_input(fields, dtype), model, COEF_FD[model], dt, dx, steps, stencil)
    assert_parity(list(got), list(ref), dtype, ("unequal spacings", model, n, dx, stencil))
