"""Equations read at run time (Sec. 2.4.2 split) stepped by the forward-Euler
finite-difference solver (Sec. 2.4.1, stencils of Sec. 2.2.2) on the GPU,
element by element against the oracle's Euler form of the split on the same
seeded inputs, for every stencil in 2D and 3D, FP64 and FP32."""
import numpy as np
import pytest

from oracle import fd_euler
from oracle import operator_split as osp
from tests import _equations as eqs
from tests._common import COEF, TOL, as_input, assert_parity, need_gpu, rel_l2, say, synth_fields

pytestmark = pytest.mark.gpu

COEF_FD = dict(COEF)
COEF_FD["pfc"] = (-0.25, 1.0, 0.3, 1.0)
# explicit time steps inside each fixed model's stability limit at dx = 1
DT_FIXED = {"allen_cahn": 0.05, "cahn_hilliard": 0.01, "pfc": 0.0005, "gray_scott": 0.1, "model_c": 0.01}
CASES = [((64, 32), 0), ((32, 64), 9), ((32, 64), 4), ((16, 8, 32), 0), ((16, 16, 16), 19),
         ((16, 16, 16), 27), ((16, 8, 32), 4),
         # grids the marching kernels tile (rows of 256, tiles of 64 x 4 x 8)
         ((256, 16), 9), ((512, 8), 4), ((64, 8, 16), 27), ((64, 8, 16), 0),
         # the 2D axis-wise and the 3D fourth-order marching tiles (two rows a
         # thread, a two-cell rim), in both precisions
         ((256, 32), 0), ((64, 8, 32), 4),
         # the 2D fourth-order and 3D 15- and 21-point isotropic stencils, on
         # the marching tiles and on the grids they do not tile
         ((256, 16), 17), ((32, 64), 21), ((16, 16, 16), 15), ((64, 8, 16), 21)]


def gpu_euler_eq(text, coefs, n, dx, dt, steps, fields, dtype, stencil):
    torch, specstep = need_gpu()
    g = specstep.Grid(n, dx, dtype=dtype, equations=text, coefs=coefs, dt=dt, solver="euler", stencil=stencil)
    assert g.nfields == len(fields)
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
    g.step(steps)
    out = [g.get_field(i).double().cpu().numpy() for i in range(len(fields))]
    g.close()
    return out


def stable_dt(split, ndim, stencil, h=1.0, frac=0.4):
    """frac / max |L| over the stencils' eigenvalue range (an upper bound of
    the Laplacian's magnitude: 4 per axis / h^2, 16/3 for the fourth-order
    axis-wise and 17-point stencils)."""
    lam = 4.0 * ndim / (h * h) * (4.0 / 3.0 if stencil in (4, 17) else 1.0)
    x = -np.linspace(0.0, lam, 2001)
    big = 1e-3
    for Lj in split.L:
        big = max(big, np.abs(sum(c * x ** p for p, c in Lj.items())).max())
    for ch in split.channels:
        for p, _, _ in ch:
            big = max(big, lam ** p)
    return frac / big


def check(got, want, dtype, what):
    assert_parity(got, want, dtype, what)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc", "gray_scott", "model_c"])
@pytest.mark.parametrize("n,stencil", CASES)
def test_fixed_models_written_as_equations(model, n, stencil, dtype):
    torch, specstep = need_gpu()
    dx = (1.0,) * len(n)
    dt = DT_FIXED[model] * (0.5 if stencil in (4, 17) else 1.0)
    text, coefs = eqs.fixed(model, COEF_FD[model])
    f0 = as_input(synth_fields(model, n, dx, 600 + len(n)), dtype)
    got = gpu_euler_eq(text, coefs, n, dx, dt, 20, f0, dtype, stencil)
    check(got, osp.euler_n(f0, osp.parse(text, coefs), dt, dx, 20, stencil), dtype, (model, n, stencil))
    if dtype == "f64":
        # the fixed-model kernels on the same input: the same step, rounding aside
        g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF_FD[model], dt=dt, solver="euler",
                          stencil=stencil)
        for i, f in enumerate(f0):
            g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
        g.step(20)
        for i in range(len(f0)):
            assert rel_l2(got[i], g.get_field(i).double().cpu().numpy()) <= 1e-12
        g.close()


def smooth_fields(nf, shape, seed, amp=0.1, offsets=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    return [offsets[f] + amp * (rng.random(shape) - 0.5) for f in range(nf)]


NEW = {
    "swift_hohenberg": (eqs.SWIFT_HOHENBERG, (0.0, 0.0)),
    "fitzhugh_nagumo": (eqs.FITZHUGH_NAGUMO, (0.1, -0.05)),
    "conserved_quartic": (eqs.CONSERVED_QUARTIC, (0.1, 0.0)),
    "paired_under_lap": (("a' = -a + lap(b + 0.2*b^2); b' = 0.5*lap(b) - a*b + 0.05", {}), (0.2, 0.3)),
    "constant_source": (("c' = 0.3*lap(c) - 0.1*c + 0.02 - c^2*0.5 + c^3/7", {}), (0.3, 0.0)),
    "no_derivative": (("u' = 0.5*u - u^3 + 0.2*v; v' = u - v - 0.1*u*v^2", {}), (0.1, 0.2)),
    "conserved_pair": (("p' = lap(p^3 - p + 0.5*q) - 0.3*bilap(p); q' = 0.2*lap(q - p^2)", {}), (0.05, 0.1)),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(NEW))
@pytest.mark.parametrize("n,stencil", CASES)
def test_new_equations(name, n, stencil, dtype):
    (text, coefs), offsets = NEW[name]
    sp = osp.parse(text, coefs)
    dx = (1.0,) * len(n)
    dt = stable_dt(sp, len(n), stencil)
    f0 = as_input(smooth_fields(len(sp.fields), n[::-1], 31 + len(n) + stencil, offsets=offsets), dtype)
    got = gpu_euler_eq(text, coefs, n, dx, dt, 20, f0, dtype, stencil)
    check(got, osp.euler_n(f0, sp, dt, dx, 20, stencil), dtype, (name, n, stencil))


@pytest.mark.parametrize("stencil,n", [(0, (128, 64)), (9, (64, 64)), (19, (32, 32, 32)), (27, (32, 32, 32)),
                                       (4, (64, 128)), (17, (256, 64)), (21, (64, 64)), (15, (32, 32, 32)),
                                       (21, (64, 16, 32))])
def test_conserved_equation_keeps_its_sum(stencil, n):
    """Every term of a conserved equation sits under a Laplacian whose
    stencil weights sum to zero: the field's sum stays put to rounding."""
    text, coefs = eqs.CONSERVED_QUARTIC
    sp = osp.parse(text, coefs)
    dx = (1.0,) * len(n)
    f0 = smooth_fields(1, n[::-1], 5, offsets=(0.1, 0.0))
    out = gpu_euler_eq(text, coefs, n, dx, stable_dt(sp, len(n), stencil), 200, f0, "f64", stencil)[0]
    drift = abs(out.sum() - f0[0].sum()) / f0[0].size
    say("conserved drift per cell", stencil, drift)
    assert drift < 1e-14


def test_edge_shapes_and_a_single_step():
    """Thin and small grids (8-cell axes, which the fourth-order and the
    nested stencils wrap around more than once) and a single step."""
    text, coefs = eqs.fixed("cahn_hilliard", COEF_FD["cahn_hilliard"])
    sp = osp.parse(text, coefs)
    for n, stencil, steps in [((4096, 8), 0, 3), ((8, 1024), 9, 3), ((16, 8, 8), 27, 3), ((8, 8), 4, 1),
                              ((8, 8, 8), 0, 2), ((8, 16), 17, 2), ((16, 8), 21, 2), ((8, 8, 8), 15, 2),
                              ((8, 16, 8), 21, 2)]:
        dx = (1.0,) * len(n)
        dt = stable_dt(sp, len(n), stencil)
        f0 = smooth_fields(1, n[::-1], 3, offsets=(0.1, 0.0))
        got = gpu_euler_eq(text, coefs, n, dx, dt, steps, f0, "f64", stencil)
        check(got, osp.euler_n(f0, sp, dt, dx, steps, stencil), "f64", (n, stencil))


def test_the_implicit_scheme_is_refused():
    torch, specstep = need_gpu()
    text, coefs = eqs.fixed("allen_cahn", COEF_FD["allen_cahn"])
    with pytest.raises(specstep.SpecStepError):
        specstep.Grid((32, 32), (1.0, 1.0), equations=text, coefs=coefs, dt=0.01, solver="euler",
                      scheme="implicit")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "gray_scott", "model_c"])
@pytest.mark.parametrize("n,dx,stencil", [((64, 32), (1.0, 0.8), 0), ((256, 32), (0.9, 1.2), 0),
                                          ((32, 64), (0.8, 1.25), 4), ((16, 8, 32), (1.0, 0.8, 1.3), 0),
                                          ((64, 8, 32), (1.3, 1.0, 0.8), 4), ((64, 8, 16), (1.2, 0.9, 1.0), 0)])
def test_equations_unequal_spacings(model, n, dx, stencil, dtype):
    """The equation kernels with a spacing per axis (the axis-wise stencils
    take unequal ones; the other tests use 1): against the oracle's Euler
    form of the split."""
    text, coefs = eqs.fixed(model, (0.9, 1.3, 0.7, 1.2, 0.8)[:len(COEF_FD[model])]
                            if model != "gray_scott" else (0.14, 0.07, 0.04, 0.06))
    split = osp.parse(text, coefs)
    dt = stable_dt(split, len(n), stencil, h=min(dx))
    f0 = as_input(synth_fields(model, n, dx, 800 + len(n)), dtype)
    got = gpu_euler_eq(text, coefs, n, dx, dt, 20, f0, dtype, stencil)
    check(got, osp.euler_n(f0, split, dt, dx, 20, stencil), dtype, ("unequal spacings", model, n, dx, stencil))
