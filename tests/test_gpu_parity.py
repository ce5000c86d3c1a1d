"""HIP path vs the FP64 oracle, element by element (relative L2 and the
largest element-wise difference per field).

Bars: 1e-10 (FP64) and 1e-4 (FP32) after 50 steps.  Sizes span several
blocks of every kernel, non-square grids, the smallest supported axis
(8) and the largest (4096), 2D and 3D, every model.
"""
import math

import numpy as np
import pytest

from tests._common import (COEF, TOL, as_input, assert_parity, need_gpu, oracle_run, rel_l2, run_gpu, say,
                           synth_fields)

pytestmark = pytest.mark.gpu

# every transform plan: x lengths 8 .. 4096 (16 points per thread: first
# stage of radix 2, 4, 8 or 16 and one to three radix-16 stages; 8 points for
# 8-point rows) and line lengths 8 .. 4096 (8 points per thread)
SHAPES_2D = [(8, 8), (16, 64), (64, 16), (256, 32), (128, 128), (32, 512), (2048, 16),
             (4096, 8), (8, 1024), (512, 8), (1024, 16), (16, 4096), (16, 2048)]
SHAPES_3D = [(8, 8, 8), (16, 32, 8), (32, 16, 64), (64, 8, 32)]
DX = {"pfc": math.pi / 4}


def case(model, n, dtype, steps=50, dt=None, seed=11):
    h = DX.get(model, 1.0)
    dx = tuple(h * (1.0 + 0.1 * i) for i in range(len(n)))   # anisotropic spacing
    dt = dt if dt is not None else {"allen_cahn": 0.5, "cahn_hilliard": 0.1, "pfc": 0.5,
                                    "gray_scott": 1.0, "model_c": 0.05}[model]
    say("case", model, n, dtype, "steps", steps, "dt", dt)
    f0 = as_input(synth_fields(model, n, dx, seed), dtype)
    got, _ = run_gpu(model, n, dx, dt, steps, f0, dtype)
    want = oracle_run(model, n, dx, dt, steps, f0)
    assert_parity(got, want, dtype, (model, n))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", SHAPES_2D)
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc"])
def test_parity_2d_single_field(model, n, dtype):
    case(model, n, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(8, 8), (64, 16), (128, 256), (512, 32)])
@pytest.mark.parametrize("model", ["gray_scott", "model_c"])
def test_parity_2d_two_fields(model, n, dtype):
    case(model, n, dtype)


# two fields on the longest rows and lines: the two-field x pass (8 points
# per thread in FP64, 16 in FP32) on 2048- and 4096-point rows, and the
# k-space pass on 2048- and 4096-point lines
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(2048, 16), (4096, 8), (16, 2048), (8, 4096)])
@pytest.mark.parametrize("model", ["gray_scott", "model_c"])
def test_parity_2d_two_fields_long_axes(model, n, dtype):
    case(model, n, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", SHAPES_3D)
@pytest.mark.parametrize("model", ["allen_cahn", "cahn_hilliard", "pfc", "gray_scott", "model_c"])
def test_parity_3d(model, n, dtype):
    case(model, n, dtype)


# 3D grids with one long axis: x rows and y lines of 1024 and 2048 points,
# z lines of 1024 (the longest z the library takes)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(2048, 16, 8), (16, 2048, 8), (8, 16, 1024), (1024, 8, 16), (8, 1024, 16)])
@pytest.mark.parametrize("model", ["cahn_hilliard", "gray_scott", "model_c"])
def test_parity_3d_long_axes(model, n, dtype):
    case(model, n, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(8, 8), (64, 32), (2048, 8), (16, 8, 32)])
def test_set_get_round_trip(n, dtype):
    import torch
    from tests._common import need_gpu
    torch, specstep = need_gpu()
    f = as_input(synth_fields("allen_cahn", n, (1.0,) * len(n), 5), dtype)[0]
    g = specstep.Grid(n, (1.0,) * len(n), dtype=dtype, model="allen_cahn", coef=COEF["allen_cahn"], dt=0.1)
    g.set_field(0, f.astype(np.float32) if dtype == "f32" else f)        # host path
    back = g.get_field_host(0).astype(np.float64)
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert np.max(np.abs(back - f)) <= tol * np.max(np.abs(f))
    g.step(0)
    back2 = g.get_field(0).double().cpu().numpy()
    assert np.array_equal(back, back2)
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,model", [((256, 64), "cahn_hilliard"), ((64, 128), "gray_scott"),
                                     ((32, 16, 64), "pfc")])
def test_tilings_are_bitwise_identical(n, model, dtype):
    """Every valid tiling of every pass gives bit-identical fields, and the
    autotuner's pick is one of them."""
    from tests._common import need_gpu
    torch, specstep = need_gpu()
    dx = (1.0,) * len(n)
    f0 = as_input(synth_fields(model, n, dx, 3), dtype)
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=0.05)
    base = None
    esz = 16 if dtype == "f64" else 8
    cands = [(r, l, y, pp) for r in (2, 4, 8, 16, 32, 64) for l in (1, 2, 4, 8, 16, 32, 64)
             for y in ((1, 2, 4, 8, 16) if len(n) == 3 else (0,)) for pp in (0, 2, 3)]
    tried = 0
    for r, l, y, pp in cands:
        try:
            g.set_tiles([r, l, y, 0, pp])
        except specstep.SpecStepError:
            continue
        for i, f in enumerate(f0):
            g.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
        g.step(7)
        out = [g.get_field(i).cpu().numpy() for i in range(len(f0))]
        if base is None:
            base = out
        else:
            for a, b in zip(out, base):
                assert np.array_equal(a, b), (r, l, y, pp)
        tried += 1
    assert tried >= 3
    # the row block of the layout (chosen before any field is set)
    for blk in (1, 2, 8, 1 << 30):
        gb = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=0.05)
        rows = int(np.prod(n[1:]))
        b = min(blk, rows)
        if len(n) == 3 and b > n[2]:
            gb.close()
            continue
        gb.set_tiles([0, 0, 0, 0, 0, b])
        for i, f in enumerate(f0):
            gb.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
        gb.step(7)
        for i, ref in enumerate(base):
            assert np.array_equal(gb.get_field(i).cpu().numpy(), ref), ("row block", b)
        assert gb.tiles()[5] == b
        gb.close()
        tried += 1
    tiles = g.autotune(2)
    for i, f in enumerate(f0):
        g.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
    g.step(7)
    for i, b in enumerate(base):
        assert np.array_equal(g.get_field(i).cpu().numpy(), b), tiles
    say("tilings tried", tried, "autotuned", tiles)
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,model", [((256, 64), "cahn_hilliard"), ((64, 128), "gray_scott"),
                                     ((32, 16, 64), "pfc"), ((16, 16, 32), "model_c")])
def test_step_arrangements_are_bitwise_identical(n, model, dtype):
    """The three arrays arrangements of a step (in place on the state; G in
    scratch; G in scratch with T over it and the arrays swapping roles) give
    the same bits, across calls of odd length and a reload of the fields."""
    from tests._common import need_gpu
    torch, specstep = need_gpu()
    dx = (1.0,) * len(n)
    f0 = as_input(synth_fields(model, n, dx, 5), dtype)
    f1 = as_input(synth_fields(model, n, dx, 6), dtype)
    outs = {}
    for arr in (1, 0, 2):
        g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=0.05)
        specstep.ss_set_step_arrangement(g.h, arr)
        assert specstep.ss_get_step_arrangement(g.h) == arr
        for i, f in enumerate(f0):
            g.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
        g.step(3)
        g.step(4)
        assert specstep.ss_get_step_arrangement(g.h) == arr   # not replaced by tuned tiles of the shape
        mid = [g.get_field(i).cpu().numpy() for i in range(len(f0))]
        for i, f in enumerate(f1):
            g.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
        g.step(5)
        outs[arr] = mid + [g.get_field(i).cpu().numpy() for i in range(len(f1))]
        g.close()
    for arr in (0, 2):
        for a, b in zip(outs[arr], outs[1]):
            assert np.array_equal(a, b), arr
    with pytest.raises(specstep.SpecStepError):
        specstep.ss_set_step_arrangement(specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model],
                                                       dt=0.05).h, 3)


def test_mass_log_host_copy():
    """ss_mass_log copies the logged rows to the host: the steps up to the
    bound capacity, at most `max` of them, equal to the device log."""
    torch, specstep = need_gpu()
    n, dx = (64, 64), (1.0, 1.0)
    f0 = synth_fields("cahn_hilliard", n, dx, 66)
    g = specstep.Grid(n, dx, dtype="f64", model="cahn_hilliard", coef=COEF["cahn_hilliard"], dt=0.1)
    g.set_field(0, torch.from_numpy(f0[0]).to("cuda:0"))
    g.enable_mass_log(30)
    g.step(40)
    dev = g.mass_log()
    host = specstep.ss_mass_log(g.h, 100, 1)
    assert host.shape == (30, 1) and np.array_equal(host, dev)
    assert np.array_equal(specstep.ss_mass_log(g.h, 10, 1), dev[:10])
    assert specstep.ss_mass_log(g.h, 0, 1).shape == (0, 1)
    assert abs(float(host[-1, 0]) - float(np.mean(f0[0]))) <= 1e-15
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model,n", [("gray_scott", (64, 32)), ("model_c", (32, 64)), ("allen_cahn", (16, 8, 32)),
                                     ("gray_scott", (16, 16, 8)), ("pfc", (32, 32))])
def test_mass_log_is_each_fields_mean_after_each_step(model, n, dtype):
    """The per-step log of every field of every model (conserved or not) is
    the mean of that field after the step, as the oracle steps it, across
    calls of the step."""
    torch, specstep = need_gpu()
    dx = (1.0,) * len(n)
    dt = {"allen_cahn": 0.5, "pfc": 0.5, "gray_scott": 1.0, "model_c": 0.05}[model]
    f0 = as_input(synth_fields(model, n, dx, 67), dtype)
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=dt)
    for i, f in enumerate(f0):
        g.set_field(i, f.astype(np.float32) if dtype == "f32" else f)
    g.enable_mass_log(12)
    g.step(5)
    g.step(7)
    log = g.mass_log()
    g.close()
    assert log.shape == (12, len(f0))
    cur = f0
    tol = 1e-13 if dtype == "f64" else 2e-6
    worst = 0.0
    for s in range(12):
        cur = oracle_run(model, n, dx, dt, 1, cur)
        for f, c in enumerate(cur):
            worst = max(worst, abs(float(log[s, f]) - float(np.mean(c))))
    say(model, n, dtype, "max |log - oracle mean| %.3e" % worst)
    assert worst <= tol


# distinct coefficients, none equal to 1 (q0 = 0.9 in PFC): a coefficient
# read in place of another, or a missing power of one, cannot hide behind
# the value 1 of the workloads' coefficients
DISTINCT = {
    "allen_cahn": (1.3, 0.7, 0.6, 1.4),
    "cahn_hilliard": (0.8, 1.3, 0.7, 1.6),
    "pfc": (-0.2, 0.9, 0.4, 1.3),
    "gray_scott": (0.14, 0.07, 0.04, 0.06),
    "model_c": (0.8, 1.2, 0.7, 1.3, 0.9),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(64, 32), (16, 32, 8)])
@pytest.mark.parametrize("model", sorted(DISTINCT))
def test_parity_distinct_coefficients(model, n, dtype):
    h = DX.get(model, 1.0)
    dx = tuple(h * (1.0 + 0.1 * i) for i in range(len(n)))
    dt = {"allen_cahn": 0.3, "cahn_hilliard": 0.05, "pfc": 0.4, "gray_scott": 0.7, "model_c": 0.04}[model]
    f0 = as_input(synth_fields(model, n, dx, 13), dtype)
    got, _ = run_gpu(model, n, dx, dt, 50, f0, dtype, coef=DISTINCT[model])
    want = oracle_run(model, n, dx, dt, 50, f0, coef=DISTINCT[model])
    assert_parity(got, want, dtype, ("distinct coefficients", model, n))
