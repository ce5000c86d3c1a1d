"""The stepping entry point that allocates nothing (ss_step_fields_noalloc):
its state lives in the library's fixed device array.  It must give what
ss_set_field + ss_step_n + ss_get_field give on a grid with a bound
workspace, bit for bit, on consecutive calls that reuse the array with a
smaller input the second time, and refuse grids the array cannot hold."""
import numpy as np
import pytest

from tests._common import COEF, as_input, assert_parity, need_gpu, oracle_run, say, synth_fields

pytestmark = pytest.mark.gpu

DT = {"cahn_hilliard": 0.1, "gray_scott": 1.0, "pfc": 0.5, "model_c": 0.05}


def existing_path(specstep, torch, model, n, dx, dt, steps, fields, dtype):
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=dt)
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
    g.step(steps)
    out = [g.get_field(i).cpu().numpy() for i in range(len(fields))]
    g.close()
    return out


def bare_handle(specstep, torch, model, n, dx, dt, dtype):
    """A grid handle with a model and no workspace (C entry points only)."""
    h = specstep.ss_create_grid(n, dx, specstep.SS_F64 if dtype == "f64" else specstep.SS_F32,
                                torch.cuda.current_stream().cuda_stream)
    specstep.ss_set_model(h, specstep.MODELS[model], COEF[model], dt)
    return h


def noalloc_path(specstep, torch, model, n, dx, dt, steps, fields, dtype):
    h = bare_handle(specstep, torch, model, n, dx, dt, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ts = [torch.from_numpy(np.ascontiguousarray(f)).to(device="cuda:0", dtype=tdt) for f in fields]
    need, limit = specstep.ss_noalloc_scratch_bytes(h)
    say("noalloc", model, n, dtype, "needs", need, "of", limit, "bytes")
    torch.cuda.synchronize()
    specstep.ss_step_fields_noalloc(h, [t.data_ptr() for t in ts], steps)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in ts]
    specstep.ss_destroy_grid(h)
    return out


CASES = [
    # (model, first grid, second (smaller) grid, dtype, steps)
    ("cahn_hilliard", (1024, 1024), (256, 128), "f64", 20),
    ("cahn_hilliard", (2048, 2048), (512, 64), "f32", 20),
    ("gray_scott", (512, 256), (128, 64), "f32", 30),
    ("pfc", (64, 64, 64), (32, 16, 16), "f64", 10),
    ("model_c", (32, 64, 16), (16, 8, 8), "f32", 10),
]


@pytest.mark.parametrize("model,n1,n2,dtype,steps", CASES)
def test_noalloc_equals_existing_entry_points(model, n1, n2, dtype, steps):
    torch, specstep = need_gpu()
    dx0 = np.pi / 4 if model == "pfc" else 1.0
    for call, n in enumerate((n1, n2)):
        dx = tuple(dx0 for _ in n)
        f0 = as_input(synth_fields(model, n, dx, 900 + call), dtype)
        want = existing_path(specstep, torch, model, n, dx, DT[model], steps, f0, dtype)
        got = noalloc_path(specstep, torch, model, n, dx, DT[model], steps, f0, dtype)
        for i, (a, b) in enumerate(zip(got, want)):
            say("call", call, model, n, dtype, "field", i, "bitwise equal:", bool(np.array_equal(a, b)))
            assert np.array_equal(a, b), (call, model, n, dtype, i)
        if call == 1 or np.prod(n) <= 1 << 18:
            assert_parity([a.astype(np.float64) for a in got],
                          oracle_run(model, n, dx, DT[model], steps, f0), dtype, ("noalloc", model, n))


def test_noalloc_leaves_the_grids_own_fields_alone():
    torch, specstep = need_gpu()
    n, dx, model = (128, 64), (1.0, 1.0), "cahn_hilliard"
    fa = synth_fields(model, n, dx, 31)[0]
    fb = synth_fields(model, n, dx, 32)[0]
    g = specstep.Grid(n, dx, dtype="f64", model=model, coef=COEF[model], dt=0.1)
    g.set_field(0, torch.from_numpy(fa).to("cuda:0"))
    g.step(5)
    before = g.get_field(0).cpu().numpy()
    tb = torch.from_numpy(fb).to("cuda:0")
    torch.cuda.synchronize()
    specstep.ss_step_fields_noalloc(g.h, [tb.data_ptr()], 5)
    torch.cuda.synchronize()
    assert np.array_equal(g.get_field(0).cpu().numpy(), before)
    g.step(5)
    ref = existing_path(specstep, torch, model, n, dx, 0.1, 10, [fa], "f64")[0]
    assert np.array_equal(g.get_field(0).cpu().numpy(), ref)
    g.close()


def test_noalloc_refusals():
    torch, specstep = need_gpu()
    # PFC 256^3 FP32: two 64 MiB arrays do not fit the 64 MiB array
    h = bare_handle(specstep, torch, "pfc", (256, 256, 256), (1.0, 1.0, 1.0), 0.5, "f32")
    need, limit = specstep.ss_noalloc_scratch_bytes(h)
    assert need > limit
    dummy = torch.empty(8, device="cuda:0")
    with pytest.raises(specstep.SpecStepError) as e:
        specstep.ss_step_fields_noalloc(h, [dummy.data_ptr()], 1)
    assert e.value.code == specstep.SS_ERR_ARG
    say("refused:", specstep.ss_last_error())
    specstep.ss_destroy_grid(h)
    h = bare_handle(specstep, torch, "cahn_hilliard", (64, 64), (1.0, 1.0), 0.1, "f64")
    with pytest.raises(specstep.SpecStepError) as e:
        specstep.ss_step_fields_noalloc(h, [0], 1)
    assert e.value.code == specstep.SS_ERR_ARG
    with pytest.raises(specstep.SpecStepError) as e:
        specstep.ss_step_fields_noalloc(h, [dummy.data_ptr()], -1)
    assert e.value.code == specstep.SS_ERR_ARG
    specstep.ss_destroy_grid(h)
    h = specstep.Grid((64, 64), (1.0, 1.0), dtype="f64", model="cahn_hilliard", coef=COEF["cahn_hilliard"],
                      dt=0.01, solver="euler")
    t = torch.zeros((64, 64), dtype=torch.float64, device="cuda:0")
    with pytest.raises(specstep.SpecStepError) as e:
        specstep.ss_step_fields_noalloc(h.h, [t.data_ptr()], 1)
    assert e.value.code == specstep.SS_ERR_UNSUPPORTED
    h.close()


@pytest.mark.parametrize("n,dtype", [((64, 32), "f64"), ((16, 8, 32), "f32")])
def test_noalloc_with_two_explicit_channels(n, dtype):
    """Equations read at run time with two explicit channels per field: the
    second channel's arrays are carved from the fixed array too."""
    torch, specstep = need_gpu()
    text = "u' = 0.2*lap(u) - u*v^2 + 0.03*(1 - u) + 0.01*lap(u^2*v); v' = 0.1*lap(v) + u*v^2 - 0.09*v"
    dx = tuple(1.0 for _ in n)
    f0 = as_input(synth_fields("gray_scott", n, dx, 77), dtype)
    g = specstep.Grid(n, dx, dtype=dtype, equations=text, coefs={}, dt=0.5)
    for i, f in enumerate(f0):
        g.set_field(i, torch.from_numpy(f).to("cuda:0"))
    g.step(20)
    want = [g.get_field(i).cpu().numpy() for i in range(2)]
    g.close()
    h = specstep.ss_create_grid(n, dx, specstep.SS_F64 if dtype == "f64" else specstep.SS_F32,
                                torch.cuda.current_stream().cuda_stream)
    specstep.ss_set_equations(h, text, {}, 0.5)
    need, limit = specstep.ss_noalloc_scratch_bytes(h)
    cells = int(np.prod(n))
    assert need == (3 if len(n) == 2 else 4) * 2 * cells * (8 if dtype == "f64" else 4)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ts = [torch.from_numpy(f).to(device="cuda:0", dtype=tdt) for f in f0]
    torch.cuda.synchronize()
    specstep.ss_step_fields_noalloc(h, [t.data_ptr() for t in ts], 20)
    torch.cuda.synchronize()
    for i in range(2):
        assert np.array_equal(ts[i].cpu().numpy(), want[i]), i
    specstep.ss_destroy_grid(h)
