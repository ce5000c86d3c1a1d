"""Grids on separate streams share nothing a step writes: stepped with
their launches interleaved on two HIP streams (no synchronisation between
the grids), every grid gives the bits and the mass log it gives alone, and
results read through the binding are ordered after the grid's stream."""
import numpy as np
import pytest

from tests._common import COEF, need_gpu, synth_fields

pytestmark = pytest.mark.gpu

CASES = [("cahn_hilliard", (256, 128), 0.1, "f64"), ("gray_scott", (128, 64), 1.0, "f32"),
         ("pfc", (32, 16, 16), 0.5, "f64"), ("allen_cahn", (64, 64), 0.5, "f32"),
         ("model_c", (64, 128), 0.1, "f64")]


def make(specstep, case, stream, seed):
    model, n, dt, dtype = case
    dx = (1.0,) * len(n)
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=COEF[model], dt=dt, stream=stream)
    for i, f in enumerate(synth_fields(model, n, dx, seed)):
        g.set_field(i, f)
    g.enable_mass_log(64)
    return g


def read(g):
    return [g.get_field(i).double().cpu().numpy() for i in range(g.nfields)], g.mass_log()


def test_grids_on_two_streams_match_their_solo_runs():
    torch, specstep = need_gpu()
    solo = []
    for k, case in enumerate(CASES):
        g = make(specstep, case, None, 80 + k)
        g.step(40)
        solo.append(read(g))
        g.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    grids = [make(specstep, case, streams[k % 2].cuda_stream, 80 + k) for k, case in enumerate(CASES)]
    for _ in range(8):
        for g in grids:
            g.step(5)
    for k, g in enumerate(grids):
        got, log = read(g)       # the binding orders these reads after the grid's stream
        assert log.shape == solo[k][1].shape == (40, g.nfields), CASES[k]
        assert np.array_equal(log, solo[k][1]), CASES[k]
        for a, b in zip(got, solo[k][0]):
            assert np.array_equal(a, b), CASES[k]
        g.close()


def test_structure_factor_on_a_side_stream():
    torch, specstep = need_gpu()
    case = ("cahn_hilliard", (128, 128), 0.1, "f64")
    g0 = make(specstep, case, None, 90)
    g0.step(30)
    s0, n0 = [t.cpu().numpy() for t in g0.structure_factor()]
    g0.close()
    side = torch.cuda.Stream()
    g1 = make(specstep, case, side.cuda_stream, 90)
    g1.step(30)
    s1, n1 = g1.structure_factor()     # returned after the grid's stream
    s1, n1 = s1.cpu().numpy(), n1.cpu().numpy()
    g1.close()
    assert np.array_equal(n0, n1)
    assert np.allclose(s1, s0, rtol=1e-13, atol=0.0)


def test_moving_a_grid_between_streams():
    """ss_set_stream between calls: the run continues with the bits of a
    run on one stream."""
    torch, specstep = need_gpu()
    case = ("gray_scott", (128, 128), 1.0, "f64")
    ref = make(specstep, case, None, 95)
    ref.step(30)
    want, wlog = read(ref)
    ref.close()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    g = make(specstep, case, s1.cuda_stream, 95)
    g.step(10)
    g.set_stream(s2.cuda_stream)
    g.step(10)
    g.set_stream()
    g.step(10)
    got, log = read(g)
    g.close()
    assert np.array_equal(log, wlog)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
