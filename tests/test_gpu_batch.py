"""Batched step: many uneven grids (Cahn-Hilliard, and every fixed one-field
model mixed in one batch) in grouped launches.

Each member must match the plain single-grid path bit for bit (both run
the same per-line code, and multiply-adds are contracted per source
expression, not per inlining context), match the FP64 oracle to the
parity bar, and a captured HIP graph replayed several times (with eager
work and synchronisations in between) must give exactly what eager
stepping gives.
"""
import numpy as np
import pytest

from oracle import spectral
from paper_2109_02598_amd import inputs
from tests._common import TOL, as_input, assert_parity, need_gpu, oracle_fft, rel_l2, say

pytestmark = pytest.mark.gpu


def same_as_plain(got, want):
    return np.array_equal(got, want)


def make_members(sizes, dtype, seed0=4000):
    ws = []
    for i, (nx, ny) in enumerate(sizes):
        m = 0.5 + 1.5 * inputs.uniform(77, 2 * len(sizes))[2 * i]
        k = 0.5 + 1.5 * inputs.uniform(77, 2 * len(sizes))[2 * i + 1]
        f = inputs.uniform_field(seed0 + i, (ny, nx), -0.05, 0.05)
        ws.append(inputs.Workload("m%d" % i, "cahn_hilliard", (nx, ny), (1.0, 1.0), 0.1,
                                  (m, k, 1.0, 1.0), 0, as_input([f], dtype)))
    return ws


def grids_for(specstep, ws, dtype, stream):
    gs = []
    for w in ws:
        g = specstep.Grid(w.n, w.dx, dtype=dtype, model=w.model, coef=w.coef, dt=w.dt, stream=stream)
        g.set_field(0, w.fields[0].astype(np.float32) if dtype == "f32" else w.fields[0])
        gs.append(g)
    return gs


SIZES = [(64, 64), (128, 64), (64, 256), (256, 256), (512, 128), (128, 128), (1024, 64), (64, 512)]
# the single-launch form runs both passes with one block size (256 threads):
# rows of at least 128 points (the workload's sizes)
PSIZES = [(128, 64), (256, 256), (512, 128), (128, 128), (1024, 64), (128, 512), (256, 1024)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_matches_plain_and_oracle(dtype):
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members(SIZES, dtype)
    steps = 20
    plain = grids_for(specstep, ws, dtype, stream.cuda_stream)
    for g in plain:
        g.step(steps)
    want_plain = [g.get_field(0).cpu().numpy() for g in plain]
    gs = grids_for(specstep, ws, dtype, stream.cuda_stream)
    b = specstep.Batch(gs, autotune=True, reps=2)
    say("batch info (threads, x tiles, k tiles):", b.info())
    b.step(steps)
    torch.cuda.synchronize()
    for i, (g, w) in enumerate(zip(gs, ws)):
        got = g.get_field(0).cpu().numpy()
        say("member", i, w.n, "vs plain rel %.3e" % rel_l2(got, want_plain[i]))
        assert same_as_plain(got, want_plain[i]), (i, w.n)
        ref = spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, steps)[0]
        assert_parity(got, ref, dtype, ("member", i, w.n))
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_graph_replay_equals_eager(dtype):
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members(SIZES[:5], dtype, seed0=4100)
    eager = grids_for(specstep, ws, dtype, stream.cuda_stream)
    be = specstep.Batch(eager, autotune=False)
    graph = grids_for(specstep, ws, dtype, stream.cuda_stream)
    bg = specstep.Batch(graph, autotune=False)
    bg.capture(4)
    for rep in range(3):
        bg.launch()
        be.step(4)
        torch.cuda.synchronize()
        # eager work on the side between replays
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        for a, c in zip(graph, eager):
            assert np.array_equal(a.get_field(0).cpu().numpy(), c.get_field(0).cpu().numpy()), rep
    be.close()
    bg.close()


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_single_launch_matches_plain_grouped_and_oracle(dtype, mode):
    """One launch per run gives the bits of the plain path and of the
    grouped launches: mode 1 (a workgroup per work item, items drawn from a
    ticket counter, per-member counters ordering the passes) and mode 2
    (resident workgroups, two device-wide barriers a step)."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members(PSIZES, dtype, seed0=4200)
    steps = 20
    plain = grids_for(specstep, ws, dtype, stream.cuda_stream)
    for g in plain:
        g.step(steps)
    want = [g.get_field(0).cpu().numpy() for g in plain]
    gp = grids_for(specstep, ws, dtype, stream.cuda_stream)
    bp = specstep.Batch(gp, autotune=False)
    bp.set_mode(mode)
    assert bp.mode() == mode
    bp.step(7)
    bp.step(steps - 7)          # two launches: the counters restart per launch
    bp.check()
    gg = grids_for(specstep, ws, dtype, stream.cuda_stream)
    bg = specstep.Batch(gg, autotune=False)
    bg.set_mode(0)
    bg.step(steps)
    torch.cuda.synchronize()
    for i, w in enumerate(ws):
        got = gp[i].get_field(0).cpu().numpy()
        assert same_as_plain(got, want[i]), (i, w.n, "single launch vs plain", mode)
        assert same_as_plain(gg[i].get_field(0).cpu().numpy(), want[i]), (i, w.n, "grouped vs plain")
        ref = spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, steps)[0]
        assert_parity(got, ref, dtype, ("single-launch member", i, w.n))
    bp.close()
    bg.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_single_launch_graph_replay_equals_eager(mode):
    """Captured runs replayed (mode 1: a graph; mode 2: the cooperative
    launch issued again) equal eager steps, with other work in between."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members(PSIZES[:6], "f32", seed0=4300)
    eager = grids_for(specstep, ws, "f32", stream.cuda_stream)
    be = specstep.Batch(eager, autotune=False)
    be.set_mode(mode)
    graph = grids_for(specstep, ws, "f32", stream.cuda_stream)
    bg = specstep.Batch(graph, autotune=False)
    bg.set_mode(mode)
    bg.capture(5)
    for rep in range(3):
        bg.launch()
        be.step(5)
        bg.check()
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        for a, c in zip(graph, eager):
            assert np.array_equal(a.get_field(0).cpu().numpy(), c.get_field(0).cpu().numpy()), rep
    be.close()
    bg.close()


def test_single_launch_forms_take_small_members_and_refuse_bad_modes():
    """Members of 64-point rows share the block size of the others (their x
    pass takes 4 points per thread), so both single-launch forms accept a
    mixed batch and give the plain path's bits; unknown forms are refused."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members([(64, 64), (256, 128)], "f32", seed0=4500)
    plain = grids_for(specstep, ws, "f32", stream.cuda_stream)
    for g in plain:
        g.step(6)
    want = [g.get_field(0).cpu().numpy() for g in plain]
    for mode in (1, 2):
        gs = grids_for(specstep, ws, "f32", stream.cuda_stream)
        b = specstep.Batch(gs, autotune=False)
        b.set_mode(mode)
        assert b.mode() == mode
        b.step(6)
        b.check()
        for g, w in zip(gs, want):
            assert same_as_plain(g.get_field(0).cpu().numpy(), w), mode
        for bad in (3, -1):
            with pytest.raises(specstep.SpecStepError) as e:
                b.set_mode(bad)
            assert e.value.code == specstep.SS_ERR_ARG
        assert b.mode() == mode
        b.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_single_launch_wait_limit_is_reported_and_recovered(mode):
    """A wait bound of zero gives up at the first unmet wait: every
    workgroup leaves, the launch ends, ss_batch_check reports it; with the
    bound restored the batch steps correctly again."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members(PSIZES[:4], "f32", seed0=4400)
    gs = grids_for(specstep, ws, "f32", stream.cuda_stream)
    b = specstep.Batch(gs, autotune=False)
    b.set_mode(mode)
    specstep.ss_batch_set_wait_limit(b.b, 0)
    b.step(10)
    with pytest.raises(specstep.SpecStepError) as e:
        b.check()
    assert e.value.code == specstep.SS_ERR_DEVICE
    say("reported:", specstep.ss_last_error())
    specstep.ss_batch_set_wait_limit(b.b, 1 << 22)
    for g, w in zip(gs, ws):
        g.set_field(0, w.fields[0].astype(np.float32))
    b.step(10)
    b.check()
    for g, w in zip(gs, ws):
        ref = spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, 10)[0]
        assert_parity(g.get_field(0).cpu().numpy(), ref, "f32", ("recovered", w.n))
    b.close()


@pytest.mark.timeout(1200)
def test_batch_64_uneven_members():
    """The 64-member workload (sizes from {128, 256, 512, 1024}^2, M and kappa
    in [0.5, 2)), FP32, autotuned, run through a captured graph for 50
    steps: every member equals the plain single-grid path bit for bit and
    matches its own FP64 oracle run to the parity bar."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = inputs.cahn_hilliard_batch(count=64)
    for w in ws:
        w.fields = as_input(w.fields, "f32")
    steps = 50
    gs = grids_for(specstep, ws, "f32", stream.cuda_stream)
    b = specstep.Batch(gs, autotune=True, reps=2)
    b_mode = b.mode()
    say("64-member batch info:", b.info(), "mode", b_mode, "cells", sum(w.cells for w in ws))
    b.capture(steps)
    b.launch()
    b.check()
    got = [g.get_field(0).cpu().numpy() for g in gs]
    b.close()
    # the other forms of the batched step on the same members: the same bits
    for other in (m for m in (0, 1, 2) if m != b_mode):
        go = grids_for(specstep, ws, "f32", stream.cuda_stream)
        bo = specstep.Batch(go, autotune=False)
        bo.set_mode(other)
        bo.capture(steps)
        bo.launch()
        bo.check()
        for i in range(len(ws)):
            assert same_as_plain(go[i].get_field(0).cpu().numpy(), got[i]), (i, "mode", other)
        bo.close()
        for g in go:
            g.close()
    for i, w in enumerate(ws):
        p = specstep.Grid(w.n, w.dx, dtype="f32", model=w.model, coef=w.coef, dt=w.dt,
                          stream=stream.cuda_stream)
        p.set_field(0, w.fields[0].astype(np.float32))
        p.step(steps)
        plain = p.get_field(0).cpu().numpy()
        p.close()
        assert same_as_plain(got[i], plain), (i, w.n, "differs from the plain path")
    say("all 64 members equal the plain path bit for bit")
    fft = oracle_fft()
    for i, w in enumerate(ws):
        ref = spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, steps, fft=fft)[0]
        assert_parity(got[i], ref, "f32", ("member", i, w.n, "coef", tuple(round(c, 4) for c in w.coef)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_one_member_cooperative_run_of_the_small_workload(dtype):
    """The Allen-Cahn 128^2 workload (dt 0.5, 100 steps) as a one-member
    batch in one cooperative launch: the plain path's bits, and the oracle
    to the parity bar."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    w = inputs.allen_cahn_2d(n=128, seed=1)
    f0 = as_input(w.fields, dtype)
    p = specstep.Grid(w.n, w.dx, dtype=dtype, model=w.model, coef=w.coef, dt=w.dt, stream=stream.cuda_stream)
    p.set_field(0, f0[0])
    p.step(100)
    want = p.get_field(0).cpu().numpy()
    g = specstep.Grid(w.n, w.dx, dtype=dtype, model=w.model, coef=w.coef, dt=w.dt, stream=stream.cuda_stream)
    g.set_field(0, f0[0])
    b = specstep.Batch([g], autotune=False)
    b.set_mode(2)
    b.step(40)
    b.step(60)
    b.check()
    got = g.get_field(0).cpu().numpy()
    say("cooperative one-member batch, workgroups:", b.info())
    assert same_as_plain(got, want)
    assert_parity(got, spectral.step_n(f0, w.model, w.coef, w.dt, w.dx, 100)[0], dtype, "cooperative AC 128^2")
    b.close()
    g.close()
    p.close()


def test_check_after_grouped_steps_on_a_dirty_workspace():
    """Binding clears the counters and the error flag, so ss_batch_check
    after grouped launches (which never touch them) reports no error even
    when the workspace held other data."""
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    ws = make_members(PSIZES[:3], "f32", seed0=4600)
    gs = grids_for(specstep, ws, "f32", stream.cuda_stream)
    b = specstep.Batch(gs, autotune=False)
    nbytes = specstep.ss_batch_workspace_size(b.b)
    dirty = torch.full((nbytes,), 255, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    specstep.ss_batch_bind_workspace(b.b, dirty.data_ptr(), nbytes)
    b.workspace = dirty
    b.set_mode(0)
    b.step(3)
    b.check()
    for g, w in zip(gs, ws):
        ref = spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, 3)[0]
        assert_parity(g.get_field(0).cpu().numpy(), ref, "f32", ("dirty workspace", w.n))
    b.close()


# every member its own coefficients (none shared between members of a model)
MIXED = [("allen_cahn", (128, 64), (1.0, 0.7), (1.2, 0.8, 0.9, 1.1), 0.4),
         ("pfc", (256, 128), (0.785, 0.864), (-0.25, 0.9, 0.3, 1.2), 0.5),
         ("cahn_hilliard", (64, 256), (0.9, 1.0), (1.0, 1.5, 0.8, 1.3), 0.1),
         ("pfc", (64, 64), (0.785, 0.785), (-0.2, 1.1, 0.0, 0.9), 0.5),
         ("allen_cahn", (512, 128), (1.0, 1.0), (1.0, 1.0, 1.0, 1.0), 0.5),
         ("cahn_hilliard", (1024, 64), (1.0, 1.1), (0.7, 1.3, 1.1, 0.8), 0.1)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_of_mixed_models_and_spacings(dtype):
    """Allen-Cahn, Cahn-Hilliard and PFC members (every fixed one-field
    model), each with its own spacings, coefficients and dt, in one batch:
    every member matches its plain run bit for bit and its oracle run to
    the bar."""
    from tests._common import synth_fields
    torch, specstep = need_gpu()
    stream = torch.cuda.Stream()
    steps = 20
    f0 = [as_input(synth_fields(m, n, dx, 300 + i), dtype) for i, (m, n, dx, c, dt) in enumerate(MIXED)]

    def grids():
        out = []
        for (m, n, dx, c, dt), f in zip(MIXED, f0):
            g = specstep.Grid(n, dx, dtype=dtype, model=m, coef=c, dt=dt, stream=stream.cuda_stream)
            g.set_field(0, f[0])
            out.append(g)
        return out

    plain = grids()
    for g in plain:
        g.step(steps)
    want = [g.get_field(0).cpu().numpy() for g in plain]
    gs = grids()
    b = specstep.Batch(gs, autotune=True, reps=2)
    b.step(steps)
    torch.cuda.synchronize()
    for i, ((m, n, dx, c, dt), g) in enumerate(zip(MIXED, gs)):
        got = g.get_field(0).cpu().numpy()
        assert same_as_plain(got, want[i]), (i, m, n)
        ref = spectral.step_n(f0[i], m, c, dt, dx, steps)[0]
        assert_parity(got, ref, dtype, ("mixed member", i, m, n))
    b.close()
    for g in plain + gs:
        g.close()
