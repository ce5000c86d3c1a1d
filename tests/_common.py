"""Helpers shared by the GPU parity tests: run the HIP path and the oracle
on the same seeded inputs and compare them."""
import math
import os
import sys

import numpy as np
import pytest

from oracle import spectral
from paper_2109_02598_amd import inputs

COEF = {
    "allen_cahn": (1.0, 1.0, 1.0, 1.0),
    "cahn_hilliard": (1.0, 1.0, 1.0, 1.0),
    "pfc": (-0.25, 1.0, 0.0, 1.0),
    "gray_scott": (0.16, 0.08, 0.035, 0.065),
    "model_c": (1.0, 1.0, 1.0, 1.0, 1.0),
}
# parity bars on relative L2 after the stated number of steps
TOL = {"f64": 1e-10, "f32": 1e-4}
# element-wise bar beside it: max |gpu - oracle| <= MAXABS_C * TOL * max |oracle|.
# An error confined to one line of a 2048^2 grid moves the relative L2 by
# only 1/45 of its size; this bound catches it at the bar itself.
MAXABS_C = 1.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def need_gpu():
    try:
        import torch
    except Exception:  # pragma: no cover
        pytest.skip("torch missing")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_02598_amd import specstep
    if not os.path.exists(specstep.LIB_PATH):
        pytest.fail("libspecstep.so is not built: the HIP path is required")
    return torch, specstep


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_abs_ratio(a, b):
    """max |a - b| / max |b| (element by element)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def assert_parity(got, want, dtype, what, tol=None):
    """Relative L2 <= tol and max |got - want| <= MAXABS_C * tol * max |want|,
    per field; prints both figures."""
    tol = TOL[dtype] if tol is None else tol
    got = got if isinstance(got, (list, tuple)) else [got]
    want = want if isinstance(want, (list, tuple)) else [want]
    assert len(got) == len(want)
    for i, (a, b) in enumerate(zip(got, want)):
        assert np.shape(a) == np.shape(b), (what, i, np.shape(a), np.shape(b))
        e = rel_l2(a, b)
        m = max_abs_ratio(a, b)
        say("  ", what, "field", i, dtype, "rel_l2 %.3e max_abs/max %.3e" % (e, m))
        assert np.all(np.isfinite(a)), (what, i, "non-finite values")
        assert e <= tol, (what, i, "rel_l2", e)
        assert m <= MAXABS_C * tol, (what, i, "max_abs", m)


def host_workers():
    """Threads for the oracle's transforms: the CPUs this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_fft(workers=None):
    """(forward, inverse) complex transforms over every axis on several host
    threads (scipy's pocketfft): the same unnormalised/1/N transforms as
    numpy's, only faster.  None (numpy's) when scipy is absent."""
    try:
        import scipy.fft as sfft
    except ImportError:  # pragma: no cover
        return None
    w = host_workers() if workers is None else workers
    return (lambda a: sfft.fftn(a, workers=w), lambda a: sfft.ifftn(a, workers=w))


def synth_fields(model, n, dx, seed):
    """Seeded fields with the value structure of each model's workload."""
    shape = tuple(reversed(n))
    if model == "pfc":
        return [-0.285 + inputs.uniform_field(seed, shape, -0.05, 0.05)]
    if model == "gray_scott":
        u = 1.0 - 0.5 * inputs.uniform_field(seed, shape, 0.0, 0.5)
        v = inputs.uniform_field(seed + 1, shape, 0.0, 0.25)
        return [u, v]
    if model == "model_c":
        return [inputs.uniform_field(seed, shape, -0.1, 0.1),
                inputs.uniform_field(seed + 1, shape, -0.1, 0.1)]
    if model == "allen_cahn":
        return [inputs.uniform_field(seed, shape, -0.1, 0.1)]
    return [inputs.uniform_field(seed, shape, -0.05, 0.05)]


def run_gpu(model, n, dx, dt, steps, fields, dtype, coef=None, mass_capacity=0, tune=False):
    """Step `fields` on a fresh grid and read them back.  tune: pick tiles
    and arrangement with the autotuner first, as the benchmark does."""
    torch, specstep = need_gpu()
    coef = COEF[model] if coef is None else coef
    g = specstep.Grid(n, dx, dtype=dtype, model=model, coef=coef, dt=dt)
    if tune:
        say("autotuned tiles", g.autotune(5), "arrangement", specstep.ss_get_step_arrangement(g.h))
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
    if mass_capacity:
        g.enable_mass_log(mass_capacity)
    g.step(steps)
    out = [g.get_field(i).double().cpu().numpy() for i in range(len(fields))]
    mass = g.mass_log() if mass_capacity else None
    g.close()
    return out, mass


def as_input(fields, dtype):
    """The exact values the GPU sees (rounded to float32 for f32 runs)."""
    if dtype == "f32":
        return [np.asarray(f, dtype=np.float32).astype(np.float64) for f in fields]
    return [np.asarray(f, dtype=np.float64) for f in fields]


def oracle_run(model, n, dx, dt, steps, fields, coef=None, mass_log=None, fft=None):
    coef = COEF[model] if coef is None else coef
    return spectral.step_n(fields, model, coef, dt, dx, steps, mass_log=mass_log, fft=fft)
