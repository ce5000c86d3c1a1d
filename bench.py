#!/usr/bin/env python3
"""Benchmark of the semi-implicit Fourier spectral step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload ch2048] [--dtype f64]

Workload (default): 2D Cahn-Hilliard on a 2048x2048 periodic grid, dx=1,
dt=0.1, M=kappa=c1=c2=1, phi ~ U[-0.05, 0.05) from seed 2, with the
per-step mass log on.  A "step" is one full spectral time step (nonlinear
term, forward transforms, ETD1 update, inverse transforms, mass entry).
Inputs are resident in HBM before the timed region; the K steps are
bracketed by torch.cuda.synchronize() and HIP events on the stream the
library launches on.  The metric is cell-updates/s = cells * K / time.

Also reported: the roofline of the dominant kernel (its algorithmic bytes
per launch divided by its mean launch time from per-launch HIP events),
the FP32 run of the same workload, and the FP64 oracle on the host CPU
over a bounded sample of steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s


def workloads():
    from paper_2109_02598_amd import inputs
    return {
        "ch2048": lambda: inputs.cahn_hilliard_2d(n=2048, seed=2, steps=1000),
        "ac128": lambda: inputs.allen_cahn_2d(n=128, seed=1, steps=100),
        "pfc256": lambda: inputs.pfc_3d(n=256, seed=3, steps=500),
        "gs512": lambda: inputs.gray_scott_2d(n=512),
        # the shapes of the paper's own timing table (Sec. 3.1): context
        "ac512": lambda: inputs.allen_cahn_2d(n=512, seed=1, steps=100),
        "mc512": lambda: inputs.model_c_2d(n=512),
    }


def kernel_source_hash():
    """Hash of the device code of the single-grid step kernels."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2109_02598_amd", "csrc")
    for name in ("ss_fft.hpp", "ss_kernels.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(pass_name, w, esz):
    """HBM bytes one launch of a pass must move at minimum (read + write).

    Every array is cells*esz bytes (half spectrum with the kx=0/Nyquist
    packing).  x pass: reads the state of each field, writes the
    nonlinear term of each field.  k-space pass (stepping form): reads the
    state's spectrum and the nonlinear term, writes the new spectrum and
    the new state (one launch covers every field).  y passes: read and
    write one array of one field.
    """
    n = w.cells * esz
    nf = len(w.fields)
    return {"xpass": 2 * nf * n, "kpass": 4 * nf * n,
            "ypass_inv": 2 * n, "ypass_fwd": 2 * n}[pass_name]


PASSES = {2: ("xpass", "kpass"), 3: ("xpass", "kpass", "ypass_inv", "ypass_fwd")}


def step_bytes(w, esz):
    """Byte model of one whole step (every pass): 6 F N s in 2D (x pass 2,
    k-space pass 4 arrays per field), 10 F N s in 3D (y passes 2 + 2 more)."""
    return (6 if len(w.n) == 2 else 10) * len(w.fields) * w.cells * esz


def run_gpu(w, dtype, steps, warmup, profile_steps, autotune=True):
    import torch
    from paper_2109_02598_amd import specstep
    g = specstep.Grid(w.n, w.dx, dtype=dtype, model=w.model, coef=w.coef, dt=w.dt)
    tiles = g.autotune(5) if autotune else g.tiles()
    # mean launch of each pass from back-to-back launches between two events
    # (per-launch events add a completion fence to every launch), taken
    # before the fields are loaded, when the passes run on the step's own
    # arrays
    b2b = {k: g.time_pass(k, 200) for k in PASSES[len(w.n)]}
    for i, f in enumerate(w.fields):
        g.set_field(i, torch.from_numpy(f).to("cuda:0"))
    g.enable_mass_log(warmup + steps + profile_steps)
    g.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    prof = g.step_profiled(profile_steps)
    prof["mean_b2b"] = b2b
    mass = g.mass_log()
    # one radially averaged structure factor of the evolved field (x pass with
    # the occupancy threshold, line transforms, binning), back to back
    L = [n * d for n, d in zip(w.n, w.dx)]
    if max(L) - min(L) <= 1e-12 * max(L):
        s_k, n_k = g.structure_factor(0)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(20):
            g.structure_factor(0)
        e1.record(stream)
        torch.cuda.synchronize()
        prof["structure_factor"] = {"ms_per_call": round(e0.elapsed_time(e1) / 20, 4),
                                    "nbins": int(s_k.numel())}
    g.close()
    prof["tiles"] = tiles
    return ms, wall, prof, mass


def run_batch(steps=500, reps=3, forms=(0, 1, 2)):
    """64 uneven Cahn-Hilliard grids (FP32): one captured run of `steps`
    batched steps in each form (grouped launches in a graph, one launch, one
    cooperative launch), the tuned form eager, and the same members stepped
    one grid at a time."""
    import torch
    from paper_2109_02598_amd import inputs, specstep
    ws = inputs.cahn_hilliard_batch(count=64, steps=steps)
    stream = torch.cuda.Stream()
    gs = []
    for w in ws:
        g = specstep.Grid(w.n, w.dx, dtype="f32", model=w.model, coef=w.coef, dt=w.dt,
                          stream=stream.cuda_stream)
        g.set_field(0, w.fields[0].astype(np.float32))
        gs.append(g)
    cells = sum(w.cells for w in ws)
    b = specstep.Batch(gs, autotune=False)
    if tuple(sorted(forms)) != (0, 1, 2):
        b.set_mode(0)               # the tuner then times block sizes only
    specstep.ss_batch_autotune(b.b, reps)
    tuned_mode = b.mode()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def graph_ms(mode):
        b.set_mode(mode)
        b.capture(steps)
        b.launch()                  # warm-up replay
        b.check()
        e0.record(stream)
        b.launch()
        e1.record(stream)
        b.check()
        return e0.elapsed_time(e1)

    # every form, each one captured run of `steps` steps (the single and the
    # cooperative launch need one block size for both passes)
    ms_modes = {0: graph_ms(0), 1: None, 2: None}
    for m in (1, 2):
        if m not in forms:
            continue
        try:
            ms_modes[m] = graph_ms(m)
        except specstep.SpecStepError:
            pass
    if tuned_mode not in forms or ms_modes[tuned_mode] is None:
        tuned_mode = 0
    b.set_mode(tuned_mode)
    ms_graph = ms_modes[tuned_mode]
    e0.record(stream)
    b.step(steps)                   # the same steps, eager
    e1.record(stream)
    b.check()
    ms_eager = e0.elapsed_time(e1)
    # the plain path: every member on its own, one after another
    for g in gs:
        g.autotune(2)
    e0.record(stream)
    for g in gs:
        g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    info = b.info()
    b.close()
    for g in gs:
        g.close()
    # the byte model of one step of every member (6 arrays of N_i floats each)
    bpass = sum(6 * w.cells * 4 for w in ws)
    agg = bpass * steps / (ms_graph * 1e-3) / 1e9
    return {"workload": "cahn_hilliard batch of 64 (sizes %s, M, kappa ~ U[0.5, 2)), f32, %d steps"
                        % (sorted(set(w.n[0] for w in ws)), steps),
            "roofline": {"bound": "hbm", "what": "aggregate: sum over members of 6 N_i s bytes per step "
                                                 "over the graph launch time per step",
                         "bytes_per_step": bpass, "achieved": round(agg, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(agg / HBM_PEAK_GBS, 4)},
            "cells": cells, "value": round(cells * steps / (ms_graph * 1e-3), 1),
            "unit": "cell-updates/s", "ms_graph_launch": round(ms_graph, 3),
            "mode": {0: "grouped launches", 1: "single launch", 2: "cooperative launch"}[tuned_mode],
            "ms_graph_grouped": round(ms_modes[0], 3),
            "ms_graph_single_launch": None if ms_modes[1] is None else round(ms_modes[1], 3),
            "ms_cooperative_launch": None if ms_modes[2] is None else round(ms_modes[2], 3),
            "ms_eager": round(ms_eager, 3), "ms_sequential_plain": round(ms_plain, 3),
            "speedup_vs_sequential_plain": round(ms_plain / ms_graph, 2),
            "threads_per_block": info[0], "x_tiles": info[1], "k_tiles": info[2]}


def run_adjoint(steps=200, K=20, dtype="f32"):
    """Gray-Scott 512x512: checkpointed forward + reverse sweep, against the
    plain forward of the same steps."""
    import torch
    from paper_2109_02598_amd import inputs, specstep
    w = inputs.gray_scott_2d(n=512, steps=steps)
    vstar = torch.from_numpy(inputs.gray_scott_target(n=512)).to("cuda")
    g = specstep.Grid(w.n, w.dx, dtype=dtype, model=w.model, coef=w.coef, dt=w.dt)
    g.autotune(3)
    g.bind_adjoint(steps, K)

    def reset():
        for i, f in enumerate(w.fields):
            g.set_field(i, torch.from_numpy(f).to("cuda"))

    reset()
    g.step(steps)                       # warm-up
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    reset()
    g.step_checkpointed()
    (du0, dv0), dc = g.adjoint([torch.zeros(g.shape, device="cuda", dtype=g.tdtype),
                                (g.get_field(1) - vstar.to(g.tdtype))])   # warm-up
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_checkpointed()
    vT = g.get_field(1)
    (du0, dv0), dc = g.adjoint([torch.zeros(g.shape, device="cuda", dtype=g.tdtype),
                                (vT - vstar.to(g.tdtype))])
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    g.close()
    return {"workload": "gray_scott 512x512, %s, %d steps, checkpoint every %d" % (dtype, steps, K),
            "ms_plain_forward": round(t_plain * 1e3, 3),
            "ms_forward_plus_adjoint": round(t_adj * 1e3, 3),
            "ratio_to_plain": round(t_adj / t_plain, 2),
            "dJ_dcoef": [float(x) for x in dc]}


def run_euler(w, dtype, steps=500):
    """The forward-Euler finite-difference solver on the same grid and
    fields (every Laplacian stencil of the dimension), with the
    fixed-model kernels and with the model's equation read at run time; for
    a 2D workload also Cahn-Hilliard on 256^3 with the 3D stencils.  A
    Cahn-Hilliard step is two launches, mu from psi, then psi + dt M L mu
    (5 arrays), except with the 2D axis-wise stencil on grids the
    row-marching kernel does not tile: one launch that recomputes mu at
    the stencil points (2 arrays)."""
    from paper_2109_02598_amd import inputs
    out = euler_times(w, dtype, steps)
    if len(w.n) == 2:
        w3 = inputs.cahn_hilliard_3d(n=256)
        out["3d"] = euler_times(w3, dtype, 200)
    return out


def euler_times(w, dtype, steps):
    import torch
    from paper_2109_02598_amd import specstep
    out = {"workload": "%s, forward Euler, %s, %d steps (dt 0.01)" % (w.name, dtype, steps)}
    esz = 8 if dtype == "f64" else 4
    nfa = {"allen_cahn": 2, "cahn_hilliard": 5, "pfc": 8, "gray_scott": 4, "model_c": 6}[w.model]
    text, names = MODEL_TEXT.get(w.model, (None, ()))
    variants = [(st, eq) for st in ((0, 9, 4, 17, 21) if len(w.n) == 2 else (0, 15, 19, 21, 27, 4))
                for eq in ((False, True) if text else (False,))]
    for st, eq in variants:
        kw = (dict(equations=text, coefs=dict(zip(names, w.coef))) if eq else dict(model=w.model, coef=w.coef))
        g = specstep.Grid(w.n, w.dx, dtype=dtype, dt=0.01, solver="euler", stencil=st, **kw)
        for i, f in enumerate(w.fields):
            g.set_field(i, torch.from_numpy(f).to("cuda:0"))
        g.step(20)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        g.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        g.close()
        name = {0: "axis-wise", 4: "fourth-order axis-wise"}.get(
            st, ("fourth-order isotropic %d-point" if len(w.n) == 2 and st in (17, 21) else "isotropic %d-point") % st)
        name += ", equation text" if eq else ""
        # arrays moved per step: the fused Cahn-Hilliard launch (2D axis-wise,
        # grids the row-marching kernel does not tile) moves 2; otherwise one
        # launch per Laplacian, for the equation text too
        fused = (w.model == "cahn_hilliard" and st == 0 and len(w.n) == 2 and not eq
                 and (w.n[0] % 256 or w.n[1] % 8))
        arrays = 2 if fused else nfa
        out[name] = {"value": round(w.cells * steps / (ms * 1e-3), 1), "unit": "cell-updates/s",
                     "us_per_step": round(ms * 1e3 / steps, 2),
                     "achieved_GBs": round(arrays * w.cells * esz * steps / (ms * 1e-3) / 1e9, 1)}
    return out


# the fixed models' equations as text, for the run-time split (coefficient
# names in the order of each model's coefficient vector)
MODEL_TEXT = {
    "cahn_hilliard": ("psi' = M*lap(c2*psi^3 - c1*psi - kappa*lap(psi))", ("M", "kappa", "c1", "c2")),
    "allen_cahn": ("psi' = M*(kappa*lap(psi) + c1*psi - c2*psi^3)", ("M", "kappa", "c1", "c2")),
    "pfc": ("psi' = lap((r + q0^4)*psi + 2*q0^2*lap(psi) + bilap(psi) + g2*psi^2 + g3*psi^3)",
            ("r", "q0", "g2", "g3")),
    "gray_scott": ("u' = Du*lap(u) - u*v^2 + F*(1 - u); v' = Dv*lap(v) + u*v^2 - (F + k)*v",
                   ("Du", "Dv", "F", "k")),
}


def run_equations(w, dtype, steps=300):
    """The same workload driven by its equation read at run time (the x pass
    evaluates a monomial table, the k-space pass the split's symbol), with
    the ETD1 and the linearly implicit factors, against the fixed-model
    kernels: time per step and the mean launch of each pass."""
    import torch
    from paper_2109_02598_amd import specstep
    text, names = MODEL_TEXT[w.model]
    coefs = dict(zip(names, w.coef))
    esz = 8 if dtype == "f64" else 4
    out = {"workload": "%s as the text  %s, %s, %d steps" % (w.name, text, dtype, steps)}
    for label, kw in (("fixed_model", dict(model=w.model, coef=w.coef)),
                      ("equations_etd1", dict(equations=text, coefs=coefs, scheme="etd1")),
                      ("equations_implicit", dict(equations=text, coefs=coefs, scheme="implicit"))):
        g = specstep.Grid(w.n, w.dx, dtype=dtype, dt=w.dt, **kw)
        g.autotune(3)
        passes = {k: g.time_pass(k, 200) for k in PASSES[len(w.n)]}   # before the fields: step's arrays
        for i, f in enumerate(w.fields):
            g.set_field(i, torch.from_numpy(f).to("cuda:0"))
        g.step(20)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        g.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        g.close()
        out[label] = {"value": round(w.cells * steps / (ms * 1e-3), 1), "unit": "cell-updates/s",
                      "us_per_step": round(ms * 1e3 / steps, 2),
                      "mean_launch_us": {k: round(v * 1e3, 2) for k, v in passes.items()},
                      "achieved_GBs": {k: round(algorithmic_bytes(k, w, esz) / (v * 1e-3) / 1e9, 1)
                                       for k, v in passes.items()}}
    return out


def run_others(skip, steps=200):
    """The other workloads of the benchmark set (PFC 256^3, GS 512^2, AC
    128^2) and two shapes of the paper's timing table (Allen-Cahn and
    Model C at 512^2), both precisions, 200 timed steps each:
    cell-updates/s and the roofline of each one's dominant kernel."""
    out = {}
    for name in ("pfc256", "gs512", "ac128", "ac512", "mc512"):
        if name == skip:
            continue
        w = workloads()[name]()
        res = {"workload": w.name}
        for dt in ("f64", "f32"):
            ms, _, prof, _ = run_gpu(w, dt, steps, 20, 50)
            prof.pop("structure_factor", None)
            r = roofline(w, dt, prof, load_traffic(name, dt), ms / steps)
            res[dt] = {"value": round(w.cells * steps / (ms * 1e-3), 1), "unit": "cell-updates/s",
                       "ms_per_step": round(ms / steps, 5),
                       "roofline": {k: r[k] for k in ("kernel", "achieved", "frac", "traffic", "mean_launch_us",
                                                      "whole_step", "tiles")}}
        out[name] = res
    return out


def roofline(w, dtype, prof, traffic_rec, ms_per_step=None):
    """Roofline of the dominant kernel: algorithmic bytes per launch over its
    mean launch duration inside steps (HIP events around every launch of
    the profiled steps, on the library's stream).  The back-to-back means
    (200 launches between two events, before the fields were loaded) are
    reported beside it."""
    esz = 8 if dtype == "f64" else 4
    tiles = prof.pop("tiles", None)
    b2b = prof.pop("mean_b2b")
    evt = {k: (v[0] / v[1]) for k, v in prof.items()}
    dom = max(evt, key=evt.get)
    algo = algorithmic_bytes(dom, w, esz)
    achieved = algo / (evt[dom] * 1e-3) / 1e9
    traffic = None
    if traffic_rec:
        traffic = traffic_rec.get("bytes_per_launch", {}).get(dom)
    step = None
    if ms_per_step:
        sb = step_bytes(w, esz)
        sg = sb / (ms_per_step * 1e-3) / 1e9
        step = {"bytes_per_step": sb, "achieved": round(sg, 1), "frac": round(sg / HBM_PEAK_GBS, 4)}
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": algo, "whole_step": step,
            "mean_launch_us": {k: round(v * 1e3, 2) for k, v in evt.items()},
            "mean_launch_us_back_to_back": {k: round(v * 1e3, 2) for k, v in b2b.items()},
            "tiles": tiles}


def load_traffic(workload, dtype):
    """HBM bytes per launch from rocprofv3 counters, if taken on the current kernels."""
    p = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, dtype))
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def counter_rows(d):
    """Rows (kernel name, counter name, value) of a rocprofv3 --pmc output
    directory, in dispatch order."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit("expected one counter_collection.csv under %s, found %d" % (d, len(files)))
    rows = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    rows.sort()
    return [(k, c, v) for _, k, c, v in rows]


def traffic_record(workload, fetch_dir, write_dir, copyf_dir, copyw_dir, copy_mb=64, out_dir=None):
    """Write profiles/traffic_<workload>_<dtype>.json from two counter runs of
    the bench (FETCH_SIZE, then WRITE_SIZE) and two of --copy-calibration:
    HBM bytes per launch of each pass, the counters (KiB per dispatch)
    scaled by what they read for a plain device copy of copy_mb MiB.  Only
    the dispatches after each precision's refresh of the carried spectrum
    (kfwd_kernel) count: the timed configuration, not the tuner's trials."""
    import re
    kib = copy_mb * 1024.0

    def copy_factor(d, name):
        vals = [v for k, c, v in counter_rows(d) if c == name and "copyBuffer" in k]
        if not vals:
            raise SystemExit("no device copy in %s" % d)
        return kib / (sum(vals) / len(vals))

    ff, fw = copy_factor(copyf_dir, "FETCH_SIZE"), copy_factor(copyw_dir, "WRITE_SIZE")
    pat = re.compile(r"ss::(kpass|xpass|xpass_pp|ypass|kfwd)_kernel<(double|float), (\d+)(?:, (.*))?>")
    out = {}
    for dtype, tname in (("f64", "double"), ("f32", "float")):
        per = {}
        for d, cname, factor in ((fetch_dir, "FETCH_SIZE", ff), (write_dir, "WRITE_SIZE", fw)):
            started = False
            for k, c, v in counter_rows(d):
                m = pat.search(k)
                if c != cname or not m or m.group(2) != tname:
                    continue
                kind, rest = m.group(1), m.group(4) or ""
                if kind == "kfwd":
                    started = True
                    continue
                if not started:
                    continue
                if kind == "kpass" and not rest.startswith("true, 0"):
                    continue
                if kind in ("xpass", "xpass_pp") and not (rest.startswith("1, 2, 0") or (kind == "xpass_pp" and rest.startswith("1, 0"))):
                    continue
                key = "xpass" if kind == "xpass_pp" else kind
                per.setdefault(key, {}).setdefault(cname, []).append(v * 1024.0 * factor)
        bpl = {k: sum(sum(x) / len(x) for x in cs.values()) for k, cs in per.items() if len(cs) == 2}
        rec = {"workload": workload, "dtype": dtype, "source_hash": kernel_source_hash(),
               "copy_factor_fetch": ff, "copy_factor_write": fw, "bytes_per_launch": bpl,
               "command": "see profiles/%s_kernels.md" % workload}
        path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), "traffic_%s_%s.json" % (workload, dtype))
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        out[dtype] = bpl
    return out


def trace_summary(d, last=0):
    """Markdown table of a rocprofv3 --kernel-trace output directory: per
    kernel, the dispatches after each precision's refresh of the carried
    spectrum (kfwd_kernel; the timed configuration, not the tuner's trials
    before it), or with last > 0 the last `last` dispatches of each kernel;
    their count, mean and minimum duration in microseconds."""
    import csv
    import glob
    import re
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit("expected one kernel_trace.csv under %s, found %d" % (d, len(files)))
    rows = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"],
                         (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3))
    rows.sort()
    prec = re.compile(r"<(double|float)\b")
    started, stats = set(), {}
    for _, k, us in rows:
        m = prec.search(k)
        p = m.group(1) if m else None
        if "ss::kfwd_kernel<" in k:
            started.add(p)
        if p not in started and not last:
            continue
        stats.setdefault(k, []).append(us)
    if last:
        stats = {k: v[-last:] for k, v in stats.items()}
    return _trace_table(stats)


def _trace_table(stats):
    lines = ["| kernel | calls | mean us | min us |", "|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| `%s` | %d | %.2f | %.2f |" % (k[:90], len(v), sum(v) / len(v), min(v)))
    return "\n".join(lines)


def trace_per_load(d, n):
    """One kernel table per refresh of the carried spectrum (kfwd_kernel,
    which follows every field load) in a rocprofv3 --kernel-trace output:
    the n dispatches right after it (a grid's first n/2 steps when a step
    is two launches)."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit("expected one kernel_trace.csv under %s, found %d" % (d, len(files)))
    with open(files[0]) as f:
        rows = sorted((int(r["Dispatch_Id"]), r["Kernel_Name"],
                       (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3) for r in csv.DictReader(f))
    out = []
    for j, i in enumerate(i for i, r in enumerate(rows) if "ss::kfwd_kernel<" in r[1]):
        stats = {}
        for _, k, us in rows[i + 1:i + 1 + n]:
            stats.setdefault(k, []).append(us)
        out.append("load %d (dispatch %d)\n\n%s" % (j + 1, rows[i][0], _trace_table(stats)))
    return "\n\n".join(out)


SQ_KERNELS = [("x pass FP64", "xpass_kernel<double, 2048, 1, 2, 0"),
              ("k-space pass FP64", "kpass_kernel<double, 2048, true, 0, false>"),
              ("x pass FP32", "xpass_kernel<float, 2048, 1, 2, 0"),
              ("k-space pass FP32", "kpass_kernel<float, 2048, true, 0, false>")]


def sq_table(dirs):
    """Markdown table of SQ counters per wave for the two passes of a 2D
    step at 2048 x 2048 (both precisions), from rocprofv3 --pmc output
    directories (each pass of counters in its own run), over the dispatches
    after each precision's refresh of the carried spectrum."""
    import csv
    import glob
    vals = {label: {} for label, _ in SQ_KERNELS}
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if len(files) != 1:
            raise SystemExit("expected one counter_collection.csv under %s, found %d" % (d, len(files)))
        disp, names = {}, {}
        with open(files[0]) as f:
            for r in csv.DictReader(f):
                i = int(r["Dispatch_Id"])
                disp.setdefault(i, {})[r["Counter_Name"]] = float(r["Counter_Value"])
                names[i] = r["Kernel_Name"]
        start = {}
        for i in sorted(disp):
            for prec in ("double", "float"):
                if "kfwd_kernel<%s" % prec in names[i]:
                    start[prec] = i
        for i in sorted(disp):
            prec = "double" if "<double" in names[i] else "float"
            if prec not in start or i <= start[prec]:
                continue
            for label, key in SQ_KERNELS:
                if key in names[i]:
                    for c, v in disp[i].items():
                        vals[label].setdefault(c, []).append(v)

    def mean(label, c):
        v = vals[label].get(c, [])
        return sum(v) / len(v) if v else float("nan")

    fp = ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
          "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32")
    lines = ["| kernel | waves | VALU instr | of which FP add/mul/fma | INT32 | LDS instr | SALU | wave cycles | "
             "VALU active | LDS wait | any wait | LDS conflict / LDS active |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    def num(x, fmt="%d"):
        return "-" if x != x else fmt % (round(x) if fmt == "%d" else x)

    for label, key in SQ_KERNELS:
        if not vals[label].get("SQ_WAVES"):
            continue                                 # kernel absent from these runs
        w = mean(label, "SQ_WAVES")
        per = [mean(label, "SQ_INSTS_VALU") / w, sum(mean(label, c) for c in fp) / w]
        per += [mean(label, c) / w for c in ("SQ_INSTS_VALU_INT32", "SQ_INSTS_LDS", "SQ_INSTS_SALU",
                                             "SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_LDS",
                                             "SQ_WAIT_INST_ANY")]
        lines.append("| %s (`%s`) | %d | %s | %s |" % (
            label, key + ("" if key.endswith(">") else "...>"), round(w), " | ".join(num(x) for x in per),
            num(mean(label, "SQ_LDS_BANK_CONFLICT") / mean(label, "SQ_ACTIVE_INST_LDS"), "%.2f")))
    return "\n".join(lines)


def counter_table(workload, fetch_dir, write_dir, copyf_dir, copyw_dir, copy_mb=64):
    """Markdown table of the memory counters per dispatch of the timed
    configuration (dispatches after each precision's kfwd_kernel): raw
    FETCH_SIZE and WRITE_SIZE means (KiB), the bytes they stand for (scaled
    by a plain device copy of copy_mb MiB) and, for the step's passes, the
    algorithmic bytes and the ratio."""
    import re
    kib = copy_mb * 1024.0
    fc = [v for k, c, v in counter_rows(copyf_dir) if c == "FETCH_SIZE" and "copyBuffer" in k]
    wc = [v for k, c, v in counter_rows(copyw_dir) if c == "WRITE_SIZE" and "copyBuffer" in k]
    ff, fw = kib / (sum(fc) / len(fc)), kib / (sum(wc) / len(wc))
    w = workloads()[workload]()
    prec = re.compile(r"<(double|float)\b")
    kind = re.compile(r"ss::(kpass|xpass|xpass_pp|ypass)_kernel<(double|float), \d+, (.*)>")
    vals = {}
    for d, cname in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        started = set()
        for k, c, v in counter_rows(d):
            if c != cname:
                continue
            m = prec.search(k)
            p = m.group(1) if m else None
            if "ss::kfwd_kernel<" in k:
                started.add(p)
            if p in started:
                vals.setdefault(k, {}).setdefault(cname, []).append(v)
    lines = ["Copy calibration: a %d MiB device copy reads FETCH_SIZE = %.1f KiB (factor %.4f) and "
             "WRITE_SIZE = %.1f KiB (factor %.4f)." % (copy_mb, kib / ff, ff, kib / fw, fw), "",
             "| kernel | dispatches | FETCH raw | WRITE raw | scaled bytes | algorithmic bytes | ratio |",
             "|---|---|---|---|---|---|---|"]
    for k in sorted(vals, key=lambda k: (prec.search(k).group(1) if prec.search(k) else "", k)):
        cs = vals[k]
        if len(cs) != 2:
            continue
        f = sum(cs["FETCH_SIZE"]) / len(cs["FETCH_SIZE"])
        wr = sum(cs["WRITE_SIZE"]) / len(cs["WRITE_SIZE"])
        scaled = (f * ff + wr * fw) * 1024.0
        algo, ratio = "", ""
        m = kind.search(k)
        if m:
            esz = 8 if m.group(2) == "double" else 4
            rest = m.group(3)
            name = {"kpass": "kpass", "xpass": "xpass", "xpass_pp": "xpass", "ypass": "ypass_inv"}[m.group(1)]
            step_x = rest.startswith("1, 2, 0") or (m.group(1) == "xpass_pp")
            if (name == "kpass" and rest.startswith("true, 0")) or (name == "xpass" and step_x) or name == "ypass_inv":
                a = algorithmic_bytes(name, w, esz)
                algo, ratio = "%d" % a, "%.3f" % (scaled / a)
        lines.append("| `%s` | %d | %.1f | %.1f | %.0f | %s | %s |" % (
            k[:90], len(cs["FETCH_SIZE"]), f, wr, scaled, algo, ratio))
    return "\n".join(lines)


def host_cpu():
    """CPU model name, logical CPUs and the CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model or platform.processor() or platform.machine(),
            "nproc": os.cpu_count(), "usable_cpus": usable}


def oracle_rate(w, fft, budget_s):
    """Cell-updates/s of the FP64 oracle over about budget_s seconds of steps."""
    from oracle import spectral
    t = time.perf_counter()
    q = spectral.step_n(w.fields, w.model, w.coef, w.dt, w.dx, 1, fft=fft)
    one = time.perf_counter() - t
    nsteps = int(max(1, min(200, budget_s // max(one, 1e-6))))
    t = time.perf_counter()
    spectral.step_n(q, w.model, w.coef, w.dt, w.dx, nsteps, fft=fft)
    dt = time.perf_counter() - t
    return w.cells * nsteps / dt, nsteps


def cpu_baseline(w, budget_s=10.0):
    """The FP64 oracle on the host: its transforms on every usable core (at
    most 16, the host share of one GPU), and on one thread."""
    host = host_cpu()
    threads = max(1, min(16, host["usable_cpus"]))
    fft = None
    try:
        import scipy.fft as sfft
        fft = (lambda a: sfft.fftn(a, workers=threads), lambda a: sfft.ifftn(a, workers=threads))
    except ImportError:
        threads = 1
    v, n = oracle_rate(w, fft, budget_s)
    v1, n1 = oracle_rate(w, None, budget_s)
    return {"value": round(v, 1), "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the %s workload (after 1 untimed step), numpy FP64 oracle with its "
                      "FFTs in scipy's pocketfft on %d threads (pointwise work on one)" % (n, w.name, threads),
            "single_thread": {"value": round(v1, 1), "cores": 1, "steps": n1,
                              "sample": "numpy's pocketfft, one thread"},
            "host": host}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ch2048", choices=sorted(workloads()))
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-autotune", action="store_true", help="use the default tiles")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-grid run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-euler", action="store_true", help="skip the finite-difference solver timing")
    ap.add_argument("--no-equations", action="store_true", help="skip the run-time equations timing")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads (PFC 256^3, GS, AC)")
    ap.add_argument("--only", choices=["equations", "euler", "batch", "adjoint"],
                    help="run only this leg on the workload and print its JSON object (for profiling)")
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--batch-forms", default="0,1,2",
                    help="forms the batch leg times beside the grouped graph (a profiler that "
                         "cannot follow a cooperative launch takes 0,1)")
    ap.add_argument("--traffic-record", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPYF_DIR", "COPYW_DIR"),
                    help="only write the traffic records of --workload from rocprofv3 --pmc output "
                         "directories (FETCH_SIZE and WRITE_SIZE runs of the bench, then of "
                         "--copy-calibration 64) and exit; no GPU is used")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="only print the kernel table of a rocprofv3 --kernel-trace output "
                         "directory (the timed configuration's dispatches) and exit; no GPU is used")
    ap.add_argument("--counter-table", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPYF_DIR", "COPYW_DIR"),
                    help="only print the memory-counter table of --workload from the same four "
                         "rocprofv3 --pmc output directories as --traffic-record and exit; no GPU is used")
    ap.add_argument("--trace-last", type=int, default=0, metavar="N",
                    help="with --trace-summary: the last N dispatches of each kernel instead")
    ap.add_argument("--sq-table", nargs="+", metavar="PMC_DIR",
                    help="only print the per-wave SQ counter table of the 2048^2 passes from --pmc runs")
    ap.add_argument("--trace-per-load", type=int, default=0, metavar="N",
                    help="with --trace-summary: one table per field load, the N dispatches after it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run 20 plain device copies of MB megabytes (for scaling "
                         "the memory counters of a profiler) and exit")
    args = ap.parse_args()
    if args.sq_table:
        print(sq_table(args.sq_table), flush=True)
        return
    if args.trace_summary:
        if args.trace_per_load:
            print(trace_per_load(args.trace_summary, args.trace_per_load), flush=True)
        else:
            print(trace_summary(args.trace_summary, args.trace_last), flush=True)
        return
    if args.counter_table:
        print(counter_table(args.workload, *args.counter_table), flush=True)
        return
    if args.traffic_record:
        print(json.dumps(traffic_record(args.workload, *args.traffic_record)), flush=True)
        return
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration * 1024 * 1024
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 20}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(independent simulations shard with no communication; one large grid "
              "would need an all-to-all transpose per FFT)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from paper_2109_02598_amd import specstep
    if not os.path.exists(specstep.LIB_PATH):
        from paper_2109_02598_amd import build
        build.build()
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    w = workloads()[args.workload]()
    if args.only:
        leg = {"equations": lambda: run_equations(w, args.dtype), "euler": lambda: run_euler(w, args.dtype),
               "batch": lambda: run_batch(forms=tuple(int(v) for v in args.batch_forms.split(","))),
               "adjoint": run_adjoint}[args.only]
        print(json.dumps({args.only: leg()}), flush=True)
        return
    print("bench: workload %s cells %d dtype %s steps %d warmup %d" %
          (w.name, w.cells, args.dtype, args.steps, args.warmup), file=sys.stderr, flush=True)
    ms, wall, prof, mass = run_gpu(w, args.dtype, args.steps, args.warmup, args.profile_steps,
                                   not args.no_autotune)
    value = w.cells * args.steps / (ms * 1e-3)
    sf1 = prof.pop("structure_factor", None)
    roof = roofline(w, args.dtype, prof, load_traffic(args.workload, args.dtype), ms / args.steps)
    other = "f32" if args.dtype == "f64" else "f64"
    print("bench: %s done, %.3f ms/step; running %s" % (args.dtype, ms / args.steps, other),
          file=sys.stderr, flush=True)
    ms2, _, prof2, _ = run_gpu(w, other, args.steps, args.warmup, args.profile_steps,
                               not args.no_autotune)
    sf2 = prof2.pop("structure_factor", None)
    roof2 = roofline(w, other, prof2, load_traffic(args.workload, other), ms2 / args.steps)
    drift = float(abs(mass[-1][0] - mass[0][0])) if len(mass) else None
    adj = None
    if not args.no_adjoint:
        print("bench: adjoint workload", file=sys.stderr, flush=True)
        adj = run_adjoint()
    euler = None
    if not args.no_euler:
        print("bench: forward-Euler finite differences", file=sys.stderr, flush=True)
        euler = run_euler(w, args.dtype)
    equations = None
    if w.model in MODEL_TEXT and not args.no_equations:
        print("bench: equations read at run time", file=sys.stderr, flush=True)
        equations = run_equations(w, args.dtype)
    others = None
    if not args.no_others:
        print("bench: the other workloads", file=sys.stderr, flush=True)
        others = run_others(args.workload)
    batch = None
    if not args.no_batch:
        print("bench: batched 64-grid workload", file=sys.stderr, flush=True)
        batch = run_batch()
    summary = {"%s_%s" % (args.workload, args.dtype): {"kernel_frac": roof["frac"],
                                                        "step_frac": roof["whole_step"]["frac"]},
               "%s_%s" % (args.workload, other): {"kernel_frac": roof2["frac"],
                                                  "step_frac": roof2["whole_step"]["frac"]}}
    for name, res in (others or {}).items():
        for dt in ("f64", "f32"):
            r = res[dt]["roofline"]
            summary["%s_%s" % (name, dt)] = {"kernel_frac": r["frac"], "step_frac": r["whole_step"]["frac"]}
    if batch:
        summary["batch64_f32"] = {"step_frac": batch["roofline"]["frac"]}
    out = {
        "metric": "grid cell-updates/sec per spectral step + % peak HBM BW",
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded SplitMix64 uniform noise)",
        "config": {"workload": w.name, "equation": w.model, "grid": list(w.n), "dx": list(w.dx),
                   "dt": w.dt, "coef": list(w.coef), "mass_log": True, "parallelism": "1 GPU"},
        "roofline": roof,
        "rooflines": summary,
        "other_dtype": {"dtype": other, "value": round(w.cells * args.steps / (ms2 * 1e-3), 1),
                        "ms_per_step": round(ms2 / args.steps, 5), "roofline": roof2},
        "mass_drift_over_run": drift,
        "structure_factor": {
            "what": "radially averaged S(k) of [psi > 0] of the evolved field, one call",
            args.dtype: sf1, other: sf2},
        "batched": batch,
        "euler_fd": euler,
        "equations": equations,
        "other_workloads": others,
        "adjoint": adj,
        "wall_s_timed_region": round(wall, 4),
    }
    if not args.no_cpu:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
