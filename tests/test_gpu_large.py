"""Arrays past 4 GiB: byte offsets beyond 32 bits (FP64, 1024 x 1024 x 512)
and 2^31 cells (FP32, 2048 x 2048 x 512), sizes the oracle cannot step.

Closed form (Sec. 2.4.2, Eqs. 3-4): with c2 = 0 Allen-Cahn is linear, its
explicit term is exactly zero, and every Fourier mode is multiplied by
A = exp(L dt), L = M (c1 - kappa |k|^2), per step.  Two cosine modes, one in
the interior and one in the kx = 0 plane (stored packed with the Nyquist
plane), therefore give after n steps

    psi = a1 A1^n cos(theta1) + a2 A2^n cos(theta2)

in every cell, up to the transforms' rounding.  The whole array is compared
with that on the GPU (torch, in z chunks), not sampled.
"""
import math

import numpy as np
import pytest

from tests._common import need_gpu, say

pytestmark = pytest.mark.gpu

M, KAPPA, C1 = 1.0, 1.0, 0.5
DT = 0.25
MODES = [((3, 5, 7), 0.04), ((0, 11, 2), 0.03)]   # (mx, my, mz), amplitude


def phase(torch, n, m, zs, dtype):
    """theta(x, y, z) = 2 pi (mx x / nx + my y / ny + mz z / nz) for z in zs."""
    nx, ny, nz = n
    x = torch.arange(nx, device="cuda", dtype=torch.float64) * (2 * math.pi * m[0] / nx)
    y = torch.arange(ny, device="cuda", dtype=torch.float64) * (2 * math.pi * m[1] / ny)
    z = torch.arange(zs.start, zs.stop, device="cuda", dtype=torch.float64) * (2 * math.pi * m[2] / nz)
    return (z[:, None, None] + y[None, :, None] + x[None, None, :]).to(dtype)


def factor(n, m):
    k2 = sum((2 * math.pi * mj / nj) ** 2 for mj, nj in zip(m, n))
    return math.exp(M * (C1 - KAPPA * k2) * DT)


@pytest.mark.parametrize("dtype,n,tol", [("f64", (1024, 1024, 512), 1e-12), ("f32", (2048, 2048, 512), 2e-5)])
def test_two_modes_closed_form_past_4_gib(dtype, n, tol):
    torch, specstep = need_gpu()
    nx, ny, nz = n
    tdt = torch.float64 if dtype == "f64" else torch.float32
    esz = 8 if dtype == "f64" else 4
    say("grid %dx%dx%d %s: %.1f GiB per real array" % (nx, ny, nz, dtype, nx * ny * nz * esz / 2**30))
    chunk = 64
    psi0 = torch.empty((nz, ny, nx), device="cuda", dtype=tdt)
    for z0 in range(0, nz, chunk):
        zs = range(z0, z0 + chunk)
        acc = torch.zeros((chunk, ny, nx), device="cuda", dtype=torch.float64)
        for m, a in MODES:
            acc += a * torch.cos(phase(torch, n, m, zs, torch.float64))
        psi0[z0:z0 + chunk] = acc.to(tdt)
        del acc
    g = specstep.Grid(n, (1.0, 1.0, 1.0), dtype=dtype, model="allen_cahn", coef=(M, KAPPA, C1, 0.0), dt=DT)
    g.set_field(0, psi0)
    del psi0
    steps = 3
    g.step(steps)
    got = g.get_field(0)
    g.close()
    del g
    worst = 0.0
    for z0 in range(0, nz, chunk):
        zs = range(z0, z0 + chunk)
        want = torch.zeros((chunk, ny, nx), device="cuda", dtype=torch.float64)
        for m, a in MODES:
            want += a * factor(n, m) ** steps * torch.cos(phase(torch, n, m, zs, torch.float64))
        worst = max(worst, float((got[z0:z0 + chunk].double() - want).abs().max()))
        del want
    scale = sum(a for _, a in MODES)
    say("max |psi - closed form| / (a1 + a2) = %.3e (bar %.0e); A1^n = %.6f, A2^n = %.6f"
        % (worst / scale, tol, factor(n, MODES[0][0]) ** steps, factor(n, MODES[1][0]) ** steps))
    del got
    torch.cuda.empty_cache()
    assert np.isfinite(worst) and worst <= tol * scale
