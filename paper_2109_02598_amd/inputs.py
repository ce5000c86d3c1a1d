"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the spectral method: it only draws
random numbers and lays them out as fields.  Both the CPU oracle tests
and the GPU tests take their inputs from here, so the two sides see
bit-identical initial data.

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  State advances by the
golden-gamma constant; each output is the state passed through the
published 64-bit finaliser.  A uniform double in [0, 1) is the top 53
bits of an output times 2**-53.  Values are assigned in flat order of
a C-contiguous array whose last axis is x (x fastest), field 0 first.

The paper's runs start from uniform noise (Sec. 3: initial conditions
of models A, B and C are uniformly distributed noise); the recipes
below reproduce that structure at the sizes of each workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs ``offset .. offset+count-1`` of the SplitMix64 stream of ``seed``.

    Output i is mix(seed + (i+1)*gamma) (all arithmetic mod 2**64).
    """
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, lo: float = 0.0, hi: float = 1.0,
            offset: int = 0) -> np.ndarray:
    """``count`` doubles lo + (hi-lo)*u with u = (x >> 11) * 2**-53."""
    u = (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64)
    u *= 2.0 ** -53
    return lo + (hi - lo) * u


def uniform_field(seed: int, shape, lo: float, hi: float,
                  offset: int = 0) -> np.ndarray:
    """C-contiguous float64 array of ``shape`` (.., y, x) filled x-fastest."""
    n = int(np.prod(shape))
    return uniform(seed, n, lo, hi, offset).reshape(shape)


# ---------------------------------------------------------------------------
# Workload recipes.  Sizes are given as (nx, ny[, nz]); arrays are shaped
# (nz, ny, nx) / (ny, nx).
# ---------------------------------------------------------------------------

MODEL_IDS = {"allen_cahn": 1, "cahn_hilliard": 2, "pfc": 3, "gray_scott": 4,
             "model_c": 5}
NFIELDS = {"allen_cahn": 1, "cahn_hilliard": 1, "pfc": 1, "gray_scott": 2,
           "model_c": 2}


@dataclass
class Workload:
    """One simulation: grid, model, coefficients, time step and fields."""
    name: str
    model: str
    n: tuple            # (nx, ny[, nz])
    dx: tuple           # spacing per axis, same order as n
    dt: float
    coef: tuple
    steps: int
    fields: list = field(default_factory=list)   # float64 arrays (..., y, x)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def cells(self):
        return int(np.prod(self.n))


def allen_cahn_2d(n=128, seed=1, steps=100) -> Workload:
    """2D Allen-Cahn, dx=1, dt=0.5, M=kappa=c1=c2=1, phi ~ U[-0.1, 0.1)."""
    shape = (n, n)
    return Workload("allen_cahn_%dx%d" % (n, n), "allen_cahn", (n, n),
                    (1.0, 1.0), 0.5, (1.0, 1.0, 1.0, 1.0), steps,
                    [uniform_field(seed, shape, -0.1, 0.1)])


def model_c_2d(n=512, seed=8, steps=100) -> Workload:
    """2D Model C (psi non-conserved, m conserved), dx=1, dt=0.05,
    c1..c5 = 1, both fields ~ U[-0.1, 0.1) (field 1 from seed + 1)."""
    shape = (n, n)
    return Workload("model_c_%dx%d" % (n, n), "model_c", (n, n), (1.0, 1.0), 0.05,
                    (1.0, 1.0, 1.0, 1.0, 1.0), steps,
                    [uniform_field(seed, shape, -0.1, 0.1), uniform_field(seed + 1, shape, -0.1, 0.1)])


def cahn_hilliard_2d(n=2048, seed=2, steps=1000) -> Workload:
    """2D Cahn-Hilliard, dx=1, dt=0.1, M=kappa=c1=c2=1, phi ~ U[-0.05, 0.05).

    The noise is not re-centred: conservation is judged against the mean
    of the sample itself.
    """
    shape = (n, n)
    return Workload("cahn_hilliard_%dx%d" % (n, n), "cahn_hilliard", (n, n),
                    (1.0, 1.0), 0.1, (1.0, 1.0, 1.0, 1.0), steps,
                    [uniform_field(seed, shape, -0.05, 0.05)])


def cahn_hilliard_3d(n=256, seed=9, steps=500) -> Workload:
    """3D Cahn-Hilliard, dx=1, dt=0.01, M=kappa=c1=c2=1, phi ~ U[-0.05, 0.05)
    (the forward-Euler solver's 3D case)."""
    shape = (n, n, n)
    return Workload("cahn_hilliard_%d^3" % n, "cahn_hilliard", (n, n, n),
                    (1.0, 1.0, 1.0), 0.01, (1.0, 1.0, 1.0, 1.0), steps,
                    [uniform_field(seed, shape, -0.05, 0.05)])


def pfc_3d(n=256, seed=3, steps=500) -> Workload:
    """3D phase-field crystal, dx=pi/4, dt=0.5, r=-0.25, q0=1, g2=0, g3=1.

    psi = -0.285 + U[-0.05, 0.05).
    """
    shape = (n, n, n)
    h = math.pi / 4
    return Workload("pfc_%d^3" % n, "pfc", (n, n, n), (h, h, h), 0.5,
                    (-0.25, 1.0, 0.0, 1.0), steps,
                    [-0.285 + uniform_field(seed, shape, -0.05, 0.05)])


def gray_scott_2d(n=512, patch_seed=5, npatch=20, patch=16,
                  steps=200) -> Workload:
    """2D Gray-Scott, Du=0.16, Dv=0.08, F=0.035, k=0.065, dx=1, dt=1.

    u = 1, v = 0 except inside ``npatch`` square patches of side ``patch``
    whose lower corner (x0, y0) = floor(n*U) each (two draws per patch,
    x first), wrapped periodically; inside a patch v = 0.25, u stays 1.
    """
    u = np.ones((n, n))
    v = np.zeros((n, n))
    corners = uniform(patch_seed, 2 * npatch)
    for p in range(npatch):
        x0 = int(math.floor(n * corners[2 * p]))
        y0 = int(math.floor(n * corners[2 * p + 1]))
        ys = (y0 + np.arange(patch)) % n
        xs = (x0 + np.arange(patch)) % n
        v[np.ix_(ys, xs)] = 0.25
    return Workload("gray_scott_%dx%d" % (n, n), "gray_scott", (n, n),
                    (1.0, 1.0), 1.0, (0.16, 0.08, 0.035, 0.065), steps, [u, v])


def gray_scott_target(n=512, seed=6) -> np.ndarray:
    """Target field v* ~ U[0, 0.5) for the Gray-Scott misfit."""
    return uniform_field(seed, (n, n), 0.0, 0.5)


BATCH_SIZES = (128, 256, 512, 1024)


def cahn_hilliard_batch(count=64, seed=4, steps=500, sizes=BATCH_SIZES,
                        field_seed_base=4000) -> list:
    """``count`` independent 2D Cahn-Hilliard runs of uneven size.

    Per simulation i, three draws from stream ``seed``: size index
    floor(4U), then M ~ U[0.5, 2), then kappa ~ U[0.5, 2).  Fields are
    U[-0.05, 0.05) from seed field_seed_base+i; dx=1, dt=0.1, c1=c2=1.
    """
    draws = uniform(seed, 3 * count)
    out = []
    for i in range(count):
        n = sizes[int(math.floor(len(sizes) * draws[3 * i]))]
        m = 0.5 + 1.5 * draws[3 * i + 1]
        kap = 0.5 + 1.5 * draws[3 * i + 2]
        out.append(Workload("ch_batch_%d_%d" % (i, n), "cahn_hilliard", (n, n),
                            (1.0, 1.0), 0.1, (m, kap, 1.0, 1.0), steps,
                            [uniform_field(field_seed_base + i, (n, n),
                                           -0.05, 0.05)]))
    return out


def smooth_modes(shape, dx, seed, amp=0.1, mmax=3, offset=0.0) -> np.ndarray:
    """Band-limited field: a few seeded Fourier modes with |m_j| <= mmax.

    Used where a smooth initial condition is needed (cross-checks against
    an independent finite-difference discretisation).  ``shape`` is
    (..., y, x) and ``dx`` is (dx, dy[, dz]).
    """
    nd = len(shape)
    axes = [np.arange(s) * d for s, d in zip(shape, reversed(dx))]
    grids = np.meshgrid(*axes, indexing="ij")
    lengths = [s * d for s, d in zip(shape, reversed(dx))]
    r = uniform(seed, 8 * (nd + 2))
    f = np.full(shape, float(offset))
    for t in range(8):
        ms = [int(math.floor((2 * mmax + 1) * r[t * (nd + 2) + a])) - mmax
              for a in range(nd)]
        phase = 2 * math.pi * r[t * (nd + 2) + nd]
        weight = amp * (r[t * (nd + 2) + nd + 1] - 0.5)
        arg = sum(2 * math.pi * m * g / ln for m, g, ln in zip(ms, grids, lengths))
        f += weight * np.cos(arg + phase)
    return f
