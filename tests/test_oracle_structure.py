"""Pins of the structure-factor oracle (Sec. 3, radially averaged S(k) of
the occupancy rho = [psi > 0]) against what the definition and the
mathematics fix: a brute-force DFT with integer bin bounds, Parseval, the
k = 0 bin, the closed form of a sampled square wave, and invariances."""
import itertools

import numpy as np
import pytest

from oracle import structure as osf
from paper_2109_02598_amd import inputs


def brute(psi):
    """Direct O(N^2) DFT; bins by the integer test b^2 - b < m2 <= b^2 + b
    (the same rounding rule as floor(sqrt(m2) + 1/2), without sqrt)."""
    shape = psi.shape
    n = psi.size
    rho = [(1.0 if v > 0 else 0.0) for v in psi.ravel()]
    coords = list(itertools.product(*[range(s) for s in shape]))
    freqs = list(itertools.product(*[range(s) for s in shape]))
    nb = 2 + int(np.sqrt(sum((s // 2) ** 2 for s in shape)))
    sums = [0.0] * nb
    cnt = [0] * nb
    for f in freqs:
        acc = 0j
        for r, c in zip(rho, coords):
            if r:
                ph = sum(fj * cj / sj for fj, cj, sj in zip(f, c, shape))
                acc += np.exp(-2j * np.pi * ph)
        s = abs(acc) ** 2 / n
        m = [fj - sj if fj >= sj // 2 else fj for fj, sj in zip(f, shape)]
        m2 = sum(x * x for x in m)
        b = 0
        while not (b * b - b < m2 <= b * b + b) and m2 != 0:
            b += 1
        sums[b] += s
        cnt[b] += 1
    last = max(i for i, c in enumerate(cnt) if c)
    sums, cnt = sums[: last + 1], cnt[: last + 1]
    avg = [s / c if c else 0.0 for s, c in zip(sums, cnt)]
    return np.array(avg), np.array(cnt)


@pytest.mark.parametrize("shape,seed", [((6, 8), 11), ((8, 8), 12), ((4, 4, 6), 13)])
def test_brute_force_dft(shape, seed):
    psi = inputs.uniform_field(seed, shape, -1.0, 1.0)
    got, cnt = osf.structure_factor(psi)
    ref, rcnt = brute(psi)
    assert len(got) == len(ref) == osf.nbins(shape)
    assert np.array_equal(cnt, rcnt)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_parseval_and_k0():
    psi = inputs.uniform_field(21, (64, 48), -1.0, 1.0)
    s, c = osf.structure_factor(psi)
    npos = int((psi > 0).sum())
    # sum over modes of |rho_hat|^2 / N = sum over cells of rho^2 = npos
    assert abs(float(np.sum(s * c)) - npos) <= 1e-9 * npos
    # bin 0 holds only m = 0, where rho_hat = npos
    assert c[0] == 1
    assert abs(s[0] - npos ** 2 / psi.size) <= 1e-12 * s[0]
    assert int(c.sum()) == psi.size


def test_exact_zeros_are_empty_cells():
    """rho = [psi > 0]: cells where psi is exactly 0 are not occupied (the
    k = 0 bin counts the cells with psi > 0 only)."""
    psi = np.zeros((8, 12))
    psi[1, 2] = psi[3, 7] = psi[6, 1] = 0.5            # three occupied cells
    psi[2, 2] = psi[5, 5] = -0.25
    s, c = osf.structure_factor(psi)
    assert c[0] == 1 and s[0] == 3 ** 2 / psi.size
    assert abs(float(np.sum(s * c)) - 3.0) <= 1e-12


def test_sampled_square_wave_closed_form():
    """psi = cos(pi (x + 1/2) / 8) on 64 x 64: rho is a square wave of
    period 16 (8 ones), constant along y.  Its DFT is nonzero only at
    (mx, 0) with mx = 4h: |rho_hat| = 64 * 4 / |sin(pi h / 16)| for odd h,
    N/2 for h = 0, 0 for even h != 0 (a geometric sum)."""
    ny = nx = 64
    x = np.arange(nx)
    psi = np.tile(np.cos(np.pi * (x + 0.5) / 8.0), (ny, 1))
    s, c = osf.structure_factor(psi)
    n = nx * ny
    expect = np.zeros(len(s))
    for h in range(-8, 8):
        m = 4 * h
        if h == 0:
            amp = n / 2
        elif h % 2:
            amp = ny * 4 / abs(np.sin(np.pi * h / 16))
        else:
            amp = 0.0
        b = int(np.floor(abs(m) + 0.5))
        expect[b] += amp * amp / n
    # counts by brute force over the integer lattice of the grid's modes
    cnt = np.zeros(len(s), dtype=np.int64)
    for my in range(-32, 32):
        for mx in range(-32, 32):
            m2 = mx * mx + my * my
            b = 0
            while m2 and not (b * b - b < m2 <= b * b + b):
                b += 1
            cnt[b] += 1
    assert np.array_equal(c, cnt)
    np.testing.assert_allclose(s, expect / np.maximum(cnt, 1), rtol=1e-12, atol=1e-9)


def test_invariances():
    psi = inputs.uniform_field(31, (32, 32), -1.0, 1.0)
    s0, c0 = osf.structure_factor(psi)
    s1, _ = osf.structure_factor(np.roll(psi, (5, -7), axis=(0, 1)))
    s2, _ = osf.structure_factor(psi.T)
    s3, _ = osf.structure_factor(psi[::-1, :])
    for s in (s1, s2, s3):
        np.testing.assert_allclose(s, s0, rtol=1e-12, atol=1e-12)
    # all cells occupied: only k = 0 survives, S(0) = N
    s4, _ = osf.structure_factor(np.ones((16, 16)))
    assert abs(s4[0] - 256.0) < 1e-12 and np.all(np.abs(s4[1:]) < 1e-20)


def test_porod_slope_of_a_power_law():
    s = np.array([0.0] + [b ** -3.0 for b in range(1, 40)])
    c = np.ones(40, dtype=np.int64)
    assert abs(osf.porod_slope(s, c, 4, 30) + 3.0) < 1e-12
