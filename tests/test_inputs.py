"""Seeded input generator: published test vector and recipe shapes."""
import os

import numpy as np

from paper_2109_02598_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_vector():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    got = [int(v) for v in inputs.splitmix64(0, len(want))]
    assert got == want


def test_offset_continues_stream():
    a = inputs.splitmix64(123, 10)
    b = inputs.splitmix64(123, 4, offset=6)
    assert np.array_equal(a[6:], b)


def test_uniform_range_and_layout():
    f = inputs.uniform_field(2, (4, 8), -0.05, 0.05)
    assert f.shape == (4, 8) and f.flags.c_contiguous
    assert f.min() >= -0.05 and f.max() < 0.05
    flat = inputs.uniform(2, 32, -0.05, 0.05)
    assert np.array_equal(f.ravel(), flat)      # x fastest


def test_recipes():
    w = inputs.allen_cahn_2d()
    assert w.fields[0].shape == (128, 128) and w.dt == 0.5
    g = inputs.gray_scott_2d(n=64, npatch=3, patch=4)
    u, v = g.fields
    assert np.all(u == 1.0) and np.count_nonzero(v) <= 3 * 16 and v.max() == 0.25
    b = inputs.cahn_hilliard_batch(count=8)
    assert all(x.n[0] in inputs.BATCH_SIZES for x in b)
    assert all(0.5 <= x.coef[0] < 2.0 and 0.5 <= x.coef[1] < 2.0 for x in b)
