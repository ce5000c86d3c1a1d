"""Radially averaged structure factor, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.

What is computed (Sec. 3, coarsening check, with Porod's law Eq. 14):
  * the occupancy field rho = 1 where psi > 0 and 0 elsewhere (the
    positive phase stands for the solid);
  * its discrete Fourier transform rho_hat (unnormalised, every axis);
  * the structure factor S(k) = |rho_hat_k|^2, here divided by the cell
    count N so that sum_k S(k) equals the number of occupied cells;
  * the radial average: modes are binned by b = floor(|m| + 1/2), |m| the
    length of the integer mode vector (m_j in -N_j/2 .. N_j/2 - 1); a bin's
    value is the mean of S over its modes.

Readings (listed in the design notes): the text defines S through the
occupancy rho, a figure caption writes |psi_hat|^2 -- the text is
followed; the box must have the same length along every axis so that |k|
is 2 pi |m| / L and the integer |m| bins are radial shells; the 1/N
normalisation is a convention (Porod's law fixes only the k dependence).
"""
from __future__ import annotations

import numpy as np


def occupancy(psi):
    """rho = [psi > 0] as float64 (Sec. 3)."""
    return (np.asarray(psi) > 0).astype(np.float64)


def mode_norm_sq(shape):
    """Integer |m|^2 of every DFT mode of an array of this shape (numpy
    axis order), m_j in the DFT frequency order of each axis."""
    grids = np.meshgrid(*[np.fft.fftfreq(n, d=1.0 / n) for n in shape], indexing="ij")
    m2 = np.zeros(shape, dtype=np.int64)
    for g in grids:
        gi = np.rint(g).astype(np.int64)
        m2 += gi * gi
    return m2


def radial_bin(m2):
    """b = floor(sqrt(m2) + 1/2) for integer m2 (exact: sqrt(m2) is never
    within 1e-5 of a half-integer for the sizes used, far above FP64
    rounding)."""
    return np.floor(np.sqrt(m2.astype(np.float64)) + 0.5).astype(np.int64)


def nbins(shape):
    """Number of radial bins: one past the largest bin of any mode."""
    return int(radial_bin(np.array([sum((n // 2) ** 2 for n in shape)]))[0]) + 1


def structure_factor(psi):
    """Return (S_bins, counts): the mean of |rho_hat|^2 / N over the modes
    of each radial bin (0 where a bin has no mode) and the number of modes
    per bin.  psi: real array in numpy axis order (z, y, x)."""
    psi = np.asarray(psi, dtype=np.float64)
    rho = occupancy(psi)
    n_cells = rho.size
    s = np.abs(np.fft.fftn(rho)) ** 2 / n_cells
    b = radial_bin(mode_norm_sq(psi.shape)).ravel()
    nb = nbins(psi.shape)
    sums = np.bincount(b, weights=s.ravel(), minlength=nb)
    counts = np.bincount(b, minlength=nb).astype(np.int64)
    avg = np.where(counts > 0, sums / np.maximum(counts, 1), 0.0)
    return avg, counts


def porod_slope(s_bins, counts, kmin, kmax):
    """Least-squares slope of log S against log |m| over bins kmin..kmax
    (Porod's law, Eq. 14, predicts -(d + 1) in the scaling regime)."""
    b = np.arange(len(s_bins))
    sel = (b >= kmin) & (b <= kmax) & (counts > 0) & (s_bins > 0)
    x = np.log(b[sel].astype(np.float64))
    y = np.log(s_bins[sel])
    return float(np.polyfit(x, y, 1)[0])
