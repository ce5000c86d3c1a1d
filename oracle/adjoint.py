"""Discrete adjoint of the Gray-Scott ETD1 spectral map, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY.

The paper has no adjoint; this is the exact transpose of the forward map
implemented in ``spectral.step_n`` (Sec. 2.4.2, Eqs. 3-4) for the
two-field Gray-Scott model, derived by hand:

  forward   q_j^{n+1} = Acal_j q_j^n + Bcal_j g_j(q^n; theta)
            Acal_j = IFFT diag(A_j) FFT,  Bcal_j = IFFT diag(B_j) FFT,
            g_u = F - u v^2,  g_v = u v^2   (N = 1 for both fields).
  A_j and B_j are real and even in k, so Acal_j and Bcal_j are symmetric.

  misfit    J = 1/2 sum_cells (v^T - v*)^2
  backward  lambda^T = (0, v^T - v*);  for n = T-1 .. 0:
              mu_j      = Bcal_j lambda_j^{n+1}
              lambda_u^n = Acal_u lambda_u^{n+1} - v^2 mu_u + v^2 mu_v
              lambda_v^n = Acal_v lambda_v^{n+1} - 2uv mu_u + 2uv mu_v
            (u, v at level n), and for each coefficient theta
              dJ/dtheta += sum_j < lambda_j^{n+1}, dAcal_j/dtheta q_j^n
                                                + dBcal_j/dtheta g_j^n >
                         + sum_j < mu_j, dg_j/dtheta >.
            dJ/du^0 = lambda_u^0, dJ/dv^0 = lambda_v^0.
  dA/dL = dt A;  dB/dL = dt^2 phi1'(z), phi1'(z) = (z e^z - e^z + 1)/z^2.

Checkpointing: states are kept at steps 0, K, 2K, ...; each segment is
recomputed forward from its checkpoint before it is swept backwards.
"""
from __future__ import annotations

import numpy as np

from . import spectral


def dphi1(z):
    """Derivative of phi1(z) = (e^z - 1)/z: (z e^z - expm1(z)) / z^2.

    Taylor series 1/2 + z/3 + z^2/8 + z^3/30 + z^4/144 for |z| < 1e-3.
    """
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-3
    zs = z[small]
    out[small] = 0.5 + zs / 3.0 + zs ** 2 / 8.0 + zs ** 3 / 30.0 + zs ** 4 / 144.0
    zb = z[~small]
    out[~small] = (zb * np.exp(zb) - np.expm1(zb)) / zb ** 2
    return out


def _apply(sym, f):
    """IFFT(sym * FFT(f)), real part (sym real and even in k)."""
    return np.real(np.fft.ifftn(sym * np.fft.fftn(f)))


def gray_scott_misfit_grad(u0, v0, coef, dt, dx, nsteps, vstar, K=1):
    """J and its gradient w.r.t. (u0, v0) and (Du, Dv, F, k).

    Returns dict with keys J, uT, vT, du0, dv0, dcoef (array of 4).
    """
    du_, dv_, F, kk = [float(c) for c in coef]
    u0 = np.asarray(u0, dtype=np.float64)
    v0 = np.asarray(v0, dtype=np.float64)
    k2 = spectral.wavenumber_sq(u0.shape, dx)
    Lu = -du_ * k2 - F
    Lv = -dv_ * k2 - (F + kk)
    Au, Bu = spectral.etd1_factors(Lu, dt)
    Av, Bv = spectral.etd1_factors(Lv, dt)
    dAu, dBu = dt * Au, dt * dt * dphi1(Lu * dt)     # d/dL_u
    dAv, dBv = dt * Av, dt * dt * dphi1(Lv * dt)     # d/dL_v

    def step(q):
        return spectral.step_n(q, "gray_scott", coef, dt, dx, 1)

    K = max(1, int(K))
    ckpt = {0: (u0, v0)}
    q = (u0, v0)
    for n in range(nsteps):
        q = tuple(step(q))
        if (n + 1) % K == 0 and n + 1 < nsteps:
            ckpt[n + 1] = q
    uT, vT = q
    r = vT - vstar
    J = 0.5 * float(np.sum(r * r))

    lam_u = np.zeros_like(u0)
    lam_v = r.copy()
    g = np.zeros(4)              # dJ/d(Du, Dv, F, k)
    seg_starts = list(range(0, nsteps, K))
    for s0 in reversed(seg_starts):
        s1 = min(s0 + K, nsteps)
        states = [ckpt[s0]]
        for _ in range(s0, s1 - 1):
            states.append(tuple(step(states[-1])))
        for n in reversed(range(s0, s1)):
            u, v = states[n - s0]
            gu = F - u * v * v
            gv = u * v * v
            mu_u = _apply(Bu, lam_u)
            mu_v = _apply(Bv, lam_v)
            # derivatives of the linear parts with respect to L_j, applied
            # to the level-n state and nonlinear term
            Tu = _apply(dAu, u) + _apply(dBu, gu)
            Tv = _apply(dAv, v) + _apply(dBv, gv)
            Tu_k2 = _apply(-k2 * dAu, u) + _apply(-k2 * dBu, gu)
            Tv_k2 = _apply(-k2 * dAv, v) + _apply(-k2 * dBv, gv)
            g[0] += np.sum(lam_u * Tu_k2)                  # dL_u/dDu = -k^2
            g[1] += np.sum(lam_v * Tv_k2)                  # dL_v/dDv = -k^2
            g[2] += -np.sum(lam_u * Tu) - np.sum(lam_v * Tv) + np.sum(mu_u)
            g[3] += -np.sum(lam_v * Tv)                    # dL_v/dk = -1
            new_u = _apply(Au, lam_u) - v * v * mu_u + v * v * mu_v
            new_v = _apply(Av, lam_v) - 2.0 * u * v * mu_u + 2.0 * u * v * mu_v
            lam_u, lam_v = new_u, new_v
    return {"J": J, "uT": uT, "vT": vT, "du0": lam_u, "dv0": lam_v,
            "dcoef": g}


def gray_scott_misfit(u0, v0, coef, dt, dx, nsteps, vstar):
    """J = 1/2 sum (v^T - v*)^2 from the forward map alone."""
    uT, vT = spectral.step_n([u0, v0], "gray_scott", coef, dt, dx, nsteps)
    r = vT - vstar
    return 0.5 * float(np.sum(r * r))
