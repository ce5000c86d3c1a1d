"""ETD1 semi-implicit Fourier spectral scheme, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.

What is computed (Sec. 2.4.2):
  * the equation of motion is split into a linear operator applied to
    the field and linear operators N_i applied to nonlinear functions
    f_i of the fields (Eq. 1);
  * in Fourier space each mode obeys a linear ODE with forcing
    (Eq. 2), with the derivative symbols grad -> i k, lap -> -|k|^2;
  * one time step is psi_hat <- A psi_hat + B sum_i N_i f_i_hat with
    A = exp(L dt) and B = (exp(L dt) - 1)/L (Eqs. 3-4, and the update
    rule Eq. 8).

Readings taken where the paper is silent (each one is listed in the
design notes):
  * B is evaluated as dt * expm1(z)/z with z = L dt, and B = dt where
    L = 0 (the limit of Eq. 4);
  * every term linear in a field, zeroth-order terms included, belongs
    to L; constant sources ride with the nonlinear term (Gray-Scott's F);
  * the symbol of the Laplacian is the continuous -|k|^2 with
    k_j = 2 pi m_j / (N_j dx_j); no dealiasing;
  * forward FFT unnormalised, inverse scaled by 1/N;
  * with several fields all nonlinear terms use the fields of the
    current step (the equation()/step() split of Sec. 2.2.4);
  * the state is carried in real space between steps.
"""
from __future__ import annotations

import numpy as np

# Coefficient vectors (four doubles per model, five for model C):
#   allen_cahn    (M, kappa, c1, c2)  d psi/dt = M (kappa lap psi + c1 psi - c2 psi^3)
#   cahn_hilliard (M, kappa, c1, c2)  d psi/dt = M lap (c2 psi^3 - c1 psi - kappa lap psi)
#   pfc           (r, q0, g2, g3)     d psi/dt = lap [ (r + (q0^2 + lap)^2) psi + g2 psi^2 + g3 psi^3 ]
#   gray_scott    (Du, Dv, F, k)      u_t = Du lap u - u v^2 + F (1 - u)
#                                     v_t = Dv lap v + u v^2 - (F + k) v
#   model_c       (c1, c2, c3, c4, c5)
#                 psi_t = lap psi + c1 psi - c2 psi^3 + 2 c5 psi m
#                 m_t   = -lap^2 m - lap (c3 m - c4 m^3 + c5 psi^2)
NCOEF = {"allen_cahn": 4, "cahn_hilliard": 4, "pfc": 4, "gray_scott": 4,
         "model_c": 5}
NFIELDS = {"allen_cahn": 1, "cahn_hilliard": 1, "pfc": 1, "gray_scott": 2,
           "model_c": 2}


def wavenumber_sq(shape, dx):
    """|k|^2 on the unshifted FFT grid of an array of ``shape`` (..., y, x).

    ``dx`` is the spacing per axis in (x, y[, z]) order.  Sec. 2.4.2:
    lap -> -|k|^2 with k_j = 2 pi m_j / (N_j dx_j).
    """
    shape = tuple(shape)
    dxs = tuple(reversed(tuple(dx)))          # array-axis order
    k2 = np.zeros(shape)
    for ax, (n, h) in enumerate(zip(shape, dxs)):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
        sl = [None] * len(shape)
        sl[ax] = slice(None)
        k2 = k2 + (k ** 2)[tuple(sl)]
    return k2


def symbols(model, coef, k2):
    """Linear symbol L(k) and nonlinear terms [(N_i(k), f_i)] per field.

    This is the split of Eq. 1 into L{psi} + sum_i N_i{f_i(psi)}, written
    out by hand for each model of Sec. 3 (Eqs. 9, 10, 11-12, 13) and for
    Gray-Scott.  Each f_i takes the list of all fields at the current step.
    """
    c = [float(v) for v in coef]
    if len(c) != NCOEF[model]:
        raise ValueError("%s takes %d coefficients" % (model, NCOEF[model]))
    one = np.ones_like(k2)
    if model == "allen_cahn":
        M, kap, c1, c2 = c
        L = M * (c1 - kap * k2)
        return [(L, [(-M * c2 * one, lambda q: q[0] ** 3)])]
    if model == "cahn_hilliard":
        M, kap, c1, c2 = c
        L = M * (c1 * k2 - kap * k2 ** 2)
        return [(L, [(-M * c2 * k2, lambda q: q[0] ** 3)])]
    if model == "pfc":
        r, q0, g2, g3 = c
        L = -k2 * (r + (q0 ** 2 - k2) ** 2)
        return [(L, [(-k2, lambda q: g2 * q[0] ** 2 + g3 * q[0] ** 3)])]
    if model == "gray_scott":
        du, dv, F, kk = c
        Lu = -du * k2 - F
        Lv = -dv * k2 - (F + kk)
        return [(Lu, [(one, lambda q: F - q[0] * q[1] ** 2)]),
                (Lv, [(one, lambda q: q[0] * q[1] ** 2)])]
    if model == "model_c":
        c1, c2, c3, c4, c5 = c
        Lp = c1 - k2
        Lm = c3 * k2 - k2 ** 2
        return [(Lp, [(one, lambda q: -c2 * q[0] ** 3 + 2.0 * c5 * q[0] * q[1])]),
                (Lm, [(k2.copy(), lambda q: -c4 * q[1] ** 3 + c5 * q[0] ** 2)])]
    raise ValueError("unknown model %r" % (model,))


def phi1(z):
    """(exp(z) - 1)/z with the limit 1 at z = 0 (B of Eq. 4 is dt*phi1(L dt))."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def etd1_factors(L, dt):
    """A = exp(L dt) and B = (exp(L dt) - 1)/L (Eq. 4), B = dt where L = 0."""
    z = L * dt
    return np.exp(z), dt * phi1(z)


def _default_fft():
    return np.fft.fftn, np.fft.ifftn


def step_n(fields, model, coef, dt, dx, nsteps, fft=None, mass_log=None,
           check_hermitian=True):
    """Advance ``fields`` by ``nsteps`` ETD1 spectral steps; returns new fields.

    One step (Eq. 3 / Eq. 8): for every field j,
        psi_j_hat' = A_j psi_j_hat + B_j sum_i N_ij FFT(f_ij(psi^n)),
        psi_j'     = IFFT(psi_j_hat').
    ``fft`` optionally replaces (forward, inverse) transforms (the pin
    against a naive DFT uses it).  If ``mass_log`` is a list, the mean of
    every field after each step is appended to it.
    """
    fwd, inv = fft or _default_fft()
    q = [np.array(f, dtype=np.float64, copy=True) for f in fields]
    if len(q) != NFIELDS[model]:
        raise ValueError("%s has %d fields" % (model, NFIELDS[model]))
    k2 = wavenumber_sq(q[0].shape, dx)
    tables = []
    for L, terms in symbols(model, coef, k2):
        A, B = etd1_factors(L, dt)
        tables.append((A, [(B * Nk, f) for Nk, f in terms]))
    for _ in range(int(nsteps)):
        new = []
        for j, (A, terms) in enumerate(tables):
            acc = A * fwd(q[j])
            for BN, f in terms:
                acc = acc + BN * fwd(f(q))
            r = inv(acc)
            if check_hermitian:
                scale = max(float(np.max(np.abs(r.real))),
                            float(np.max(np.abs(q[j]))), 1e-300)
                if float(np.max(np.abs(r.imag))) > 1e-10 * scale:
                    raise AssertionError("inverse transform not real")
            new.append(np.ascontiguousarray(r.real))
        q = new
        if mass_log is not None:
            mass_log.append([float(np.mean(f)) for f in q])
    return q

