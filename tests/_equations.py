"""The fixed models (Sec. 3 equations of motion and Gray-Scott) written as
equation text for the run-time split, with the names of their coefficient
vectors; plus equations outside the fixed set."""

FIXED = {
    "allen_cahn": ("psi' = M*(kappa*lap(psi) + c1*psi - c2*psi^3)", ("M", "kappa", "c1", "c2")),
    "cahn_hilliard": ("psi' = M*lap(c2*psi^3 - c1*psi - kappa*lap(psi))", ("M", "kappa", "c1", "c2")),
    "pfc": ("psi' = lap((r + q0^4)*psi + 2*q0^2*lap(psi) + bilap(psi) + g2*psi^2 + g3*psi^3)",
            ("r", "q0", "g2", "g3")),
    "gray_scott": ("u' = Du*lap(u) - u*v^2 + F*(1 - u); v' = Dv*lap(v) + u*v^2 - (F + k)*v",
                   ("Du", "Dv", "F", "k")),
    "model_c": ("psi' = lap(psi) + c1*psi - c2*psi^3 + 2*c5*psi*m\n"
                "m' = -bilap(m) - lap(c3*m - c4*m^3 + c5*psi^2)", ("c1", "c2", "c3", "c4", "c5")),
}


def fixed(model, values):
    text, names = FIXED[model]
    return text, dict(zip(names, values))


# Swift-Hohenberg (non-conserved PFC): psi_t = r psi - (q0^2 + lap)^2 psi - psi^3
SWIFT_HOHENBERG = ("psi' = (r - q0^4)*psi - 2*q0^2*lap(psi) - bilap(psi) - psi^3", {"r": 0.3, "q0": 1.0})
# FitzHugh-Nagumo: terms linear in the other field are explicit (paired with
# the nonlinear term under the same derivative)
FITZHUGH_NAGUMO = ("u' = Du*lap(u) + u - u^3 - v; v' = Dv*lap(v) + eps*(u - a1*v - a0)",
                   {"Du": 1.0, "Dv": 4.0, "eps": 0.05, "a1": 2.0, "a0": -0.03})
# conserved form with a cubic-quartic free energy and a constant mobility
CONSERVED_QUARTIC = ("phi' = lap(0.5*phi^2 + phi^3 - 0.8*phi - 1.2*lap(phi))", {})
