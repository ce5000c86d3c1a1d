"""Mutation check of the oracle's pins: each plausible mistake below (a
flipped sign, a dropped or misplaced term, a transposed operand, a wrong
power, factor or stencil weight), planted in a copy of the oracle inside a
temporary directory, makes the oracle's own tests fail.  The repository's
oracle is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the oracle's tests, the ones that exercise a file first
PIN_FILES = {
    "spectral.py": ["tests/test_oracle_pins.py", "tests/test_oracle_split.py", "tests/test_oracle_adjoint.py",
                    "tests/test_oracle_structure.py"],
    "fd_euler.py": ["tests/test_oracle_fd.py", "tests/test_oracle_pins.py"],
    "adjoint.py": ["tests/test_oracle_adjoint.py"],
    "structure.py": ["tests/test_oracle_structure.py"],
    "operator_split.py": ["tests/test_oracle_split.py"],
}

MUTATIONS = [
    # AC: sign of the cubic term
    ("spectral.py", "-M * c2 * one", "M * c2 * one"),
    # AC: sign in L
    ("spectral.py", "M * (c1 - kap * k2)", "M * (c1 + kap * k2)"),
    # CH: derivative dropped
    ("spectral.py", "-M * c2 * k2, lambda", "-M * c2 * one, lambda"),
    # CH: wrong power in L
    ("spectral.py", "kap * k2 ** 2", "kap * k2"),
    # PFC: quadratic term dropped
    ("spectral.py", "g2 * q[0] ** 2 + g3 * q[0] ** 3", "g3 * q[0] ** 3"),
    # PFC: q0 not squared
    ("spectral.py", "(q0 ** 2 - k2) ** 2", "(q0 - k2) ** 2"),
    # PFC: sign in L
    ("spectral.py", "L = -k2 * (r + (q0 ** 2 - k2) ** 2)", "L = -k2 * (r - (q0 ** 2 - k2) ** 2)"),
    # GS: operands transposed
    ("spectral.py", "F - q[0] * q[1] ** 2", "F - q[0] ** 2 * q[1]"),
    # GS: F dropped from L_v
    ("spectral.py", "Lv = -dv * k2 - (F + kk)", "Lv = -dv * k2 - kk"),
    # GS: wrong diffusivity
    ("spectral.py", "Lu = -du * k2 - F", "Lu = -dv * k2 - F"),
    # Model C: factor 2 dropped
    ("spectral.py", "2.0 * c5 * q[0] * q[1]", "c5 * q[0] * q[1]"),
    # Model C: sign in L_psi
    ("spectral.py", "Lp = c1 - k2", "Lp = c1 + k2"),
    # Model C: sign in L_m
    ("spectral.py", "Lm = c3 * k2 - k2 ** 2", "Lm = c3 * k2 + k2 ** 2"),
    # Model C: lap of N_m dropped
    ("spectral.py", "(k2.copy(), lambda", "(one, lambda"),
    # Model C: wrong field
    ("spectral.py", "c5 * q[0] ** 2)", "c5 * q[1] ** 2)"),
    # Model C: wrong field
    ("spectral.py", "-c4 * q[1] ** 3", "-c4 * q[0] ** 3"),
    # phi1 not divided by z
    ("spectral.py", "np.expm1(z[nz]) / z[nz]", "np.expm1(z[nz])"),
    # B = dt (explicit Euler)
    ("spectral.py", "return np.exp(z), dt * phi1(z)", "return np.exp(z), dt"),
    # A dropped
    ("spectral.py", "acc = A * fwd(q[j])", "acc = fwd(q[j])"),
    # wavenumbers halved
    ("spectral.py", "2.0 * np.pi * np.fft.fftfreq(n, d=h)", "np.pi * np.fft.fftfreq(n, d=h)"),
    # spacings in the wrong order
    ("spectral.py", "dxs = tuple(reversed(tuple(dx)))", "dxs = tuple(dx)"),
    # finite differences (zero-sum kept where a weight moves: the mistake
    # survives the k = 0 checks and must be caught by the symbol and order)
    # 4th order, one side
    ("fd_euler.py", "16.0 * np.roll(f, 1, axis=ax)", "15.0 * np.roll(f, 1, axis=ax)"),
    ("fd_euler.py", "(4.0 * ring(1, 0) + ring(1, 1) - 20.0 * f) / (6.0 * h * h)",
     "(4.0 * ring(1, 0) + 2.0 * ring(1, 1) - 24.0 * f) / (6.0 * h * h)"),             # 9-point weights
    ("fd_euler.py", "3.0 * ring(1, 1, 0) + ring(1, 1, 1) - 128.0 * f",
     "2.0 * ring(1, 1, 0) + ring(1, 1, 1) - 116.0 * f"),                               # 27-point weights
    ("fd_euler.py", "(4.0 * ring(1, 1, 0) - ring(1, 1, 1) - 40.0 * f)",
     "(4.0 * ring(1, 1, 0) + ring(1, 1, 1) - 56.0 * f)"),                              # 21-point (3D) sign
    # 17-point
    ("fd_euler.py", "- 8.0 * ring(2, 0) - ring(2, 2)", "- 7.0 * ring(2, 0) - 5.0 * ring(2, 2)"),
    ("fd_euler.py", "16.0 * ring(1, 1) - ring(2, 0) - 2.0 * ring(1, 2)",
     "16.0 * ring(1, 1) - 2.0 * ring(2, 0) - 1.5 * ring(1, 2)"),                       # 21-point (2D)
    ("fd_euler.py", "M * (kap * lap(p) + c1 * p - c2 * p ** 3)", "M * (kap * lap(p) - c1 * p - c2 * p ** 3)"),
    ("fd_euler.py", "F * (1.0 - u)", "F * (1.0 + u)"),
    ("fd_euler.py", "2.0 * q0 ** 2 * lp", "q0 ** 2 * lp"),
    ("fd_euler.py", "+ 2.0 * c5 * p * m,", "+ c5 * p * m,"),
    # reverse mode: Jacobian transpose, coefficient sums, phi1 derivative
    ("adjoint.py", "- 2.0 * u * v * mu_u + 2.0 * u * v * mu_v", "- 2.0 * u * v * mu_u + u * v * mu_v"),
    ("adjoint.py", "- v * v * mu_u + v * v * mu_v", "- v * v * mu_u - v * v * mu_v"),
    ("adjoint.py", "+ np.sum(mu_u)", "- np.sum(mu_u)"),
    ("adjoint.py", "g[3] += -np.sum(lam_v * Tv)", "g[3] += -np.sum(lam_u * Tu)"),
    ("adjoint.py", "dt * dt * dphi1(Lu * dt)", "dt * dphi1(Lu * dt)"),
    ("adjoint.py", "_apply(Au, lam_u) -", "_apply(Av, lam_u) -"),
    # structure factor: threshold, normalisation, binning, integer modes
    ("structure.py", "return (np.asarray(psi) > 0).astype", "return (np.asarray(psi) >= 0).astype"),
    ("structure.py", "np.abs(np.fft.fftn(rho)) ** 2 / n_cells", "np.abs(np.fft.fftn(rho)) ** 2 / n_cells ** 2"),
    ("structure.py", "np.floor(np.sqrt(m2.astype(np.float64)) + 0.5)", "np.floor(np.sqrt(m2.astype(np.float64)))"),
    ("structure.py", "np.fft.fftfreq(n, d=1.0 / n)", "np.fft.fftfreq(n, d=1.0)"),
    ("structure.py", "sum((n // 2) ** 2 for n in shape)", "sum((n // 2) for n in shape)"),
    # the split: the Laplacian's symbol, pairing, linear part, factors
    ("operator_split.py", "out = out + c * (-k2) ** p", "out = out + c * k2 ** p"),
    ("operator_split.py", "if sum(k[1]) <= 1}", "if sum(k[1]) <= 0}"),
    ("operator_split.py", "if any(e):                      # the Laplacian of a constant is zero",
     "if True:"),
    ("operator_split.py", "return 1.0 / den, dt / den", "return 1.0 / den, dt"),
    ("operator_split.py", "r._add(k, sign * c)", "r._add(k, c)"),
]


@pytest.fixture(scope="module")
def sandbox(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("oracle_mutations"))
    skip = shutil.ignore_patterns("__pycache__", "*.so", "csrc", "golden")
    for sub in ("oracle", "tests", "paper_2109_02598_amd"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub), ignore=skip)
    shutil.copy(os.path.join(ROOT, "pytest.ini"), d)
    return d


def run_pins(cwd, files):
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *files],
                          cwd=cwd, capture_output=True, text=True, timeout=600)


def test_unmutated_copy_passes(sandbox):
    r = run_pins(sandbox, sorted({f for fs in PIN_FILES.values() for f in fs}))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,old,new", MUTATIONS)
def test_planted_mistake_is_caught(sandbox, name, old, new):
    with open(os.path.join(ROOT, "oracle", name)) as f:
        src = f.read()
    assert src.count(old) == 1, old
    with open(os.path.join(sandbox, "oracle", name), "w") as f:
        f.write(src.replace(old, new))
    try:
        r = run_pins(sandbox, PIN_FILES[name])
    finally:
        with open(os.path.join(sandbox, "oracle", name), "w") as f:
            f.write(src)
    # exit status 1: tests ran and at least one failed (not a collection error)
    assert r.returncode == 1 and " failed" in r.stdout, (old, new, r.returncode, r.stdout[-1500:])
