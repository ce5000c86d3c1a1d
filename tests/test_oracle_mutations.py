"""Mutation check of the oracle's pins: each plausible mistake below (a
flipped sign, a dropped or misplaced term, a transposed operand, a wrong
power or factor), planted in a copy of oracle/spectral.py inside a
temporary directory, makes the oracle's own tests fail.  The repository's
oracle is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_split.py", "tests/test_oracle_adjoint.py",
             "tests/test_oracle_structure.py"]

MUTATIONS = [
    ("-M * c2 * one", "M * c2 * one"),                                     # AC: sign of the cubic term
    ("M * (c1 - kap * k2)", "M * (c1 + kap * k2)"),                        # AC: sign in L
    ("-M * c2 * k2, lambda", "-M * c2 * one, lambda"),                     # CH: derivative dropped
    ("kap * k2 ** 2", "kap * k2"),                                         # CH: wrong power in L
    ("g2 * q[0] ** 2 + g3 * q[0] ** 3", "g3 * q[0] ** 3"),                 # PFC: quadratic term dropped
    ("(q0 ** 2 - k2) ** 2", "(q0 - k2) ** 2"),                             # PFC: q0 not squared
    ("L = -k2 * (r + (q0 ** 2 - k2) ** 2)", "L = -k2 * (r - (q0 ** 2 - k2) ** 2)"),   # PFC: sign in L
    ("F - q[0] * q[1] ** 2", "F - q[0] ** 2 * q[1]"),                      # GS: operands transposed
    ("Lv = -dv * k2 - (F + kk)", "Lv = -dv * k2 - kk"),                    # GS: F dropped from L_v
    ("Lu = -du * k2 - F", "Lu = -dv * k2 - F"),                            # GS: wrong diffusivity
    ("2.0 * c5 * q[0] * q[1]", "c5 * q[0] * q[1]"),                        # Model C: factor 2 dropped
    ("Lp = c1 - k2", "Lp = c1 + k2"),                                      # Model C: sign in L_psi
    ("Lm = c3 * k2 - k2 ** 2", "Lm = c3 * k2 + k2 ** 2"),                  # Model C: sign in L_m
    ("(k2.copy(), lambda", "(one, lambda"),                                # Model C: lap of N_m dropped
    ("c5 * q[0] ** 2)", "c5 * q[1] ** 2)"),                                # Model C: wrong field
    ("-c4 * q[1] ** 3", "-c4 * q[0] ** 3"),                                # Model C: wrong field
    ("np.expm1(z[nz]) / z[nz]", "np.expm1(z[nz])"),                        # phi1 not divided by z
    ("return np.exp(z), dt * phi1(z)", "return np.exp(z), dt"),            # B = dt (explicit Euler)
    ("acc = A * fwd(q[j])", "acc = fwd(q[j])"),                            # A dropped
    ("2.0 * np.pi * np.fft.fftfreq(n, d=h)", "np.pi * np.fft.fftfreq(n, d=h)"),   # wavenumbers halved
    ("dxs = tuple(reversed(tuple(dx)))", "dxs = tuple(dx)"),               # spacings in the wrong order
]


@pytest.fixture(scope="module")
def sandbox(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("oracle_mutations"))
    skip = shutil.ignore_patterns("__pycache__", "*.so", "csrc", "golden")
    for sub in ("oracle", "tests", "paper_2109_02598_amd"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub), ignore=skip)
    shutil.copy(os.path.join(ROOT, "pytest.ini"), d)
    return d


def run_pins(cwd):
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_FILES],
                          cwd=cwd, capture_output=True, text=True, timeout=600)


def test_unmutated_copy_passes(sandbox):
    r = run_pins(sandbox)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_planted_mistake_is_caught(sandbox, old, new):
    with open(os.path.join(ROOT, "oracle", "spectral.py")) as f:
        src = f.read()
    assert src.count(old) == 1, old
    with open(os.path.join(sandbox, "oracle", "spectral.py"), "w") as f:
        f.write(src.replace(old, new))
    try:
        r = run_pins(sandbox)
    finally:
        with open(os.path.join(sandbox, "oracle", "spectral.py"), "w") as f:
            f.write(src)
    # exit status 1: tests ran and at least one failed (not a collection error)
    assert r.returncode == 1 and " failed" in r.stdout, (old, new, r.returncode, r.stdout[-1500:])
