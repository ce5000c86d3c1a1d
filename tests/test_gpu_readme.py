"""The README's usage example runs as written (taken from the file)."""
import os

import pytest

from tests._common import need_gpu

pytestmark = pytest.mark.gpu


def test_readme_example_runs():
    torch, specstep = need_gpu()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "README.md")) as f:
        text = f.read()
    a = text.index("```python\n") + len("```python\n")
    code = text[a:text.index("```", a)]
    env = {}
    exec(compile(code, "README.md", "exec"), env)
    assert tuple(env["psi"].shape) == (2048, 2048)
    assert env["mass"].shape == (1000, 1)
    assert abs(float(env["mass"][-1, 0]) - float(env["mass"][0, 0])) <= 1e-15   # Cahn-Hilliard keeps the mean
    assert env["s"].shape == env["counts"].shape and int(env["counts"].sum()) > 0
