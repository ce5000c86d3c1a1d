"""C-ABI library: loads, exports every declared symbol, validates arguments.

No compute call is made: everything here runs without a GPU.
"""
import ctypes
import os
import re

import pytest

from paper_2109_02598_amd import specstep as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "specstep.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ss.LIB_PATH):
        pytest.skip("library not built")
    return ss.lib()


def test_header_declares_the_abi():
    syms = declared_symbols()
    for s in ("ss_create_grid", "ss_set_model", "ss_workspace_size", "ss_bind_workspace",
              "ss_set_field", "ss_get_field", "ss_step_n", "ss_destroy_grid", "ss_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol(L):
    for s in declared_symbols():
        assert hasattr(L, s), s


def test_version(L):
    assert "gfx950" in ss.ss_version()


def code_of(fn, *a):
    with pytest.raises(ss.SpecStepError) as e:
        fn(*a)
    return e.value.code


def test_create_grid_validation(L):
    assert code_of(ss.ss_create_grid, (64, 48), (1, 1), ss.SS_F64) == ss.SS_ERR_UNSUPPORTED
    assert code_of(ss.ss_create_grid, (64, 8192), (1, 1), ss.SS_F64) == ss.SS_ERR_UNSUPPORTED
    assert code_of(ss.ss_create_grid, (4, 64), (1, 1), ss.SS_F64) == ss.SS_ERR_UNSUPPORTED
    assert code_of(ss.ss_create_grid, (64, 64, 2048), (1, 1, 1), ss.SS_F32) == ss.SS_ERR_UNSUPPORTED
    assert code_of(ss.ss_create_grid, (64, 64), (1, 0), ss.SS_F64) == ss.SS_ERR_ARG
    assert code_of(ss.ss_create_grid, (64, 64), (1, float("nan")), ss.SS_F64) == ss.SS_ERR_ARG
    assert code_of(ss.ss_create_grid, (64,), (1,), ss.SS_F64) == ss.SS_ERR_ARG
    assert code_of(ss.ss_create_grid, (64, 64), (1, 1), 5) == ss.SS_ERR_ARG
    h = ss.ss_create_grid((64, 32), (1, 0.5), ss.SS_F32)
    ss.ss_destroy_grid(h)


def test_model_and_workspace_validation(L):
    h = ss.ss_create_grid((64, 32), (1, 1), ss.SS_F64)
    try:
        assert code_of(ss.ss_workspace_size, h) == ss.SS_ERR_STATE
        assert code_of(ss.ss_set_model, h, 9, (1, 1, 1, 1), 0.1) == ss.SS_ERR_ARG
        assert code_of(ss.ss_set_model, h, 1, (1, 1, 1), 0.1) == ss.SS_ERR_ARG
        assert code_of(ss.ss_set_model, h, 1, (1, 1, 1, float("inf")), 0.1) == ss.SS_ERR_ARG
        assert code_of(ss.ss_set_model, h, 1, (1, 1, 1, 1), 0.0) == ss.SS_ERR_ARG
        assert code_of(ss.ss_set_model, h, 5, (1, 1, 1, 1), 0.1) == ss.SS_ERR_ARG
        ss.ss_set_model(h, 1, (1, 1, 1, 1), 0.5)
        need = ss.ss_workspace_size(h)
        assert need >= 3 * 64 * 32 * 8
        ss.ss_set_model(h, 4, (0.16, 0.08, 0.035, 0.065), 1.0)
        assert ss.ss_workspace_size(h) >= 5 * 64 * 32 * 8
        fake = 1 << 40                         # never dereferenced by these calls
        assert code_of(ss.ss_bind_workspace, h, fake + 8, 1 << 30) == ss.SS_ERR_ARG
        assert code_of(ss.ss_bind_workspace, h, fake, 16) == ss.SS_ERR_ARG
        ss.ss_bind_workspace(h, fake, ss.ss_workspace_size(h))
        # no field set yet: the step and read-out refuse before touching the GPU
        assert code_of(ss.ss_step_n, h, 1) == ss.SS_ERR_STATE
        assert code_of(ss.ss_get_field, h, 0, fake, True) == ss.SS_ERR_STATE
        assert code_of(ss.ss_set_field, h, 2, fake, True) == ss.SS_ERR_ARG
        assert code_of(ss.ss_step_n, h, -1) == ss.SS_ERR_ARG
        assert "nsteps" in ss.ss_last_error()
    finally:
        ss.ss_destroy_grid(h)


def test_null_handles(L):
    assert L.ss_step_n(None, 1) == ss.SS_ERR_ARG
    assert L.ss_destroy_grid(None) == ss.SS_OK
    out = ctypes.c_void_p()
    assert L.ss_create_grid(2, None, None, 8, None, ctypes.byref(out)) == ss.SS_ERR_ARG


def test_batch_validation(L):
    fake = 1 << 40
    hs = []
    try:
        for i, (n, model) in enumerate([((64, 128), 2), ((256, 256), 2), ((32, 64), 2)]):
            h = ss.ss_create_grid(n, (1, 1), ss.SS_F32)
            ss.ss_set_model(h, model, (1, 1, 1, 1), 0.1)
            ss.ss_bind_workspace(h, fake + (i << 32), ss.ss_workspace_size(h))
            hs.append(h)
        b = ss.ss_batch_create(hs[:2])
        assert ss.ss_batch_workspace_size(b) >= 2 * 2 * 100
        assert code_of(ss.ss_batch_step_n, b, 1) == ss.SS_ERR_STATE     # no workspace
        assert code_of(ss.ss_batch_capture, b, 1) == ss.SS_ERR_ARG      # null stream
        assert code_of(ss.ss_batch_launch, b) == ss.SS_ERR_STATE
        ss.ss_batch_destroy(b)
        assert code_of(ss.ss_batch_create, hs) == ss.SS_ERR_UNSUPPORTED  # 32 < 64
        # members share no state: a repeated grid, overlapping workspaces
        assert code_of(ss.ss_batch_create, [hs[0], hs[1], hs[0]]) == ss.SS_ERR_ARG
        assert "share workspace" in ss.ss_last_error()
        ss.ss_bind_workspace(hs[1], fake + ss.ss_workspace_size(hs[0]) - 256, ss.ss_workspace_size(hs[1]))
        assert code_of(ss.ss_batch_create, hs[:2]) == ss.SS_ERR_ARG
        ss.ss_bind_workspace(hs[1], fake + ss.ss_workspace_size(hs[0]), ss.ss_workspace_size(hs[1]))
        ss.ss_batch_destroy(ss.ss_batch_create(hs[:2]))                  # adjacent: fine
        h64 = ss.ss_create_grid((64, 64), (1, 1), ss.SS_F64)
        ss.ss_set_model(h64, 2, (1, 1, 1, 1), 0.1)
        ss.ss_bind_workspace(h64, fake + (8 << 32), ss.ss_workspace_size(h64))
        hs.append(h64)
        assert code_of(ss.ss_batch_create, [hs[0], h64]) == ss.SS_ERR_ARG  # mixed dtype
        hgs = ss.ss_create_grid((64, 64), (1, 1), ss.SS_F32)
        ss.ss_set_model(hgs, 4, (0.16, 0.08, 0.035, 0.065), 1.0)
        ss.ss_bind_workspace(hgs, fake + (9 << 32), ss.ss_workspace_size(hgs))
        hs.append(hgs)
        assert code_of(ss.ss_batch_create, [hs[0], hgs]) == ss.SS_ERR_UNSUPPORTED  # two fields
        h3 = ss.ss_create_grid((64, 64, 64), (1, 1, 1), ss.SS_F32)
        ss.ss_set_model(h3, 2, (1, 1, 1, 1), 0.1)
        hs.append(h3)
        assert code_of(ss.ss_batch_create, [hs[0], h3]) == ss.SS_ERR_UNSUPPORTED  # 3D
    finally:
        for h in hs:
            ss.ss_destroy_grid(h)


def test_finite_check_validation(L):
    """Argument and state checks of ss_check_finite (refused before any
    device work)."""
    fake = 1 << 40
    m = ctypes.c_int()
    assert L.ss_check_finite(None, ctypes.byref(m)) == ss.SS_ERR_ARG
    h = ss.ss_create_grid((64, 32), (1, 1), ss.SS_F64)
    try:
        assert L.ss_check_finite(h, None) == ss.SS_ERR_ARG
        assert L.ss_check_finite(h, ctypes.byref(m)) == ss.SS_ERR_STATE       # no model
        ss.ss_set_model(h, 2, (1, 1, 1, 1), 0.1)
        assert L.ss_check_finite(h, ctypes.byref(m)) == ss.SS_ERR_STATE       # no workspace
        ss.ss_bind_workspace(h, fake, ss.ss_workspace_size(h))
        assert L.ss_check_finite(h, ctypes.byref(m)) == ss.SS_ERR_STATE       # no field
    finally:
        ss.ss_destroy_grid(h)


def test_noalloc_validation(L):
    """Argument and state checks of ss_step_fields_noalloc (refused before
    any device work)."""
    fake = 1 << 40
    h = ss.ss_create_grid((64, 32), (1, 1), ss.SS_F64)
    try:
        assert code_of(ss.ss_step_fields_noalloc, h, [fake], 1) == ss.SS_ERR_STATE
        assert code_of(ss.ss_noalloc_scratch_bytes, h) == ss.SS_ERR_STATE
        ss.ss_set_model(h, 2, (1, 1, 1, 1), 0.1)
        need, limit = ss.ss_noalloc_scratch_bytes(h)
        assert need == 2 * 64 * 32 * 8 and limit == 64 << 20
        assert code_of(ss.ss_step_fields_noalloc, h, [0], 1) == ss.SS_ERR_ARG
        assert code_of(ss.ss_step_fields_noalloc, h, [fake], -1) == ss.SS_ERR_ARG
        assert L.ss_step_fields_noalloc(h, None, 1) == ss.SS_ERR_ARG
    finally:
        ss.ss_destroy_grid(h)
    big = ss.ss_create_grid((256, 256, 256), (1, 1, 1), ss.SS_F32)
    try:
        ss.ss_set_model(big, 3, (-0.25, 1, 0, 1), 0.5)
        need, limit = ss.ss_noalloc_scratch_bytes(big)
        assert need == 2 * 256 ** 3 * 4 > limit
        assert code_of(ss.ss_step_fields_noalloc, big, [fake], 1) == ss.SS_ERR_ARG
        assert "scratch" in ss.ss_last_error()
    finally:
        ss.ss_destroy_grid(big)


def test_mass_log_copy_validation(L):
    """ss_mass_log (the host copy of the per-step log) checks its arguments
    and the bound log before touching the device."""
    buf = (ctypes.c_double * 8)()
    rows = ctypes.c_int64(7)
    assert L.ss_mass_log(None, buf, 8, ctypes.byref(rows)) == ss.SS_ERR_ARG
    assert rows.value == 0
    h = ss.ss_create_grid((64, 32), (1, 1), ss.SS_F64)
    try:
        assert L.ss_mass_log(h, buf, -1, None) == ss.SS_ERR_ARG
        assert L.ss_mass_log(h, None, 4, None) == ss.SS_ERR_ARG
        assert L.ss_mass_log(h, buf, 4, ctypes.byref(rows)) == ss.SS_ERR_STATE   # no log bound
        assert "no mass log" in ss.ss_last_error()
    finally:
        ss.ss_destroy_grid(h)


def test_header_is_plain_c(tmp_path):
    """include/specstep.h is a C header (no C++ in the boundary): it compiles
    as pedantic C99 and C++11 with warnings as errors."""
    import shutil
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "use.c"
    src.write_text('#include "specstep.h"\nint main(void) { ss_grid g = 0; (void)g; return 0; }\n')
    for cc, args in (("gcc", ["-std=c99", "-x", "c"]), ("g++", ["-std=c++11", "-x", "c++"])):
        if not shutil.which(cc):
            pytest.skip("%s not available" % cc)
        r = subprocess.run([cc, *args, "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc, "-c", str(src),
                            "-o", str(tmp_path / "use.o")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
