"""Optional finite check of the fields (ss_check_finite, SS_ERR_NONFINITE):
clean fields pass, a NaN or an infinity in any cell of any field is
reported for that field, and a run that blows up is caught."""
import numpy as np
import pytest

from tests._common import COEF, need_gpu, say, synth_fields

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(64, 32), (16, 8, 32)])
def test_finite_fields_pass_and_bad_cells_are_found(n, dtype):
    torch, specstep = need_gpu()
    dx = (1.0,) * len(n)
    fields = synth_fields("gray_scott", n, dx, 5)
    g = specstep.Grid(n, dx, dtype=dtype, model="gray_scott", coef=COEF["gray_scott"], dt=1.0)
    for i, f in enumerate(fields):
        g.set_field(i, torch.from_numpy(f).to("cuda:0"))
    g.step(3)
    assert g.check_finite() == 0
    for bad, field, want in ((np.nan, 0, 1), (np.inf, 1, 2), (-np.inf, 0, 1)):
        f = fields[field].copy()
        f.flat[(f.size * 3) // 7] = bad
        g.set_field(field, torch.from_numpy(f).to("cuda:0"))
        got = g.check_finite()
        say(n, dtype, "planted", bad, "in field", field, "mask", got)
        assert got == want
        with pytest.raises(specstep.SpecStepError) as e:
            specstep._check(specstep.lib().ss_check_finite(g.h, specstep.ctypes.byref(specstep.ctypes.c_int())))
        assert e.value.code == specstep.SS_ERR_NONFINITE
        g.set_field(field, torch.from_numpy(fields[field]).to("cuda:0"))
        assert g.check_finite() == 0
    g.close()


def test_a_blown_up_run_is_caught():
    """Forward Euler far beyond its stability limit overflows."""
    torch, specstep = need_gpu()
    n, dx = (64, 64), (1.0, 1.0)
    f0 = synth_fields("allen_cahn", n, dx, 9)[0]
    g = specstep.Grid(n, dx, dtype="f64", model="allen_cahn", coef=COEF["allen_cahn"], dt=5.0,
                      solver="euler", stencil=0)
    g.set_field(0, torch.from_numpy(f0).to("cuda:0"))
    assert g.check_finite() == 0
    g.step(200)
    assert g.check_finite() == 1
    assert not np.all(np.isfinite(g.get_field(0).cpu().numpy()))
    g.close()
