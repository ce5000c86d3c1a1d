"""ss_step_n captured by the caller into a HIP graph (torch.cuda.graph on
the grid's stream) and replayed several times, with other work between
the replays, gives the bits of the same steps taken eagerly.  Conditions:
the carried spectrum is current before the capture (a step taken since the
last set_field), and the captured step count is even (the tuned step
arrangement may swap two arrays every step)."""
import numpy as np
import pytest

from paper_2109_02598_amd import inputs
from tests._common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["ac128", "gs512"])
def test_captured_steps_replay_like_eager_steps(case, dtype):
    torch, specstep = need_gpu()
    w = inputs.allen_cahn_2d(n=128, seed=1) if case == "ac128" else inputs.gray_scott_2d(n=512)
    s = torch.cuda.Stream()

    def grid():
        g = specstep.Grid(w.n, w.dx, dtype=dtype, model=w.model, coef=w.coef, dt=w.dt, stream=s.cuda_stream)
        g.autotune(1)
        for i, f in enumerate(w.fields):
            g.set_field(i, torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0"))
        g.step(2)                           # the carried spectrum is current
        return g

    eager = grid()
    eager.step(3 * 40)
    want = [eager.get_field(i).cpu().numpy() for i in range(len(w.fields))]
    g = grid()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g.step(40)
    for _ in range(3):
        with torch.cuda.stream(s):
            graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 18, device="cuda").sum().item()
    say("graph replays", case, dtype, "arrangement", specstep.ss_get_step_arrangement(g.h))
    for i in range(len(w.fields)):
        assert np.array_equal(g.get_field(i).cpu().numpy(), want[i]), i
    g.close()
    eager.close()
