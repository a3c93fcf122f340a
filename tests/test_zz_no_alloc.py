"""The allocation-free ray-tracing adjoint (static device scratch) against the
workspace entry point through the C-ABI: bitwise equal on two calls in a row,
the second on a smaller grid, and the size limit rejected on the host."""
import numpy as np
import pytest

import synth

from helpers import gpu_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2105_09465_amd as G
    return G


def _case(G, index, n, ss, seed):
    w = synth.workload(index).replace(n=n, ss=ss)
    prob = gpu_problem(w)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, w.N)).astype(np.float32)
    gpx = torch.as_tensor(g[0], device="cuda")
    gpy = torch.as_tensor(g[1], device="cuda")
    return prob, gpx, gpy


def test_noalloc_adjoint_matches_workspace_entry(G):
    """Two calls in a row, 200 x 200 at 2x supersampling (160,000 points, 625
    blocks) then 24 x 24 at 1x (576 points, 3 blocks): the second reads only the
    blocks it wrote, whatever the first left in the shared array."""
    for index, n, ss, seed in [(2, 200, 2, 70), (0, 24, 1, 71)]:
        print(f"[case] noalloc adjoint workload {index} n={n} ss={ss}", flush=True)
        prob, gpx, gpy = _case(G, index, n, ss, seed)
        want = G.ops.lens_raytrace_backward(prob.grid, prob.lens, gpx, gpy)
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        got = G.ops.lens_raytrace_backward_noalloc(prob.grid, prob.lens, gpx, gpy, out)
        torch.cuda.synchronize()
        assert torch.equal(got.cpu(), want.cpu()), (got, want)


def test_noalloc_adjoint_rejects_oversized_grid(G):
    """(n ss)^2 above 4,194,304 points is refused before anything is launched."""
    print("[case] noalloc adjoint size limit", flush=True)
    w = synth.workload(0).replace(n=2049, ss=1)
    prob = gpu_problem(w)
    tiny = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception, match="static scratch"):
        G.ops.lens_raytrace_backward_noalloc(prob.grid, prob.lens, tiny, tiny, out)
