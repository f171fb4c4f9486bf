"""The library's calls enqueue kernels on the caller's stream only (no
allocation, no memset, no synchronisation), so a caller can capture them in a
graph.  Captured here with torch's graph API: the sampler, the dielectric
sampler and the one-pass albedo value and gradient; the graph is replayed
several times with unrelated eager work and synchronisation in between, and
every replay must equal the eager results bit for bit."""

import numpy as np
import pytest
import torch

import workloads
from _gpu import to_dev

pytestmark = pytest.mark.gpu

cv = pytest.importorskip("paper_2306_05044_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cv.load_library()


def test_hot_path_in_a_captured_graph():
    d = workloads.tuples_small(65536 + 5, seed=2)
    t = to_dev(d)
    g = workloads.lut_grid(8, 8)
    c = to_dev(g)
    n = 1 << 14
    outs = tuple(torch.empty_like(t["wx"]) for _ in range(4))
    douts = tuple(torch.empty_like(t["wx"]) for _ in range(5))
    ws = torch.empty(cv.albedo_workspace_size(64, n, 2) // 4 + 4, device="cuda")
    vals = [torch.empty(64, device="cuda") for _ in range(4)]

    def run():
        cv.vndf_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], seed=3, out=outs)
        cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, seed=4, out=douts)
        r = cv.albedo_value_and_grad(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 5,
                                     workspace=ws)
        for v, x in zip(vals, r):
            v.copy_(x)

    run()
    torch.cuda.synchronize()
    eager = [x.clone() for x in outs + douts + tuple(vals)]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    torch.cuda.synchronize()

    for rep in range(4):
        for x in outs + douts + tuple(vals):
            x.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda")
        _ = (junk * 3).sum().item()  # unrelated eager work and a synchronisation
        graph.replay()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(eager, outs + douts + tuple(vals))):
            assert torch.equal(a, b), f"replay {rep}, output {k}"
    assert np.isfinite(eager[0].cpu().numpy()).all()
