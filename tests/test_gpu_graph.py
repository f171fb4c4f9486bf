"""The library's calls enqueue kernels on the caller's stream only (no
allocation, no memset, no synchronisation), so a caller can capture them in a
graph.  Captured here with torch's graph API: the sampler, the pdf and inverse map at
its normals, the dielectric sampler and its pdf, the one-pass albedo value and
gradient, the direct-illumination estimator, and the autograd helpers (view
directions from angles, the Jacobian product); the graph is replayed
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
    pouts = tuple(torch.empty_like(t["wx"]) for _ in range(4))  # pdf, u1, u2, dielectric pdf
    ws = torch.empty(cv.albedo_workspace_size(64, [n] * 64, 1) // 4 + 4, device="cuda")
    wr = torch.empty(cv.albedo_workspace_size(64, None, 0) // 4 + 4, device="cuda")
    vals = [torch.empty(64, device="cuda") for _ in range(5)]
    lobes = torch.tensor([[0.0, 0.0, 1.0, 4.0, 2.0], [0.6, 0.0, 0.8, 30.0, 5.0]],
                         dtype=torch.float32, device="cuda")
    th = torch.linspace(0.0, 1.5, 64, device="cuda")
    ph = torch.linspace(-3.0, 3.0, 64, device="cuda")
    vdirs = tuple(torch.empty(64, device="cuda") for _ in range(3))
    jvals = [torch.empty(64, device="cuda") for _ in range(4)]

    def run():
        cv.vndf_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], seed=3, out=outs)
        cv.vndf_pdf(t["wx"], t["wy"], t["wz"], outs[0], outs[1], outs[2], t["ax"], t["ay"],
                    out=pouts[0])
        cv.vndf_inverse(t["wx"], t["wy"], t["wz"], outs[0], outs[1], outs[2], t["ax"], t["ay"],
                        out=(pouts[1], pouts[2]))
        cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, seed=4, out=douts)
        cv.dielectric_pdf(t["wx"], t["wy"], t["wz"], douts[0], douts[1], douts[2], t["ax"],
                          t["ay"], 1.5, out=pouts[3])
        r = cv.albedo_value_and_grad(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 5,
                                     workspace=ws)
        for v, x in zip(vals, r):
            v.copy_(x)
        vals[4].copy_(cv.radiance_estimate(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 6,
                                           lobes, workspace=wr))
        cv.albedo_view_from_angles(th, ph, out=vdirs)
        j = cv.albedo_apply_jacobian(vals[0], vals[1], vals[2], vals[3], vals[0], vals[4])
        for v, x in zip(jvals, j):
            v.copy_(x)

    run()
    torch.cuda.synchronize()
    eager = [x.clone() for x in outs + douts + pouts + tuple(vals) + vdirs + tuple(jvals)]

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
        for x in outs + douts + pouts + tuple(vals) + vdirs + tuple(jvals):
            x.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda")
        _ = (junk * 3).sum().item()  # unrelated eager work and a synchronisation
        graph.replay()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(eager, outs + douts + pouts + tuple(vals) + vdirs + tuple(jvals))):
            assert torch.equal(a, b), f"replay {rep}, output {k}"
    assert np.isfinite(eager[0].cpu().numpy()).all()
