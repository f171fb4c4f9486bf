"""GPU parity of the direct-illumination estimator against the FP64 oracle
on the same Philox streams.  The albedo bar (1e-4 absolute for weights in
[0, 1]) is scaled by the radiance bound sum(lambda): |err| <= 1e-4 sum(lambda).
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from _gpu import golden, host, to_dev

pytestmark = pytest.mark.gpu

cv = pytest.importorskip("paper_2306_05044_amd")

LOBES = np.array([[0.0, 0.0, 1.0, 4.0, 2.0],
                  [0.6, 0.0, 0.8, 30.0, 5.0],
                  [-0.5, 0.5, np.sqrt(0.5), 10.0, 1.5],
                  [0.0, 0.0, 1.0, 0.0, 0.3]], dtype=np.float32)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cv.load_library()


def _cells(n_side, seed):
    gg = workloads.grad_grid(n_side, seed=seed)
    wx, wy, wz = workloads.view_from_angles(gg["theta"], gg["phi"])
    return {"wx": wx, "wy": wy, "wz": wz, "ax": gg["ax"], "ay": gg["ay"]}


# every lobe count has its own kernel instantiation (0 lobes: see the edges test)
@pytest.mark.parametrize("n,nl", [(1 << 12, 4), (4097, 1), (1, 4), (1 << 14, 8), (2049, 2),
                                  (2049, 3), (2049, 5), (2049, 6), (2049, 7)])
def test_radiance_matches_oracle(n, nl):
    g = _cells(8, seed=21)
    t = to_dev(g)
    lobes = np.tile(LOBES, (2, 1))[:nl].copy()
    f0 = np.where(np.arange(64) % 2 == 0, 1.0, 0.04).astype(np.float32)
    r = cv.radiance_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 8,
                             torch.from_numpy(lobes).cuda(), f0=torch.from_numpy(f0).cuda())
    ref = oracle.radiance((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], n, 8,
                          lobes.astype(np.float64), f0=f0)
    bound = float(lobes[:, 4].sum())
    assert np.abs(host(r) - ref).max() <= 1e-4 * bound


def test_constant_radiance_and_edges():
    g = workloads.lut_grid(8, 8)
    t = to_dev(g)
    const = torch.tensor([[0.0, 0.0, 1.0, 0.0, 2.5]], device="cuda")
    r = cv.radiance_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 5000, 3, const)
    s1, _ = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 5000, 3)
    assert torch.allclose(r, 2.5 * s1, rtol=2e-6, atol=1e-7)
    empty = torch.zeros((0, 5), device="cuda")
    r0 = cv.radiance_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 5000, 3, empty)
    assert torch.all(r0 == 0)
    with pytest.raises(cv.CapvndfError):
        cv.radiance_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 10, 3,
                             torch.zeros((9, 5), device="cuda"))


def test_radiance_full_table_every_cell():
    """64 x 64 cells x 2^20 samples under 4 lobes: every cell against the
    oracle's stored values, and four cells against the oracle run live."""
    gold = golden("radiance")
    g = workloads.lut_grid(64, 64)
    t = to_dev(g)
    n, seed = int(gold["radiance_n"]), int(gold["radiance_seed"])
    lobes = np.ascontiguousarray(gold["radiance_lobes"])
    r = cv.radiance_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, seed,
                             torch.from_numpy(lobes).cuda())
    torch.cuda.synchronize()
    got = host(r)
    tol = 1e-4 * float(lobes[:, 4].sum())
    err = np.abs(got - gold["radiance_value"]).max()
    print(f"radiance, every cell: max |err| {err:.2e} (tolerance {tol:.1e})")
    assert err <= tol
    cells = np.array([5, 1234, 2900, 4094])
    sub = {k: v[cells] for k, v in g.items()}
    ref = oracle.radiance((sub["wx"], sub["wy"], sub["wz"]), sub["ax"], sub["ay"], n, seed,
                          lobes.astype(np.float64), units=cells)
    assert np.abs(got[cells] - ref).max() <= tol
    assert np.abs(gold["radiance_value"][cells] - ref).max() <= 1e-12
