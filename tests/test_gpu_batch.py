"""GPU parity of the batched persistent estimator (graph-replayed) and its
per-request baseline against the FP64 oracle, replay stability, and the
autotuner."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from _gpu import host, to_dev

pytestmark = pytest.mark.gpu

cv = pytest.importorskip("paper_2306_05044_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cv.load_library()


def _jobs(n_jobs, seed, lo=4, hi=15):
    j = workloads.batch_jobs(n_jobs, seed=seed, log2_min=lo, log2_max=hi)
    j["n"][0] = 0      # an empty job
    j["n"][1] = 1      # a single sample
    j["n"][2] = 3      # odd count
    return j


def _check(plan, j, f0, with_grad):
    wo = (j["wx"], j["wy"], j["wz"])
    A, rx, ry, rt = oracle.albedo_grad(wo, j["ax"], j["ay"], j["n"], 4, f0=f0)
    assert np.abs(host(plan.albedo) - A).max() <= 1e-4
    if with_grad:
        for got, ref in ((plan.grad_ax, rx), (plan.grad_ay, ry), (plan.grad_theta_o, rt)):
            d = np.abs(host(got) - ref)
            assert np.all(d <= 1e-4 + 1e-3 * np.abs(ref)), np.max(d / (1e-4 + 1e-3 * np.abs(ref)))


@pytest.mark.parametrize("tiling", [None, (256, 8, 2), (512, 16, 4), (256, 64, 16),
                                    (256, 8, 4, 1), (512, 128, 8, 1), (256, 32, 16, 1),
                                    (256, 8, 2, 0, 1), (512, 64, 8, 0, 1), (256, 16, 16, 1, 1),
                                    (512, 8, 1, 1, 1)])
def test_batch_matches_oracle(tiling):
    j = _jobs(97, seed=5)
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    f0 = torch.from_numpy(np.where(np.arange(97) % 3 == 0, 0.04, 1.0).astype(np.float32)).cuda()
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, f0=f0,
                        with_grad=True, tiling=tiling)
    plan.run()
    torch.cuda.synchronize()
    _check(plan, j, host(f0).astype(np.float64), True)
    info = plan.info()
    assert info["total_samples"] == int(j["n"].sum())
    plan.close()


@pytest.mark.parametrize("tiling", [None, (256, 16, 4, 1), (256, 32, 8, 0, 1), (256, 8, 8, 1, 1)])
def test_batch_forward_only(tiling):
    j = _jobs(50, seed=6)
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, with_grad=False,
                        tiling=tiling)
    plan.run()
    torch.cuda.synchronize()
    _check(plan, j, 1.0, False)


def test_replays_and_per_request_baseline():
    j = _jobs(64, seed=7)
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, with_grad=True)
    plan.run()
    torch.cuda.synchronize()
    first = [o.clone() for o in (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o)]
    for r in range(4):
        for o in (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o):
            o.fill_(123.0)
        x = torch.randn(1 << 16, device="cuda")
        _ = (x * 2).sum().item()          # unrelated eager work between replays
        plan.run()
        torch.cuda.synchronize()
        for a, b in zip(first, (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o)):
            assert torch.equal(a, b), f"replay {r} differs"
    plan.run_per_request()
    torch.cuda.synchronize()
    _check(plan, j, 1.0, True)
    for a, b in zip(first, (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o)):
        assert torch.allclose(a, b, rtol=1e-5, atol=2e-6)


@pytest.mark.parametrize("tiling", [(256, 16, 8, 0, 1), (256, 8, 8, 1, 1)])
def test_dynamic_replays_are_bitwise_stable(tiling):
    """Dynamic chunk assignment changes which owner runs a chunk from replay to
    replay but not its result slot: every replay gives the same bits, equal to
    the static assignment's."""
    j = _jobs(80, seed=13, lo=6, hi=16)
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    static = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, with_grad=True,
                          tiling=tiling[:4] + (0,))
    static.run()
    torch.cuda.synchronize()
    ref = [o.clone() for o in (static.albedo, static.grad_ax, static.grad_ay, static.grad_theta_o)]
    static.close()
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, with_grad=True,
                        tiling=tiling)
    for r in range(5):
        for o in (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o):
            o.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        for a, b in zip(ref, (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o)):
            assert torch.equal(a, b), f"replay {r}"
    plan.close()


def test_full_batch_sampled():
    """4096 uneven jobs (2^10 .. 2^22 samples); 72 jobs checked by the oracle."""
    j = workloads.batch_jobs(4096, seed=4)
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, with_grad=True)
    plan.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    small = np.flatnonzero(j["n"] <= (1 << 16))
    large = np.flatnonzero(j["n"] >= (1 << 21))
    mid = np.flatnonzero((j["n"] > (1 << 16)) & (j["n"] < (1 << 21)))
    idx = np.concatenate([rng.choice(small, 48, replace=False), rng.choice(mid, 16, replace=False),
                          rng.choice(large, 8, replace=False)])
    sub = {k: v[idx] for k, v in j.items()}
    A, rx, ry, rt = oracle.albedo_grad((sub["wx"], sub["wy"], sub["wz"]), sub["ax"], sub["ay"],
                                       sub["n"], 4, units=idx)
    assert np.abs(host(plan.albedo)[idx] - A).max() <= 1e-4
    for got, ref in ((plan.grad_ax, rx), (plan.grad_ay, ry), (plan.grad_theta_o, rt)):
        d = np.abs(host(got)[idx] - ref)
        assert np.all(d <= 1e-4 + 1e-3 * np.abs(ref))
    assert torch.all(torch.isfinite(plan.grad_ax))


def test_autotune_small(tmp_path, monkeypatch):
    monkeypatch.setenv("CAPVNDF_TUNE_CACHE", str(tmp_path / "tune.txt"))
    j = _jobs(32, seed=8, lo=8, hi=14)
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    best, ms = cv.albedo_batch_autotune(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4)
    assert best[0] in (256, 512) and best[1] % 8 == 0 and best[3] in (0, 1) and ms > 0
    assert best[4] in (0, 1)
    text = (tmp_path / "tune.txt").read_text().split()
    assert [int(x) for x in text[1:6]] == list(best)
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4)
    assert plan.info()["tiling"] == best   # picked up from the cache
    plan.run()
    torch.cuda.synchronize()
    _check(plan, j, 1.0, True)
    plan.close()
    # lines of another layout for the same problem are skipped, not misread:
    # a six-field line (no dynamic field) whose time would parse as a valid
    # dynamic flag, and a truncated line
    sig = text[0]
    other = (512, 16, 2, 1) if tuple(best[:4]) != (512, 16, 2, 1) else (256, 16, 2, 1)
    with open(tmp_path / "tune.txt", "a") as f:
        f.write(f"{sig} {other[0]} {other[1]} {other[2]} {other[3]} 1.250000\n")
        f.write(f"{sig} {other[0]} {other[1]}\n")
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4)
    assert plan.info()["tiling"] == best
    plan.close()


@pytest.mark.parametrize("tiling", [None, (256, 8, 4, 1), (512, 32, 8, 0, 1)])
@pytest.mark.parametrize("n_samples", [1, 2, 1 << 20])
def test_single_job(n_samples, tiling):
    """A batch of one job: one sample, one pair, and a job large enough to be
    split over many chunks and blocks."""
    j = workloads.batch_jobs(1, seed=9)
    j["n"][0] = n_samples
    t = to_dev({k: v for k, v in j.items() if k != "n"})
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], j["n"], 4, with_grad=True,
                        tiling=tiling)
    plan.run()
    torch.cuda.synchronize()
    _check(plan, j, 1.0, True)
    assert plan.info()["total_samples"] == n_samples
    plan.close()


def test_too_many_chunks_is_refused_before_building():
    """2048 jobs of 2^40 - 1 samples in chunks of 512 pairs are 2^41 chunks:
    refused with a message before any table is built (no host blow-up)."""
    n = 2048
    t = {k: torch.full((n,), v, device="cuda") for k, v in
         (("wx", 0.0), ("wy", 0.0), ("wz", 1.0), ("ax", 0.5), ("ay", 0.5))}
    with pytest.raises(cv.CapvndfError) as e:
        cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                     np.full(n, (1 << 40) - 1, dtype=np.int64), 4, tiling=(256, 8, 2, 1, 0))
    assert "exceed 2^31 - 2" in str(e.value)


def test_autotune_refuses_when_no_tiling_fits():
    n = 2048
    t = {k: torch.full((n,), v, device="cuda") for k, v in
         (("wx", 0.0), ("wy", 0.0), ("wz", 1.0), ("ax", 0.5), ("ay", 0.5))}
    with pytest.raises(cv.CapvndfError) as e:
        cv.albedo_batch_autotune(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                                 np.full(n, (1 << 40) - 1, dtype=np.int64), 4)
    assert e.value.code == -2 and "exceed 2^31 - 2" in str(e.value)


def test_per_request_path_refuses_a_job_beyond_one_launch():
    """A job of 2^38 samples is 2^24 per-request chunks of 16384 samples,
    one more than a launch of 256-lane blocks can count: refused before
    anything is enqueued (the plan itself, with large chunks, is fine)."""
    t = {k: torch.full((1,), v, device="cuda") for k, v in
         (("wx", 0.0), ("wy", 0.0), ("wz", 1.0), ("ax", 0.5), ("ay", 0.5))}
    plan = cv.BatchPlan(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                        np.array([1 << 38], dtype=np.int64), 4, tiling=(512, 4096, 1, 0, 0))
    with pytest.raises(cv.CapvndfError) as e:
        plan.run_per_request()
    assert e.value.code == -2 and "more than one launch" in str(e.value)
    plan.close()
