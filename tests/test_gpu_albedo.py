"""GPU parity of the albedo estimator, its pathwise adjoint, the autograd
Function and the batched plan, against the FP64 oracle on the same Philox
streams.  Albedo within 1e-4 absolute; gradients within
1e-4 + 1e-3 |g| of the oracle's dual-number gradient."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from _gpu import golden, host, to_dev

pytestmark = pytest.mark.gpu

cv = pytest.importorskip("paper_2306_05044_amd")

ATOL_A = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cv.load_library()


def _oracle_sums(g, n, seed, units=None):
    wo = (g["wx"], g["wy"], g["wz"])
    a1 = oracle.albedo(wo, g["ax"], g["ay"], n, seed, f0=1.0, units=units)
    a5 = oracle.albedo(wo, g["ax"], g["ay"], n, seed, f0=0.0, units=units)
    return a1, a5


@pytest.mark.parametrize("n", [1, 2, 3, 4097, 1 << 14, (1 << 14) + 1, 70001])
def test_lut_subgrid(n):
    g = workloads.lut_grid(16, 16)
    t = to_dev(g)
    s1, s5 = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 2)
    a1, a5 = _oracle_sums(g, n, 2)
    e1 = np.abs(host(s1) - a1).max()
    e5 = np.abs(host(s5) - a5).max()
    print(f"n={n}: max |err| S1 {e1:.2e} S5 {e5:.2e}")
    assert e1 <= ATOL_A and e5 <= ATOL_A
    # both Fresnel values from the one stream
    for f0 in (0.04, 1.0):
        a = f0 * host(s1) + (1 - f0) * host(s5)
        ref = oracle.albedo((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], n, 2, f0=f0)
        assert np.abs(a - ref).max() <= ATOL_A


def test_lut_edges():
    wx = torch.tensor([0.0, 0.0, 0.6, 0.0], device="cuda")
    wy = torch.zeros(4, device="cuda")
    wz = torch.tensor([1.0, -1.0, 0.8, 1.0], device="cuda")
    ax = torch.tensor([0.5, 0.5, 0.0, 1.0], device="cuda")
    s1, s5 = cv.albedo_estimate(wx, wy, wz, ax, ax.clone(), 1000, 1)
    assert host(s1)[1] == 0 and host(s1)[2] == 0 and host(s5)[1] == 0
    assert host(s1)[0] > 0 and host(s1)[3] > 0
    s1, s5 = cv.albedo_estimate(wx, wy, wz, ax, ax.clone(), 0, 1)
    assert torch.all(s1 == 0) and torch.all(s5 == 0)
    z = torch.zeros(0, device="cuda")
    s1, s5 = cv.albedo_estimate(z, z, z, z, z, 100, 1)
    assert s1.numel() == 0


def _uneven_counts(ncells):
    """Per-cell counts: empty, single, odd, chunk boundaries (16384 samples
    per chunk), and one cell with more chunks (257) than a call of this many
    cells gives it slots (128), so that slots loop over several chunks."""
    base = [0, 1, 2, 3, 4097, 16383, 16384, 16385, 32769, 70001, (1 << 22) + 12345]
    rng = np.random.default_rng(31)
    rest = rng.integers(0, 1 << 15, ncells - len(base))
    return np.concatenate([base, rest]).astype(np.int64)


def test_uneven_counts():
    """Every table estimator with its own sample count per cell (host counts
    and a device count tensor), against the oracle on the same counts."""
    g = workloads.lut_grid(8, 8)
    t = to_dev(g)
    ns = _uneven_counts(64)
    wo = (g["wx"], g["wy"], g["wz"])
    a1 = oracle.albedo(wo, g["ax"], g["ay"], ns, 12, f0=1.0)
    a5 = oracle.albedo(wo, g["ax"], g["ay"], ns, 12, f0=0.0)
    f0 = np.where(np.arange(64) % 2 == 0, 0.04, 1.0).astype(np.float32)
    A, rx, ry, rt = oracle.albedo_grad(wo, g["ax"], g["ay"], ns, 12, f0=f0)
    gf = torch.from_numpy(f0).cuda()
    for counts in (ns, torch.from_numpy(ns).cuda()):
        s1, s5 = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], counts, 12)
        assert np.abs(host(s1) - a1).max() <= ATOL_A
        assert np.abs(host(s5) - a5).max() <= ATOL_A
        assert host(s1)[0] == 0 and host(s5)[0] == 0  # an empty cell
        a, gx, gy, gt = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                                                 counts, 12, f0=gf)
        assert np.abs(host(a) - A).max() <= ATOL_A
        _check_grad(host(gx), rx, "uneven d/d alpha_x")
        _check_grad(host(gy), ry, "uneven d/d alpha_y")
        _check_grad(host(gt), rt, "uneven d/d theta_o")
        bx, by, bt = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                                                 counts, 12, f0=gf)
        for u, v in ((gx, bx), (gy, by), (gt, bt)):
            assert torch.allclose(u, v, rtol=1e-5, atol=1e-6)
    # host counts size the workspace for at most the largest cell's chunks,
    # device counts for the most slots: with one chunk per slot in both, the
    # bits agree; the big cell (257 chunks) is summed over different slots
    h1, _ = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], ns, 12)
    d1, _ = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                               torch.from_numpy(ns).cuda(), 12)
    small = ns < 128 * 16384
    assert torch.equal(h1[torch.from_numpy(small).cuda()], d1[torch.from_numpy(small).cuda()])


def test_one_slot_per_cell():
    """The smallest workspace (one partial per cell): every slot sums all of
    its cell's chunks; results stay within the parity bounds."""
    g = workloads.lut_grid(4, 4)
    t = to_dev(g)
    ns = np.array([0, 1, 70001, 1 << 18] * 4, dtype=np.int64)
    # 16 cells x (4 sums x (s, c) + a 32-byte horizon record)
    ws = torch.empty(16 * (4 * 2 + 8), device="cuda")
    a, gx, gy, gt = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], ns, 14,
                                             workspace=ws)
    A, rx, ry, rt = oracle.albedo_grad((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], ns, 14)
    assert np.abs(host(a) - A).max() <= ATOL_A
    _check_grad(host(gx), rx, "one slot d/d alpha_x")
    _check_grad(host(gy), ry, "one slot d/d alpha_y")
    _check_grad(host(gt), rt, "one slot d/d theta_o")


def test_invalid_count_gives_nan():
    """A device count outside [0, 2^40) cannot be checked on the host: that
    cell's outputs are NaN and the other cells are unaffected."""
    g = workloads.lut_grid(2, 2)
    t = to_dev(g)
    ns = torch.tensor([1000, -5, 1 << 40, 3000], dtype=torch.int64, device="cuda")
    s1, s5 = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], ns, 1)
    r1 = oracle.albedo((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], [1000, 0, 0, 3000], 1)
    v = host(s1)
    assert np.isnan(v[1]) and np.isnan(v[2]) and np.isnan(host(s5)[1])
    assert abs(v[0] - r1[0]) <= ATOL_A and abs(v[3] - r1[3]) <= ATOL_A


def test_lut_full_size_every_cell():
    """64 x 64 cells x 2^20 samples (the table workload): S1 and S5 of every
    cell against the oracle's values, and the one-pass value and Jacobian at
    F0 = 0.04 (what the autograd Function and the benchmark's forward +
    backward run) of every cell against the oracle's dual-number gradient."""
    gold = golden("lut")
    g = workloads.lut_grid(64, 64)
    t = to_dev(g)
    n = int(gold["lut_n"])
    s1, s5 = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 2)
    f0 = torch.full((4096,), float(gold["lut_f0"]), device="cuda")
    a, gx, gy, gt = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 2,
                                             f0=f0)
    torch.cuda.synchronize()
    S1, S5 = host(s1), host(s5)
    assert np.all(S1 >= 0) and np.all(S1 <= 1.0 + 1e-6) and np.all(S5 >= 0) and np.all(S5 <= S1)
    e1 = np.abs(S1 - gold["lut_s1"]).max()
    e5 = np.abs(S5 - gold["lut_s5"]).max()
    ea = np.abs(host(a) - gold["lut_value"]).max()
    print(f"table, every cell: max |err| S1 {e1:.2e}, S5 {e5:.2e}, A(0.04) {ea:.2e}")
    assert e1 <= ATOL_A and e5 <= ATOL_A and ea <= ATOL_A
    _check_grad(host(gx), gold["lut_gax"], "table d/d alpha_x", gold["lut_band_ax"])
    _check_grad(host(gy), gold["lut_gay"], "table d/d alpha_y", gold["lut_band_ay"])
    _check_grad(host(gt), gold["lut_gth"], "table d/d theta_o", gold["lut_band_th"])
    # normal incidence row (mu = 1) at alpha = 1: 1 - ln 2 within MC error
    c = 64 * 63 + 63
    assert abs(S1[c] - (1 - np.log(2))) < 4 * 0.366 / np.sqrt(n)


def _grad_cells(n_side, seed=3):
    gg = workloads.grad_grid(n_side, seed=seed)
    wx, wy, wz = workloads.view_from_angles(gg["theta"], gg["phi"])
    return {"wx": wx, "wy": wy, "wz": wz, "ax": gg["ax"], "ay": gg["ay"]}


def _check_grad(got, ref, name, band=None):
    """Within 1e-4 + 1e-3 |g| of the oracle's dual-number gradient, plus (for
    the full-size workloads) the oracle's bound on what samples within FP32
    rounding of the horizon can move (they may land on either side)."""
    diff = np.abs(got - ref)
    lim = 1e-4 + 1e-3 * np.abs(ref)
    if band is not None:
        lim = lim + band
    print(f"{name}: worst {np.max(diff / lim):.3f} of the limit, "
          f"{np.max(diff / (1e-4 + 1e-3 * np.abs(ref))):.3f} of the plain tolerance")
    assert np.all(diff <= lim), f"{name}: worst {np.max(diff / lim):.2f}x of the limit"


@pytest.mark.parametrize("n", [1 << 12, 4097])
def test_backward_subgrid(n):
    g = _grad_cells(8)
    t = to_dev(g)
    f0 = np.where(np.arange(64) % 2 == 0, 1.0, 0.04).astype(np.float32)
    gf = torch.from_numpy(f0).cuda()
    up = torch.linspace(0.5, 2.0, 64, device="cuda")
    gx, gy, gt = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 3,
                                             f0=gf, grad_albedo=up)
    A, rx, ry, rt = oracle.albedo_grad((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], n, 3, f0=f0)
    u = host(up).astype(np.float64)
    _check_grad(host(gx), u * rx, "d/d alpha_x")
    _check_grad(host(gy), u * ry, "d/d alpha_y")
    _check_grad(host(gt), u * rt, "d/d theta_o")


def test_grad_grid_every_cell():
    """32 x 32 anisotropic cells x 2^18 samples (the gradient workload): the
    recompute-style backward and the one-pass value and Jacobian of every
    cell against the oracle's dual-number gradient."""
    gold = golden("grad")
    g = _grad_cells(32)
    t = to_dev(g)
    n = int(gold["grad_n"])
    gx, gy, gt = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 3)
    a, vx, vy, vt = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 3)
    torch.cuda.synchronize()
    assert np.abs(host(a) - gold["grad_value"]).max() <= ATOL_A
    for (x, y), ref, band, name in zip(((gx, vx), (gy, vy), (gt, vt)),
                                       (gold["grad_gax"], gold["grad_gay"], gold["grad_gth"]),
                                       (gold["grad_band_ax"], gold["grad_band_ay"],
                                        gold["grad_band_th"]),
                                       ("alpha_x", "alpha_y", "theta_o")):
        _check_grad(host(x), ref, f"grid backward d/d {name}", band)
        _check_grad(host(y), ref, f"grid value_and_grad d/d {name}", band)


@pytest.mark.parametrize("n", [1 << 12, 4097, 1])
def test_value_and_grad(n):
    g = _grad_cells(8, seed=13)
    t = to_dev(g)
    f0 = np.where(np.arange(64) % 3 == 0, 0.04, 1.0).astype(np.float32)
    gf = torch.from_numpy(f0).cuda()
    a, gx, gy, gt = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 6,
                                             f0=gf)
    A, rx, ry, rt = oracle.albedo_grad((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], n, 6, f0=f0)
    assert np.abs(host(a) - A).max() <= ATOL_A
    _check_grad(host(gx), rx, "value_and_grad alpha_x")
    _check_grad(host(gy), ry, "value_and_grad alpha_y")
    _check_grad(host(gt), rt, "value_and_grad theta_o")
    # value only: same value bits as the F0 combination of one stream
    a2, n1, n2, n3 = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 6,
                                              f0=gf, with_grad=False)
    assert n1 is None and n2 is None and n3 is None
    assert np.abs(host(a2) - A).max() <= ATOL_A
    # the backward entry point gives the same gradients (different summation order)
    bx, by, bt = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 6,
                                             f0=gf)
    for u, v in ((gx, bx), (gy, by), (gt, bt)):
        assert torch.allclose(u, v, rtol=1e-5, atol=1e-6)


def test_backward_vs_central_differences():
    """The gradient configuration's check: the GPU gradient on the 32 x 32
    grid (2^12 samples per cell) against the oracle's FP64 central
    differences with step 1e-4 on the same random numbers, within
    1e-4 + 1e-3 |g| (the parity bound) + 1e-6 + 1e-5 |g| (the bound between
    the exact derivative and FD(1e-4) that the oracle's pin establishes), on
    the cells where the step resolves the derivative: no horizon kink within
    the step and both roughness values at least 0.2 (the same selection as
    the oracle's pin)."""
    n = 1 << 12
    gg = workloads.grad_grid(32, seed=3)
    wx, wy, wz = workloads.view_from_angles(gg["theta"], gg["phi"])
    g = {"wx": wx, "wy": wy, "wz": wz, "ax": gg["ax"], "ay": gg["ay"]}
    wo = (wx, wy, wz)
    kinks = oracle.albedo_kinks(wo, g["ax"], g["ay"], n, 3, step=1e-4)
    smooth = np.minimum(g["ax"], g["ay"]) >= 0.2
    t = to_dev(g)
    got = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 3)
    fd = oracle.albedo_fd(wo, g["ax"], g["ay"], n, 3, step=1e-4)
    for name, x, f, k in zip(("alpha_x", "alpha_y", "theta_o"), got, fd, kinks):
        m = (k == 0) & smooth
        gpu = host(x)
        lim = 1e-4 + 1e-3 * np.abs(f) + 1e-6 + 1e-5 * np.abs(f)
        r = np.abs(gpu - f) / lim
        print(f"GPU vs FD(1e-4) d/d {name}: {m.sum()} cells, worst {r[m].max():.3f} of the limit")
        assert m.sum() >= 60 and np.all(r[m] <= 1.0)


def test_autograd_function():
    gg = workloads.grad_grid(6, seed=11)
    ax = torch.from_numpy(gg["ax"]).cuda().requires_grad_(True)
    ay = torch.from_numpy(gg["ay"]).cuda().requires_grad_(True)
    th = torch.from_numpy(gg["theta"]).cuda().requires_grad_(True)
    ph = torch.from_numpy(gg["phi"]).cuda()
    f0 = torch.full_like(ph, 0.04)
    n = 1 << 12
    a = cv.albedo(ax, ay, th, ph, f0, n, 5)
    w = torch.linspace(-1, 1, a.numel(), device="cuda")
    (a * w).sum().backward()
    st = torch.sin(th.detach())
    wo = [host(x) for x in (st * torch.cos(ph), st * torch.sin(ph), torch.cos(th.detach()))]
    A, rx, ry, rt = oracle.albedo_grad(wo, gg["ax"], gg["ay"], n, 5, f0=0.04)
    assert np.abs(host(a.detach()) - A).max() <= ATOL_A
    W = host(w).astype(np.float64)
    _check_grad(host(ax.grad), W * rx, "autograd alpha_x")
    _check_grad(host(ay.grad), W * ry, "autograd alpha_y")
    _check_grad(host(th.grad), W * rt, "autograd theta_o")


def test_autograd_f0_gradient():
    """dA/dF0 = S1 - S5 (the estimate is linear in F0), against the oracle's
    two sums on the same stream; phi_o gets no gradient."""
    gg = workloads.grad_grid(5, seed=12)
    ax = torch.from_numpy(gg["ax"]).cuda()
    ay = torch.from_numpy(gg["ay"]).cuda()
    th = torch.from_numpy(gg["theta"]).cuda()
    ph = torch.from_numpy(gg["phi"]).cuda()
    f0 = torch.full_like(ph, 0.3).requires_grad_(True)
    n = 4097
    a = cv.albedo(ax, ay, th, ph, f0, n, 6)
    a.sum().backward()
    wo = [host(x) for x in (torch.sin(th) * torch.cos(ph), torch.sin(th) * torch.sin(ph),
                            torch.cos(th))]
    s1 = oracle.albedo(wo, gg["ax"], gg["ay"], n, 6, f0=1.0)
    s5 = oracle.albedo(wo, gg["ax"], gg["ay"], n, 6, f0=0.0)
    assert np.abs(host(f0.grad) - (s1 - s5)).max() <= 2e-4
    assert np.abs(host(a.detach()) - (0.3 * s1 + 0.7 * s5)).max() <= ATOL_A


def test_view_from_angles():
    """wo = (sin t cos p, sin t sin p, cos t) in FP32, against float64 at the
    same FP32 angles, over the hemisphere and a ragged length."""
    rng = np.random.default_rng(21)
    n = 100003
    th = rng.uniform(0.0, np.pi / 2, n).astype(np.float32)
    ph = rng.uniform(-np.pi, np.pi, n).astype(np.float32)
    th[:4] = [0.0, np.float32(np.pi / 2), 1e-6, 1.5]
    wx, wy, wz = cv.albedo_view_from_angles(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda())
    t, p = th.astype(np.float64), ph.astype(np.float64)
    ref = (np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t))
    for got, want in zip((wx, wy, wz), ref):
        assert np.abs(host(got).astype(np.float64) - want).max() <= 4e-7
    assert cv.albedo_view_from_angles(torch.empty(0, device="cuda"),
                                      torch.empty(0, device="cuda"))[0].numel() == 0


def test_apply_jacobian_is_the_fp32_product():
    """Each output is one correctly rounded FP32 product (F0: of the sums'
    difference), so it equals torch's on the same inputs bit for bit; also
    with outputs written over their inputs."""
    rng = np.random.default_rng(22)
    n = 70001
    g, dx, dy, dt, s1, s5 = (torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
                             for _ in range(6))
    ox, oy, ot, of = cv.albedo_apply_jacobian(g, dx, dy, dt, s1, s5)
    assert torch.equal(ox, g * dx) and torch.equal(oy, g * dy) and torch.equal(ot, g * dt)
    assert torch.equal(of, g * (s1 - s5))
    only = cv.albedo_apply_jacobian(g, d_theta_o=dt)
    assert only[0] is None and only[1] is None and only[3] is None
    assert torch.equal(only[2], g * dt)
    # in place: grad_ax over d_ax, grad_f0 over s_f1
    want_x, want_f = g * dx, g * (s1 - s5)
    lib = cv.load_library()
    P = lambda t: cv._ptr(t)  # noqa: E731
    rc = lib.albedo_apply_jacobian(n, P(g), P(dx), None, None, P(s1), P(s5), P(dx), None, None,
                                   P(s1), cv._stream(None))
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(dx, want_x) and torch.equal(s1, want_f)


def test_estimator_determinism():
    g = workloads.lut_grid(8, 8)
    t = to_dev(g)
    a = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 50000, 9)
    b = cv.albedo_estimate(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 50000, 9)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    c = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 50000, 9)
    d = cv.albedo_estimate_backward(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 50000, 9)
    for x, y in zip(c, d):
        assert torch.equal(x, y)


def test_estimator_microbench_runs():
    """The register-resident estimator benchmark (the mix ceiling the table
    kernels are measured against): every kind runs, gives finite per-lane
    sums and the same bits twice; a ragged lane count leaves the words
    beyond it untouched; bad arguments are refused."""
    lobes = torch.tensor([[0.0, 0.0, 1.0, 4.0, 2.0], [0.6, 0.0, 0.8, 30.0, 5.0],
                          [-0.5, 0.5, 0.70710678, 10.0, 1.5], [0.0, 0.0, 1.0, 0.0, 0.3]],
                         dtype=torch.float32, device="cuda")
    for kind in (0, 1, 2):
        a = cv.estimator_microbench(kind, 1000, 16, 3, lobes)
        b = cv.estimator_microbench(kind, 1000, 16, 3, lobes)
        assert torch.equal(a, b)
        assert np.all(np.isfinite(host(a).view(np.float32)))
        out = torch.full((1024,), 7, dtype=torch.int32, device="cuda")
        cv.estimator_microbench(kind, 1000, 16, 3, lobes, out=out)
        assert torch.equal(out[:1000], a) and torch.all(out[1000:] == 7)
    with pytest.raises(cv.CapvndfError):
        cv.estimator_microbench(3, 10, 1, 3, lobes)
    with pytest.raises(cv.CapvndfError):
        cv.estimator_microbench(2, 10, 1, 3, None)


def _grazing_cells(n=32, seed=12):
    """Grazing views (cos theta_o in [1e-3, 4e-3]) of strongly anisotropic
    roughness (one alpha log-uniform in [10^-0.5, 1], the other in
    [1e-3, 10^-2.5]): the pathwise derivative's slope jump at the horizon
    makes single per-sample terms reach hundreds, so one sample that FP32
    puts on the wrong side of the horizon moves a 2^16-sample cell by up to
    2000 times the gradient tolerance (the oracle's FP32 band bound)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(1e-3, 4e-3, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    big = 10.0 ** rng.uniform(-0.5, 0.0, n)
    small = 10.0 ** rng.uniform(-3.0, -2.5, n)
    swap = rng.random(n) < 0.5
    return {"wx": (s * np.cos(phi)).astype(np.float32), "wy": (s * np.sin(phi)).astype(np.float32),
            "wz": mu.astype(np.float32), "ax": np.where(swap, big, small).astype(np.float32),
            "ay": np.where(swap, small, big).astype(np.float32)}


def test_horizon_fix_on_grazing_cells():
    """The horizon fix pass where it matters: on grazing, strongly anisotropic
    cells (most with samples in the oracle's FP32 horizon band, whose bound
    reaches 2000 times the tolerance) the value and its derivatives match
    the oracle within the plain tolerance, the same bits come back twice,
    the backward entry point agrees, and so do workspaces of one to three
    slots per cell (a slot then walks several of the four chunks, and the
    fix pass with it)."""
    g = _grazing_cells()
    t = to_dev(g)
    n = 1 << 16
    wo = (g["wx"], g["wy"], g["wz"])
    _, _, _, cnt = oracle.albedo_horizon_band(wo, g["ax"], g["ay"], n, 21, c0=44, c1=192,
                                             kappa_max=1024.0)
    assert (cnt > 0).sum() >= 24  # the fix pass has work in most cells
    A, rx, ry, rt = oracle.albedo_grad(wo, g["ax"], g["ay"], n, 21)
    args = (t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], n, 21)
    first = cv.albedo_value_and_grad(*args)
    again = cv.albedo_value_and_grad(*args)
    for x, y in zip(first, again):
        assert torch.equal(x, y)
    assert np.abs(host(first[0]) - A).max() <= ATOL_A
    for got, ref, name in zip(first[1:], (rx, ry, rt), ("alpha_x", "alpha_y", "theta_o")):
        _check_grad(host(got), ref, f"grazing d/d {name}")
    back = cv.albedo_estimate_backward(*args)
    for got, ref, name in zip(back, (rx, ry, rt), ("alpha_x", "alpha_y", "theta_o")):
        _check_grad(host(got), ref, f"grazing backward d/d {name}")
    # 1, 2 and 3 slots per cell (4 sums x (s, c) and a 32-byte horizon
    # record each): the fix pass then walks 4, 2 or 1-2 chunks per slot
    for slots in (1, 2, 3):
        ws = torch.empty(32 * slots * (4 * 2 + 8), device="cuda")
        few = cv.albedo_value_and_grad(*args, workspace=ws)
        for x, y in zip(few, cv.albedo_value_and_grad(*args, workspace=ws)):
            assert torch.equal(x, y)
        assert np.abs(host(few[0]) - A).max() <= ATOL_A
        for got, ref, name in zip(few[1:], (rx, ry, rt), ("alpha_x", "alpha_y", "theta_o")):
            _check_grad(host(got), ref, f"grazing {slots} slot(s) d/d {name}")
