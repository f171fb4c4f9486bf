"""The variant of albedo_value_and_grad that allocates nothing (its partials
live in a buffer the library owns on each device), called through the C ABI:
the same values and gradients as the workspace entry point on the same
inputs, within the parity bounds, on two calls in a row (the second on fewer
cells and other counts, so stale partials of the first would show), plus its
size limit."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from _gpu import host, to_dev

pytestmark = pytest.mark.gpu

cv = pytest.importorskip("paper_2306_05044_amd")

_P = ctypes.c_void_p


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = cv.load_library()
    fn = L.albedo_value_and_grad_noalloc
    fn.argtypes = [ctypes.c_int64] + [_P] * 6 + [ctypes.c_uint64] + [_P] * 6
    fn.restype = ctypes.c_int32
    return L


def _ptr(t):
    return None if t is None else _P(t.data_ptr())


def _call(lib, g, counts, seed, f0, grad=True):
    n = g["wx"].numel()
    outs = [torch.full((n,), float("nan"), device="cuda") for _ in range(4 if grad else 1)]
    if not grad:
        outs += [None, None, None]
    rc = lib.albedo_value_and_grad_noalloc(
        n, *[_ptr(g[k]) for k in ("wx", "wy", "wz", "ax", "ay")], _ptr(counts), seed, _ptr(f0),
        *[_ptr(o) for o in outs], _P(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.capvndf_last_error()
    torch.cuda.synchronize()
    return outs


def _check(got, ref, tol_value=1e-4):
    assert np.abs(host(got[0]) - ref[0]).max() <= tol_value
    for a, b in zip(got[1:], ref[1:]):
        d = np.abs(host(a) - b)
        assert np.all(d <= 1e-4 + 1e-3 * np.abs(b)), np.max(d / (1e-4 + 1e-3 * np.abs(b)))


def test_no_alloc_matches_the_workspace_entry_point(lib):
    # first call: the 64 x 64 table at 2^16 samples per cell, F0 = 0.04
    g = workloads.lut_grid(64, 64)
    t = to_dev(g)
    n1 = np.full(4096, 1 << 16, dtype=np.int64)
    c1 = torch.from_numpy(n1).cuda()
    f0 = torch.full((4096,), 0.04, device="cuda")
    got = _call(lib, t, c1, 2, f0)
    ref = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], c1, 2, f0=f0)
    _check(got, [host(x).astype(np.float64) for x in ref])
    # second call: fewer cells, uneven counts (0, 1, odd, several chunks)
    g2 = workloads.lut_grid(6, 5)
    t2 = to_dev(g2)
    n2 = np.array([0, 1, 3, 4097, 70001, 1 << 15] * 5, dtype=np.int64)
    c2 = torch.from_numpy(n2).cuda()
    got2 = _call(lib, t2, c2, 7, None)
    ref2 = cv.albedo_value_and_grad(t2["wx"], t2["wy"], t2["wz"], t2["ax"], t2["ay"], c2, 7)
    _check(got2, [host(x).astype(np.float64) for x in ref2])
    A, rx, ry, rt = oracle.albedo_grad((g2["wx"], g2["wy"], g2["wz"]), g2["ax"], g2["ay"], n2, 7)
    _check(got2, (A, rx, ry, rt))
    assert host(got2[0])[0] == 0.0
    # values only
    got3 = _call(lib, t2, c2, 7, None, grad=False)
    assert np.abs(host(got3[0]) - A).max() <= 1e-4


def test_no_alloc_size_limit(lib):
    # one cell more than the buffer holds with gradients (4 sums x (s, c) and
    # a 32-byte horizon record per cell)
    big = (16 << 20) // 64 + 1
    fake = _P(0x1000)
    rc = lib.albedo_value_and_grad_noalloc(big, *[fake] * 6, 0, None, fake, fake, fake, fake, None)
    assert rc == -2
    assert b"at most" in lib.capvndf_last_error()
    assert lib.albedo_value_and_grad_noalloc(0, *[None] * 6, 0, None, None, None, None, None,
                                             None) == 0


def test_no_alloc_binding_with_given_outputs(lib):
    """The Python binding with caller-given outputs (nothing allocated per
    call): values and gradients, then values only, equal to the workspace
    entry point bit for bit on the same inputs."""
    g = workloads.lut_grid(5, 7)
    t = to_dev(g)
    c = torch.full((35,), 3000, dtype=torch.int64, device="cuda")
    outs = [torch.empty(35, device="cuda") for _ in range(4)]
    got = cv.albedo_value_and_grad_noalloc(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], c, 5,
                                           out=outs)
    ref = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], c, 5)
    torch.cuda.synchronize()
    assert all(x is y for x, y in zip(got, outs))
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    a = torch.empty(35, device="cuda")
    only = cv.albedo_value_and_grad_noalloc(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], c, 5,
                                            with_grad=False, out=(a,))
    torch.cuda.synchronize()
    assert only[0] is a and only[1:] == (None, None, None)
    ref_value = cv.albedo_value_and_grad(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], c, 5,
                                         with_grad=False)[0]
    torch.cuda.synchronize()
    assert torch.equal(a, ref_value)
    with pytest.raises(ValueError):
        cv.albedo_value_and_grad_noalloc(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], c, 5,
                                         out=(a,))
