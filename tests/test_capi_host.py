"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/capvndf.h, and rejects bad arguments on
the host before any HIP call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "capvndf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


@pytest.fixture(scope="module")
def lib():
    import paper_2306_05044_amd as cv
    if not os.path.exists(cv.LIB_PATH):
        pytest.fail("libcapvndf.so is not built (run python paper_2306_05044_amd/build.py)")
    return cv.load_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("vndf_sample", "vndf_pdf", "albedo_estimate", "albedo_estimate_backward",
                     "albedo_workspace_size", "albedo_batch_plan_create", "albedo_batch_run",
                     "albedo_batch_plan_destroy", "capvndf_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(__import__("paper_2306_05044_amd").LIB_PATH)
    for name in _declared_functions():
        assert hasattr(raw, name), name


def test_binding_covers_the_header():
    import paper_2306_05044_amd as cv
    assert set(_declared_functions()) == set(cv.exported_symbols())


def test_version(lib):
    import re
    hdr = open(os.path.join(ROOT, "include", "capvndf.h")).read()
    assert lib.capvndf_version() == int(re.search(r"#define CAPVNDF_VERSION (\d+)", hdr).group(1))
    # the binding's tiling struct matches the header's field list
    import paper_2306_05044_amd as cv
    fields = re.search(r"typedef struct capvndf_tiling \{(.*?)\}", hdr, re.S).group(1)
    names = re.findall(r"int32_t (\w+);", fields)
    assert [f[0] for f in cv.Tiling._fields_] == names


def _err(lib):
    return lib.capvndf_last_error().decode()


def test_sample_argument_errors(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: validation fails first
    args = [fake] * 5
    assert lib.vndf_sample(-1, *args, None, None, 0, 0, 0, fake, fake, fake, None, None) == -2
    assert "n = -1" in _err(lib)
    assert lib.vndf_sample(8, *args, None, None, 0, 0, 7, fake, fake, fake, None, None) == -4
    assert lib.vndf_sample(8, *args, fake, None, 0, 0, 0, fake, fake, fake, None, None) == -1
    assert lib.vndf_sample(8, None, fake, fake, fake, fake, None, None, 0, 0, 0, fake, fake, fake,
                           None, None) == -1
    assert "wix is NULL" in _err(lib)
    mis = P(0x1002)
    assert lib.vndf_sample(8, mis, fake, fake, fake, fake, None, None, 0, 0, 0, fake, fake, fake,
                           None, None) == -3
    # n == 0 enqueues nothing and succeeds even with NULL arrays
    assert lib.vndf_sample(0, None, None, None, None, None, None, None, 0, 0, 0, None, None, None,
                           None, None) == 0
    assert lib.vndf_inverse(-5, *[None] * 10, None) == -2
    assert lib.vndf_inverse(3, *[fake] * 9, None, None) == -1
    assert lib.vndf_pdf(-5, *[None] * 9, None) == -2
    assert lib.vndf_pdf(0, *[None] * 9, None) == 0


def test_albedo_argument_errors(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)
    i64 = ctypes.c_int64

    def counts(*v):
        return (i64 * len(v))(*v)

    # workspace: ncells * slots * partial sums * 8 bytes, plus with gradients
    # a 32-byte horizon record per slot; slots per cell aim at 8192 blocks with
    # at least 32, below 2^24 blocks, and (given host counts) no more than the
    # largest cell's chunks of 16384 samples
    assert lib.albedo_workspace_size(-1, None, 0) == 0
    assert lib.albedo_workspace_size(0, None, 0) == 0
    assert lib.albedo_workspace_size(1 << 24, None, 0) == 0
    assert lib.albedo_workspace_size(16, None, 2) == 0
    assert lib.albedo_workspace_size(4096, None, 0) == 4096 * 32 * 2 * 8
    assert lib.albedo_workspace_size(4096, None, 1) == 4096 * 32 * (4 * 8 + 32)
    assert lib.albedo_workspace_size(4096, counts(*[1 << 20] * 4096), 0) == 4096 * 32 * 2 * 8
    assert lib.albedo_workspace_size(4096, counts(*[4096] * 4096), 1) == 4096 * 1 * (4 * 8 + 32)
    assert lib.albedo_workspace_size(1, None, 0) == 8192 * 2 * 8
    assert lib.albedo_workspace_size(1, counts(1 << 20), 0) == 64 * 2 * 8
    assert lib.albedo_workspace_size(1, counts(1 << 30), 1) == 8192 * (4 * 8 + 32)
    assert lib.albedo_workspace_size(3, counts(0, 1, 0), 0) == 3 * 1 * 2 * 8
    assert lib.albedo_workspace_size(2, counts(0, 0), 0) == 2 * 1 * 2 * 8
    assert lib.albedo_workspace_size(1 << 20, None, 0) == (1 << 20) * 15 * 2 * 8
    assert lib.albedo_workspace_size(2, counts(5, -1), 0) == 0
    assert lib.albedo_workspace_size(2, counts(5, 1 << 40), 0) == 0
    five = [fake] * 5
    assert lib.albedo_estimate(-1, *five, fake, 0, fake, fake, fake, 1 << 20, None) == -2
    assert lib.albedo_estimate(1 << 24, *five, fake, 0, fake, fake, fake, 1 << 62, None) == -2
    assert "below 2^24" in _err(lib)
    assert lib.radiance_estimate(1 << 24, *five, None, fake, 0, None, 0, fake, fake, 1 << 62,
                                 None) == -2
    assert lib.albedo_estimate(4, *five, None, 0, fake, fake, fake, 1 << 20, None) == -1
    assert "nsamples" in _err(lib)
    assert lib.albedo_estimate(4, *five, P(0x1004), 0, fake, fake, fake, 1 << 20, None) == -3
    assert lib.albedo_estimate(4, *five, fake, 0, fake, fake, fake, 4 * 16 - 1, None) == -5
    assert "workspace" in _err(lib)
    assert lib.albedo_estimate(4, *five, fake, 0, fake, fake, None, 1 << 20, None) == -5
    assert lib.albedo_estimate(4, *five, fake, 0, fake, fake, P(0x1008), 1 << 20, None) == -3
    assert lib.albedo_estimate(4, *five, fake, 0, None, fake, fake, 1 << 20, None) == -1
    assert lib.albedo_estimate(0, *[None] * 5, None, 0, None, None, None, 0, None) == 0
    assert lib.albedo_estimate_backward(4, *five, fake, 0, None, None, fake, fake, fake, fake,
                                        4 * (24 + 32) - 1, None) == -5
    # value_and_grad: partial gradient outputs, small workspace, no value output
    assert lib.albedo_value_and_grad(4, *five, fake, 0, None, fake, fake, None, None, fake,
                                     1 << 20, None) == -1
    assert lib.albedo_value_and_grad(4, *five, fake, 0, None, fake, fake, fake, fake, fake,
                                     4 * (32 + 32) - 1, None) == -5
    assert lib.albedo_value_and_grad(4, *five, fake, 0, None, None, None, None, None, fake,
                                     4 * 8 - 1, None) == -1
    assert lib.albedo_value_and_grad(4, *five, fake, 0, None, fake, None, None, None, fake,
                                     4 * 8 - 1, None) == -5
    assert lib.radiance_estimate(4, *five, None, fake, 0, fake, 9, fake, fake, 1 << 20, None) == -2
    assert lib.radiance_estimate(4, *five, None, fake, 0, None, 2, fake, fake, 1 << 20, None) == -1
    assert lib.radiance_estimate(4, *five, None, fake, 0, fake, 2, fake, fake, 4 * 8 - 1,
                                 None) == -5
    out = P()
    ns = (ctypes.c_int64 * 2)(10, 20)
    assert lib.albedo_batch_plan_create(0, *five, None, ns, 0, 1, fake, fake, fake, fake, None,
                                        None, ctypes.byref(out)) == -2
    assert lib.albedo_batch_plan_create(2, *five, None, None, 0, 1, fake, fake, fake, fake, None,
                                        None, ctypes.byref(out)) == -1
    bad = (ctypes.c_int64 * 2)(10, -20)
    assert lib.albedo_batch_plan_create(2, *five, None, bad, 0, 1, fake, fake, fake, fake, None,
                                        None, ctypes.byref(out)) == -2
    assert lib.albedo_batch_plan_create(2, *five, None, ns, 0, 2, fake, fake, fake, fake, None,
                                        None, ctypes.byref(out)) == -7
    assert lib.albedo_batch_run(None, None) == -1
    lib.albedo_batch_plan_destroy(None)  # no-op


def test_no_alloc_argument_errors(lib):
    """albedo_value_and_grad_noalloc validates before it touches a device:
    its cell limit (64 bytes per cell with gradients, 8 without, in a 16 MiB
    buffer), partial gradient outputs, and an empty call."""
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: validation fails first
    five = [fake] * 5
    fn = lib.albedo_value_and_grad_noalloc
    limit_grad, limit_value = (16 << 20) // 64, (16 << 20) // 8
    assert fn(limit_grad + 1, *five, fake, 0, None, fake, fake, fake, fake, None) == -2
    assert "at most %d cells" % limit_grad in _err(lib)
    assert fn(limit_value + 1, *five, fake, 0, None, fake, None, None, None, None) == -2
    assert "at most %d cells" % limit_value in _err(lib)
    assert fn(4, *five, fake, 0, None, fake, fake, None, None, None) == -1
    assert fn(4, *five, fake, 0, None, None, fake, fake, fake, None) == -1
    assert fn(0, *[None] * 5, None, 0, None, None, None, None, None, None) == 0
    assert fn(-1, *[None] * 5, None, 0, None, None, None, None, None, None) == -2


def test_gradient_helper_argument_errors(lib):
    P = ctypes.c_void_p
    fake, odd = P(0x1000), P(0x1002)
    assert lib.albedo_view_from_angles(-1, fake, fake, fake, fake, fake, None) == -2
    assert lib.albedo_view_from_angles(0, None, None, None, None, None, None) == 0
    assert lib.albedo_view_from_angles(4, fake, None, fake, fake, fake, None) == -1
    assert "phi_o" in _err(lib)
    assert lib.albedo_view_from_angles(4, fake, fake, odd, fake, fake, None) == -3
    none4 = [None] * 4
    assert lib.albedo_apply_jacobian(-1, fake, *[None] * 5, *none4, None) == -2
    # an input without its output, and the reverse
    assert lib.albedo_apply_jacobian(4, fake, fake, None, None, None, None, *none4, None) == -1
    assert "d_ax" in _err(lib)
    assert lib.albedo_apply_jacobian(4, fake, None, None, None, None, None, None, None, fake, None,
                                     None) == -1
    assert "d_theta_o" in _err(lib)
    # F0 needs both sums
    assert lib.albedo_apply_jacobian(4, fake, None, None, None, fake, None, None, None, None, fake,
                                     None) == -1
    assert "s_f5" in _err(lib)
    assert lib.albedo_apply_jacobian(4, None, fake, None, None, None, None, fake, None, None, None,
                                     None) == -1
    assert "grad_albedo" in _err(lib)
    assert lib.albedo_apply_jacobian(4, fake, odd, None, None, None, None, fake, None, None, None,
                                     None) == -3
    assert lib.albedo_apply_jacobian(0, None, fake, None, None, None, None, fake, None, None, None,
                                     None) == 0


def test_dielectric_argument_errors(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: validation fails first
    nou = [None] * 3
    assert lib.dielectric_sample(-1, *[fake] * 5, *nou, 1.5, 0, 0, *[fake] * 5, None) == -2
    for bad in (1.0, 0.0, -1.5, float("inf"), float("nan")):
        assert lib.dielectric_sample(4, *[fake] * 5, *nou, bad, 0, 0, *[fake] * 5, None) == -7
        assert "eta" in _err(lib)
        assert lib.dielectric_pdf(4, *[fake] * 8, bad, fake, None) == -7
    assert lib.dielectric_sample(4, *[fake] * 5, *nou, 1.5, 0, 0, *[fake] * 4, None, None) == -1
    assert "weight is NULL" in _err(lib)
    assert lib.dielectric_sample(4, *[fake] * 5, fake, None, fake, 1.5, 0, 0, *[fake] * 5,
                                 None) == -1
    assert "u1, u2, u3" in _err(lib)
    assert lib.dielectric_sample(4, P(0x1002), *[fake] * 4, *nou, 1.5, 0, 0, *[fake] * 5,
                                 None) == -3
    assert lib.dielectric_pdf(-3, *[None] * 8, 1.5, None, None) == -2
    assert lib.dielectric_pdf(0, *[None] * 8, 1.5, None, None) == 0
    assert lib.dielectric_sample(0, *[None] * 5, *nou, 1.5, 0, 0, *[None] * 5, None) == 0
