"""Spherical-cap GGX VNDF sampling on MI355X -- Python binding of libcapvndf.so.

Method: Dupuy and Benyoub, "Sampling Visible GGX Normals with Spherical Caps"
(arXiv 2306.05044).  Every step of the path runs in the HIP kernels of
``libcapvndf.so``; this module only marshals torch tensors (device memory and
the current stream) into the C ABI declared in ``include/capvndf.h``.  There is
no CPU fallback: without the built library every call raises.

Names mirror the C entry points: ``vndf_sample``, ``vndf_pdf``, ``vndf_inverse``,
``albedo_estimate``, ``albedo_estimate_backward``, ``albedo_value_and_grad``
(and ``albedo_value_and_grad_noalloc``),
``albedo_workspace_size``, ``radiance_estimate``,
``BatchPlan`` (``albedo_batch_plan_create`` / ``albedo_batch_run`` /
``albedo_batch_run_per_request``), ``albedo_batch_autotune``, and the hooks
``capvndf_uniforms``, ``capvndf_philox_blocks``, ``vndf_microbench`` and
``capvndf_stream_probe``.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime that libcapvndf.so links against

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcapvndf.so")

CAP = 0
DISK2018 = 1
CAP_F64 = 2
TAG_SAMPLE = 2
TAG_ALBEDO = 3

_METHODS = {"cap": CAP, "disk2018": DISK2018, "cap_f64": CAP_F64, CAP: CAP,
            DISK2018: DISK2018, CAP_F64: CAP_F64}


class CapvndfError(RuntimeError):
    """A libcapvndf call returned an error code."""

    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with code {code}: {msg}")
        self.code = code


class Tiling(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("pairs_per_thread", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("per_wave", ctypes.c_int32),
                ("dynamic", ctypes.c_int32)]

    def as_tuple(self):
        return (self.block, self.pairs_per_thread, self.blocks_per_cu, self.per_wave,
                self.dynamic)


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32

_SIGNATURES = {
    "capvndf_version": ([], _I32),
    "capvndf_last_error": ([], ctypes.c_char_p),
    "vndf_sample": ([_I64, _P, _P, _P, _P, _P, _P, _P, _U64, _U64, _I32, _P, _P, _P, _P, _P], _I32),
    "vndf_pdf": ([_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "vndf_inverse": ([_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "dielectric_sample": ([_I64, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_float, _U64, _U64, _P,
                           _P, _P, _P, _P, _P], _I32),
    "dielectric_pdf": ([_I64, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_float, _P, _P], _I32),
    "albedo_workspace_size": ([_I64, _P, _I32], ctypes.c_size_t),
    "albedo_estimate": ([_I64, _P, _P, _P, _P, _P, _P, _U64, _P, _P, _P, ctypes.c_size_t, _P],
                        _I32),
    "albedo_estimate_backward": ([_I64, _P, _P, _P, _P, _P, _P, _U64, _P, _P, _P, _P, _P, _P,
                                  ctypes.c_size_t, _P], _I32),
    "albedo_value_and_grad": ([_I64, _P, _P, _P, _P, _P, _P, _U64, _P, _P, _P, _P, _P, _P,
                               ctypes.c_size_t, _P], _I32),
    "albedo_value_and_grad_noalloc": ([_I64, _P, _P, _P, _P, _P, _P, _U64, _P, _P, _P, _P, _P,
                                       _P], _I32),
    "radiance_estimate": ([_I64, _P, _P, _P, _P, _P, _P, _P, _U64, _P, _I32, _P, _P,
                           ctypes.c_size_t, _P], _I32),
    "albedo_view_from_angles": ([_I64, _P, _P, _P, _P, _P, _P], _I32),
    "albedo_apply_jacobian": ([_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "albedo_batch_plan_create": ([_I64, _P, _P, _P, _P, _P, _P, _P, _U64, _I32, _P, _P, _P, _P,
                                  ctypes.POINTER(Tiling), _P, ctypes.POINTER(_P)], _I32),
    "albedo_batch_run": ([_P, _P], _I32),
    "albedo_batch_run_per_request": ([_P, _P], _I32),
    "albedo_batch_plan_info": ([_P, ctypes.POINTER(Tiling), ctypes.POINTER(_I64),
                                ctypes.POINTER(_I64)], _I32),
    "albedo_batch_plan_destroy": ([_P], None),
    "albedo_batch_autotune": ([_I64, _P, _P, _P, _P, _P, _P, _P, _U64, _I32, _P, _P, _P, _P, _P,
                               ctypes.POINTER(Tiling), ctypes.POINTER(ctypes.c_float)], _I32),
    "capvndf_uniforms": ([_U64, _U32, _U32, _U64, _I64, _P, _P, _P], _I32),
    "capvndf_philox_blocks": ([_I64, _P, _U32, _U32, _P, _P], _I32),
    "vndf_microbench": ([_I32, _I64, _I32, _U64, _P, _P], _I32),
    "estimator_microbench": ([_I32, _I64, _I32, _U64, _P, _P, _P], _I32),
    "capvndf_stream_probe": ([_I32, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcapvndf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libcapvndf.so not found at {path}: build it first "
            "(python paper_2306_05044_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(fn, rc):
    if rc != 0:
        msg = load_library().capvndf_last_error().decode(errors="replace")
        raise CapvndfError(fn, rc, msg)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name, dtype=torch.float32):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (there is no CPU path)")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on {t.device}, but the current device is "
                         f"cuda:{torch.cuda.current_device()}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _same_len(n, **ts):
    for k, t in ts.items():
        if t is not None and t.numel() != n:
            raise ValueError(f"{k} has {t.numel()} elements, expected {n}")


def version() -> int:
    return int(load_library().capvndf_version())


def vndf_sample(wix, wiy, wiz, ax, ay, u1=None, u2=None, seed=0, index_base=0, method="cap_f64",
                with_pdf=True, out=None, stream=None):
    """GGX VNDF samples h (and pdf) for SoA float32 GPU tensors; see
    include/capvndf.h.  Returns (hx, hy, hz, pdf_or_None)."""
    lib = load_library()
    n = wix.numel()
    for k, t in dict(wix=wix, wiy=wiy, wiz=wiz, ax=ax, ay=ay, u1=u1, u2=u2).items():
        _dev(t, k)
    _same_len(n, wiy=wiy, wiz=wiz, ax=ax, ay=ay, u1=u1, u2=u2)
    if out is None:
        hx, hy, hz = (torch.empty_like(wix) for _ in range(3))
        pdf = torch.empty_like(wix) if with_pdf else None
    else:
        hx, hy, hz, pdf = out
        for k, t in dict(hx=hx, hy=hy, hz=hz, pdf=pdf).items():
            _dev(t, k)
        _same_len(n, hx=hx, hy=hy, hz=hz, pdf=pdf)
    m = _METHODS.get(method, method)
    rc = lib.vndf_sample(n, _ptr(wix), _ptr(wiy), _ptr(wiz), _ptr(ax), _ptr(ay), _ptr(u1),
                         _ptr(u2), seed, index_base, m, _ptr(hx), _ptr(hy), _ptr(hz), _ptr(pdf),
                         _stream(stream))
    _check("vndf_sample", rc)
    return hx, hy, hz, pdf


def vndf_pdf(wix, wiy, wiz, hx, hy, hz, ax, ay, out=None, stream=None):
    """VNDF pdf of Eq. (1) at given unit normals."""
    lib = load_library()
    n = wix.numel()
    for k, t in dict(wix=wix, wiy=wiy, wiz=wiz, hx=hx, hy=hy, hz=hz, ax=ax, ay=ay).items():
        _dev(t, k)
    _same_len(n, wiy=wiy, wiz=wiz, hx=hx, hy=hy, hz=hz, ax=ax, ay=ay)
    pdf = torch.empty_like(wix) if out is None else _dev(out, "out")
    rc = lib.vndf_pdf(n, _ptr(wix), _ptr(wiy), _ptr(wiz), _ptr(hx), _ptr(hy), _ptr(hz), _ptr(ax),
                      _ptr(ay), _ptr(pdf), _stream(stream))
    _check("vndf_pdf", rc)
    return pdf


def vndf_inverse(wix, wiy, wiz, hx, hy, hz, ax, ay, out=None, stream=None):
    """Uniforms (u1, u2) that the cap sampler maps to the given normals."""
    lib = load_library()
    n = wix.numel()
    for k, t in dict(wix=wix, wiy=wiy, wiz=wiz, hx=hx, hy=hy, hz=hz, ax=ax, ay=ay).items():
        _dev(t, k)
    _same_len(n, wiy=wiy, wiz=wiz, hx=hx, hy=hy, hz=hz, ax=ax, ay=ay)
    if out is None:
        u1, u2 = torch.empty_like(wix), torch.empty_like(wix)
    else:
        u1, u2 = (_dev(x, "out") for x in out)
        _same_len(n, u1=u1, u2=u2)
    rc = lib.vndf_inverse(n, _ptr(wix), _ptr(wiy), _ptr(wiz), _ptr(hx), _ptr(hy), _ptr(hz),
                          _ptr(ax), _ptr(ay), _ptr(u1), _ptr(u2), _stream(stream))
    _check("vndf_inverse", rc)
    return u1, u2


def dielectric_sample(wix, wiy, wiz, ax, ay, eta, seed=0, index_base=0, u=None, out=None,
                      stream=None):
    """Rough-dielectric sampling with the cap VNDF: (wox, woy, woz, pdf, weight).
    ``u`` is None (Philox stream) or a tuple (u1, u2, u3) of float32 tensors."""
    lib = load_library()
    n = wix.numel()
    us = (None, None, None) if u is None else tuple(u)
    if len(us) != 3:
        raise ValueError("u must be None or (u1, u2, u3)")
    for k, t in dict(wix=wix, wiy=wiy, wiz=wiz, ax=ax, ay=ay, u1=us[0], u2=us[1], u3=us[2]).items():
        _dev(t, k)
    _same_len(n, wiy=wiy, wiz=wiz, ax=ax, ay=ay, u1=us[0], u2=us[1], u3=us[2])
    if out is None:
        outs = tuple(torch.empty_like(wix) for _ in range(5))
    else:
        outs = tuple(_dev(x, "out") for x in out)
        if len(outs) != 5:
            raise ValueError("out must hold (wox, woy, woz, pdf, weight)")
        _same_len(n, **{f"out{i}": x for i, x in enumerate(outs)})
    rc = lib.dielectric_sample(n, _ptr(wix), _ptr(wiy), _ptr(wiz), _ptr(ax), _ptr(ay),
                               *[_ptr(x) for x in us], float(eta), int(seed), int(index_base),
                               *[_ptr(x) for x in outs], _stream(stream))
    _check("dielectric_sample", rc)
    return outs


def dielectric_pdf(wix, wiy, wiz, wox, woy, woz, ax, ay, eta, out=None, stream=None):
    """Density of dielectric_sample at given unit pairs (wi, wo)."""
    lib = load_library()
    n = wix.numel()
    for k, t in dict(wix=wix, wiy=wiy, wiz=wiz, wox=wox, woy=woy, woz=woz, ax=ax, ay=ay).items():
        _dev(t, k)
    _same_len(n, wiy=wiy, wiz=wiz, wox=wox, woy=woy, woz=woz, ax=ax, ay=ay)
    pdf = torch.empty_like(wix) if out is None else _dev(out, "out")
    _same_len(n, pdf=pdf)
    rc = lib.dielectric_pdf(n, _ptr(wix), _ptr(wiy), _ptr(wiz), _ptr(wox), _ptr(woy), _ptr(woz),
                            _ptr(ax), _ptr(ay), float(eta), _ptr(pdf), _stream(stream))
    _check("dielectric_pdf", rc)
    return pdf


def albedo_workspace_size(ncells: int, nsamples_host=None, with_grad: int = 0) -> int:
    """Workspace bytes of the table estimators for ncells cells; nsamples_host
    (host int64 counts per cell, or None) lets the call use fewer slots."""
    if nsamples_host is None:
        ptr = None
    else:
        nsamples_host = np.ascontiguousarray(np.asarray(nsamples_host, dtype=np.int64))
        if nsamples_host.size != ncells:
            raise ValueError("nsamples_host must have one entry per cell")
        ptr = nsamples_host.ctypes.data_as(ctypes.c_void_p)
    return int(load_library().albedo_workspace_size(ncells, ptr, int(with_grad)))


def _workspace(nbytes, device):
    return torch.empty(max(1, (nbytes + 3) // 4), dtype=torch.float32, device=device)


def _counts(nsamples, n, device):
    """Per-cell sample counts as (device int64 tensor, host int64 array or
    None).  An int gives every cell that count; a host sequence or CPU tensor
    is copied to the device; a GPU tensor is used as it is (no host copy, so
    the workspace is sized without the counts)."""
    if isinstance(nsamples, torch.Tensor) and nsamples.is_cuda:
        _dev(nsamples, "nsamples", torch.int64)
        _same_len(n, nsamples=nsamples)
        return nsamples, None
    if isinstance(nsamples, (int, np.integer)):
        host = np.full(n, int(nsamples), dtype=np.int64)
        return torch.full((n,), int(nsamples), dtype=torch.int64, device=device), host
    if isinstance(nsamples, torch.Tensor):
        nsamples = nsamples.numpy()
    host = np.ascontiguousarray(np.asarray(nsamples, dtype=np.int64).reshape(-1))
    if host.size != n:
        raise ValueError(f"nsamples has {host.size} entries, expected {n}")
    return torch.from_numpy(host).to(device), host


def _table_setup(wox, n, nsamples, with_grad, workspace):
    dev_counts, host = _counts(nsamples, n, wox.device)
    if workspace is None:
        nbytes = albedo_workspace_size(n, host, with_grad) if n > 0 else 0
        workspace = _workspace(nbytes, wox.device)
    else:
        _dev(workspace, "workspace")
    return dev_counts, workspace


def albedo_estimate(wox, woy, woz, ax, ay, nsamples, seed, workspace=None, stream=None):
    """(s_f1, s_f5) per cell: A(F0) = F0 s_f1 + (1 - F0) s_f5.  nsamples: an
    int for every cell, or one count per cell (host sequence or int64 tensor)."""
    lib = load_library()
    n = wox.numel()
    for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay).items():
        _dev(t, k)
    _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay)
    ns, ws = _table_setup(wox, n, nsamples, 0, workspace)
    s1 = torch.empty_like(wox)
    s5 = torch.empty_like(wox)
    rc = lib.albedo_estimate(n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay), _ptr(ns),
                             seed, _ptr(s1), _ptr(s5), _ptr(ws), ws.numel() * 4, _stream(stream))
    _check("albedo_estimate", rc)
    return s1, s5


def albedo_estimate_backward(wox, woy, woz, ax, ay, nsamples, seed, f0=None, grad_albedo=None,
                             workspace=None, stream=None):
    """(grad_ax, grad_ay, grad_theta_o) per cell for A(F0), times grad_albedo."""
    lib = load_library()
    n = wox.numel()
    for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0,
                     grad_albedo=grad_albedo).items():
        _dev(t, k)
    _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0, grad_albedo=grad_albedo)
    ns, ws = _table_setup(wox, n, nsamples, 1, workspace)
    gx, gy, gt = (torch.empty_like(wox) for _ in range(3))
    rc = lib.albedo_estimate_backward(n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay),
                                      _ptr(ns), seed, _ptr(f0), _ptr(grad_albedo), _ptr(gx),
                                      _ptr(gy), _ptr(gt), _ptr(ws), ws.numel() * 4,
                                      _stream(stream))
    _check("albedo_estimate_backward", rc)
    return gx, gy, gt


def albedo_value_and_grad(wox, woy, woz, ax, ay, nsamples, seed, f0=None, with_grad=True,
                          workspace=None, stream=None):
    """(A(F0), dA/d alpha_x, dA/d alpha_y, dA/d theta_o) per cell from one pass;
    the gradients are None when with_grad is False."""
    lib = load_library()
    n = wox.numel()
    for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0).items():
        _dev(t, k)
    _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0)
    ns, ws = _table_setup(wox, n, nsamples, 1 if with_grad else 0, workspace)
    a = torch.empty_like(wox)
    g = [torch.empty_like(wox) for _ in range(3)] if with_grad else [None, None, None]
    rc = lib.albedo_value_and_grad(n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay),
                                   _ptr(ns), seed, _ptr(f0), _ptr(a), *[_ptr(x) for x in g],
                                   _ptr(ws), ws.numel() * 4, _stream(stream))
    _check("albedo_value_and_grad", rc)
    return (a, *g)


def albedo_value_and_grad_noalloc(wox, woy, woz, ax, ay, nsamples, seed, f0=None,
                                  with_grad=True, stream=None, out=None):
    """albedo_value_and_grad on the library's own device buffer (no workspace
    argument).  `nsamples` must already be a GPU int64 tensor and `out`, if
    given, the (albedo, grad_ax, grad_ay, grad_theta_o) tensors (the grads
    None without gradients), so that the call allocates nothing."""
    lib = load_library()
    n = wox.numel()
    for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0).items():
        _dev(t, k)
    _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0)
    if not (isinstance(nsamples, torch.Tensor) and nsamples.is_cuda):
        raise TypeError("nsamples must be a GPU int64 tensor")
    _dev(nsamples, "nsamples", torch.int64)
    _same_len(n, nsamples=nsamples)
    if out is None:
        a = torch.empty_like(wox)
        g = [torch.empty_like(wox) for _ in range(3)] if with_grad else [None, None, None]
    else:
        a = out[0]
        g = list(out[1:4]) if with_grad else []
        if len(g) != (3 if with_grad else 0):
            raise ValueError("out must hold albedo and, with gradients, the three gradient tensors")
        g += [None] * (3 - len(g))
        for k, x in zip(("albedo", "grad_ax", "grad_ay", "grad_theta_o"), [a] + g):
            if x is not None:
                _dev(x, k)
                _same_len(n, **{k: x})
    rc = lib.albedo_value_and_grad_noalloc(n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay),
                                           _ptr(nsamples), seed, _ptr(f0), _ptr(a),
                                           *[_ptr(x) for x in g], _stream(stream))
    _check("albedo_value_and_grad_noalloc", rc)
    return (a, *g)


def radiance_estimate(wox, woy, woz, ax, ay, nsamples, seed, lobes, f0=None, workspace=None,
                      stream=None):
    """Direct illumination per cell under spherical-Gaussian lobes; lobes is a
    float32 GPU tensor of shape (nlobes, 5): (mu_x, mu_y, mu_z, kappa, lambda)."""
    lib = load_library()
    n = wox.numel()
    for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0, lobes=lobes).items():
        _dev(t, k)
    _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0)
    if lobes.dim() != 2 or lobes.shape[1] != 5:
        raise ValueError("lobes must have shape (nlobes, 5)")
    ns, ws = _table_setup(wox, n, nsamples, 0, workspace)
    out = torch.empty_like(wox)
    rc = lib.radiance_estimate(n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay), _ptr(f0),
                               _ptr(ns), seed, _ptr(lobes), lobes.shape[0], _ptr(out), _ptr(ws),
                               ws.numel() * 4, _stream(stream))
    _check("radiance_estimate", rc)
    return out


def albedo_view_from_angles(theta_o, phi_o, out=None, stream=None):
    """View directions (sin t cos p, sin t sin p, cos t) from their angles;
    returns (wox, woy, woz)."""
    lib = load_library()
    _dev(theta_o, "theta_o")
    _dev(phi_o, "phi_o")
    n = theta_o.numel()
    _same_len(n, phi_o=phi_o)
    wox, woy, woz = out if out is not None else [torch.empty_like(theta_o) for _ in range(3)]
    for k, t in dict(wox=wox, woy=woy, woz=woz).items():
        _dev(t, k)
    _same_len(n, wox=wox, woy=woy, woz=woz)
    _check("albedo_view_from_angles",
           lib.albedo_view_from_angles(n, _ptr(theta_o), _ptr(phi_o), _ptr(wox), _ptr(woy),
                                       _ptr(woz), _stream(stream)))
    return wox, woy, woz


def albedo_apply_jacobian(grad_albedo, d_ax=None, d_ay=None, d_theta_o=None, s_f1=None,
                          s_f5=None, stream=None):
    """Chain rule through the diagonal Jacobian: g * d_ax, g * d_ay,
    g * d_theta_o and g * (s_f1 - s_f5) (None where the input is None)."""
    lib = load_library()
    _dev(grad_albedo, "grad_albedo")
    n = grad_albedo.numel()
    ins = dict(d_ax=d_ax, d_ay=d_ay, d_theta_o=d_theta_o, s_f1=s_f1, s_f5=s_f5)
    for k, t in ins.items():
        _dev(t, k)
    _same_len(n, **ins)
    if (s_f1 is None) != (s_f5 is None):
        raise ValueError("give both s_f1 and s_f5 or neither")
    outs = [None if t is None else torch.empty_like(grad_albedo) for t in (d_ax, d_ay, d_theta_o, s_f1)]
    _check("albedo_apply_jacobian",
           lib.albedo_apply_jacobian(n, _ptr(grad_albedo), _ptr(d_ax), _ptr(d_ay),
                                     _ptr(d_theta_o), _ptr(s_f1), _ptr(s_f5), *[_ptr(o) for o in outs],
                                     _stream(stream)))
    return tuple(outs)


class BatchPlan:
    """Batched forward (+ adjoint) estimation of uneven jobs; one graph replay
    per run().  Holds the output tensors it writes."""

    def __init__(self, wox, woy, woz, ax, ay, nsamples, seed, f0=None, with_grad=True,
                 tiling=None, stream=None):
        lib = load_library()
        n = wox.numel()
        for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0).items():
            _dev(t, k)
        _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0)
        ns = torch.as_tensor(nsamples, dtype=torch.int64).cpu().contiguous()
        if ns.numel() != n:
            raise ValueError("nsamples must have one entry per job")
        self._inputs = (wox, woy, woz, ax, ay, f0, ns)
        self.albedo = torch.empty_like(wox)
        self.grad_ax = torch.empty_like(wox) if with_grad else None
        self.grad_ay = torch.empty_like(wox) if with_grad else None
        self.grad_theta_o = torch.empty_like(wox) if with_grad else None
        t = None
        if tiling is not None:
            t = Tiling(int(tiling[0]), int(tiling[1]), int(tiling[2]),
                       int(tiling[3]) if len(tiling) > 3 else 0,
                       int(tiling[4]) if len(tiling) > 4 else 0)
        plan = ctypes.c_void_p()
        rc = lib.albedo_batch_plan_create(
            n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay), _ptr(f0),
            ctypes.c_void_p(ns.data_ptr()), seed, 1 if with_grad else 0, _ptr(self.albedo),
            _ptr(self.grad_ax), _ptr(self.grad_ay), _ptr(self.grad_theta_o),
            ctypes.byref(t) if t is not None else None, _stream(stream), ctypes.byref(plan))
        _check("albedo_batch_plan_create", rc)
        self._plan = plan

    def run(self, stream=None):
        _check("albedo_batch_run", load_library().albedo_batch_run(self._plan, _stream(stream)))

    def run_per_request(self, stream=None):
        _check("albedo_batch_run_per_request",
               load_library().albedo_batch_run_per_request(self._plan, _stream(stream)))

    def info(self):
        t = Tiling()
        nch = _I64()
        tot = _I64()
        _check("albedo_batch_plan_info",
               load_library().albedo_batch_plan_info(self._plan, ctypes.byref(t),
                                                     ctypes.byref(nch), ctypes.byref(tot)))
        return {"tiling": t.as_tuple(), "nchunks": nch.value, "total_samples": tot.value}

    def close(self):
        if getattr(self, "_plan", None):
            load_library().albedo_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def albedo_batch_autotune(wox, woy, woz, ax, ay, nsamples, seed, f0=None, with_grad=True,
                          stream=None):
    """Time candidate tilings on these jobs; returns
    ((block, ppt, bpc, per_wave, dynamic), ms)."""
    lib = load_library()
    n = wox.numel()
    for k, t in dict(wox=wox, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0).items():
        _dev(t, k)
    _same_len(n, woy=woy, woz=woz, ax=ax, ay=ay, f0=f0)
    ns = torch.as_tensor(nsamples, dtype=torch.int64).cpu().contiguous()
    if ns.numel() != n:
        raise ValueError("nsamples must have one entry per job")
    outs = [torch.empty_like(wox) for _ in range(4)]
    best = Tiling()
    ms = ctypes.c_float()
    rc = lib.albedo_batch_autotune(n, _ptr(wox), _ptr(woy), _ptr(woz), _ptr(ax), _ptr(ay),
                                   _ptr(f0), ctypes.c_void_p(ns.data_ptr()), seed,
                                   1 if with_grad else 0, *[_ptr(o) for o in outs],
                                   _stream(stream), ctypes.byref(best), ctypes.byref(ms))
    _check("albedo_batch_autotune", rc)
    return best.as_tuple(), ms.value


def capvndf_uniforms(seed, tag, unit, k0, n, device="cuda", out=None, stream=None):
    """(u1, u2) of samples k0..k0+n-1 of Philox stream (seed, tag, unit);
    ``out`` optionally gives the two float32 tensors of n elements to fill."""
    if out is None:
        u1 = torch.empty(n, dtype=torch.float32, device=device)
        u2 = torch.empty(n, dtype=torch.float32, device=device)
    else:
        u1, u2 = out
        _dev(u1, "u1")
        _dev(u2, "u2")
        _same_len(n, u1=u1, u2=u2)
    _check("capvndf_uniforms", load_library().capvndf_uniforms(
        seed, tag, unit, k0, n, _ptr(u1), _ptr(u2), _stream(stream)))
    return u1, u2


def capvndf_philox_blocks(ctr, key0, key1, stream=None):
    """Raw Philox4x32-10 of an int32 (n, 4) counter tensor (bit patterns)."""
    _dev(ctr, "ctr", torch.int32)
    out = torch.empty_like(ctr)
    _check("capvndf_philox_blocks", load_library().capvndf_philox_blocks(
        ctr.numel() // 4, _ptr(ctr), key0, key1, _ptr(out), _stream(stream)))
    return out


def vndf_microbench(method, lanes, iters, seed=1, out=None, stream=None):
    """Register-resident sampler benchmark; returns the per-lane int32 fold."""
    o = torch.empty(lanes, dtype=torch.int32, device="cuda") if out is None else out
    _check("vndf_microbench", load_library().vndf_microbench(
        _METHODS.get(method, method), lanes, iters, seed, _ptr(o), _stream(stream)))
    return o


def estimator_microbench(kind, lanes, pairs, seed=1, lobes=None, out=None, stream=None):
    """Register-resident benchmark of an estimator's per-sample arithmetic
    (kind 0 forward, 1 value + adjoint, 2 radiance under 4 lobes given as a
    (4, 5) float32 GPU tensor); returns the per-lane int32 fold."""
    o = torch.empty(lanes, dtype=torch.int32, device="cuda") if out is None else out
    if lobes is not None:
        _dev(lobes, "lobes")
        if lobes.numel() != 20:
            raise ValueError("lobes must hold 4 lobes of 5 values")
    _check("estimator_microbench", load_library().estimator_microbench(
        int(kind), lanes, pairs, seed, _ptr(lobes), _ptr(o), _stream(stream)))
    return o


def capvndf_stream_probe(ins, outs, mode=0, stream=None):
    """Streaming probe over 5 input and 4 output float32 GPU tensors: mode 0
    the sampler's traffic, 1 the reads only, 2 the writes only."""
    n = ins[0].numel()
    for k, t in enumerate(list(ins) + list(outs)):
        _dev(t, f"probe array {k}")
    _same_len(n, **{f"a{k}": t for k, t in enumerate(list(ins) + list(outs))})
    _check("capvndf_stream_probe", load_library().capvndf_stream_probe(
        int(mode), n, *[_ptr(t) for t in ins], *[_ptr(t) for t in outs], _stream(stream)))


from .autograd import AlbedoFunction, albedo  # noqa: E402,F401
