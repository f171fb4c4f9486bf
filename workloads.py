"""Seeded synthetic inputs for the VNDF sampler and the albedo estimator.

This module is shared by the tests, the benchmark and the smoke check, and
feeds both the GPU library and the CPU oracle.  It holds none of the method's
arithmetic: it only draws view directions, roughness values, grids and sample
counts with numpy's PCG64 generator, in double precision, and rounds them to
float32 (the precision of the library's inputs).  The oracle receives those same
float32 values widened to float64.

Recipes (directions are uniform in solid angle over the upper hemisphere,
i.e. cos(theta) uniform; roughness is log-uniform, alpha = a_min ** U):

* ``tuples_small``  -- 65,536 tuples, isotropic alpha in [0.01, 1],
  cos(theta) in (0, 1].
* ``tuples_streaming`` -- 2**26 tuples, alpha_x and alpha_y independent in
  [1e-3, 1], cos(theta) in [1e-3, 1].
* ``lut_grid``      -- 64 x 64 cells: cos(theta_o) = (i + 1) / 64, isotropic
  alpha = 0.01 + 0.99 j / 63, azimuth 0.
* ``grad_grid``     -- 32 x 32 cells: alpha_x = 10^(-2 + 2 j / 31),
  alpha_y = 10^(-2 + 2 k / 31), a random view direction per cell.
* ``batch_jobs``    -- 4096 jobs: random view direction, alpha_x and alpha_y
  independent in [1e-3, 1], sample count floor(2^(10 + 12 U)) capped at 2^22.
"""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _hemisphere(rng, n, mu_min=0.0):
    """Directions uniform in solid angle with cos(theta) in (mu_min, 1]."""
    mu = 1.0 - (1.0 - mu_min) * rng.random(n)          # (mu_min, 1]
    phi = 2.0 * np.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return (s * np.cos(phi)).astype(np.float32), (s * np.sin(phi)).astype(np.float32), \
        mu.astype(np.float32)


def _log_uniform(rng, n, a_min):
    return (a_min ** rng.random(n)).astype(np.float32)


def tuples_small(n: int = 65536, seed: int = 0):
    """Dict of float32 arrays wx, wy, wz, ax, ay (ax == ay)."""
    rng = _rng(seed)
    wx, wy, wz = _hemisphere(rng, n, 0.0)
    a = _log_uniform(rng, n, 0.01)
    return {"wx": wx, "wy": wy, "wz": wz, "ax": a, "ay": a.copy()}


def tuples_streaming(n: int = 1 << 26, seed: int = 1):
    """Dict of float32 arrays wx, wy, wz, ax, ay (anisotropic)."""
    rng = _rng(seed)
    wx, wy, wz = _hemisphere(rng, n, 1e-3)
    ax = _log_uniform(rng, n, 1e-3)
    ay = _log_uniform(rng, n, 1e-3)
    return {"wx": wx, "wy": wy, "wz": wz, "ax": ax, "ay": ay}


def explicit_uniforms(n: int, seed: int):
    """Caller-supplied (u1, u2) in [0, 1) on the 2^-24 lattice, float32."""
    rng = _rng(seed)
    u1 = (rng.integers(0, 1 << 24, n) * 2.0 ** -24).astype(np.float32)
    u2 = (rng.integers(0, 1 << 24, n) * 2.0 ** -24).astype(np.float32)
    return u1, u2


def lut_grid(n_mu: int = 64, n_alpha: int = 64):
    """Cells of the directional-albedo table, row-major (mu index, alpha index)."""
    mu = (np.arange(n_mu, dtype=np.float64) + 1.0) / n_mu
    alpha = 0.01 + 0.99 * np.arange(n_alpha, dtype=np.float64) / max(1, n_alpha - 1)
    m, a = np.meshgrid(mu, alpha, indexing="ij")
    m = m.ravel()
    a = a.ravel()
    s = np.sqrt(np.maximum(0.0, 1.0 - m * m))
    return {"wx": s.astype(np.float32), "wy": np.zeros_like(s, dtype=np.float32),
            "wz": m.astype(np.float32), "ax": a.astype(np.float32),
            "ay": a.astype(np.float32)}


def grad_grid(n_side: int = 32, seed: int = 3, a_lo: float = -2.0):
    """Anisotropic cells with a random view direction each; also returns the
    spherical angles (theta_o, phi_o) of the view direction in float32."""
    rng = _rng(seed)
    e = a_lo + (-a_lo) * np.arange(n_side, dtype=np.float64) / max(1, n_side - 1)
    ax, ay = np.meshgrid(10.0 ** e, 10.0 ** e, indexing="ij")
    n = n_side * n_side
    mu = 1.0 - rng.random(n)
    phi = 2.0 * np.pi * rng.random(n)
    theta = np.arccos(mu).astype(np.float32)
    phi = phi.astype(np.float32)
    return {"theta": theta, "phi": phi, "ax": ax.ravel().astype(np.float32),
            "ay": ay.ravel().astype(np.float32)}


def batch_jobs(n_jobs: int = 4096, seed: int = 4, log2_min: int = 10, log2_max: int = 22):
    """Uneven estimation jobs: view direction, anisotropic alpha, sample count."""
    rng = _rng(seed)
    wx, wy, wz = _hemisphere(rng, n_jobs, 0.0)
    ax = _log_uniform(rng, n_jobs, 1e-3)
    ay = _log_uniform(rng, n_jobs, 1e-3)
    span = log2_max - log2_min
    n = np.floor(2.0 ** (log2_min + span * rng.random(n_jobs))).astype(np.int64)
    n = np.minimum(n, 1 << log2_max)
    return {"wx": wx, "wy": wy, "wz": wz, "ax": ax, "ay": ay, "n": n}


def view_from_angles(theta, phi):
    """Unit view directions (float32) from spherical angles (float32)."""
    t = np.asarray(theta, dtype=np.float64)
    p = np.asarray(phi, dtype=np.float64)
    return ((np.sin(t) * np.cos(p)).astype(np.float32),
            (np.sin(t) * np.sin(p)).astype(np.float32),
            np.cos(t).astype(np.float32))
