"""Pins of the oracle's direct-illumination estimator (CPU only).

The estimator of Appendix A with a non-constant incident radiance L(w_b),
here a sum of spherical-Gaussian lobes L(w) = sum lambda exp(kappa (mu.w - 1)):

* the lobe function itself: lambda at w = mu, lambda exp(-kappa) at w _|_ mu;
* a constant radiance reduces the estimator to lambda times the albedo;
* the estimator is additive over lobes (same samples);
* 2-D quadrature of int L(w_l) f_r(w_o, w_l) cos(theta_l) dw_l vs Monte Carlo
  within 4 sigma / sqrt(N), sigma estimated from independent streams.
"""

import numpy as np
import pytest

from _hemi import hemi_grid

LOBES = np.array([[0.0, 0.0, 1.0, 4.0, 2.0],
                  [0.6, 0.0, 0.8, 30.0, 5.0],
                  [-0.5, 0.5, np.sqrt(0.5), 10.0, 1.5],
                  [0.0, 0.0, 1.0, 0.0, 0.3]])


def test_lobe_function(orc):
    mu = LOBES[1, :3]
    perp = np.array([0.0, 1.0, 0.0])
    L = orc.radiance_at(tuple(np.array([[c] for c in mu])), LOBES[1:2])
    assert abs(L[0] - 5.0) < 1e-14
    L = orc.radiance_at(tuple(np.array([[c] for c in perp])), LOBES[1:2])
    assert abs(L[0] - 5.0 * np.exp(-30.0)) < 1e-20


def test_constant_radiance_is_scaled_albedo(orc):
    wo = ([0.6, 0.0, 0.3], [0.0, 0.0, 0.4], [0.8, 1.0, np.sqrt(0.75)])
    ax, ay = [0.3, 0.05, 1.0], [0.3, 0.5, 0.2]
    A = orc.albedo(wo, ax, ay, [8192] * 3, 5, f0=0.04)
    R = orc.radiance(wo, ax, ay, [8192] * 3, 5, [[0, 0, 1, 0.0, 2.5]], f0=0.04)
    assert np.allclose(R, 2.5 * A, rtol=1e-13, atol=0)


def test_additive_over_lobes(orc):
    wo = ([0.6], [0.0], [0.8])
    parts = [orc.radiance(wo, [0.3], [0.5], [4096], 9, LOBES[k:k + 1])[0] for k in range(4)]
    total = orc.radiance(wo, [0.3], [0.5], [4096], 9, LOBES)[0]
    assert abs(total - sum(parts)) < 1e-12 * max(1.0, total)


def _quad(orc, wo, ax, ay, lobes, f0, nb=384, nphi=384):
    h, w = hemi_grid(ax, ay, nb, nphi)
    wo = np.asarray(wo, dtype=np.float64)
    c = h @ wo
    wl = 2.0 * c[:, None] * h - wo
    n = h.shape[0]
    fr = orc.brdf(np.full(n, ax), np.full(n, ay), tuple(np.full(n, x) for x in wo), tuple(wl.T), f0)
    L = orc.radiance_at(tuple(wl.T), lobes)
    integrand = np.where((c > 0) & (wl[:, 2] > 0), L * fr * wl[:, 2] * 4.0 * c, 0.0)
    return (integrand * w).sum()


@pytest.mark.parametrize("ax,ay,mu,phi,f0", [
    (0.5, 0.5, 0.5, 0.0, 1.0),
    (0.2, 0.6, 0.8, 0.3, 0.04),
    (1.0, 1.0, 0.1, 2.0, 1.0),
])
def test_quadrature_vs_mc(orc, ax, ay, mu, phi, f0):
    s = np.sqrt(1 - mu * mu)
    wo = (s * np.cos(phi), s * np.sin(phi), mu)
    ref = _quad(orc, wo, ax, ay, LOBES, f0)
    N = 1 << 20
    R = orc.radiance(tuple([c] for c in wo), [ax], [ay], [N], 11, LOBES, f0=f0)[0]
    small = [orc.radiance(tuple([c] for c in wo), [ax], [ay], [4096], 100 + k, LOBES, f0=f0)[0]
             for k in range(24)]
    sig = np.std(small) * np.sqrt(4096)
    assert abs(R - ref) <= 4.0 * sig / np.sqrt(N), (R, ref, sig)
