"""Pins of the oracle's densities (CPU only).

* Eq. (1) integrates to one over the hemisphere (Gauss-Legendre quadrature);
* the NDF is normalised, int D(h) h_z dh = 1, and G1's denominator is the
  projected area, int D(h) max(0, w.h) dh = w_z / G1(w) (Appendix A);
* closed form at alpha = 1 (the ellipsoid is the hemisphere itself):
  pdf = 2 max(0, wi.h) / (pi (1 + z_i));
* the two routes of the paper to the pdf agree: Eq. (1) equals
  G1(wi) max(0, wi.h) D(h) / z_i built from the Appendix A functions;
* D, G1, G2 and f_r against textbook closed forms (Walter et al. 2007 for D;
  Smith's Lambda for G1 and the height-correlated G2 = 1 / (1 + L_i + L_o)),
  which the oracle does not use;
* f_r is reciprocal, f_r(a, b) = f_r(b, a).
"""

import numpy as np
import pytest

from _hemi import hemi_grid
import workloads

CASES = [
    (0.3, 0.6, 0.2, 0.7),
    (0.05, 0.05, 0.05, 0.0),
    (1.0, 1.0, 1.0, 0.0),
    (0.001, 0.01, 0.5, 1.0),
    (1.0, 0.05, 0.02, 2.0),
    (0.5, 0.5, 0.999, 3.0),
]


def _dirs(mu, phi, n):
    s = np.sqrt(1.0 - mu * mu)
    return (np.full(n, s * np.cos(phi)), np.full(n, s * np.sin(phi)), np.full(n, mu))


@pytest.mark.parametrize("ax,ay,mu,phi", CASES)
def test_normalisations(orc, ax, ay, mu, phi):
    h, w = hemi_grid(ax, ay, 512, 512)
    n = h.shape[0]
    hh = (h[:, 0], h[:, 1], h[:, 2])
    wi = _dirs(mu, phi, n)
    pdf = orc.vndf_pdf(wi, hh, np.full(n, ax), np.full(n, ay))
    assert abs((pdf * w).sum() - 1.0) < 1e-6
    D = orc.ggx_ndf(hh, ax, ay)
    assert abs((D * h[:, 2] * w).sum() - 1.0) < 1e-9
    wv = np.array([c[0] for c in wi])
    g1 = orc.smith_g1((np.zeros(1), np.zeros(1), np.ones(1)), tuple(np.array([c]) for c in wv),
                      ax, ay)[0]
    proj = (D * np.maximum(0.0, h @ wv) * w).sum()
    assert abs(proj / (mu / g1) - 1.0) < 1e-6


def test_alpha_one_closed_form(orc):
    d = workloads.tuples_small(5000, seed=3)
    n = 5000
    wi = (d["wx"], d["wy"], d["wz"])
    one = np.ones(n)
    h, pdf = orc.vndf_sample(wi, one, one, seed=8)
    w = np.stack([c.astype(np.float64) for c in wi], axis=1)
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    ref = 2.0 * np.maximum(0.0, np.einsum("ij,ij->i", w, h)) / (np.pi * (1.0 + w[:, 2]))
    assert np.allclose(pdf, ref, rtol=1e-12)


def test_two_routes_to_the_pdf(orc):
    d = workloads.tuples_streaming(5000, seed=4)
    n = 5000
    wi = tuple(c.astype(np.float64) for c in (d["wx"], d["wy"], d["wz"]))
    h, pdf = orc.vndf_sample(wi, d["ax"], d["ay"], seed=9)
    hh = (h[:, 0], h[:, 1], h[:, 2])
    D = orc.ggx_ndf(hh, d["ax"], d["ay"])
    z = np.zeros(n)
    G1 = orc.smith_g1((z, z, np.ones(n)), wi, d["ax"], d["ay"])
    w = np.stack(wi, axis=1)
    nw = np.linalg.norm(w, axis=1)
    alt = G1 * np.maximum(0.0, np.einsum("ij,ij->i", w, h)) * D / w[:, 2]
    assert np.allclose(pdf, alt * 1.0, rtol=1e-11)
    assert np.all(nw > 0)


def _lambda(w, ax, ay):
    """Smith's Lambda for the anisotropic GGX NDF (Heitz 2014)."""
    t2 = (ax * ax * w[:, 0] ** 2 + ay * ay * w[:, 1] ** 2) / w[:, 2] ** 2
    return (-1.0 + np.sqrt(1.0 + t2)) / 2.0


def test_textbook_closed_forms(orc):
    rng = np.random.default_rng(5)
    n = 4000
    ax = 10 ** (-2 * rng.random(n))
    ay = 10 ** (-2 * rng.random(n))

    def rand_dirs():
        mu = 1 - rng.random(n) * 0.98
        phi = 2 * np.pi * rng.random(n)
        s = np.sqrt(1 - mu * mu)
        return np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)

    wa, wb = rand_dirs(), rand_dirs()
    wh = wa + wb
    wh /= np.linalg.norm(wh, axis=1, keepdims=True)
    # Walter et al. 2007 anisotropic GGX
    k = wh[:, 0] ** 2 / ax ** 2 + wh[:, 1] ** 2 / ay ** 2 + wh[:, 2] ** 2
    D_ref = 1.0 / (np.pi * ax * ay * k * k)
    D = orc.ggx_ndf(tuple(wh.T), ax, ay)
    assert np.allclose(D, D_ref, rtol=1e-12)
    La, Lb = _lambda(wa, ax, ay), _lambda(wb, ax, ay)
    G1 = orc.smith_g1(tuple(wh.T), tuple(wa.T), ax, ay)
    assert np.allclose(G1, 1.0 / (1.0 + La), rtol=1e-12)
    for f0 in (1.0, 0.04):
        x = np.einsum("ij,ij->i", wh, wb)
        F = f0 + (1 - f0) * (1 - x) ** 5
        fr_ref = F * D_ref / (1.0 + La + Lb) / (4.0 * wa[:, 2] * wb[:, 2])
        fr = orc.brdf(ax, ay, tuple(wa.T), tuple(wb.T), f0)
        assert np.allclose(fr, fr_ref, rtol=1e-11)
        fr_swapped = orc.brdf(ax, ay, tuple(wb.T), tuple(wa.T), f0)
        assert np.allclose(fr, fr_swapped, rtol=1e-12)
    # below the horizon everything vanishes
    wb_low = wb.copy()
    wb_low[:, 2] *= -1
    assert np.all(orc.brdf(ax, ay, tuple(wa.T), tuple(wb_low.T), 1.0) == 0.0)
    assert np.all(orc.smith_g1(tuple(wh.T), tuple(wb_low.T), ax, ay) == 0.0)
