"""Quadrature over the upper hemisphere of microfacet normals (test helper).

Directions are parameterised in the stretched slope space of a GGX surface:
h = p / |p| with p = (ax r cos(phi), ay r sin(phi), 1) and r = tan(beta),
beta in [0, pi/2).  The solid-angle element of this map is
ax ay r / |p|^3 dr dphi (the triple product of p with its two partial
derivatives over |p|^3), and dr = sec^2(beta) dbeta.  Gauss-Legendre nodes in
beta and phi then concentrate where a GGX lobe of that roughness has its mass.
"""

import numpy as np


def hemi_grid(ax, ay, nb=512, nphi=512, beta_lo=0.0, beta_hi=np.pi / 2):
    xb, wb = np.polynomial.legendre.leggauss(nb)
    xp, wp = np.polynomial.legendre.leggauss(nphi)
    beta = beta_lo + (beta_hi - beta_lo) * (xb + 1.0) / 2.0
    wbeta = wb * (beta_hi - beta_lo) / 2.0
    phi = np.pi * (xp + 1.0)
    wphi = wp * np.pi
    B, P = np.meshgrid(beta, phi, indexing="ij")
    WB, WP = np.meshgrid(wbeta, wphi, indexing="ij")
    r = np.tan(B)
    px = ax * r * np.cos(P)
    py = ay * r * np.sin(P)
    norm = np.sqrt(px * px + py * py + 1.0)
    h = np.stack([px / norm, py / norm, 1.0 / norm], axis=-1).reshape(-1, 3)
    jac = ax * ay * r / norm ** 3 / np.cos(B) ** 2
    w = (jac * WB * WP).reshape(-1)
    return h, w


def slope_coords(h, ax, ay):
    """Inverse of the parameterisation: (beta, phi in [0, 2 pi)) of normals h."""
    sx = h[:, 0] / (ax * h[:, 2])
    sy = h[:, 1] / (ay * h[:, 2])
    beta = np.arctan(np.hypot(sx, sy))
    phi = np.mod(np.arctan2(sy, sx), 2 * np.pi)
    return beta, phi


def binned_grid(ax, ay, b_edges, p_edges, nq=12):
    """Gauss-Legendre nodes inside every (beta, phi) bin.

    Returns h of shape (nbeta_bins * nphi_bins * nq * nq, 3), the matching
    solid-angle weights, and the flat bin index of every node."""
    x, wq = np.polynomial.legendre.leggauss(nq)
    b_lo, b_hi = np.asarray(b_edges[:-1]), np.asarray(b_edges[1:])
    p_lo, p_hi = np.asarray(p_edges[:-1]), np.asarray(p_edges[1:])
    beta = b_lo[:, None] + (b_hi - b_lo)[:, None] * (x[None, :] + 1.0) / 2.0   # (nb, nq)
    wbeta = (b_hi - b_lo)[:, None] * wq[None, :] / 2.0
    phi = p_lo[:, None] + (p_hi - p_lo)[:, None] * (x[None, :] + 1.0) / 2.0    # (np, nq)
    wphi = (p_hi - p_lo)[:, None] * wq[None, :] / 2.0
    nb, npb = len(b_lo), len(p_lo)
    B = np.broadcast_to(beta[:, None, :, None], (nb, npb, nq, nq))
    P = np.broadcast_to(phi[None, :, None, :], (nb, npb, nq, nq))
    W = wbeta[:, None, :, None] * wphi[None, :, None, :]
    r = np.tan(B)
    px = ax * r * np.cos(P)
    py = ay * r * np.sin(P)
    norm = np.sqrt(px * px + py * py + 1.0)
    h = np.stack([px / norm, py / norm, 1.0 / norm], axis=-1).reshape(-1, 3)
    w = (ax * ay * r / norm ** 3 / np.cos(B) ** 2 * W).reshape(-1)
    idx = np.broadcast_to(np.arange(nb * npb).reshape(nb, npb, 1, 1), (nb, npb, nq, nq))
    return h, w, idx.reshape(-1)
