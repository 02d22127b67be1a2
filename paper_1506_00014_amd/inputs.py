"""Seeded synthetic inputs: ellipse phantoms, Gaussian blobs, random images.

This module holds no arithmetic of the transform itself; it only draws inputs
(numpy PCG64 generators, FP64) that the tests, the benchmark and the smoke
check feed to both the HIP path and the CPU reference.

The phantoms stand in for the modified Shepp-Logan phantom the paper uses
(sec. 6): sums of ellipse indicator functions with densities of mixed sign,
supported inside the unit disc.  Pixels are node samples x = -1 + i*2/N,
row index = x2, column index = x1.
"""

from __future__ import annotations

import numpy as np


def _nodes(n):
    return -1.0 + (2.0 / n) * np.arange(n)


def draw_ellipses(rng, count, centre=0.6, axes=(0.05, 0.4), dens=(-0.5, 1.0), reach=0.95):
    """count ellipses (cx, cy, a, b, phi, rho0); each is redrawn until |c| + max(a, b) <= reach."""
    out = []
    while len(out) < count:
        cx, cy = rng.uniform(-centre, centre, size=2)
        a, b = rng.uniform(axes[0], axes[1], size=2)
        phi = rng.uniform(0.0, np.pi)
        rho0 = rng.uniform(dens[0], dens[1])
        if np.hypot(cx, cy) + max(a, b) <= reach:
            out.append((float(cx), float(cy), float(a), float(b), float(phi), float(rho0)))
    return out


def rasterize_ellipses(n, ellipses):
    x = _nodes(n)
    X1, X2 = np.meshgrid(x, x)
    img = np.zeros((n, n))
    for cx, cy, a, b, phi, rho0 in ellipses:
        u = (X1 - cx) * np.cos(phi) + (X2 - cy) * np.sin(phi)
        v = -(X1 - cx) * np.sin(phi) + (X2 - cy) * np.cos(phi)
        img += rho0 * ((u / a) ** 2 + (v / b) ** 2 <= 1.0)
    return img


def ellipse_phantom(n, count, seed):
    """(image[n, n] float64, ellipse list) for a seeded phantom."""
    rng = np.random.default_rng(seed)
    ells = draw_ellipses(rng, count)
    return rasterize_ellipses(n, ells), ells


def draw_gaussians(rng, count, sigma=(0.02, 0.1), amp=(-0.5, 1.0), reach=0.95):
    """count blobs (cx, cy, sigma, amp) with centres uniform in the disc of radius reach - 4 sigma."""
    out = []
    for _ in range(count):
        s = rng.uniform(sigma[0], sigma[1])
        a = rng.uniform(amp[0], amp[1])
        rad = (reach - 4.0 * s) * np.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * np.pi)
        out.append((float(rad * np.cos(ang)), float(rad * np.sin(ang)), float(s), float(a)))
    return out


def rasterize_gaussians(n, blobs):
    x = _nodes(n)
    X1, X2 = np.meshgrid(x, x)
    img = np.zeros((n, n))
    for cx, cy, s, a in blobs:
        img += a * np.exp(-((X1 - cx) ** 2 + (X2 - cy) ** 2) / (s * s))
    return img


def mixed_phantom(n, n_ell, n_gauss, seed):
    """Ellipses plus Gaussian blobs from one seeded generator: (image, ellipses, blobs)."""
    rng = np.random.default_rng(seed)
    ells = draw_ellipses(rng, n_ell)
    blobs = draw_gaussians(rng, n_gauss)
    return rasterize_ellipses(n, ells) + rasterize_gaussians(n, blobs), ells, blobs


def uniform_image(n, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(n, n))


def normal_array(shape, seed):
    return np.random.default_rng(seed).standard_normal(size=shape)
