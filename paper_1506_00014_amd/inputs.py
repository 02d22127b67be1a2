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


# ---------------------------------------------------------------- noisy stacks (on the device)
def rasterize_ellipses_torch(n, ellipses, device):
    """rasterize_ellipses computed with torch on `device` (FP64), returned as float32."""
    import torch

    x = -1.0 + (2.0 / n) * torch.arange(n, dtype=torch.float64, device=device)
    X2, X1 = torch.meshgrid(x, x, indexing="ij")  # row index = x2, column index = x1
    img = torch.zeros(n, n, dtype=torch.float64, device=device)
    for cx, cy, a, b, phi, rho0 in ellipses:
        c, s = float(np.cos(phi)), float(np.sin(phi))
        u = (X1 - cx) * c + (X2 - cy) * s
        v = -(X1 - cx) * s + (X2 - cy) * c
        img += rho0 * ((u / a) ** 2 + (v / b) ** 2 <= 1.0).double()
    return img.float()


def ellipse_line_integrals_torch(n_theta, n_s, ellipses, device):
    """Exact line integrals of a sum of ellipse indicators (density rho0, centre c, semi-axes a
    along angle phi and b) on the grid theta_j = j pi / n_theta, s_k = -1 + 2k / n_s, computed
    with torch on `device` in FP64.  The line x . theta = s meets the ellipse in a chord of length
    2 a b sqrt(w^2 - t^2) / w^2 where t = s - c . theta and w^2 = (a cos(theta - phi))^2 +
    (b sin(theta - phi))^2 (the ellipse's half-width along theta).  Returned as float32."""
    import torch

    th = (np.pi / n_theta) * torch.arange(n_theta, dtype=torch.float64, device=device)[:, None]
    s = -1.0 + (2.0 / n_s) * torch.arange(n_s, dtype=torch.float64, device=device)[None, :]
    out = torch.zeros(n_theta, n_s, dtype=torch.float64, device=device)
    for cx, cy, a, b, phi, rho0 in ellipses:
        t = s - (cx * torch.cos(th) + cy * torch.sin(th))
        w2 = (a * torch.cos(th - phi)) ** 2 + (b * torch.sin(th - phi)) ** 2
        out += (2.0 * rho0 * a * b) * torch.sqrt(torch.clamp(w2 - t * t, min=0.0)) / w2
    return out.float()


def poisson_log_data(p, photons, seed):
    """Log-transformed Poisson data: counts ~ Poisson(photons e^{-p}) (torch generator `seed` on
    p's device), g = -log(max(counts, 1) / photons)."""
    import torch

    gen = torch.Generator(device=p.device)
    gen.manual_seed(seed)
    counts = torch.poisson(photons * torch.exp(-p.double()), generator=gen)
    return (-torch.log(torch.clamp(counts, min=1.0) / photons)).float()


def noisy_ellipse_stack(count, n, n_theta, n_s, n_ell, photons, device, seed0=5000, noise_seed=501):
    """A stack of `count` ellipse phantoms (seeds seed0 + i, n_ell ellipses each) on `device`, with
    their analytic line integrals turned into log Poisson data at `photons` incident photons per
    ray: (phantoms [count][n][n], data [count][n_theta][n_s]), float32."""
    import torch

    imgs, ps = [], []
    for i in range(count):
        ells = draw_ellipses(np.random.default_rng(seed0 + i), n_ell)
        imgs.append(rasterize_ellipses_torch(n, ells, device))
        ps.append(ellipse_line_integrals_torch(n_theta, n_s, ells, device))
    return torch.stack(imgs), poisson_log_data(torch.stack(ps), photons, noise_seed)
