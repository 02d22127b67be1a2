"""EM reconstruction on the oracle's R and R# (sec. 7, the EM iteration), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One step, for measured data g >= 0 and an image f > 0:
    f_next = f * R#( chi_C g / R f ) / R# chi_C,
where chi_C(theta, s) is 1 on the lines that pass through the unit disc (|s| < 1: every
s-node but s = -1 on the grid s_k = -1 + k ds) and 0 elsewhere.  Readings where the paper
is silent: the ratio is 0 on lines where R f <= 0 (the approximate R can dip below zero
near the support's edge); the image lives on the unit disc, the support of f (R ignores
samples outside it): f_next is 0 at pixels with |x| >= 1 or R# chi_C <= 0.

Pins (tests/test_oracle_em.py): a positive f is a fixed point of the step for g = R f; the
step preserves the weighted flux sum_x f_next R# chi_C = (w_S / w_X) sum of g over the
lines in C with R f > 0 (an identity of the adjoint); R# chi_C is pi inside the disc (the
back-projection of ones over [0, pi)) to the method's accuracy.
"""

from __future__ import annotations

import numpy as np

from .radon import radon_adj, radon_fwd


def chi_c(geom) -> np.ndarray:
    """chi_C on the sinogram grid [n_theta][n_s]."""
    s = geom.s_nodes()
    return np.tile((np.abs(s) < 1.0).astype(np.float64), (geom.n_theta, 1))


def disc_mask(geom) -> np.ndarray:
    """Pixels x with |x| < 1 (node coordinates), the support of the EM image."""
    # node i sits at x = (2i - n)/n: decide |x| < 1 exactly in integers
    k = 2 * np.arange(geom.n) - geom.n
    return k[None, :] ** 2 + k[:, None] ** 2 < geom.n ** 2


def em_norm(geom, mode="fft") -> np.ndarray:
    """R# chi_C, the denominator of the step."""
    return radon_adj(geom, chi_c(geom), mode=mode)


def em_ratio(geom, g, rf) -> np.ndarray:
    """chi_C g / R f on lines with R f > 0, else 0."""
    g = np.asarray(g, dtype=np.float64)
    rf = np.asarray(rf, dtype=np.float64)
    out = np.zeros_like(g)
    ok = (chi_c(geom) > 0) & (rf > 0)
    out[ok] = g[ok] / rf[ok]
    return out


def em_step(geom, g, f, norm=None, mode="fft") -> np.ndarray:
    if norm is None:
        norm = em_norm(geom, mode)
    f = np.asarray(f, dtype=np.float64)
    back = radon_adj(geom, em_ratio(geom, g, radon_fwd(geom, f, mode=mode)), mode=mode)
    out = np.zeros_like(f)
    ok = disc_mask(geom) & (norm > 0)
    out[ok] = f[ok] * back[ok] / norm[ok]
    return out


def em(geom, g, f0, iters, mode="fft") -> np.ndarray:
    norm = em_norm(geom, mode)
    f = np.asarray(f0, dtype=np.float64)
    for _ in range(iters):
        f = em_step(geom, g, f, norm, mode)
    return f
