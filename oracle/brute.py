"""Brute-force line integrals of the cubic-spline image (oracle pin, FP64).

Test infrastructure only (see the package docstring).

The exact quantity the method approximates, for an image given by its samples:
    g(theta, s) = int_{line(theta, s) cap unit disc} F(x) dl ,
with F the periodic bicubic B-spline interpolant of the samples (sec. 4, eq.
Bsplineinterp with the prefilter Q) and the line {x . theta = s} of eq.
(radon_def).  Along a line, F restricted to one grid cell is a polynomial of
degree <= 6 in the arc length, so 4-point Gauss-Legendre on every piece between
consecutive cell-boundary crossings integrates it exactly (to rounding).  Only
for small N (the cost is O(N_theta N_s N)).
"""

from __future__ import annotations

import numpy as np

from . import bspline


def line_integrals(geom, f, thetas=None, svals=None):
    f = np.asarray(f, dtype=np.float64)
    c = bspline.prefilter_2d(f)
    dx = geom.dx
    thetas = geom.theta_nodes() if thetas is None else np.asarray(thetas, dtype=np.float64)
    svals = geom.s_nodes() if svals is None else np.asarray(svals, dtype=np.float64)
    xg, wg = np.polynomial.legendre.leggauss(4)
    out = np.zeros((thetas.size, svals.size))
    for a, th in enumerate(thetas):
        ct, st = np.cos(th), np.sin(th)
        for b, s in enumerate(svals):
            if abs(s) >= 1.0:
                continue
            half = np.sqrt(1.0 - s * s)
            # x(l) = s*theta + l*theta_perp, theta_perp = (-sin, cos), l in [-half, half]
            x0, y0 = s * ct, s * st
            # index coordinates X = (x1 + 1)/dx, Y = (x2 + 1)/dx along l
            X0, Y0 = (x0 + 1.0) / dx, (y0 + 1.0) / dx
            dX, dY = -st / dx, ct / dx
            cuts = [-half, half]
            for P0, dP in ((X0, dX), (Y0, dY)):
                if abs(dP) > 1e-14:
                    lo, hi = sorted((P0 + dP * -half, P0 + dP * half))
                    ks = np.arange(np.ceil(lo), np.floor(hi) + 1)
                    cuts.extend(((ks - P0) / dP).tolist())
            cuts = np.unique(np.clip(np.array(cuts), -half, half))
            l0, l1 = cuts[:-1], cuts[1:]
            mid, hw = 0.5 * (l0 + l1), 0.5 * (l1 - l0)
            ll = (mid[:, None] + hw[:, None] * xg[None, :]).ravel()
            ww = (hw[:, None] * wg[None, :]).ravel()
            F = bspline.eval_periodic_2d(c, X0 + dX * ll, Y0 + dY * ll)
            out[a, b] = np.sum(ww * F)
    return out
