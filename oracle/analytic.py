"""Closed-form Radon transforms used as pins (oracle, FP64).

Test infrastructure only (see the package docstring).

R f(theta, s) = int f(x) delta(x . theta - s) dx with x . theta = x1 cos theta +
x2 sin theta (sec. 1, eq. radon_def).  Closed forms (standard calculus, stated
so a reader can check them by hand):
  * Gaussian f = A exp(-|x - c|^2 / sigma^2):
        R f = A sigma sqrt(pi) exp(-(s - c . theta)^2 / sigma^2);
  * ellipse of density rho0, centre c, semi-axes a (along angle phi) and b:
        R f = 2 rho0 a b sqrt(a_t^2 - t^2) / a_t^2  for |t| <= a_t, else 0,
        t = s - c . theta,  a_t^2 = a^2 cos^2(theta - phi) + b^2 sin^2(theta - phi)
    (a disc of radius r centred at 0 gives 2 sqrt(r^2 - s^2));
  * back-projection over theta in [0, pi) of g(theta, s) = exp(-s^2 / sigma^2):
        R# g(x) = pi exp(-|x|^2 / (2 sigma^2)) I0(|x|^2 / (2 sigma^2)).
"""

from __future__ import annotations

import numpy as np
from scipy.special import i0e


def gaussian_sino(theta, s, cx, cy, sigma, amp=1.0):
    th = np.asarray(theta, dtype=np.float64)[:, None]
    s = np.asarray(s, dtype=np.float64)[None, :]
    t = s - (cx * np.cos(th) + cy * np.sin(th))
    return amp * sigma * np.sqrt(np.pi) * np.exp(-(t * t) / (sigma * sigma))


def gaussian_image(x, cx, cy, sigma, amp=1.0):
    x = np.asarray(x, dtype=np.float64)
    X1, X2 = np.meshgrid(x, x)  # X1 varies along columns (x1), X2 along rows (x2)
    return amp * np.exp(-((X1 - cx) ** 2 + (X2 - cy) ** 2) / (sigma * sigma))


def ellipse_sino(theta, s, ellipses):
    """ellipses: iterable of (cx, cy, a, b, phi, rho0)."""
    th = np.asarray(theta, dtype=np.float64)[:, None]
    s = np.asarray(s, dtype=np.float64)[None, :]
    out = np.zeros((th.shape[0], s.shape[1]))
    for cx, cy, a, b, phi, rho0 in ellipses:
        t = s - (cx * np.cos(th) + cy * np.sin(th))
        at2 = (a * np.cos(th - phi)) ** 2 + (b * np.sin(th - phi)) ** 2
        out += 2.0 * rho0 * a * b * np.sqrt(np.maximum(at2 - t * t, 0.0)) / at2
    return out


def backproject_gaussian_ridge(x, sigma):
    """R# of g(theta, s) = exp(-s^2/sigma^2) at image nodes (theta over [0, pi))."""
    x = np.asarray(x, dtype=np.float64)
    X1, X2 = np.meshgrid(x, x)
    z = (X1 * X1 + X2 * X2) / (2.0 * sigma * sigma)
    return np.pi * i0e(z)  # exp(-z) I0(z)
