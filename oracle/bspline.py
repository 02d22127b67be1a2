"""Cubic B-spline interpolation pieces (oracle, FP64).

Test infrastructure only (see the package docstring).

Paper passages followed (sec. 4, Interpolation)
  * B(x): the piecewise cubic before eq. (Bcoeff); the second branch reads
    (-|x|^3 + 6|x|^2 - 12|x| + 8)/6 (the printed "-12x" is taken as -12|x|, the
    only reading that keeps B even and C^2);
  * B(j) = 2/3, 1/6, 0: eq. (Bcoeff); its Fourier series 2/3 + cos(2 pi xi)/3:
    eq. (Bhat);
  * interpolation f(x) = sum_k (Qf)_k B(Nx - k): eq. (Bsplineinterp), with the
    prefilter Q defined as division by B_hat in the discrete Fourier domain (the
    "most direct way" the paper describes).  Reading: periodic boundaries, so Q is
    a circulant, symmetric matrix;
  * 4-tap form: eq. (floorx)/(wsumn).  Reading: t = index coordinate, k = floor(t),
    alpha = t - k, taps k-1..k+2 with weights B(alpha+1), B(alpha), B(1-alpha),
    B(2-alpha) (the printed alpha = x - floor(x) and the reversed weight list are
    taken as typos).

Pins (tests/test_oracle_bspline.py): B(j) values, B_hat against a direct
sum, Q followed by evaluation at the nodes reproduces the samples, O(h^4)
convergence of interpolation, the recursive filter of eq. (Qfrecursive) run on
a long periodic signal agrees with the Fourier-domain Q.
"""

from __future__ import annotations

import numpy as np


def B(x):
    """Cubic cardinal B-spline."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a < 1.0
    m2 = (a >= 1.0) & (a < 2.0)
    out[m1] = (3.0 * a[m1] ** 3 - 6.0 * a[m1] ** 2 + 4.0) / 6.0
    out[m2] = (-a[m2] ** 3 + 6.0 * a[m2] ** 2 - 12.0 * a[m2] + 8.0) / 6.0
    return out


def B_hat(xi):
    """Fourier series of the samples B(j): 2/3 + cos(2 pi xi)/3 (eq. Bhat)."""
    return 2.0 / 3.0 + np.cos(2.0 * np.pi * np.asarray(xi, dtype=np.float64)) / 3.0


def prefilter_1d(f, axis=-1):
    """Periodic prefilter Q along one axis: divide the DFT by B_hat(k/N)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    k = np.fft.fftfreq(n)
    shape = [1] * f.ndim
    shape[axis] = n
    F = np.fft.fft(f, axis=axis) / B_hat(k).reshape(shape)
    return np.real(np.fft.ifft(F, axis=axis))


def prefilter_2d(f):
    """Separable 2-D prefilter Q (rows, then columns), periodic."""
    return prefilter_1d(prefilter_1d(f, axis=-1), axis=-2)


def prefilter_recursive_1d(f, n_warm=None):
    """The causal/anticausal recursion of eq. (Qfrecursive), z = sqrt(3) - 2.

    (Qf+)_k = 6 f_k + z (Qf+)_{k-1};  (Qf)_k = z ((Qf)_{k+1} - (Qf+)_k).
    Periodic boundary: each recursion is started after running it once over the
    periodic extension (the geometric tail z^n makes this exact to rounding for
    n_warm ~ 40).  Used only as a pin for prefilter_1d."""
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    z = np.sqrt(3.0) - 2.0
    if n_warm is None:
        n_warm = 64
    reps = n_warm // n + 2
    ext = np.tile(f, reps)
    cp = 0.0
    causal = np.empty(ext.size)
    for i in range(ext.size):
        cp = 6.0 * ext[i] + z * cp
        causal[i] = cp
    causal = causal[-n:]  # periodic steady state of the causal pass
    ext2 = np.tile(causal, reps)
    out = np.empty(ext2.size)
    c = 0.0
    for i in range(ext2.size - 1, -1, -1):
        c = z * (c - ext2[i])
        out[i] = c
    return out[:n]  # periodic steady state of the anticausal pass


def taps(t):
    """Integer base k = floor(t) and the 4 weights for taps k-1, k, k+1, k+2."""
    t = np.asarray(t, dtype=np.float64)
    k = np.floor(t)
    a = t - k
    w0 = (1.0 - a) ** 3 / 6.0
    w1 = (3.0 * a ** 3 - 6.0 * a ** 2 + 4.0) / 6.0
    w2 = (-3.0 * a ** 3 + 3.0 * a ** 2 + 3.0 * a + 1.0) / 6.0
    w3 = a ** 3 / 6.0
    return k.astype(np.int64), np.stack([w0, w1, w2, w3])


def eval_periodic_1d(c, t):
    """Evaluate sum_k c_k B(t - k) with periodic c at index positions t."""
    c = np.asarray(c, dtype=np.float64)
    n = c.size
    k, w = taps(t)
    out = np.zeros(np.shape(t))
    for a in range(4):
        out = out + w[a] * c[(k - 1 + a) % n]
    return out


def eval_periodic_2d(c, X, Y):
    """Evaluate the bicubic spline with periodic coefficients c[iy, ix] at (X, Y) index positions."""
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    kx, wx = taps(X)
    ky, wy = taps(Y)
    out = np.zeros(np.shape(X))
    for b in range(4):
        row = (ky - 1 + b) % ny
        acc = np.zeros(np.shape(X))
        for a in range(4):
            acc = acc + wx[a] * c[row, (kx - 1 + a) % nx]
        out = out + wy[b] * acc
    return out
