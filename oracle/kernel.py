"""Fourier multiplier of the partial log-polar Radon transform (oracle, FP64).

Test infrastructure only (see the package docstring).

Paper passages followed
  * zeta(theta, rho) = delta(cos theta - e^rho): sec. 2, eq. (logdef);
  * its Fourier coefficients on the period [-beta, beta] x [log a_r, 0]:
    sec. 3, eq. (exprcoef1),
        zeta_hat(k_theta, k_rho) = int_{-beta}^{beta} e^{-2 pi i k_theta u / P}
                                   (cos u)^{-2 pi i k_rho / L - 1} du ,
    with P the theta period of the FFT lattice (P = 2 beta for K = 2 N_theta/M,
    exactly as printed; P = K * Delta theta_c in general) and L = -log a_r;
  * the prefilter in rho folded into the multiplier (sec. 4, the remark that
    1/B_hat can be applied in the Fourier domain; Algorithm 1 step 6).

Readings
  * zeta_hat is the exact integral.  The paper's FFT-trapezoid evaluation with
    end-point weights (eq. weightsa) is replaced by composite 16-point
    Gauss-Legendre quadrature with at most 8 rad of phase per panel, written
    as one complex matrix product (k_theta x nodes) @ (nodes x k_rho).
  * 1/B_hat is applied in rho only: outputs are read at lattice angles, so no
    spline evaluation happens in theta.
  * The theta decimation filter d (see radon.py) is divided out: H also carries
    1/D_hat(k_theta), D_hat being the filter's response at the coarse frequency.
  * At the rho Nyquist bin k_rho = -N_rho/2 the real part is kept, so the
    circulant kernel ifft2(H) is real.

Pins (tests/test_oracle_kernel.py): the paper's closed form (eq. P_closed_form,
appendix) evaluated with mpmath at 30 digits for k_rho != 0; the k = 0 value
2 atanh(sin beta); the line-integral form of zeta against a smooth test function
(sec. 2, the identity after eq. logdef); evenness in k_theta and conjugate
symmetry in k_rho.
"""

from __future__ import annotations

import math

import numpy as np

from .bspline import B, B_hat

GL_NODES = 16
PANEL_PHASE = 8.0  # max phase (radians) swept by the integrand inside one panel


def decimation_taps(r: int, kind: int = 0) -> np.ndarray:
    """Taps d_n, n = -(2r-1) .. 2r-1, of the theta low-pass of Algorithm 1 step 4 (sum d_n = 1).

    kind 0: the cubic B-spline d_n = B(n / r) / r.
    kind 1: the box of one coarse cell centred on the coarse node, |phi - theta'_i| <= Delta
            theta_c / 2, sampled by the trapezoid rule on the fine rows: 1/r inside, 1/(2r) on
            the two cell edges when r is even (they fall on fine rows), 0 outside."""
    n = np.arange(-(2 * r - 1), 2 * r)
    if kind == 0:
        return B(n / r) / r
    if kind == 1:
        d = np.where(2 * np.abs(n) < r, 1.0 / r, 0.0)
        return np.where(2 * np.abs(n) == r, 0.5 / r, d)
    raise ValueError(f"unknown decimation filter {kind}")


def decimation_response(r: int, k_theta: int, kind: int = 0) -> np.ndarray:
    """D_hat at coarse frequencies kt = 0..K/2: sum_n d_n cos(2 pi kt n / (r K))."""
    d = decimation_taps(r, kind)
    n = np.arange(-(2 * r - 1), 2 * r)
    kt = np.arange(k_theta // 2 + 1)
    return (d[None, :] * np.cos(2.0 * np.pi * np.outer(kt, n) / (r * k_theta))).sum(axis=1)


def gauss_legendre_panels(a: float, b: float, n_panels: int, n_nodes: int = GL_NODES):
    x, w = np.polynomial.legendre.leggauss(n_nodes)
    edges = np.linspace(a, b, n_panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    u = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    wu = (half[:, None] * w[None, :]).ravel()
    return u, wu


def zeta_hat_half(geom, kt_max=None, kr_max=None) -> np.ndarray:
    """zeta_hat(k_theta, k_rho) for k_theta = 0..K/2 and k_rho = 0..N_rho/2 (complex128)."""
    beta = geom.beta
    P = geom.k_theta * geom.dtheta_c
    L = geom.L
    nkt = geom.k_theta // 2 + 1 if kt_max is None else kt_max + 1
    nkr = geom.n_rho // 2 + 1 if kr_max is None else kr_max + 1
    max_rate = 2.0 * math.pi * (nkt - 1) / P + 2.0 * math.pi * (nkr - 1) / L * math.tan(beta)
    n_panels = max(4, int(math.ceil(2.0 * beta * max_rate / PANEL_PHASE)))
    u, wu = gauss_legendre_panels(-beta, beta, n_panels)
    lc = np.log(np.cos(u))
    amp = wu / np.cos(u)
    kt = np.arange(nkt)
    kr = np.arange(nkr)
    out = np.zeros((nkt, nkr), dtype=np.complex128)
    chunk = 2048
    for s in range(0, u.size, chunk):
        us, ls, a = u[s:s + chunk], lc[s:s + chunk], amp[s:s + chunk]
        A = np.exp(-2j * math.pi * np.outer(kt, us) / P) * a[None, :]
        Bm = np.exp(-2j * math.pi * np.outer(ls, kr) / L)
        out += A @ Bm
    return out


def multiplier_half(geom, zeta_half=None) -> np.ndarray:
    """H = zeta_hat / (B_hat(k_rho/N_rho) * D_hat(k_theta)) on k_theta = 0..K/2, k_rho = 0..N_rho/2.

    The column k_rho = N_rho/2 holds the real part (Nyquist reading)."""
    if zeta_half is None:
        zeta_half = zeta_hat_half(geom)
    kr = np.arange(geom.n_rho // 2 + 1)
    bh = B_hat(kr / geom.n_rho)
    dh = decimation_response(geom.r_dec, geom.k_theta, geom.dec_filter)
    H = zeta_half / (dh[:, None] * bh[None, :])
    H[:, -1] = H[:, -1].real
    return H


def multiplier_full(geom, H_half=None) -> np.ndarray:
    """H on the full K x N_rho lattice in numpy FFT index order, from the half table by
    evenness in k_theta and conjugate symmetry in k_rho."""
    if H_half is None:
        H_half = multiplier_half(geom)
    K, Nr = geom.k_theta, geom.n_rho
    ikt = np.arange(K)
    kt = np.minimum(ikt, K - ikt)  # |k_theta| for index ikt (index K/2 is k_theta = -K/2)
    ikr = np.arange(Nr)
    out = np.empty((K, Nr), dtype=np.complex128)
    pos = ikr <= Nr // 2
    out[:, pos] = H_half[kt][:, ikr[pos]]
    neg = ~pos
    out[:, neg] = np.conj(H_half[kt][:, Nr - ikr[neg]])
    return out
