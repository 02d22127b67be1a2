"""Algorithm 2 (fast back-projection) step by step in FP64.

Test infrastructure only (see the package docstring).

Algorithm 2 computes the back-projection R# g(x) = int_0^pi g(theta, x . theta) d theta
by partial back-projections in log-polar coordinates, one per partition m
(beta = pi/M), and sums them (sec. 2 eq. backproj_lpp and the partition identity
after it; sec. 5 Algorithm 2):

  P1  c = Q g: spline coefficients of the sinogram      Alg. 2 step 1; eq. (Qfrecursive)
  for each partition m:
    P2  w(theta'_i, rho_q) = g(S_m^-1(theta'_i, rho_q)) on the coarse lattice Omega_p:
        the line of normal angle theta'_i + m beta and offset
        s = (e^rho - (1 - a_R) cos theta'_i) / a_R      Alg. 2 step 3; eq. (Sm_def),
                                                         (Lopolargrid_polar)
    P3  c_lp = periodic convolution with zeta# on the K x N_rho lattice, as
        Re IDFT2( DFT2(w) * H# ), H# = zeta#_hat / (B_hat_theta B_hat_rho)
                                                         Alg. 2 step 4; eq. (exprcoef2),
                                                         (ghatdef), (Rad_bck_lp_discrete)
    P4  f_m(x) = bicubic spline of c_lp at the log-polar coordinates of T_m x
                                                         Alg. 2 step 5; eq. (Tdef)
  f = sum_m f_m                                          Alg. 2 step 7

Readings (where the paper is silent or garbled):
  * P1: the lattice rows of P2 lie on sinogram rows (theta'_i + m beta = theta_j for
    the rows a partition owns, eq. Radon_all_pb), so the theta part of Q followed by
    evaluation at those rows is the identity and only the s part remains.  Beyond
    the n_s samples the sinogram is zero: c is the coefficient sequence of the
    cardinal cubic spline through the zero-extended row, c_k = sum_j sqrt(3)
    z^|k - j| g_j with z = sqrt(3) - 2 (the inverse of the filter (1, 4, 1)/6),
    kept on k = -PAD .. n_s + PAD - 1 and taken as zero outside (|c| < 1e-22 |g|
    there).
  * P2: only the rows a partition owns (|theta'| <= beta/2, each line once) carry
    data; the other rows of the K-row lattice are zero.  Rows that wrap past pi
    (partition 0, theta = theta' + pi) read the sinogram at -s.  No e^rho weight:
    with zeta#(theta, rho) = delta(e^rho cos theta - 1) the rho-integral of
    g(theta', rho') against zeta# returns g at the line through the point without
    a Jacobian (the derivative of e^rho cos theta - 1 in rho is 1 at its zero).
  * P3: zeta#_hat(k_theta, k_rho) = int_{-beta}^{beta} e^{-2 pi i k_theta u / P}
    (cos u)^{2 pi i k_rho / L} du (eq. exprcoef2; P = K Delta theta, L = -log a_r),
    evaluated like zeta_hat by composite Gauss-Legendre quadrature.  The 2-D B_hat
    of the algorithm is B_hat(k_theta/K) B_hat(k_rho/N_rho): the output is read at
    arbitrary (theta', rho), so it must be spline coefficients in both variables.
    The DFT conventions are those of the forward operator (1/(K N_rho) on the
    inverse; real part at the rho Nyquist bin).
  * P4: pixels x with |x| >= 1 are zero (T_m maps the unit disc onto D, where the
    partial back-projection is valid).  theta' = atan2 of T_m x, rho = log |T_m x|,
    row index (theta' - phi_0(m)) / Delta theta with phi_0 the angle of support row
    0, rho index (rho - rho_0) / Delta rho, periodic in rho.
  * The result approximates int_0^pi g(theta, x . theta) d theta, the same integral
    the exact transpose in radon.py (radon_adj) discretises.  The two agree to the
    method's discretisation error, not to rounding.

Pins: tests/test_oracle_bp.py (zeta#_hat against the paper's closed form and its
k_rho = 0 values; the interpolation property of the s-coefficients; the convolved
lattice's spline through the plain zeta#_hat convolution at the nodes; closed-form
back-projections of 1, s cos theta, s sin theta, s^2 and of a Gaussian's sinogram; FBP
of a phantom; linearity).
"""

from __future__ import annotations

import math

import numpy as np

from . import bspline
from .geometry import HALO
from .kernel import gauss_legendre_panels, multiplier_full, PANEL_PHASE
from .radon import fbp_filter

PAD = 40  # spline coefficients kept on k = -PAD .. n_s + PAD - 1
Z = math.sqrt(3.0) - 2.0


# ------------------------------------------------------------------ P3 tables
def zeta_sharp_half(geom, kt_max=None, kr_max=None) -> np.ndarray:
    """zeta#_hat(k_theta, k_rho) for k_theta = 0..K/2 and k_rho = 0..N_rho/2 (complex128)."""
    beta = geom.beta
    P = geom.k_theta * geom.dtheta
    L = geom.L
    nkt = geom.k_theta // 2 + 1 if kt_max is None else kt_max + 1
    nkr = geom.n_rho // 2 + 1 if kr_max is None else kr_max + 1
    max_rate = 2.0 * math.pi * (nkt - 1) / P + 2.0 * math.pi * (nkr - 1) / L * math.tan(beta)
    n_panels = max(4, int(math.ceil(2.0 * beta * max_rate / PANEL_PHASE)))
    u, wu = gauss_legendre_panels(-beta, beta, n_panels)
    lc = np.log(np.cos(u))
    kt = np.arange(nkt)
    kr = np.arange(nkr)
    out = np.zeros((nkt, nkr), dtype=np.complex128)
    chunk = 2048
    for s in range(0, u.size, chunk):
        us, ls, a = u[s:s + chunk], lc[s:s + chunk], wu[s:s + chunk]
        A = np.exp(-2j * math.pi * np.outer(kt, us) / P) * a[None, :]
        Bm = np.exp(2j * math.pi * np.outer(ls, kr) / L)  # (cos u)^(2 pi i k_rho / L)
        out += A @ Bm
    return out


def multiplier_sharp_half(geom, zeta_half=None) -> np.ndarray:
    """H# = zeta#_hat / (B_hat(k_theta/K) B_hat(k_rho/N_rho)) on k_theta = 0..K/2,
    k_rho = 0..N_rho/2; real part at the rho Nyquist column."""
    if zeta_half is None:
        zeta_half = zeta_sharp_half(geom)
    kt = np.arange(geom.k_theta // 2 + 1)
    kr = np.arange(geom.n_rho // 2 + 1)
    H = zeta_half / (bspline.B_hat(kt / geom.k_theta)[:, None] * bspline.B_hat(kr / geom.n_rho)[None, :])
    H[:, -1] = H[:, -1].real
    return H


# ------------------------------------------------------------------ P1
def s_coefficients(g) -> np.ndarray:
    """Spline coefficients along s of every sinogram row, zero-extended:
    c[:, PAD + k] = sum_j sqrt(3) z^|k - j| g[:, j] for k = -PAD .. n_s + PAD - 1."""
    g = np.asarray(g, dtype=np.float64)
    ns = g.shape[-1]
    k = np.arange(-PAD, ns + PAD)
    j = np.arange(ns)
    Hm = math.sqrt(3.0) * Z ** np.abs(k[:, None] - j[None, :]).astype(np.float64)
    return g @ Hm.T


def eval_s(c_row, t):
    """sum_k c_k B(t - k) with c_row from s_coefficients (index k stored at k + PAD), zero
    outside the stored range."""
    k, w = bspline.taps(t)
    out = np.zeros(np.shape(t))
    n = c_row.size
    for a in range(4):
        idx = k - 1 + a + PAD
        ok = (idx >= 0) & (idx < n)
        out = out + np.where(ok, w[a] * c_row[np.clip(idx, 0, n - 1)], 0.0)
    return out


# ------------------------------------------------------------------ P2-P4
def lattice_samples(geom, c, p) -> np.ndarray:
    """P2 for partition p: W[K, N_rho], owned row pos at lattice row HALO + pos."""
    a_R = geom.a_R
    E = np.exp(geom.rho_nodes())
    W = np.zeros((geom.k_theta, geom.n_rho))
    for pos, (j, wrap, nu) in enumerate(geom.partition_rows(p)):
        thp = math.pi * nu / (geom.n_theta * geom.m)
        s = (E - (1.0 - a_R) * math.cos(thp)) / a_R
        if wrap:
            s = -s
        W[HALO + pos] = eval_s(c[j], (s + 1.0) / geom.ds)
    return W


def conv_sharp(geom, W, H_full=None) -> np.ndarray:
    """P3: Re IDFT2(DFT2(W) * H#) with numpy's conventions."""
    if H_full is None:
        H_full = multiplier_full(geom, multiplier_sharp_half(geom))
    return np.real(np.fft.ifft2(np.fft.fft2(W) * H_full))


def pixel_coords(geom, p):
    """P4 positions for partition p: (mask of pixels with |x| < 1, row index, rho index)."""
    n = geom.n
    x1 = -1.0 + geom.dx * np.arange(n)
    X1, X2 = np.meshgrid(x1, x1)  # [iy, ix]: X1 = x_1 (columns), X2 = x_2 (rows)
    k = 2 * np.arange(n) - n  # node i sits at x = (2i - n)/n: |x| < 1 decided exactly
    inside = k[None, :] ** 2 + k[:, None] ** 2 < n * n
    mb = p * geom.beta
    a_R = geom.a_R
    # y = T_m x = a_R Rot(-m beta) x + (1 - a_R, 0)
    y1 = a_R * (math.cos(mb) * X1 + math.sin(mb) * X2) + (1.0 - a_R)
    y2 = a_R * (-math.sin(mb) * X1 + math.cos(mb) * X2)
    thp = np.arctan2(y2, y1)
    rho = 0.5 * np.log(y1 * y1 + y2 * y2)
    rho0 = (1 - geom.n_rho) * geom.d_rho
    T = (thp - geom.phi0(p)) / geom.dtheta
    Pr = (rho - rho0) / geom.d_rho
    return inside, T, Pr


def gather(geom, C, p) -> np.ndarray:
    """P4: bicubic spline of the lattice coefficients C[K, N_rho] at T_m x, zero for |x| >= 1."""
    inside, T, Pr = pixel_coords(geom, p)
    K, Nr = C.shape
    kt, wt = bspline.taps(np.where(inside, T, 0.0))
    kr, wr = bspline.taps(np.where(inside, Pr, 0.0))
    out = np.zeros(inside.shape)
    for a in range(4):
        rows = (kt - 1 + a) % K
        acc = np.zeros(inside.shape)
        for b in range(4):
            acc = acc + wr[b] * C[rows, (kr - 1 + b) % Nr]
        out = out + wt[a] * acc
    return np.where(inside, out, 0.0)


def radon_bp_lp(geom, g) -> np.ndarray:
    """Algorithm 2: g[N_theta, N_s] -> f[N, N] (row = x2, column = x1)."""
    g = np.asarray(g, dtype=np.float64)
    assert g.shape == (geom.n_theta, geom.n_s)
    if geom.q_theta != 1:
        raise ValueError("Algorithm 2 here uses the lattice of the sinogram rows (q_theta = 1)")
    c = s_coefficients(g)                                            # P1
    H_full = multiplier_full(geom, multiplier_sharp_half(geom))
    f = np.zeros((geom.n, geom.n))
    for p in range(geom.m):
        W = lattice_samples(geom, c, p)                              # P2
        C = conv_sharp(geom, W, H_full)                              # P3
        f += gather(geom, C, p)                                      # P4
    return f


def fbp_lp(geom, g, name="ramlak") -> np.ndarray:
    """Filtered back-projection through Algorithm 2: radon_bp_lp of the filtered sinogram."""
    return radon_bp_lp(geom, fbp_filter(geom, g, name))
