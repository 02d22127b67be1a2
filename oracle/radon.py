"""Algorithm 1 (fast Radon transform), its exact weighted transpose (the
back-projection R#) and filtered back-projection, step by step in FP64.

Test infrastructure only (see the package docstring).

The forward operator is the composition of the steps of Algorithm 1 (sec. 5),
each a linear map, in the paper's order and notation:

  S2  c = Q f                            Alg. 1 step 1; sec. 4 eq. (Bsplineinterp)
  for each partition m (beta = pi/M):
    S3  v(phi_t, rho_q) = (T_m f)(e^rho (cos phi, sin phi)) on the fine grid
        Omega_lp, by the bicubic spline of c, zero outside D
                                        Alg. 1 step 3; eq. (Tdef), (circle_D),
                                        (Lopolargrid_f), (wsumn)
    S4  u = low-pass in theta + decimation to the coarse grid Omega_p
                                        Alg. 1 step 4; eq. (Lopolargrid_polar)
    S5  w = u * e^rho                    Alg. 1 step 5
    S6  c_lp = periodic convolution with zeta on the K x N_rho lattice, as
        Re IDFT2( DFT2(w) * H ), H = zeta_hat / (B_hat_rho D_hat_theta)
                                        Alg. 1 step 6; eq. (lograd_periodic),
                                        (exprcoef1), (fhatdef)
    S7  g(theta_j, s_k) = a_R^-1 * sum_q c_lp[row(j), q] B(tau_jk - q), with
        tau from S_m(theta, s) = (theta - m beta, log(a_R s + (1 - a_R) cos(theta - m beta)))
        on the rows m owns               Alg. 1 step 7; eq. (Radon_all_pb), (Sm_def)

Readings (where the paper is silent or garbled; see also geometry.py,
bspline.py and kernel.py):
  * S4 filter (unspecified in the paper): d_n = B(n/r)/r, |n| < 2r, applied to
    the fine rows at phi_i + n*Delta theta_c/r, and divided out in H (or the box
    of one coarse cell, geom.dec_filter = 1; on a lattice of spacing Delta
    theta_c = Delta theta / q_theta, geom.q_theta = 2, the owned rows sit on every
    other lattice row);
  * S6 convolution mode "fft" (numpy FFTs) or "direct" (the circulant sum with
    the real kernel ifft2(H), for tiny sizes);
  * R# is the exact transpose of R weighted by the grids' quadrature weights:
    <R f, g>_S = <f, R# g>_X with w_S = Delta theta Delta s, w_X = Delta x^2, so
    R# = (w_S / w_X) * R^T.  (The paper's Algorithm 2 agrees with this only to
    discretisation error; the transpose gives the adjoint identity exactly and
    exact gradients.)  Each step is transposed: S6^T multiplies by conj(H),
    S2^T = S2 (periodic Q is symmetric);
  * W (eq. ramp) is the Ram-Lak kernel on the s-grid applied as a linear
    (zero-padded) convolution: h_0 = 1/(4 ds^2), h_n = -1/(pi^2 n^2 ds^2) for odd
    n, 0 for even n != 0; (W g)_k = ds * sum_n h_n g_{k-n}.  R# integrates over
    theta in [0, pi), so FBP is R# W with no extra factor.  The cosine and Shepp-Logan
    filters (eqs. cosfilt, SLfilt) multiply the ramp's DFT on the zero-padded s-axis by a
    window (filter_window), then cut the rows back to n_s samples.

Pins: tests/test_oracle_radon.py (closed forms, brute-force line integrals,
adjoint identity, direct vs FFT convolution, rotation covariance).
"""

from __future__ import annotations

import math

import numpy as np

from . import bspline
from .kernel import decimation_taps, multiplier_full

MASK_EPS = 1e-9  # samples closer than this (in e^rho) to the boundary of D count as outside

_H_CACHE: dict = {}


def _H(geom):
    key = (geom.n, geom.n_theta, geom.n_s, geom.m, geom.n_rho, geom.k_theta, geom.r_dec, geom.dec_filter,
           geom.q_theta)
    if key not in _H_CACHE:
        _H_CACHE[key] = multiplier_full(geom)
    return _H_CACHE[key]


# ----------------------------------------------------------------- S3 helpers
def fine_sample_points(geom, p):
    """In-D fine samples of partition p.

    Returns (ti, q, X, Y): index of the fine row in geom.fine_rows(p), rho index,
    and the image index coordinates of T_p^{-1}(e^rho (cos phi, sin phi))."""
    t = geom.fine_rows(p)
    phi = geom.fine_phi(p, t)
    lo, hi = geom.d_interval(phi)
    Nr, dr = geom.n_rho, geom.d_rho
    ti_list, q_list = [], []
    for ti in range(t.size):
        if not np.isfinite(lo[ti]) or hi[ti] - MASK_EPS <= lo[ti] + MASK_EPS:
            continue
        q_lo = int(math.floor(math.log(lo[ti] + MASK_EPS) / dr + Nr - 1)) + 1
        q_hi = int(math.ceil(math.log(hi[ti] - MASK_EPS) / dr + Nr - 1)) - 1
        if q_hi < q_lo:
            continue
        q = np.arange(q_lo, q_hi + 1)
        ti_list.append(np.full(q.size, ti))
        q_list.append(q)
    if not ti_list:
        e = np.zeros(0)
        return e.astype(np.int64), e.astype(np.int64), e, e
    ti = np.concatenate(ti_list)
    q = np.concatenate(q_list)
    rho = (q - Nr + 1) * dr
    ang = phi[ti]
    y1 = np.exp(rho) * np.cos(ang)
    y2 = np.exp(rho) * np.sin(ang)
    # x = T_p^{-1}(y) = Rot(p beta) (y - (1 - a_R, 0)) / a_R   (inverse of eq. Tdef)
    mb = p * geom.beta
    a_R = geom.a_R
    z1 = y1 - (1.0 - a_R)
    x1 = (math.cos(mb) * z1 - math.sin(mb) * y2) / a_R
    x2 = (math.sin(mb) * z1 + math.cos(mb) * y2) / a_R
    X = (x1 + 1.0) / geom.dx
    Y = (x2 + 1.0) / geom.dx
    return ti, q, X, Y


def _bicubic_matrix_apply(c, X, Y):
    return bspline.eval_periodic_2d(c, X, Y)


def _bicubic_transpose(vals, X, Y, shape):
    """Scatter-add vals with the same 16 weights eval_periodic_2d uses."""
    ny, nx = shape
    kx, wx = bspline.taps(X)
    ky, wy = bspline.taps(Y)
    out = np.zeros(ny * nx)
    for b in range(4):
        row = (ky - 1 + b) % ny
        for a in range(4):
            col = (kx - 1 + a) % nx
            out += np.bincount(row * nx + col, weights=vals * wx[a] * wy[b], minlength=ny * nx)
    return out.reshape(ny, nx)


# ----------------------------------------------------------------- S7 helpers
def eval_taus(geom, p):
    """For partition p: list of (lattice row i, sinogram row j, tau[k] for all s_k)."""
    rows = geom.partition_rows(p)
    s = geom.s_nodes()
    a_R = geom.a_R
    rho0 = (1 - geom.n_rho) * geom.d_rho
    out = []
    for pos, (j, wrap, nu) in enumerate(rows):
        thp = math.pi * nu / (geom.n_theta * geom.m)
        st = -s if wrap else s
        tau = (np.log(a_R * st + (1.0 - a_R) * math.cos(thp)) - rho0) / geom.d_rho
        out.append((geom.lattice_row(pos), j, tau))
    return out


# ------------------------------------------------------------------ S6
def _conv(geom, W, conj=False, mode="fft"):
    H = _H(geom)
    if conj:
        H = np.conj(H)
    if mode == "fft":
        return np.real(np.fft.ifft2(np.fft.fft2(W) * H))
    if mode == "direct":
        K, Nr = W.shape
        k = np.real(np.fft.ifft2(H))  # real circulant kernel
        out = np.zeros((K, Nr))
        # circulant matrices along rho for each theta offset: C_d[q, q'] = k[d, (q - q') mod Nr]
        qq = (np.arange(Nr)[:, None] - np.arange(Nr)[None, :]) % Nr
        nz = [i for i in range(K) if np.any(W[i])]
        for i in range(K):
            acc = np.zeros(Nr)
            for i2 in nz:
                acc += k[(i - i2) % K][qq] @ W[i2]
            out[i] = acc
        return out
    raise ValueError(mode)


# ------------------------------------------------------------- the operators
def _partition_forward(geom, c, p, mode):
    r = geom.r_dec
    t = geom.fine_rows(p)
    nfine = t.size
    ti, q, X, Y = fine_sample_points(geom, p)
    v = np.zeros((nfine, geom.n_rho))
    v[ti, q] = _bicubic_matrix_apply(c, X, Y)                       # S3
    n_sup_p = geom.n_sup_p(p)
    d = decimation_taps(r, geom.dec_filter)
    u = np.zeros((n_sup_p, geom.n_rho))
    for i in range(n_sup_p):                                         # S4
        # fine rows t = r*i + n, n = -(2r-1)..2r-1, stored at index t - t[0]
        base = r * i - (2 * r - 1) - t[0]
        u[i] = d @ v[base:base + 4 * r - 1]
    w = u * np.exp(geom.rho_nodes())[None, :]                       # S5
    W = np.zeros((geom.k_theta, geom.n_rho))
    W[:n_sup_p] = w
    return _conv(geom, W, conj=False, mode=mode)                     # S6


def radon_fwd(geom, f, mode="fft"):
    """R f on the polar grid: f[N, N] (row = x2, column = x1) -> g[N_theta, N_s]."""
    f = np.asarray(f, dtype=np.float64)
    assert f.shape == (geom.n, geom.n)
    c = bspline.prefilter_2d(f)                                      # S2
    g = np.zeros((geom.n_theta, geom.n_s))
    for p in range(geom.m):
        clp = _partition_forward(geom, c, p, mode)
        for i, j, tau in eval_taus(geom, p):                         # S7
            g[j] = bspline.eval_periodic_1d(clp[i], tau) / geom.a_R
    return g


def _partition_adjoint(geom, g, p, mode):
    """Partition p's share of R^T g before the prefilter: S3^T S4^T S5^T S6^T S7^T."""
    r = geom.r_dec
    d = decimation_taps(r, geom.dec_filter)
    Nr = geom.n_rho
    C = np.zeros((geom.k_theta, Nr))
    for i, j, tau in eval_taus(geom, p):                             # S7^T
        k, wts = bspline.taps(tau)
        for a in range(4):
            C[i] += np.bincount((k - 1 + a) % Nr, weights=wts[a] * g[j], minlength=Nr) / geom.a_R
    Wt = _conv(geom, C, conj=True, mode=mode)                        # S6^T
    n_sup_p = geom.n_sup_p(p)
    w = Wt[:n_sup_p] * np.exp(geom.rho_nodes())[None, :]            # S5^T
    t = geom.fine_rows(p)
    v = np.zeros((t.size, Nr))
    for i in range(n_sup_p):                                         # S4^T
        base = r * i - (2 * r - 1) - t[0]
        v[base:base + 4 * r - 1] += np.outer(d, w[i])
    ti, q, X, Y = fine_sample_points(geom, p)
    return _bicubic_transpose(v[ti, q], X, Y, (geom.n, geom.n))      # S3^T


def radon_adj(geom, g, mode="fft"):
    """R# g = (w_S / w_X) R^T g: g[N_theta, N_s] -> f[N, N]."""
    g = np.asarray(g, dtype=np.float64)
    assert g.shape == (geom.n_theta, geom.n_s)
    cbar = np.zeros((geom.n, geom.n))
    for p in range(geom.m):
        cbar += _partition_adjoint(geom, g, p, mode)
    return bspline.prefilter_2d(cbar) * (geom.w_S / geom.w_X)        # S2^T = S2


def ramp_filter(geom, g):
    """W g: Ram-Lak linear convolution along s (eq. ramp, reading in the module docstring)."""
    g = np.asarray(g, dtype=np.float64)
    ds = geom.ds
    ns = geom.n_s
    n = np.arange(-(ns - 1), ns)
    h = np.zeros(n.size)
    h[n == 0] = 1.0 / (4.0 * ds * ds)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (math.pi ** 2 * n[odd].astype(np.float64) ** 2 * ds * ds)
    out = np.empty_like(g)
    for j in range(g.shape[0]):
        full = np.convolve(g[j], h)  # length 3*ns - 2; entry k + ns - 1 is sum_n h_n g_{k-n}
        out[j] = ds * full[ns - 1:2 * ns - 1]
    return out


FILTERS = ("ramlak", "cosine", "shepp-logan")


def filter_length(geom):
    """Length of the zero-padded s-axis on which the filters act: the smallest power of two
    >= 2 n_s (and >= 16), so that the ramp's circular convolution is the linear one."""
    lr = 16
    while lr < 2 * geom.n_s:
        lr *= 2
    return lr


def filter_window(lr, k, name):
    """Window of the ramp at centred DFT bin k (|k| <= lr/2) of the padded s-axis (sec. 6,
    eqs. cosfilt and SLfilt, reading in DESIGN): with sigma_k = |k| / (lr ds) and the
    s-sampling's Nyquist frequency sigma_N = 1 / (2 ds) = n_s / 4 (the paper's sigma / N with
    N = n_s and the unit-disc reading of the grids),
      ramlak       1
      cosine       cos(2 pi sigma / n_s)   = cos(pi |k| / lr), zero at the Nyquist bin
      shepp-logan  sinc(sigma / n_s)       = sinc(|k| / (2 lr)), sinc(x) = sin(pi x)/(pi x)."""
    k = np.abs(np.asarray(k, dtype=np.float64))
    if name == "ramlak":
        return np.ones_like(k)
    if name == "cosine":
        return np.cos(math.pi * k / lr)
    if name == "shepp-logan":
        return np.sinc(k / (2.0 * lr))
    raise ValueError(f"unknown filter {name!r}")


def filter_circulant(geom, x, name):
    """The filter on one zero-padded row x (length lr) as a circular convolution: the DFT of
    x times the DFT of the ds-weighted Ram-Lak kernel (placed circularly) times the window."""
    lr = filter_length(geom)
    x = np.asarray(x, dtype=np.float64)
    assert x.shape[-1] == lr
    ds, ns = geom.ds, geom.n_s
    h = np.zeros(lr)
    h[0] = 1.0 / (4.0 * ds * ds)
    for n in range(1, ns, 2):
        v = -1.0 / (math.pi ** 2 * n * n * ds * ds)
        h[n] = v
        h[lr - n] = v
    kc = np.fft.fftfreq(lr) * lr                                  # centred bin indices
    mult = np.fft.fft(h).real * ds * filter_window(lr, kc, name)  # h is even: real DFT
    return np.fft.ifft(np.fft.fft(x, axis=-1) * mult, axis=-1).real


def fbp_filter(geom, g, name="ramlak"):
    """W_F g for F in FILTERS: each row zero-padded to filter_length, filtered by
    filter_circulant, cut back to n_s samples.  For "ramlak" this is ramp_filter."""
    g = np.asarray(g, dtype=np.float64)
    lr = filter_length(geom)
    x = np.zeros(g.shape[:-1] + (lr,))
    x[..., :geom.n_s] = g
    return filter_circulant(geom, x, name)[..., :geom.n_s]


def fbp(geom, g, mode="fft", name="ramlak"):
    """Filtered back-projection R# W g (eq. FBP) with the filter W of FILTERS."""
    w = ramp_filter(geom, g) if name == "ramlak" else fbp_filter(geom, g, name)
    return radon_adj(geom, w, mode=mode)
