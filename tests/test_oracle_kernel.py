"""Pins of the oracle's log-polar kernel table (sec. 3 eq. exprcoef1) against the
paper's closed form (eq. P_closed_form) evaluated with mpmath, against direct
high-precision quadrature, and against the appendix recursion (eq. hdefin)."""

import math

import numpy as np
import pytest

from oracle import closed_form, kernel
from oracle.geometry import make_geometry


@pytest.mark.parametrize("m", [3, 4])
def test_zeta_hat_matches_paper_closed_form(m):
    g = make_geometry(128, 180, 128, m=m)
    Z = kernel.zeta_hat_half(g)
    P = g.k_theta * g.dtheta
    for kt, kr in ((0, 1), (1, 1), (5, 3), (20, 50), (g.k_theta // 2, g.n_rho // 2), (33, 97)):
        mu = -2 * math.pi * kt / P
        alpha = complex(-1.0, -2 * math.pi * kr / g.L)
        ref = closed_form.P_closed(mu, alpha, g.beta)
        assert abs(Z[kt, kr] - ref) <= 1e-12 * max(1.0, abs(ref)), (kt, kr, Z[kt, kr], ref)


def test_zeta_hat_at_zero_frequency():
    for m in (3, 4, 6):
        g = make_geometry(64, 96, 64, m=m)
        Z = kernel.zeta_hat_half(g, kt_max=0, kr_max=0)
        assert abs(Z[0, 0] - 2 * math.atanh(math.sin(g.beta))) < 1e-13


def test_closed_form_is_the_defining_integral():
    # The closed form itself, against a direct mpmath quadrature of eq. (Pfor).
    for mu, alpha, beta in ((-3.0, complex(-1, -4.0), math.pi / 4), (2.5, complex(0, 3.0), math.pi / 3)):
        a = closed_form.P_closed(mu, alpha, beta)
        b = closed_form.P_quad(mu, alpha, beta)
        assert abs(a - b) < 1e-20 + 1e-15 * abs(b)


def test_appendix_recursion_holds():
    # P(mu, alpha - 2) = alpha/(alpha - 1) (1 - mu^2/alpha^2) P(mu, alpha) + h(mu, alpha)
    mu, beta = -2.7, math.pi / 4
    for alpha in (complex(2.0, -3.0), complex(3.5, 1.0)):
        lhs = closed_form.P_quad(mu, alpha - 2, beta)
        rhs = (alpha / (alpha - 1) * (1 - mu * mu / alpha ** 2) * closed_form.P_quad(mu, alpha, beta)
               + closed_form.h_term(mu, alpha, beta))
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_symmetries_and_nyquist_reading():
    g = make_geometry(64, 90, 64)
    H = kernel.multiplier_full(g)
    K, Nr = H.shape
    ik = (-np.arange(K)) % K
    ir = (-np.arange(Nr)) % Nr
    # real circulant kernel <=> Hermitian multiplier
    assert np.max(np.abs(H[ik][:, ir] - np.conj(H))) < 1e-14 * np.abs(H).max()
    k = np.fft.ifft2(H)
    assert np.max(np.abs(k.imag)) < 1e-14 * np.abs(k.real).max()
    # evenness in k_theta
    assert np.max(np.abs(H[ik] - H)) < 1e-14 * np.abs(H).max()


def test_decimation_filter_is_normalised():
    for r in (1, 2, 5, 6, 12):
        d = kernel.decimation_taps(r)
        assert abs(d.sum() - 1.0) < 1e-14
        dh = kernel.decimation_response(r, 64)
        assert abs(dh[0] - 1.0) < 1e-14
        assert np.all(dh > 0.0)
