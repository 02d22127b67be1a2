"""Pins of the oracle's geometry (sec. 2 eq. aconst/Radon_all_pb/circle_D, sec. 3 eq. vrho)."""

import json
import math
import os

import numpy as np
import pytest

from oracle import geometry
from oracle.geometry import make_geometry

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


@pytest.mark.parametrize("m", [3, 4, 5, 8])
def test_partition_constants_from_the_figure(m):
    # D (centre (1 - a_R, 0), radius a_R) is tangent to the unit circle at (1, 0) and
    # to the two rays at angle +-beta/2; a_r is the distance to the origin of the tangent
    # to D perpendicular to the direction beta/2 (the smallest s of a line in the sector).
    beta = math.pi / m
    a_R, a_r = geometry.partition_constants(m)
    assert abs((1 - a_R) * math.sin(beta / 2) - a_R) < 1e-15
    assert abs((1 - a_R) * math.cos(beta / 2) - a_R - a_r) < 1e-15


def test_rho_bound_matches_printed_ratio():
    gv = json.load(open(GOLDEN))["nrho_over_n_M3"]
    n = 4096
    ratio = geometry.rho_bound(n, gv["M"]) / n
    assert abs(ratio - gv["ratio_printed"]) < gv["tolerance"]
    a_R, a_r = geometry.partition_constants(gv["M"])
    assert abs(ratio - (-math.log(a_r) / (2 * a_R))) < 1e-3


@pytest.mark.parametrize("n_theta,m", [(180, 4), (2048, 4), (100, 3), (97, 5), (1024, 4)])
def test_ownership_covers_each_row_once(n_theta, m):
    g = geometry.Geometry(64, n_theta, 64, m, 256, 4 * n_theta, 4)
    seen = np.zeros(n_theta, dtype=int)
    for p in range(m):
        rows = g.partition_rows(p)
        for j, wrap, nu in rows:
            seen[j] += 1
            thp = math.pi * nu / (n_theta * m)
            assert -g.beta / 2 - 1e-15 <= thp < g.beta / 2
            # the line (theta_j, s) equals (theta' + m beta, s) or (theta' + pi, -s)
            ref = j * math.pi / n_theta - (math.pi if wrap else p * g.beta)
            assert abs(ref - thp) < 1e-14
            assert wrap == (p == 0 and j * math.pi / n_theta > math.pi / 2)
    assert np.all(seen == 1)


def test_half_integer_tie_goes_up():
    g = make_geometry(2048, 2048, 2048)
    # theta_256 / beta = 1/2 exactly: rounds up to partition 1
    assert g.owner(256)[0] == 1


def test_mask_interval_matches_point_test():
    g = make_geometry(64, 90, 64)
    phi = np.linspace(-g.beta / 2 + 1e-6, g.beta / 2 - 1e-6, 41)
    lo, hi = g.d_interval(phi)
    e = np.linspace(0.3, 1.0, 4001)
    for a, ph in enumerate(phi):
        y1, y2 = e * math.cos(ph), e * math.sin(ph)
        inside = (y1 - 1 + g.a_R) ** 2 + y2 ** 2 < g.a_R ** 2
        pred = (e > lo[a]) & (e < hi[a])
        assert np.array_equal(inside, pred)
    lo, hi = g.d_interval(np.array([g.beta / 2 + 1e-9]))
    assert np.isnan(lo[0]) and np.isnan(hi[0])


def test_defaults_respect_bounds():
    for n, nt in ((128, 180), (1024, 1024), (2048, 2048), (2048, 1024), (768, 768)):
        g = make_geometry(n, nt, n)
        assert g.n_rho >= geometry.rho_bound(n, g.m)
        assert g.k_theta >= 2 * math.ceil(nt / g.m) and g.k_theta >= g.n_sup
        assert g.dtheta / g.r_dec <= 2 * g.a_R / n + 1e-15
    g = make_geometry(2048, 2048, 2048)
    assert (g.n_rho, g.k_theta, g.r_dec, g.n_own) == (4096, 1024, 6, 512)


@pytest.mark.parametrize("n,n_theta,m", [(128, 192, 5), (128, 192, 6), (128, 180, 6), (128, 192, 8), (128, 180, 4)])
def test_tau_range_is_one_period_plus_one_node(n, n_theta, m):
    # On a line of the sector, a_R s + (1 - a_R) cos theta' lies in [a_r, 1]: its minimum is at
    # s = -1 on the tangent rays theta' = +-beta/2 (eq. aconst), its maximum at s = 1, theta' = 0.
    # With rho_0 = (1 - N_rho) d_rho and d_rho = -log(a_r) / N_rho that is tau in [-1, N_rho - 1].
    from oracle import radon

    g = make_geometry(n, n_theta, n, m=m)
    lo, hi = np.inf, -np.inf
    for p in range(m):
        for _, j, tau in radon.eval_taus(g, p):
            lo, hi = min(lo, tau.min()), max(hi, tau.max())
            _, wrap, nu = g.owner(j)
            if nu * 2 == -n_theta and not wrap:  # theta' = -beta/2: the sample at s = -1 sits on
                assert abs(tau[0] + 1.0) < 1e-12  # tau = -1 (a wrapped row samples s = +1 - ds)
    assert lo >= -1.0 - 1e-12 and hi <= g.n_rho - 1 + 1e-12
