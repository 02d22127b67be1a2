"""Pins of the oracle's accuracy variants of Algorithm 1 step 4 (the theta low-pass the paper
leaves open, and the spacing of the coarse lattice Omega_p of eq. Lopolargrid_polar):
dec_filter = 1 (the box of one coarse cell) and q_theta = 2 (a lattice at half the sinogram's
angular spacing).  Each variant is an operator of its own; the pins are the box's closed-form
response, the adjoint identity, Gaussian closed forms with convergence in N, and the exact
quarter-turn covariance (which fixes the lattice-row mapping of the owned rows)."""

import math

import numpy as np
import pytest

from oracle import analytic, radon
from oracle.geometry import make_geometry
from oracle.kernel import decimation_response, decimation_taps

VARIANTS = [(1, 1), (0, 2), (1, 2)]  # (dec_filter, q_theta)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("r", [3, 4, 5, 6])
def test_box_taps_and_closed_form_response(r):
    d = decimation_taps(r, 1)
    n = np.arange(-(2 * r - 1), 2 * r)
    assert abs(d.sum() - 1.0) < 1e-15
    assert np.array_equal(d, d[::-1])
    # one coarse cell: |n| <= r/2, the edge rows (r even) at half weight
    assert np.all(d[2 * np.abs(n) > r] == 0.0)
    assert np.allclose(d[2 * np.abs(n) < r], 1.0 / r)
    K = 64
    f = np.arange(K // 2 + 1) / (r * K)  # coarse frequencies in cycles per fine row
    with np.errstate(invalid="ignore", divide="ignore"):
        if r % 2:  # r samples: the Dirichlet kernel
            ref = np.sin(math.pi * f * r) / (r * np.sin(math.pi * f))
        else:  # trapezoid rule over r intervals: sin(pi f r) cot(pi f) / r
            ref = np.sin(math.pi * f * r) / (r * np.tan(math.pi * f))
    ref[0] = 1.0
    assert np.max(np.abs(decimation_response(r, K, 1) - ref)) < 1e-14


@pytest.mark.parametrize("dec,q", VARIANTS)
def test_variant_adjoint_identity_fp64(dec, q):
    g = make_geometry(48, 70, 40, dec_filter=dec, q_theta=q)
    rng = np.random.default_rng(21)
    f = rng.standard_normal((g.n, g.n))
    y = rng.standard_normal((g.n_theta, g.n_s))
    Rf = radon.radon_fwd(g, f)
    Ry = radon.radon_adj(g, y)
    lhs = g.w_S * np.sum(Rf * y)
    rhs = g.w_X * np.sum(f * Ry)
    assert abs(lhs - rhs) <= 1e-12 * g.w_S * np.linalg.norm(Rf) * np.linalg.norm(y)


@pytest.mark.parametrize("dec,q", VARIANTS)
def test_variant_gaussians_match_closed_form_and_converge(dec, q):
    errs = []
    for n in (64, 128, 256):
        g = make_geometry(n, n, n, dec_filter=dec, q_theta=q)
        e = []
        for cx, cy, sig in ((0.0, 0.0, 0.1), (0.25, 0.1, 0.08), (-0.3, 0.2, 0.12)):
            f = analytic.gaussian_image(g.x_nodes(), cx, cy, sig)
            A = analytic.gaussian_sino(g.theta_nodes(), g.s_nodes(), cx, cy, sig)
            e.append(rel(radon.radon_fwd(g, f), A))
        errs.append(max(e))
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8, errs
    assert errs[2] < 2e-6, errs


def test_half_spacing_lattice_geometry():
    g = make_geometry(128, 180, 128, q_theta=2)
    assert g.dtheta_c == g.dtheta / 2
    bound = 2.0 * g.a_R / g.n  # fine angular step bound (sec. 3, before eq. Lopolargrid_f)
    assert g.dtheta_c / g.r_dec <= bound < g.dtheta_c / (g.r_dec - 1)
    assert g.k_theta >= 4 * math.ceil(180 / 4) and g.k_theta >= g.n_sup
    assert g.n_sup == 2 * (g.n_own - 1) + 1 + 4
    # every owned row's lattice angle is its theta'
    for p in range(g.m):
        for pos, (j, wrap, nu) in enumerate(g.partition_rows(p)):
            lat = g.phi0(p) + g.lattice_row(pos) * g.dtheta_c
            assert abs(lat - math.pi * nu / (g.n_theta * g.m)) < 1e-14


@pytest.mark.parametrize("dec,q", VARIANTS)
def test_variant_quarter_turn_covariance(dec, q):
    # M = 4: rotating the image by +90 degrees maps T_m f' to T_{m-2} f exactly, so the rows
    # of partitions 2 and 3 of R f' equal rows of R f shifted by N_theta/2 (s -> -s where the
    # partner row wraps) -- whatever the low-pass and the lattice spacing.
    n, nt = 48, 64
    g = make_geometry(n, nt, n, dec_filter=dec, q_theta=q)
    rng = np.random.default_rng(8)
    f = rng.standard_normal((n, n))
    ix = np.arange(n)
    fr = f[(n - ix[None, :]) % n, ix[:, None]]
    G, Gr = radon.radon_fwd(g, f), radon.radon_fwd(g, fr)
    scale = np.abs(G).max()
    for p in (2, 3):
        for j, wrap, nu in g.partition_rows(p):
            jp = (j - nt // 2) % nt
            if g.owner(jp)[1]:
                assert np.max(np.abs(Gr[j, 1:] - G[jp, :0:-1])) < 1e-12 * scale
            else:
                assert np.max(np.abs(Gr[j] - G[jp])) < 1e-12 * scale


def test_variants_differ_from_the_default():
    # the variants are different operators (a pin that the flags reach the arithmetic)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((32, 32))
    base = radon.radon_fwd(make_geometry(32, 48, 32), f)
    for dec, q in VARIANTS:
        other = radon.radon_fwd(make_geometry(32, 48, 32, dec_filter=dec, q_theta=q), f)
        assert rel(other, base) > 1e-4, (dec, q)
