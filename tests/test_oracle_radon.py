"""Pins of the whole oracle operators (Algorithm 1, its transpose, FBP) against
closed-form Radon transforms, brute-force line integrals of the spline image,
the adjoint identity, an exact rotation covariance, and the direct circulant sum."""

import math

import numpy as np
import pytest
from scipy.special import dawsn

from oracle import analytic, brute, radon
from oracle.geometry import Geometry, make_geometry
from paper_1506_00014_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gauss_case(g, cx, cy, sig):
    f = analytic.gaussian_image(g.x_nodes(), cx, cy, sig)
    return f, analytic.gaussian_sino(g.theta_nodes(), g.s_nodes(), cx, cy, sig)


def test_gaussians_match_closed_form_and_converge():
    errs = []
    for n in (64, 128, 256):
        g = make_geometry(n, n, n)
        e = []
        for cx, cy, sig in ((0.0, 0.0, 0.1), (0.25, 0.1, 0.08), (-0.3, 0.2, 0.12)):
            f, A = gauss_case(g, cx, cy, sig)
            e.append(rel(radon.radon_fwd(g, f), A))
        errs.append(max(e))
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8, errs
    assert errs[2] < 2e-6, errs


def test_off_centre_gaussian_pins_orientation():
    # An x1 <-> x2 swap, a sign flip of s or a wrong rotation sense moves the ridge.
    g = make_geometry(128, 180, 128)
    f, A = gauss_case(g, 0.35, -0.2, 0.1)
    G = radon.radon_fwd(g, f)
    assert rel(G, A) < 1e-4
    _, Aswap = gauss_case(g, -0.2, 0.35, 0.1)
    assert rel(G, Aswap) > 0.5


def test_ellipse_phantom_and_disc_converge():
    errs_e, errs_d = [], []
    for n in (128, 256):
        g = make_geometry(n, n, n)
        img, ells = inputs.ellipse_phantom(n, 8, 101)
        errs_e.append(rel(radon.radon_fwd(g, img), analytic.ellipse_sino(g.theta_nodes(), g.s_nodes(), ells)))
        x = g.x_nodes()
        X1, X2 = np.meshgrid(x, x)
        disc = (X1 ** 2 + X2 ** 2 <= 0.25).astype(float)
        A = analytic.ellipse_sino(g.theta_nodes(), g.s_nodes(), [(0, 0, 0.5, 0.5, 0, 1.0)])
        errs_d.append(rel(radon.radon_fwd(g, disc), A))
    assert errs_e[0] < 0.03 and errs_e[1] < 0.6 * errs_e[0], errs_e
    assert errs_d[0] < 0.03 and errs_d[1] < 0.6 * errs_d[0], errs_d


def test_brute_force_line_integrals_converge():
    errs = []
    for n in (32, 64):
        g = make_geometry(n, n, n)
        x = g.x_nodes()
        f = analytic.gaussian_image(x, 0.2, -0.15, 0.15) - 0.5 * analytic.gaussian_image(x, -0.3, 0.25, 0.1)
        errs.append(rel(radon.radon_fwd(g, f), brute.line_integrals(g, f)))
    assert errs[0] < 0.05 and errs[1] < 2e-3 and errs[1] < errs[0] / 10, errs


@pytest.mark.parametrize("geom", [
    make_geometry(64, 90, 64),
    make_geometry(48, 100, 40, m=3),
    Geometry(40, 97, 50, 5, 160, 52, 5),  # M does not divide N_theta; K not a power of two
])
def test_adjoint_identity_fp64(geom):
    rng = np.random.default_rng(11)
    f = rng.standard_normal((geom.n, geom.n))
    y = rng.standard_normal((geom.n_theta, geom.n_s))
    Rf = radon.radon_fwd(geom, f)
    Ry = radon.radon_adj(geom, y)
    lhs = geom.w_S * np.sum(Rf * y)
    rhs = geom.w_X * np.sum(f * Ry)
    scale = geom.w_S * np.linalg.norm(Rf) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_direct_circulant_sum_equals_fft_convolution():
    g = make_geometry(32, 48, 32)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((32, 32))
    y = rng.standard_normal((48, 32))
    a, b = radon.radon_fwd(g, f, mode="fft"), radon.radon_fwd(g, f, mode="direct")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.abs(a).max()
    a, b = radon.radon_adj(g, y, mode="fft"), radon.radon_adj(g, y, mode="direct")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.abs(a).max()


def test_quarter_turn_covariance_is_exact_on_partitions_two_and_three():
    # M = 4: rotating the image by +90 degrees maps T_m f' to T_{m-2} f exactly (eq. Tdef),
    # so the rows owned by partitions 2 and 3 of R f' are rows of R f shifted by N_theta/2,
    # with s -> -s where the partner row is a wrapped row of partition 0.
    n, nt = 48, 64
    g = make_geometry(n, nt, n)
    rng = np.random.default_rng(7)
    f = rng.standard_normal((n, n))
    ix = np.arange(n)
    fr = f[(n - ix[None, :]) % n, ix[:, None]]  # f'[iy][ix] = f[(N - ix) mod N][iy]
    G, Gr = radon.radon_fwd(g, f), radon.radon_fwd(g, fr)
    scale = np.abs(G).max()
    checked = 0
    for p in (2, 3):
        for j, wrap, nu in g.partition_rows(p):
            jp = (j - nt // 2) % nt
            if g.owner(jp)[1]:
                # partner is a wrapped row: s_k -> s_{N_s - k}
                assert np.max(np.abs(Gr[j, 1:] - G[jp, :0:-1])) < 1e-12 * scale
            else:
                assert np.max(np.abs(Gr[j] - G[jp])) < 1e-12 * scale
            checked += 1
    assert checked == nt // 2
    # partitions 0 and 1 see the point-reflected problem: equal only to discretisation error
    assert np.max(np.abs(Gr - np.roll(G, nt // 2, axis=0))) > 1e-8 * scale


def test_backprojection_of_gaussian_ridge():
    # R# of g = exp(-s^2/sigma^2) is pi exp(-r^2/(2 sigma^2)) I0(r^2/(2 sigma^2)).  The exact
    # transpose spreads polar samples onto the log-polar lattice, so its error is set by the
    # oversampling of that lattice: at the sampling bound it is ~1e-2, at twice it ~1e-4.
    sig = 0.1
    out = []
    for g in (make_geometry(128, 128, 128), make_geometry(128, 512, 512, n_rho=512)):
        G = np.tile(np.exp(-g.s_nodes() ** 2 / sig ** 2), (g.n_theta, 1))
        A = analytic.backproject_gaussian_ridge(g.x_nodes(), sig)
        x = g.x_nodes()
        X1, X2 = np.meshgrid(x, x)
        ins = X1 ** 2 + X2 ** 2 < 0.49
        out.append(rel(radon.radon_adj(g, G)[ins], A[ins]))
    assert out[0] < 1.2e-2 and out[1] < 3e-4, out


def test_ramp_filter_of_gaussian_matches_closed_form():
    # |sigma| applied to exp(-s^2/s0^2) is (1 - 2 u F(u)) / (pi^1.5 s0), u = s/s0, F = Dawson.
    # The Ram-Lak kernel is the sampled band-limited ramp, so a Gaussian well inside the
    # band is filtered exactly up to rounding and the truncation of its tails.
    s0 = 0.1
    errs = []
    for n in (128, 256, 512):
        g = make_geometry(n, 16, n)
        s = g.s_nodes()
        G = np.tile(np.exp(-s ** 2 / s0 ** 2), (g.n_theta, 1))
        W = radon.ramp_filter(g, G)
        u = s / s0
        ref = (1.0 - 2.0 * u * dawsn(u)) / (math.pi ** 1.5 * s0)
        errs.append(rel(W[3], ref))
    assert max(errs) < 1e-12, errs


def test_fbp_recovers_smooth_object():
    # FBP = R# W R.  Like R#, its accuracy is set by the fine-lattice oversampling: ~1e-2 at
    # the sampling bounds, ~1e-4 with r and N_rho both about twice their bounds.
    errs = []
    for g in (make_geometry(128, 128, 128), make_geometry(128, 256, 256, n_rho=512, r_dec=8)):
        f = analytic.gaussian_image(g.x_nodes(), 0.2, -0.1, 0.12)
        A = analytic.gaussian_sino(g.theta_nodes(), g.s_nodes(), 0.2, -0.1, 0.12)
        x = g.x_nodes()
        X1, X2 = np.meshgrid(x, x)
        ins = X1 ** 2 + X2 ** 2 < 0.81
        errs.append(rel(radon.fbp(g, A)[ins], f[ins]))
    assert errs[0] < 2e-2 and errs[1] < 5e-4, errs
