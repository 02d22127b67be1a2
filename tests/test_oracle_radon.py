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


@pytest.mark.parametrize("name", ["cosine", "shepp-logan"])
def test_windowed_filters_of_gaussian_match_closed_form(name):
    # The windows act on the ramp's spectrum: cos(2 pi sigma / n_s) is the transform of
    # (delta(s - 1/n_s) + delta(s + 1/n_s)) / 2 and sinc(sigma / n_s) that of n_s times the
    # box of width 1/n_s, so for a Gaussian well inside the band W_cos g is the mean of the
    # ramp's closed form at s -+ 1/n_s and W_SL g its box mean; the latter integrates in
    # closed form since F' = 1 - 2 u F (F = Dawson): the antiderivative of the ramp's
    # closed form in s is F(s/s0) / pi^1.5.
    s0 = 0.1
    errs = []
    for n in (128, 256, 512):
        g = make_geometry(n, 16, n)
        s = g.s_nodes()
        G = np.tile(np.exp(-s ** 2 / s0 ** 2), (g.n_theta, 1))
        W = radon.fbp_filter(g, G, name)
        a = 1.0 / g.n_s
        if name == "cosine":
            ramp = lambda t: (1.0 - 2.0 * (t / s0) * dawsn(t / s0)) / (math.pi ** 1.5 * s0)
            ref = 0.5 * (ramp(s - a) + ramp(s + a))
        else:
            ref = (dawsn((s + a / 2) / s0) - dawsn((s - a / 2) / s0)) / (math.pi ** 1.5 * a)
        errs.append(rel(W[5], ref))
        # and not the plain ramp: the windows change the result well above that error
        assert rel(radon.ramp_filter(g, G)[5], ref) > 1e3 * errs[-1]
    assert max(errs) < 1e-11, errs


def test_windowed_filters_nyquist_and_symmetry():
    g = make_geometry(32, 8, 24)
    lr = radon.filter_length(g)
    assert lr == 64
    alt = (-1.0) ** np.arange(lr)
    ramp = radon.filter_circulant(g, alt, "ramlak")
    # the cosine filter vanishes at the s-sampling's Nyquist frequency (sec. 6) ...
    assert np.abs(radon.filter_circulant(g, alt, "cosine")).max() < 1e-12 * np.abs(ramp).max()
    # ... Shepp-Logan keeps sinc(1/4) = 2 sqrt(2) / pi of it
    sl = radon.filter_circulant(g, alt, "shepp-logan")
    assert np.allclose(sl, ramp * 2.0 * math.sqrt(2.0) / math.pi, rtol=1e-12, atol=0)
    # the ramp's Nyquist response is ds sum_n h_n (-1)^n of the Ram-Lak kernel
    ds = g.ds
    hsum = 1.0 / (4 * ds * ds) + 2 * sum(1.0 / (math.pi ** 2 * n * n * ds * ds) for n in range(1, g.n_s, 2))
    assert np.allclose(ramp, alt * ds * hsum, rtol=1e-12, atol=0)
    # even windows: filtering commutes with reversing s
    x = inputs.normal_array((g.n_theta, g.n_s), seed=4)
    for name in radon.FILTERS:
        w = radon.fbp_filter(g, x, name)
        wr = radon.fbp_filter(g, x[:, ::-1], name)
        assert np.allclose(wr, w[:, ::-1], rtol=0, atol=1e-12 * np.abs(w).max()), name


def test_windowed_filter_brute_force_dft():
    # explicit DFT sums on a tiny row, no FFT library
    g = make_geometry(8, 4, 8)
    lr = radon.filter_length(g)
    x = inputs.normal_array((1, g.n_s), seed=9)[0]
    ds, ns = g.ds, g.n_s
    h = [0.0] * lr
    h[0] = ds / (4 * ds * ds)
    for n in range(1, ns, 2):
        h[n] = h[lr - n] = -ds / (math.pi ** 2 * n * n * ds * ds)
    xp = list(x) + [0.0] * (lr - ns)
    for name in radon.FILTERS:
        out = []
        for j in range(ns):
            acc = 0.0
            for k in range(lr):
                kc = k if k <= lr // 2 else k - lr
                if name == "ramlak":
                    win = 1.0
                elif name == "cosine":
                    win = math.cos(math.pi * abs(kc) / lr)
                else:
                    t = math.pi * abs(kc) / (2 * lr)
                    win = 1.0 if kc == 0 else math.sin(t) / t
                hk = sum(h[n] * math.cos(2 * math.pi * k * n / lr) for n in range(lr))
                xk = complex(sum(xp[n] * math.cos(2 * math.pi * k * n / lr) for n in range(lr)),
                             -sum(xp[n] * math.sin(2 * math.pi * k * n / lr) for n in range(lr)))
                e = complex(math.cos(2 * math.pi * k * j / lr), math.sin(2 * math.pi * k * j / lr))
                acc += (xk * hk * win * e).real
            out.append(acc / lr)
        got = radon.fbp_filter(g, x[None, :], name)[0]
        assert np.allclose(got, out, rtol=0, atol=1e-12 * max(abs(v) for v in out)), name


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
