"""Pins of the oracle's B-spline pieces (sec. 4 of the paper) against values the
paper prints and against mathematics that does not reuse the oracle's formulas."""

import json
import os

import numpy as np

from oracle import bspline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_B_at_integers_matches_paper():
    gv = golden()["bspline_at_integers"]
    for key, val in gv.items():
        if key.startswith("B("):
            x = float(key[2:-1])
            assert abs(bspline.B(np.array([x]))[0] - val) < 1e-15


def test_B_is_convolution_of_four_boxes():
    # The cubic B-spline is box * box * box * box; compare with a numerical convolution.
    h = 1e-3
    box = np.ones(int(round(1 / h)))
    k = box
    for _ in range(3):
        k = np.convolve(k, box) * h
    xs = -2.0 + 2.0 * h + np.arange(k.size) * h  # boxes sampled at cell midpoints
    sel = slice(0, k.size, 97)
    assert np.max(np.abs(bspline.B(xs[sel]) - k[sel])) < 3e-3


def test_B_hat_matches_paper_and_direct_sum():
    gv = golden()["bspline_fourier_series"]
    assert np.allclose(bspline.B_hat(np.array(gv["xi"])), gv["B_hat"], atol=1e-15)
    xi = np.linspace(-0.5, 0.5, 11)
    j = np.arange(-3, 4)
    direct = (bspline.B(j)[None, :] * np.exp(-2j * np.pi * np.outer(xi, j))).sum(axis=1)
    assert np.max(np.abs(direct - bspline.B_hat(xi))) < 1e-15


def test_tap_weights_at_nodes_and_partition_of_unity():
    k, w = bspline.taps(np.array([5.0]))
    assert k[0] == 5
    assert np.allclose(w[:, 0], [1 / 6, 2 / 3, 1 / 6, 0.0], atol=1e-16)
    t = np.random.default_rng(1).uniform(-10, 10, 1000)
    k, w = bspline.taps(t)
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-14)
    # each weight is B at the distance from its tap
    for a in range(4):
        assert np.allclose(w[a], bspline.B(t - (k - 1 + a)), atol=1e-14)


def test_prefilter_then_evaluate_reproduces_samples():
    rng = np.random.default_rng(2)
    f = rng.standard_normal((24, 40))
    c = bspline.prefilter_2d(f)
    iy, ix = np.meshgrid(np.arange(24), np.arange(40), indexing="ij")
    back = bspline.eval_periodic_2d(c, ix.astype(float), iy.astype(float))
    assert np.max(np.abs(back - f)) < 1e-13


def test_recursive_prefilter_matches_fourier_division():
    gv = golden()["prefilter_pole"]
    assert abs((np.sqrt(3.0) - 2.0) - gv["z"]) < 1e-15
    rng = np.random.default_rng(3)
    for n in (17, 64):
        f = rng.standard_normal(n)
        assert np.max(np.abs(bspline.prefilter_recursive_1d(f) - bspline.prefilter_1d(f))) < 1e-13


def test_interpolation_converges_fourth_order():
    errs = []
    for n in (32, 64, 128):
        x = np.arange(n) / n
        f = np.sin(2 * np.pi * 3 * x) + 0.5 * np.cos(2 * np.pi * 5 * x)
        c = bspline.prefilter_1d(f)
        xt = np.linspace(0, 1, 997, endpoint=False)
        approx = bspline.eval_periodic_1d(c, xt * n)
        exact = np.sin(2 * np.pi * 3 * xt) + 0.5 * np.cos(2 * np.pi * 5 * xt)
        errs.append(np.max(np.abs(approx - exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.7), rates
