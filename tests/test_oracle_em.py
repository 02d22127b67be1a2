"""Pins of the oracle's EM step (sec. 7): fixed point, flux identity, R# chi_C = pi."""

import math

import numpy as np

from oracle import em, radon
from oracle.geometry import make_geometry
from paper_1506_00014_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_positive_image_is_a_fixed_point():
    g = make_geometry(32, 48, 32)
    f = (0.5 + inputs.uniform_image(32, seed=21)) * em.disc_mask(g)  # > 0 on the disc
    data = radon.radon_fwd(g, f)
    assert (data[:, 1:] > 0).all()
    f1 = em.em_step(g, data, f)
    assert rel(f1, f) < 1e-12


def test_step_preserves_weighted_flux():
    g = make_geometry(32, 48, 32)
    disc = em.disc_mask(g)
    f = (0.2 + inputs.uniform_image(32, seed=22)) * disc
    truth = (0.1 + inputs.uniform_image(32, seed=23)) * disc
    data = radon.radon_fwd(g, truth)
    norm = em.em_norm(g)
    assert (norm[disc] > 0).all()
    f1 = em.em_step(g, data, f, norm)
    rf = radon.radon_fwd(g, f)
    lines = (em.chi_c(g) > 0) & (rf > 0)
    lhs = float((f1 * norm)[disc].sum())
    rhs = g.w_S / g.w_X * float(data[lines].sum())
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    # a dropped chi_C or a swapped ratio breaks it
    bad = np.where(rf > 0, data / np.where(rf > 0, rf, 1.0), 0.0)
    f_bad = f * radon.radon_adj(g, bad)
    assert abs(float(f_bad[disc].sum()) - rhs) > 1e-6 * abs(rhs)


def test_norm_is_pi_inside_the_disc():
    for n, err in ((64, 5e-2), (128, 3e-2)):
        g = make_geometry(n, n, n)
        norm = em.em_norm(g)
        x = g.x_nodes()
        X1, X2 = np.meshgrid(x, x)
        ins = X1 ** 2 + X2 ** 2 < 0.6
        assert np.abs(norm[ins] / math.pi - 1.0).max() < err, n


def test_em_decreases_the_data_misfit():
    g = make_geometry(32, 48, 32)
    truth = (0.1 + inputs.uniform_image(32, seed=24)) * em.disc_mask(g)
    data = radon.radon_fwd(g, truth)
    f = em.disc_mask(g).astype(np.float64)
    lines = em.chi_c(g) > 0
    errs = []
    for _ in range(4):
        errs.append(rel(radon.radon_fwd(g, f)[lines], data[lines]))
        f = em.em_step(g, data, f)
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
