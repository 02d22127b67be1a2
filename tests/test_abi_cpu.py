"""Host-side checks of the C-ABI library: it loads without a GPU, exports every function
include/radonlp.h declares, its defaults agree with the oracle's geometry, and argument
errors come back as status codes (no device is touched by any call here)."""

import ctypes
import os
import re

import pytest

from oracle.geometry import make_geometry
from paper_1506_00014_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radonlp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libradonlp.so not built")
    return _lib.load()


def test_header_declares_the_binding_list():
    assert declared_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", out), name


@pytest.mark.parametrize("n,nt,ns", [(128, 180, 128), (1024, 1024, 1024), (2048, 2048, 2048), (2048, 1024, 2048),
                                     (256, 256, 256), (768, 768, 768), (64, 90, 64)])
def test_defaults_match_oracle_geometry(lib, n, nt, ns):
    for q in (1, 2):
        g = _lib.geom_default(n, nt, ns, 4, q)
        og = make_geometry(n, nt, ns, q_theta=q)
        assert (g.n_rho, g.k_theta, g.r_dec, g.q_theta, g.dec_filter) == (og.n_rho, og.k_theta, og.r_dec, q, 0)


def test_argument_errors_are_status_codes(lib):
    g = _lib.RlGeom()
    assert lib.rl_geom_default(7, 10, 10, 4, 1, 0, ctypes.byref(g)) == 2
    assert lib.rl_geom_default(64, 2, 64, 4, 1, 0, ctypes.byref(g)) == 2
    assert lib.rl_geom_default(64, 64, 64, 4, 1, 0, None) == 1
    p = ctypes.c_void_p()
    assert lib.rl_plan_create(None, ctypes.byref(p)) == 1
    good = _lib.geom_default(64, 90, 64)
    for field, bad in (("n_rho", 96), ("n_rho", 64), ("k_theta", 16), ("r_dec", 1), ("m", 2), ("dec_filter", 3),
                       ("q_theta", 3), ("q_theta", 0)):
        g = _lib.RlGeom.from_buffer_copy(good)
        setattr(g, field, bad)
        assert lib.rl_plan_create(ctypes.byref(g), ctypes.byref(p)) == 2, field
        assert p.value is None
        assert len(lib.rl_last_error()) > 0
    assert lib.radon_fwd(None, None, None, 1, None, 0, None) == 1
    assert lib.radon_adj(None, None, None, 1, None, 0, None) == 1
    assert lib.fbp(None, None, None, 1, 0, None, 0, None) == 1
    assert lib.rl_workspace_bytes(None, 4, 0) == 0
    lib.rl_plan_destroy(None)


def test_fft_length_validation(lib):
    """FFT lengths 2^a 3^b: N_rho a multiple of 4, K one of the theta pass's four-step splits.
    A valid geometry gets past validation and fails only for want of a device here (RL_ERR_HIP);
    an invalid one is refused with RL_ERR_GEOMETRY before any device call."""
    p = ctypes.c_void_p()
    base = _lib.geom_default(2048, 2048, 2048, 3)
    cases = [("n_rho", 4608, 4), ("n_rho", 3888 * 2, 4), ("n_rho", 4374, 2), ("n_rho", 5000, 2), ("n_rho", 8192, 4), ("n_rho", 4096, 2),
             ("k_theta", 1536, 4), ("k_theta", 1458, 2), ("k_theta", 2048, 4), ("k_theta", 3072, 2)]
    for field, value, want in cases:
        g = _lib.RlGeom.from_buffer_copy(base)
        setattr(g, field, value)
        st = lib.rl_plan_create(ctypes.byref(g), ctypes.byref(p))
        assert st in (want, 5 if want == 4 else want), (field, value, st, lib.rl_last_error())
        assert p.value is None
    small = _lib.geom_default(64, 90, 64, 4)
    for k, want in ((24, 2), (96, 4), (48, 2), (64, 4), (192, 4), (288, 2)):
        g = _lib.RlGeom.from_buffer_copy(small)
        g.k_theta = k
        st = lib.rl_plan_create(ctypes.byref(g), ctypes.byref(p))
        assert st in (want, 5 if want == 4 else want), (k, st)


def test_smooth_defaults(lib):
    """smooth = 1 picks the smallest 2^a 3^b lengths at or above the bounds."""
    g = _lib.geom_default(2048, 2048, 2048, 3, 1, 1)
    assert (g.n_rho, g.k_theta) == (4608, 1536)
    g = _lib.geom_default(2048, 2048, 2048, 4, 1, 1)
    assert (g.n_rho, g.k_theta) == (3888, 1024)
    g = _lib.geom_default(128, 180, 128, 4, 1, 1)
    assert (g.n_rho, g.k_theta) == (256, 96)
    og = make_geometry(2048, 2048, 2048, m=3)
    assert g.r_dec == make_geometry(128, 180, 128).r_dec and og.n_rho == 8192
