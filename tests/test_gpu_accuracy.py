"""Closed-form accuracy of the operator variants on the GPU at 1024 x 1024 (1024 angles x 1024 bins).

The theta low-pass of Algorithm 1 step 4 is unspecified in the paper (sec. 5); the library offers
the cubic B-spline (dec_filter 0) and the box of one coarse cell (dec_filter 1), on the sinogram's
angular lattice (q_theta 1) or one twice as fine (q_theta 2).  This study measures each choice
against closed forms (the inputs' exact line integrals and back-projections), not against the
oracle: parity with the oracle for every variant is in test_gpu_parity.py.

  R    discs (centred r = 0.5; r = 0.2 at (0.3, -0.2)) and Gaussians (sigma 0.02, 0.05, 0.1 at the
       origin and at (0.25, 0.1)) sampled at the nodes, against their exact Radon transforms;
       discs also on the bins whose line stays 2 ds inside the disc (|t| < r - 2 ds)
  R#   the ridge g = exp(-s^2 / sigma^2) (sigma 0.05, 0.1) against pi exp(-z) I0(z), z = |x|^2 / 2 sigma^2
  FBP  the exact sinogram of a Gaussian (sigma 0.05, 0.1) against the Gaussian itself
Image-side errors are taken on |x| < 0.9.  The table is printed; the asserts are loose sanity bounds
(the measured errors are recorded in the design notes)."""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import analytic  # noqa: E402

pytestmark = pytest.mark.gpu

N = 1024
VARIANTS = [(0, 1), (1, 1), (0, 2), (1, 2)]  # (dec_filter, q_theta)
DISCS = [("disc r0.5", 0.0, 0.0, 0.5), ("disc r0.2 off", 0.3, -0.2, 0.2)]
GAUSS = [(s, c) for s in (0.02, 0.05, 0.1) for c in ((0.0, 0.0), (0.25, 0.1))]


def _nodes(n):
    return -1.0 + 2.0 * np.arange(n) / n


def _rel(a, b, mask=None):
    a = np.asarray(a, np.float64)
    if mask is not None:
        a, b = a[mask], b[mask]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def test_closed_form_study_1024(dev):
    from paper_1506_00014_amd import RadonPlan

    x = _nodes(N)
    theta = np.arange(N) * math.pi / N
    s = _nodes(N)
    ds = 2.0 / N
    X1, X2 = np.meshgrid(x, x)
    inner = X1 * X1 + X2 * X2 < 0.81
    rows = []
    results = {}
    for dec_filter, q in VARIANTS:
        plan = RadonPlan(N, N, N, dec_filter=dec_filter, q_theta=q)
        tag = f"dec_filter={dec_filter} q_theta={q} (r={plan.geom['r_dec']}, K={plan.geom['k_theta']})"
        res = {}
        for name, cx, cy, r in DISCS:
            img = ((X1 - cx) ** 2 + (X2 - cy) ** 2 <= r * r).astype(np.float64)
            ref = analytic.ellipse_sino(theta, s, [(cx, cy, r, r, 0.0, 1.0)])
            got = plan.forward(torch.tensor(img, dtype=torch.float32, device=dev)).cpu().numpy()
            t = s[None, :] - (cx * np.cos(theta)[:, None] + cy * np.sin(theta)[:, None])
            res[f"R {name} all"] = _rel(got, ref)
            res[f"R {name} |t|<r-2ds"] = _rel(got, ref, np.abs(t) < r - 2 * ds)
        for sig, (cx, cy) in GAUSS:
            img = analytic.gaussian_image(x, cx, cy, sig)
            ref = analytic.gaussian_sino(theta, s, cx, cy, sig)
            got = plan.forward(torch.tensor(img, dtype=torch.float32, device=dev)).cpu().numpy()
            res[f"R gauss s{sig} c({cx},{cy})"] = _rel(got, ref)
        for sig in (0.05, 0.1):
            ridge = np.exp(-(s[None, :] ** 2) / sig**2) * np.ones((N, 1))
            got = plan.adjoint(torch.tensor(ridge, dtype=torch.float32, device=dev)).cpu().numpy()
            res[f"R# ridge s{sig}"] = _rel(got, analytic.backproject_gaussian_ridge(x, sig), inner)
            sino = analytic.gaussian_sino(theta, s, 0.1, -0.05, sig)
            got = plan.fbp(torch.tensor(sino, dtype=torch.float32, device=dev)).cpu().numpy()
            res[f"FBP gauss s{sig}"] = _rel(got, analytic.gaussian_image(x, 0.1, -0.05, sig), inner)
        results[(dec_filter, q)] = res
        rows.append(tag)
        del plan
    keys = list(results[VARIANTS[0]].keys())
    print()
    print("relative L2 error vs closed form, 1024^2, 1024 angles x 1024 bins, M = 4")
    print(f"{'case':34s}" + "".join(f"  f{d}/q{q}    " for d, q in VARIANTS))
    for k in keys:
        print(f"{k:34s}" + "".join(f"  {results[v][k]:.3e}" for v in VARIANTS))
    for tag in rows:
        print(tag)
    for v in VARIANTS:
        res = results[v]
        assert res["R gauss s0.1 c(0.0,0.0)"] < 1e-4, v
        assert res["R gauss s0.05 c(0.25,0.1)"] < 1e-3, v
        assert res["R disc r0.5 |t|<r-2ds"] < 1e-2, v
        assert res["R# ridge s0.1"] < 5e-2, v
        assert res["FBP gauss s0.1"] < 5e-2, v
