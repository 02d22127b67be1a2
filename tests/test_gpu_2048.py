"""The 2048 x 2048 workload (2048 angles x 2048 bins) in the launch configuration the
benchmark times (batch 64): parity on sampled outputs the oracle computes one partition at a
time, the adjoint identity on every slice (a property that holds at any size), and the
finite-difference check of the autograd gradient of ||R f - g||^2."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bspline as obspline  # noqa: E402
from oracle import radon as oradon  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from paper_1506_00014_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

N = 2048
BATCH = 64


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_00014_amd import RadonPlan

    dev = torch.device("cuda", 0)
    plan = RadonPlan(N, N, N)
    g = plan.geom
    og = Geometry(g["n"], g["n_theta"], g["n_s"], g["m"], g["n_rho"], g["k_theta"], g["r_dec"]).validate()
    gen = torch.Generator(device=dev)
    gen.manual_seed(303)
    f = torch.rand(BATCH, N, N, generator=gen, device=dev, dtype=torch.float32)
    ws = torch.empty(max(plan.workspace_bytes(BATCH, op) for op in (0, 1, 2)), dtype=torch.uint8, device=dev)
    return dev, plan, og, f, ws


def test_forward_sampled_partitions(setup):
    dev, plan, og, f, ws = setup
    sino = plan.forward(f, ws)
    torch.cuda.synchronize()
    s = BATCH - 1
    img = f[s].double().cpu().numpy()
    got = sino[s].double().cpu().numpy()
    c = obspline.prefilter_2d(img)
    for p in (0, 3):  # partition 0 holds the wrapped rows (theta near pi)
        clp = oradon._partition_forward(og, c, p, "fft")
        rows = []
        ref = []
        for i, j, tau in oradon.eval_taus(og, p):
            rows.append(j)
            ref.append(obspline.eval_periodic_1d(clp[i], tau) / og.a_R)
        ref = np.stack(ref)
        e = np.linalg.norm(got[rows] - ref) / np.linalg.norm(ref)
        print(f"2048^2 R, slice {s}, partition {p} ({len(rows)} rows): rel L2 vs FP64 oracle {e:.2e}")
        assert e <= 1e-5


def test_adjoint_identity_every_slice(setup):
    dev, plan, og, f, ws = setup
    gen = torch.Generator(device=dev)
    gen.manual_seed(304)
    y = torch.randn(BATCH, N, N, generator=gen, device=dev, dtype=torch.float32)
    Rf = plan.forward(f, ws).double()
    Ry = plan.adjoint(y, ws).double()
    lhs = og.w_S * (Rf * y.double()).sum(dim=(1, 2))
    rhs = og.w_X * (f.double() * Ry).sum(dim=(1, 2))
    scale = og.w_S * Rf.norm(dim=(1, 2)) * y.double().norm(dim=(1, 2))
    err = ((lhs - rhs).abs() / scale).max().item()
    print(f"2048^2 batch {BATCH}: max relative adjoint-identity defect {err:.2e}")
    assert err <= 1e-6


def test_gradient_finite_differences(setup):
    from paper_1506_00014_amd import RadonFn

    dev, plan, og, _, _ = setup
    img, _ = inputs.ellipse_phantom(N, 50, 301)
    x = torch.tensor(img, dtype=torch.float32, device=dev)
    with torch.no_grad():
        g = plan.forward(x)
        noise = torch.tensor(inputs.normal_array((N, N), 302), dtype=torch.float32, device=dev)
        g = g + 0.01 * g.abs().max() * noise
    f0 = torch.tensor(inputs.uniform_image(N, 303), dtype=torch.float32, device=dev)
    f = f0.clone().requires_grad_(True)
    loss = ((RadonFn.apply(f, plan) - g) ** 2).sum()
    loss.backward()
    grad = f.grad.double()

    def resid(z):
        with torch.no_grad():
            return plan.forward(z).double() - g.double()

    # R is linear, so L(f) = ||R f - g||^2 is exactly quadratic and its central difference
    # (L(f + h v) - L(f - h v)) / 2h equals <grad L, v> for every h.  A step h = 1 keeps the FP32
    # rounding of R(f +- h v) small against the difference (at h = 1e-3 that rounding, ~1e-3 of
    # the difference, dominates).  The difference is evaluated as sum((a - b)(a + b)) / 2h with
    # a, b the residuals at f +- h v, avoiding the cancellation of two sums of 4M squares.
    # Also checked: <grad L, v> against 2 <R v, R f - g>, which uses R on v directly.
    h = 1.0
    worst = 0.0
    r0 = resid(f0)
    for k in range(16):
        v = torch.tensor(inputs.normal_array((N, N), 310 + k), dtype=torch.float32, device=dev)
        a, b = resid(f0 + h * v), resid(f0 - h * v)
        fd = ((a - b) * (a + b)).sum().item() / (2 * h)
        with torch.no_grad():
            direct = 2.0 * (plan.forward(v).double() * r0).sum().item()
        an = (grad * v.double()).sum().item()
        rel = abs(fd - an) / abs(an)
        rel_direct = abs(direct - an) / abs(an)
        print(f"  direction {k}: analytic {an:.6e}  central difference {fd:.6e}  2<Rv,r> {direct:.6e}  "
              f"rel {rel:.2e} / {rel_direct:.2e}")
        worst = max(worst, rel, rel_direct)
    print(f"2048^2 gradient vs central differences, 16 directions: worst relative error {worst:.2e}")
    assert worst <= 1e-3
