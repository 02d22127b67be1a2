"""The 2048 x 2048 workload (2048 angles x 2048 bins) in the launch configuration the
benchmark times (batch 64).  One slice of each batch-64 launch is compared element by
element with the FP64 oracle: R on all four partitions (the oracle runs one partition at a
time), R# on a random sinogram, and FBP with each of the three filters (l_r = 4096 on the
zero-padded s-axis).  Also: the adjoint identity on every slice (a property that holds at
any size), run-twice reproducibility, and the finite-difference check of the autograd
gradient of ||R f - g||^2."""

import math
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
TOL = 1e-5


def report(label, got, ref, tol=TOL):
    """Relative L2 error (the bar) and the largest elementwise error relative to max|ref|."""
    got = np.asarray(got, np.float64)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    mx = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"{label}: rel L2 vs FP64 oracle {e:.2e}, max|d|/max|ref| {mx:.2e}", flush=True)
    assert e <= tol, label
    assert mx <= tol, label
    return e


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


@pytest.fixture(scope="module")
def sino(setup):
    dev, plan, og, f, ws = setup
    out = plan.forward(f, ws)
    torch.cuda.synchronize()
    return out


def test_forward_all_partitions(setup, sino):
    """Every sinogram row of one slice, partition by partition (partition 0 holds the wrapped
    rows near theta = pi, partition 1 the tie row j = 256 that rounds half up)."""
    dev, plan, og, f, ws = setup
    s = BATCH - 1
    img = f[s].double().cpu().numpy()
    got = sino[s].double().cpu().numpy()
    c = obspline.prefilter_2d(img)
    ref = np.zeros_like(got)
    for p in range(og.m):
        clp = oradon._partition_forward(og, c, p, "fft")
        rows = []
        for i, j, tau in oradon.eval_taus(og, p):
            rows.append(j)
            ref[j] = obspline.eval_periodic_1d(clp[i], tau) / og.a_R
        report(f"2048^2 R, slice {s}, partition {p} ({len(rows)} rows)", got[rows], ref[rows])
    report(f"2048^2 R, slice {s}, whole sinogram", got, ref)


def test_adjoint_full_slice(setup):
    """R# of a N(0, 1) sinogram: the k_splat_rfft / k_irfft_scale rows of length 4096 and the
    2048^2 splat, against the oracle's exact transpose."""
    dev, plan, og, f, ws = setup
    gen = torch.Generator(device=dev)
    gen.manual_seed(305)
    y = torch.randn(BATCH, N, N, generator=gen, device=dev, dtype=torch.float32)
    back = plan.adjoint(y, ws)
    torch.cuda.synchronize()
    s = 17
    ref = oradon.radon_adj(og, y[s].double().cpu().numpy())
    report(f"2048^2 R#, slice {s} of {BATCH}", back[s].cpu().numpy(), ref)


@pytest.fixture(scope="module")
def fbp_input(setup):
    """A batch of 64 sinograms whose slice 5 is the analytic sinogram of a 50-ellipse phantom
    (computed on the host) and the others N(0, 1)."""
    from oracle import analytic

    dev, plan, og, f, ws = setup
    _, ells = inputs.ellipse_phantom(N, 50, 306)
    g = analytic.ellipse_sino(og.theta_nodes(), og.s_nodes(), ells).astype(np.float32)
    gen = torch.Generator(device=dev)
    gen.manual_seed(307)
    batch = torch.randn(BATCH, N, N, generator=gen, device=dev, dtype=torch.float32)
    batch[5] = torch.tensor(g, device=dev)
    return 5, g.astype(np.float64), batch


@pytest.mark.parametrize("filt", ["ramlak", "cosine", "shepp-logan"])
def test_fbp_full_slice(setup, fbp_input, filt):
    """FBP: the filter on the zero-padded s-axis of length 4096, then R#."""
    dev, plan, og, f, ws = setup
    s, g, batch = fbp_input
    rec = plan.fbp(batch, ws, filter=filt)
    torch.cuda.synchronize()
    ref = oradon.radon_adj(og, oradon.fbp_filter(og, g, filt))
    report(f"2048^2 FBP {filt}, slice {s} of {BATCH}", rec[s].cpu().numpy(), ref)


def test_run_twice(setup, sino):
    """R is bitwise reproducible (no atomics).  R# accumulates each image tile with FP64 LDS
    atomics whose order varies between runs; the FP64 sums differ by rounding only, so the
    FP32 results agree to about one unit in the last place."""
    dev, plan, og, f, ws = setup
    again = plan.forward(f, ws)
    assert torch.equal(again, sino)
    b1 = plan.adjoint(sino, ws)
    b2 = plan.adjoint(sino, ws)
    d = ((b1 - b2).abs().max() / b1.abs().max()).item()
    print(f"2048^2 R# run twice: max|d|/max|R#| {d:.2e}", flush=True)
    assert d <= 1e-6


def test_adjoint_identity_every_slice(setup, sino):
    dev, plan, og, f, ws = setup
    gen = torch.Generator(device=dev)
    gen.manual_seed(304)
    y = torch.randn(BATCH, N, N, generator=gen, device=dev, dtype=torch.float32)
    Rf = sino.double()
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
    # (L(f + h v) - L(f - h v)) / 2h equals <grad L, v> for every h; the difference is
    # evaluated as sum((a - b)(a + b)) / 2h with a, b the residuals at f +- h v, avoiding the
    # cancellation of two sums of 4M squares.  What remains is FP32 rounding: of R(f +- h v)
    # (about 2e-7 of a and b) seen through a - b = 2h R v, with |R v| ~1/20 of |R f| for
    # v ~ N(0, 1) and f ~ U[0, 1]; and of the gradient (R^T in FP32).  Errors are measured against
    # the size of <grad L, v> for a random direction, s = |grad L| |v| / sqrt(n) (a direction
    # whose inner product happens to cancel to a small value must not magnify the bar).
    # h = 100: a - b dominates the rounding, bar 1e-5 of s, as for 2 <R v, R f - g> (R applied
    # to v directly, the FP32 adjoint consistency of R and R^T).  h = 1 (errors ~1e-4 observed)
    # and the configuration's h = 1e-3 (a - b ~5e-5 of a and b, comparable to their rounding:
    # errors ~1e-1) are printed, not checked.  The gradient is also pinned against the FP64
    # oracle gradient at 128^2.
    hs = (100.0, 1.0, 1e-3)
    worst = {h: 0.0 for h in hs}
    worst_direct = 0.0
    gnorm = grad.norm().item()
    r0 = resid(f0)
    for k in range(16):
        v = torch.tensor(inputs.normal_array((N, N), 310 + k), dtype=torch.float32, device=dev)
        an = (grad * v.double()).sum().item()
        scale = gnorm * v.double().norm().item() / math.sqrt(v.numel())
        with torch.no_grad():
            direct = 2.0 * (plan.forward(v).double() * r0).sum().item()
        e_direct = abs(direct - an) / scale
        worst_direct = max(worst_direct, e_direct)
        line = f"  direction {k}: <grad, v> {an:.6e} (scale {scale:.3e})  2<Rv,r> {direct:.6e} ({e_direct:.1e})"
        for h in hs:
            a, b = resid(f0 + h * v), resid(f0 - h * v)
            fd = ((a - b) * (a + b)).sum().item() / (2 * h)
            e = abs(fd - an) / scale
            line += f"  h={h:g}: fd {fd:.6e} ({e:.1e})"
            worst[h] = max(worst[h], e)
        print(line, flush=True)
    print("2048^2 gradient vs central differences, 16 directions, worst error / s: "
          + ", ".join(f"{worst[h]:.2e} (h = {h:g})" for h in hs) + f"; 2<Rv,r>: {worst_direct:.2e}")
    assert worst_direct <= TOL
    assert worst[100.0] <= TOL
