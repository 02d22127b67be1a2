"""Least-squares reconstruction by autograd (the batched gradient-descent workload): the power
iteration and the gradient-descent iterates against the same iterations run on the FP64 oracle,
and a reduced run of the full workload (Poisson data, 50 steps) whose loss and error must fall."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import radon as oradon  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from paper_1506_00014_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def make(n, nt, ns):
    from paper_1506_00014_amd import RadonPlan

    plan = RadonPlan(n, nt, ns)
    g = plan.geom
    og = Geometry(g["n"], g["n_theta"], g["n_s"], g["m"], g["n_rho"], g["k_theta"], g["r_dec"]).validate()
    return plan, og


def oracle_power(og, v0, iters):
    """Power iteration on R^T R = (w_X / w_S) R# R in FP64 (the oracle's transforms)."""
    v = v0 / np.linalg.norm(v0)
    est = 0.0
    for _ in range(iters):
        rv = oradon.radon_fwd(og, v)
        est = float(np.sum(rv * rv) / np.sum(v * v))
        w = (og.w_X / og.w_S) * oradon.radon_adj(og, rv)
        v = w / np.linalg.norm(w)
    return est


def test_power_iteration_matches_oracle(dev):
    from paper_1506_00014_amd import recon

    plan, og = make(64, 96, 64)
    v0 = inputs.normal_array((64, 64), 502)
    got = recon.power_iteration(plan, iters=20, v0=torch.tensor(v0, dtype=torch.float32))
    ref = oracle_power(og, np.asarray(v0, np.float32).astype(np.float64), 20)
    print(f"||R^T R|| by 20 power steps: GPU {got:.8e}, FP64 oracle {ref:.8e} (rel {abs(got - ref) / ref:.1e})")
    assert abs(got - ref) <= TOL * ref


def test_gradient_descent_matches_oracle(dev):
    """Ten steps of f <- f - grad / lam on a 2-slice batch, lam = 2 ||R^T R|| from the oracle's
    power iteration, against the same steps in FP64: grad = 2 R^T (R f - g)."""
    from paper_1506_00014_amd import recon

    n, nt, ns, steps = 64, 96, 64, 10
    plan, og = make(n, nt, ns)
    lam = 2.0 * oracle_power(og, inputs.normal_array((n, n), 503), 20)
    phantoms, data = inputs.noisy_ellipse_stack(2, n, nt, ns, 10, 1e4, "cpu", seed0=5100, noise_seed=504)
    g = data.double().numpy()
    losses = []
    got = recon.least_squares_gd(plan, data.to(dev), steps, lam, callback=lambda k, l: losses.append(float(l)))
    got = got.cpu().numpy()
    for b in range(2):
        f = np.zeros((n, n))
        for _ in range(steps):
            r = oradon.radon_fwd(og, f) - g[b]
            f = f - (2.0 / lam) * (og.w_X / og.w_S) * oradon.radon_adj(og, r)
        e = rel(got[b], f)
        print(f"slice {b}: {steps} gradient steps, rel L2 vs FP64 oracle {e:.2e}")
        assert e <= TOL
    assert all(b < a for a, b in zip(losses, losses[1:])), losses


def test_reduced_noisy_reconstruction(dev):
    """The batched workload at a reduced size (4 slices of 256^2, 128 angles x 256 bins, 10^4
    photons, 50 steps): the loss falls at every step and the error to the phantom falls."""
    from paper_1506_00014_amd import recon

    n, nt, ns = 256, 128, 256
    plan, og = make(n, nt, ns)
    phantoms, data = inputs.noisy_ellipse_stack(4, n, nt, ns, 30, 1e4, dev)
    lam = 2.0 * recon.power_iteration(plan, 20)
    errs, losses = [], []

    def cb(k, loss):
        losses.append(float(loss))

    f = recon.least_squares_gd(plan, data, 50, lam, callback=cb)
    err = ((f - phantoms).norm() / phantoms.norm()).item()
    fbp = plan.fbp(data)
    err_fbp = ((fbp - phantoms).norm() / phantoms.norm()).item()
    print(f"4 x 256^2: 50 gradient steps rel error {err:.3f}, FBP {err_fbp:.3f}; "
          f"loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert all(b < a for a, b in zip(losses, losses[1:]))
    assert err < 0.9
    errs.append(err)
