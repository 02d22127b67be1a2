"""GPU parity on FFT lengths with factors of 3 (N_rho and K of the form 2^a 3^b): the radix-3
Stockham passes of the rho rows and the mixed-radix register FFTs of the theta pass, against the
FP64 oracle (whose FFTs take any length) on the same seeded inputs.  The paper sizes the lattice
at the bounds of sec. 3 (eq. vrho) and sec. 5 (2 N_theta / M rows); 2^a 3^b lengths sit closer to
those bounds than powers of two (M = 3 at 2048^2: N_rho 4608 against 8192 for a bound of 4334)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bp as obp  # noqa: E402
from oracle import radon as oradon  # noqa: E402
from oracle.geometry import Geometry, rho_bound  # noqa: E402
from paper_1506_00014_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-5


def check(label, got, ref):
    got = np.asarray(got, np.float64)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    mx = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"{label}: rel L2 vs FP64 oracle {e:.2e}, max|d|/max|ref| {mx:.2e}", flush=True)
    assert e <= TOL, label


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def plan_and_geom(n, nt, ns, m, n_rho, k_theta):
    from paper_1506_00014_amd import RadonPlan

    assert n_rho >= rho_bound(n, m)
    p = RadonPlan(n, nt, ns, m=m, n_rho=n_rho, k_theta=k_theta)
    g = p.geom
    og = Geometry(g["n"], g["n_theta"], g["n_s"], g["m"], g["n_rho"], g["k_theta"], g["r_dec"]).validate()
    return p, og


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


SMALL = [
    # (n, n_theta, n_s, m, n_rho, k_theta)
    (128, 180, 128, 4, 288, 96),    # 180 angles at 128^2: N_rho 2^5 3^2 (bound 217), K 96 = 32 x 3
    (128, 180, 128, 3, 288, 128),   # M = 3 (the paper's): N_rho 288 (bound 271)
    (64, 90, 64, 4, 144, 96),       # N_rho 2^4 3^2, K 32 x 3
    (96, 97, 80, 5, 216, 192),      # odd N_theta, M = 5: N_rho 2^3 3^3, K 32 x 6
    (48, 100, 40, 3, 108, 96),      # N_rho 2^2 3^3: radix-3 passes only after one radix 2
    (32, 36, 32, 4, 72, 24),        # K = 24 (a single register FFT of 8 x 3)
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}-nr{c[4]}-k{c[5]}")
def test_smooth_lengths_parity(dev, case):
    n, nt, ns, m, nr, kt = case
    plan, og = plan_and_geom(n, nt, ns, m, nr, kt)
    img, _ = inputs.ellipse_phantom(n, 8, 111)
    img += 0.3 * inputs.uniform_image(n, 112)
    x = torch.tensor(np.asarray(img, np.float32), device=dev)
    check(f"R {case}", plan.forward(x).cpu().numpy(), oradon.radon_fwd(og, f32(img)))
    g = inputs.normal_array((nt, ns), 113)
    y = torch.tensor(np.asarray(g, np.float32), device=dev)
    check(f"R# {case}", plan.adjoint(y).cpu().numpy(), oradon.radon_adj(og, f32(g)))
    sino = oradon.radon_fwd(og, f32(img))
    s = torch.tensor(np.asarray(sino, np.float32), device=dev)
    check(f"FBP {case}", plan.fbp(s).cpu().numpy(), oradon.fbp(og, f32(sino)))
    check(f"R# Algorithm 2 {case}", plan.bp_lp(s).cpu().numpy(), obp.radon_bp_lp(og, f32(sino)))


def test_smooth_m3_2048_sampled(dev):
    """M = 3 at 2048^2 (2048 angles x 2048 bins) with N_rho = 4608 = 2^9 3^2 and K = 1536 = 32 x 48,
    the paper's partition count at about half the power-of-two N_rho: one slice of a batch of 4,
    R against the oracle on every partition's rows and R# on the whole image."""
    n = 2048
    plan, og = plan_and_geom(n, n, n, 3, 4608, 1536)
    imgs = np.stack([inputs.ellipse_phantom(n, 20, 121 + b)[0] for b in range(4)]).astype(np.float32)
    got = plan.forward(torch.tensor(imgs, device=dev)).cpu().numpy()
    check("2048^2 M=3 R, slice 2", got[2], oradon.radon_fwd(og, f32(imgs[2])))
    g = np.stack([inputs.normal_array((n, n), 131 + b) for b in range(4)]).astype(np.float32)
    got = plan.adjoint(torch.tensor(g, device=dev)).cpu().numpy()
    check("2048^2 M=3 R#, slice 1", got[1], oradon.radon_adj(og, f32(g[1])))
