"""GPU parity: the HIP path through the C-ABI against the FP64 oracle on the same seeded
inputs.  Bar: relative L2 <= 1e-5 for R, R#, FBP and R^T; the error against FP64 is printed
for every case.  Stage tests compare the intermediates rl_debug_stage exports."""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel  # noqa: E402
from oracle import radon as oradon  # noqa: E402
from oracle import bspline as obspline  # noqa: E402
from oracle.geometry import Geometry  # noqa: E402
from paper_1506_00014_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    a = np.asarray(a)
    a = a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """Largest elementwise error, relative to the largest reference value."""
    a = np.asarray(a, np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check(label, got, ref, tol=TOL):
    """Relative L2 error (the bar) with the largest elementwise error beside it."""
    e, mx = rel(got, ref), max_rel(got, ref)
    print(f"{label}: rel L2 vs FP64 oracle {e:.2e}, max|d|/max|ref| {mx:.2e}")
    assert e <= tol, label
    return e


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


_plans = {}


def get_plan(n, nt, ns, m=4, **kw):
    from paper_1506_00014_amd import RadonPlan

    key = (n, nt, ns, m, tuple(sorted(kw.items())))
    if key not in _plans:
        p = RadonPlan(n, nt, ns, m=m, **kw)
        g = p.geom
        og = Geometry(g["n"], g["n_theta"], g["n_s"], g["m"], g["n_rho"], g["k_theta"], g["r_dec"], g["dec_filter"],
                      g["q_theta"]).validate()
        _plans[key] = (p, og)
    return _plans[key]


def to_dev(x, dev):
    return torch.tensor(np.asarray(x, np.float32), device=dev)


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


CASES = [
    # (n, n_theta, n_s, m, extra): small sizes spanning several tiles and ragged tails
    (128, 180, 128, 4, {}),   # the 128 x 128, 180-angle configuration
    (64, 90, 64, 4, {}),
    (48, 100, 40, 3, {}),     # M = 3, M does not divide N_theta
    (96, 97, 80, 5, {}),      # odd N_theta, N_s != N, ragged tiles
    (32, 48, 32, 4, {"n_rho": 128, "r_dec": 8}),  # oversampled geometry
    (16, 24, 16, 4, {}),      # smaller than one tile
]

# larger theta-FFT lengths (K = 512, 1024, 2048), the 1024 x 1024 configuration, wide sectors
BIG_CASES = [
    (768, 768, 768, 4, {}),   # the odd size of the ragged-batch mix (N_rho 2048, K 512)
    # wide forward sectors: M = 6 runs all three forward tile lists (small patch at pitch 77, large
    # at pitch 93, large at each box's own pitch), M = 8 mostly the last, staged or gathering from
    # global memory where even that does not fit
    (768, 768, 768, 6, {}),
    (768, 768, 768, 8, {}),
    (256, 1024, 256, 4, {}),
    (512, 2048, 512, 4, {}),
    (256, 4096, 256, 4, {}),
    (1024, 1024, 1024, 4, {}),
]


# accuracy variants of Algorithm 1 step 4: the box low-pass (dec_filter 1), the coarse lattice at
# half the sinogram's angular spacing (q_theta 2), and both; odd and even r, M = 3 and 5
VARIANT_CASES = [
    (128, 180, 128, 4, {"dec_filter": 1}),
    (128, 180, 128, 4, {"q_theta": 2}),
    (64, 90, 64, 4, {"dec_filter": 1, "q_theta": 2}),
    (96, 97, 80, 5, {"q_theta": 2}),
    (48, 100, 40, 3, {"dec_filter": 1}),
    (256, 256, 256, 4, {"dec_filter": 1, "q_theta": 2}),
]


@pytest.mark.parametrize("case", VARIANT_CASES,
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}" + "".join(f"-{k}{v}" for k, v in c[4].items()))
def test_variant_parity(dev, case):
    """R, R# and FBP on the step-4 variants against the oracle's reading of them."""
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    assert (og.dec_filter, og.q_theta) == (kw.get("dec_filter", 0), kw.get("q_theta", 1))
    img, _ = inputs.ellipse_phantom(n, 8, 105)
    img += 0.3 * inputs.uniform_image(n, 106)
    got = plan.forward(to_dev(img, dev)).cpu().numpy()
    check(f"R {case} r={og.r_dec} K={og.k_theta}", got, oradon.radon_fwd(og, f32(img)))
    g = inputs.normal_array((nt, ns), 107)
    got = plan.adjoint(to_dev(g, dev)).cpu().numpy()
    check(f"R# {case}", got, oradon.radon_adj(og, f32(g)))
    sino = oradon.radon_fwd(og, f32(img))
    got = plan.fbp(to_dev(sino, dev)).cpu().numpy()
    check(f"FBP {case}", got, oradon.fbp(og, f32(sino)))


def test_bp_lp_rejects_half_spacing_lattice(dev):
    """Algorithm 2 reads its lattice on the sinogram rows: q_theta = 2 is refused, not run."""
    from paper_1506_00014_amd import _lib

    plan, og = get_plan(64, 90, 64, 4, q_theta=2)
    g = to_dev(inputs.normal_array((90, 64), 108), dev)
    with pytest.raises(_lib.RadonLibError) as e:
        plan.bp_lp(g)
    assert e.value.status == _lib.RL_ERR_GEOMETRY


# M = 5, 6, 8 (beta = pi/M) with rows at theta' = -beta/2 exactly, where the ray is tangent to D and
# the sample at s = -1 lands on tau = -1 up to rounding (just below it at these sizes)
TANGENT_CASES = [(128, 192, 128, 5), (128, 192, 128, 6), (128, 180, 128, 6), (128, 192, 128, 8)]


@pytest.mark.parametrize("case", TANGENT_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_more_partitions_parity(dev, case):
    """More partitions than the default, on geometries whose tangent rows put tau just below -1."""
    n, nt, ns, m = case
    plan, og = get_plan(n, nt, ns, m)
    img, _ = inputs.ellipse_phantom(n, 8, 103)
    got = plan.forward(to_dev(img, dev)).cpu().numpy()
    ref = oradon.radon_fwd(og, f32(img))
    check(f"R M={m}", got, ref)
    g = inputs.normal_array((og.n_theta, og.n_s), 104)
    got = plan.adjoint(to_dev(g, dev)).cpu().numpy()
    ref = oradon.radon_adj(og, f32(g))
    check(f"R# M={m}", got, ref)


@pytest.mark.parametrize("case", BIG_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_forward_adjoint_parity_large(dev, case):
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    img, blobs_e, blobs_g = inputs.mixed_phantom(n, 30, 5, 201)
    got = plan.forward(to_dev(img, dev)).cpu().numpy()
    ref = oradon.radon_fwd(og, f32(img))
    check(f"R {case} K={og.k_theta}", got, ref)
    g = inputs.normal_array((nt, ns), 202)
    got = plan.adjoint(to_dev(g, dev)).cpu().numpy()
    ref = oradon.radon_adj(og, f32(g))
    check(f"R# {case} K={og.k_theta}", got, ref)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_forward_parity(dev, case):
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    img, _ = inputs.ellipse_phantom(n, 8, 101)
    img += 0.3 * inputs.uniform_image(n, 103)  # nonzero up to the image border
    got = plan.forward(to_dev(img, dev)).cpu().numpy()
    ref = oradon.radon_fwd(og, f32(img))
    check(f"R {case}", got, ref)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_adjoint_parity(dev, case):
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    g = inputs.normal_array((nt, ns), 102)
    got = plan.adjoint(to_dev(g, dev)).cpu().numpy()
    ref = oradon.radon_adj(og, f32(g))
    check(f"R# {case}", got, ref)
    gt = plan.transpose(to_dev(g, dev)).cpu().numpy()
    check(f"R^T {case}", gt, ref * (og.w_X / og.w_S))


@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_fbp_parity(dev, case):
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    img, ells = inputs.ellipse_phantom(n, 8, 101)
    from oracle import analytic

    g = analytic.ellipse_sino(og.theta_nodes(), og.s_nodes(), ells)
    got = plan.fbp(to_dev(g, dev)).cpu().numpy()
    ref = oradon.fbp(og, f32(g))
    check(f"FBP {case}", got, ref)


@pytest.mark.parametrize("filt", ["cosine", "shepp-logan"])
@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_fbp_filter_parity(dev, case, filt):
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    img, ells = inputs.ellipse_phantom(n, 8, 102)
    from oracle import analytic

    g = analytic.ellipse_sino(og.theta_nodes(), og.s_nodes(), ells)
    got = plan.fbp(to_dev(g, dev), filter=filt).cpu().numpy()
    ref = oradon.fbp(og, f32(g), name=filt)
    check(f"FBP {filt} {case}", got, ref)
    # the window changes the result well above the tolerance
    assert rel(plan.fbp(to_dev(g, dev)).cpu().numpy(), ref) > 10 * TOL


def test_fbp_unknown_filter(dev):
    plan, og = get_plan(*CASES[1][:4], **CASES[1][4])
    g = torch.zeros(og.n_theta, og.n_s, device=dev)
    with pytest.raises(ValueError):
        plan.fbp(g, filter="hann")
    from paper_1506_00014_amd import _lib
    import ctypes
    lib = _lib.load()
    ws = torch.empty(plan.workspace_bytes(1, _lib.RL_OP_FBP), dtype=torch.uint8, device=dev)
    out = torch.empty(og.n, og.n, device=dev)
    st = lib.fbp(plan._ptr, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()), 1, 3,
                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == _lib.RL_ERR_INVALID_ARG


def test_stage_parity(dev):
    from paper_1506_00014_amd import _lib

    n, nt, ns = 128, 180, 128
    plan, og = get_plan(n, nt, ns)
    img = inputs.uniform_image(n, 104) - 0.5
    x = to_dev(img, dev)
    # prefilter
    c_gpu = plan.debug_stage(_lib.RL_STAGE_PREFILTER, x).cpu().numpy()
    c_ref = obspline.prefilter_2d(f32(img))
    assert rel(c_gpu, c_ref) <= 1e-6
    # kernel table (scaled by 1 / (K N_rho)), stored [k_rho][k_theta]
    Hg = plan.debug_stage(_lib.RL_STAGE_KERNEL, x).cpu().numpy()
    Hg = Hg[..., 0] + 1j * Hg[..., 1]
    Hr = okernel.multiplier_half(og).T / (og.k_theta * og.n_rho)
    assert rel(Hg, Hr) <= 1e-6
    # log-polar samples w (rows of each partition's support) and the convolution output
    w_gpu = plan.debug_stage(_lib.RL_STAGE_LOGPOLAR, x).cpu().numpy()
    conv_gpu = plan.debug_stage(_lib.RL_STAGE_CONV, x).cpu().numpy()
    c64 = obspline.prefilter_2d(f32(img))
    for p in range(og.m):
        clp = oradon._partition_forward(og, c64, p, "fft")
        # the oracle's step S5 output is recomputed here from its pieces
        n_sup_p = len(og.partition_rows(p)) + 4
        ti, q, X, Y = oradon.fine_sample_points(og, p)
        t = og.fine_rows(p)
        v = np.zeros((t.size, og.n_rho))
        v[ti, q] = obspline.eval_periodic_2d(c64, X, Y)
        d = okernel.decimation_taps(og.r_dec)
        r = og.r_dec
        u = np.stack([d @ v[r * i - (2 * r - 1) - t[0]: r * i - (2 * r - 1) - t[0] + 4 * r - 1]
                      for i in range(n_sup_p)])
        w = u * np.exp(og.rho_nodes())[None, :]
        assert rel(w_gpu[p, :n_sup_p], w) <= 1e-6, p
        own = len(og.partition_rows(p))
        assert rel(conv_gpu[p, :own], clp[2:2 + own]) <= 2e-6, p


def test_batch_equals_single_slices(dev):
    n, nt, ns = 64, 90, 64
    plan, og = get_plan(n, nt, ns)
    imgs = np.stack([inputs.ellipse_phantom(n, 5, 200 + i)[0] for i in range(3)])
    x = to_dev(imgs, dev)
    batched = plan.forward(x).cpu().numpy()
    for i in range(3):
        single = plan.forward(x[i]).cpu().numpy()
        assert np.array_equal(batched[i], single)
    g = inputs.normal_array((3, nt, ns), 5)
    gb = plan.adjoint(to_dev(g, dev)).cpu().numpy()
    for i in range(3):
        gs = plan.adjoint(to_dev(g[i], dev)).cpu().numpy()
        assert np.max(np.abs(gb[i] - gs)) <= 1e-6 * np.abs(gs).max()
    assert plan.forward(torch.empty(0, n, n, device=dev)).shape == (0, nt, ns)


def test_adjoint_identity_fp32(dev):
    n, nt, ns = 128, 180, 128
    plan, og = get_plan(n, nt, ns)
    f = inputs.normal_array((n, n), 21)
    g = inputs.normal_array((nt, ns), 22)
    Rf = plan.forward(to_dev(f, dev)).double().cpu().numpy()
    Rsg = plan.adjoint(to_dev(g, dev)).double().cpu().numpy()
    lhs = og.w_S * np.sum(Rf * g)
    rhs = og.w_X * np.sum(f * Rsg)
    scale = og.w_S * np.linalg.norm(Rf) * np.linalg.norm(g)
    print(f"adjoint identity FP32: {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_autograd_gradient_matches_oracle(dev):
    from paper_1506_00014_amd import RadonFn

    n, nt, ns = 128, 180, 128
    plan, og = get_plan(n, nt, ns)
    img, _ = inputs.ellipse_phantom(n, 8, 331)
    g = oradon.radon_fwd(og, img) + 0.01 * inputs.normal_array((nt, ns), 332)
    f0 = inputs.uniform_image(n, 333)
    f = to_dev(f0, dev).requires_grad_(True)
    y = to_dev(g, dev)
    loss = ((RadonFn.apply(f, plan) - y) ** 2).sum()
    loss.backward()
    grad = f.grad.double().cpu().numpy()
    ref = 2.0 * (og.w_X / og.w_S) * oradon.radon_adj(og, oradon.radon_fwd(og, f32(f0)) - f32(g))
    check("autograd gradient vs oracle 2 R^T (R f - g)", grad, ref)


def test_errors_on_device(dev):
    from paper_1506_00014_amd import _lib

    plan, og = get_plan(64, 90, 64)
    x = torch.zeros(2, 64, 64, device=dev)
    y = torch.zeros(2, 90, 64, device=dev)
    lib = _lib.load()
    import ctypes

    small = torch.empty(16, dtype=torch.uint8, device=dev)
    st = lib.radon_fwd(plan._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 2,
                       ctypes.c_void_p(small.data_ptr()), 16, None)
    assert st == 3  # workspace too small
    ws = torch.empty(plan.workspace_bytes(2, 0), dtype=torch.uint8, device=dev)
    st = lib.radon_fwd(plan._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr() + 4), 2,
                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == 1  # overlapping input and output
    st = lib.radon_fwd(plan._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0, None, 0, None)
    assert st == 0  # batch 0 is a no-op
    with pytest.raises(Exception):
        plan.forward(torch.zeros(64, 64, dtype=torch.float64, device=dev))


@pytest.mark.parametrize("case", CASES[:4], ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}m{c[3]}")
def test_fine_sample_count(dev, case):
    """The plan's count of in-D fine samples (work accounting) equals the oracle's sample set."""
    n, nt, ns, m, kw = case
    plan, og = get_plan(n, nt, ns, m, **kw)
    ref = sum(oradon.fine_sample_points(og, p)[0].size for p in range(og.m))
    assert plan.fine_samples() == ref


def test_adjoint_autograd_gradient_matches_oracle(dev):
    """RadonAdjFn: f = R# g with backward (R#)^T = (w_S / w_X) R.  For L(g) = ||R# g - b||^2 the
    gradient is 2 (w_S / w_X) R (R# g - b); checked against the oracle at 128^2 and against
    central differences (L is exactly quadratic, so any step gives the directional derivative)."""
    from paper_1506_00014_amd import RadonAdjFn

    n, nt, ns = 128, 180, 128
    plan, og = get_plan(n, nt, ns)
    g0 = inputs.normal_array((nt, ns), 341)
    b, _ = inputs.ellipse_phantom(n, 8, 342)
    y = to_dev(g0, dev).requires_grad_(True)
    tb = to_dev(b, dev)
    loss = ((RadonAdjFn.apply(y, plan) - tb) ** 2).sum()
    loss.backward()
    grad = y.grad.double().cpu().numpy()
    ref = 2.0 * (og.w_S / og.w_X) * oradon.radon_fwd(og, oradon.radon_adj(og, f32(g0)) - f32(b))
    check("RadonAdjFn gradient vs oracle 2 (w_S/w_X) R (R# g - b)", grad, ref)
    # the backward entry point alone: (R#)^T f = (w_S / w_X) R f
    x = inputs.normal_array((n, n), 343)
    got = plan.adjoint_transpose(to_dev(x, dev)).cpu().numpy()
    check("(R#)^T vs oracle (w_S/w_X) R", got, (og.w_S / og.w_X) * oradon.radon_fwd(og, f32(x)))
    # central differences of the loss in 8 directions, in FP64 on the host
    with torch.no_grad():
        r0 = (plan.adjoint(to_dev(g0, dev)) - tb).double()
        worst = 0.0
        for k in range(8):
            v = inputs.normal_array((nt, ns), 350 + k)
            a = (plan.adjoint(to_dev(g0 + v, dev)) - tb).double()
            bm = (plan.adjoint(to_dev(g0 - v, dev)) - tb).double()
            fd = ((a - bm) * (a + bm)).sum().item() / 2.0
            an = float(np.sum(grad * f32(v)))
            worst = max(worst, abs(fd - an) / abs(an))
    print(f"RadonAdjFn gradient vs central differences, 8 directions: worst relative error {worst:.2e}")
    assert worst <= TOL
    del r0


def test_plan_rows_match_oracle(dev):
    """rl_plan_rows: the rows each partition owns (eq. Radon_all_pb) as the oracle counts them."""
    for case in CASES + BIG_CASES:
        n, nt, ns, m, kw = case
        plan, og = get_plan(n, nt, ns, m, **kw)
        n_own, rows = plan.rows_per_partition()
        assert rows == [len(og.partition_rows(p)) for p in range(og.m)], case
        assert n_own == og.n_own, case
