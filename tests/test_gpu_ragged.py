"""Ragged batches (slices of several geometries, one call per plan, each slice read and written
in its own buffer) through the C-ABI: equality with per-slice calls, replay of a captured HIP
graph, error codes; the autotuner: results do not depend on the launch parameters, and its
cache file is written once and read back."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1506_00014_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

GEOMS = [(64, 90, 64), (96, 97, 80), (128, 180, 128)]
PLAN_OF = [0, 1, 2, 0, 2, 1, 0]


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_00014_amd import RadonPlan

    dev = torch.device("cuda", 0)
    plans = [RadonPlan(*g) for g in GEOMS]
    return dev, plans


def make_items(dev, plans, seed):
    items = []
    for i, p in enumerate(PLAN_OF):
        n, nt, ns = GEOMS[p]
        img = torch.tensor(inputs.ellipse_phantom(n, 6, seed + i)[0], dtype=torch.float32, device=dev)
        sino = torch.tensor(inputs.normal_array((nt, ns), seed + 100 + i), dtype=torch.float32, device=dev)
        items.append((plans[p], img, sino))
    return items


def test_ragged_matches_plain_calls(setup):
    from paper_1506_00014_amd import RaggedBatch

    dev, plans = setup
    items = make_items(dev, plans, 500)
    batch = RaggedBatch(items)
    batch.forward()
    torch.cuda.synchronize()
    for plan, img, sino in items:
        ref = plan.forward(img)
        assert torch.equal(sino, ref)
    sinos = [s.clone() for _, _, s in items]
    batch.adjoint()
    torch.cuda.synchronize()
    for (plan, img, _), s in zip(items, sinos):
        ref = plan.adjoint(s)
        err = (img - ref).abs().max().item() / ref.abs().max().item()
        assert err <= 1e-6  # FP64 LDS accumulation: summation order may differ


def test_ragged_bp_lp_matches_plain_calls(setup):
    """Algorithm 2 over the ragged batch (one batched call per plan, the plans concurrent)
    equals per-slice radon_bp_lp; a plan with q_theta = 2 is refused before anything runs."""
    from paper_1506_00014_amd import RadonPlan, RaggedBatch, _lib

    dev, plans = setup
    items = make_items(dev, plans, 650)
    batch = RaggedBatch(items)
    batch.bp_lp()
    torch.cuda.synchronize()
    for plan, img, sino in items:
        ref = plan.bp_lp(sino)
        err = (img - ref).abs().max().item() / ref.abs().max().item()
        assert err <= 1e-6, err
    fine = RadonPlan(64, 90, 64, q_theta=2)
    img = torch.zeros(64, 64, device=dev)
    sino = torch.zeros(90, 64, device=dev)
    b2 = RaggedBatch([(fine, img, sino)])
    with pytest.raises(_lib.RadonLibError) as exc:
        b2.bp_lp()
    assert exc.value.status == _lib.RL_ERR_GEOMETRY


@pytest.mark.parametrize("op", ["forward", "adjoint", "bp_lp"])
def test_ragged_graph_replay(setup, op):
    """Capture one call of the batch (the plans' chains as parallel branches forked from and
    joined to the capturing stream), replay it after changing the inputs in place, with eager
    work and synchronisations between replays; every replay equals eager per-slice calls."""
    from paper_1506_00014_amd import RaggedBatch

    dev, plans = setup
    items = make_items(dev, plans, 600)
    batch = RaggedBatch(items)
    run = getattr(batch, op)
    run()  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for i, (plan, img, sino) in enumerate(items):
            n, nt, ns = img.shape[0], sino.shape[0], sino.shape[1]
            if op == "forward":
                img.copy_(torch.tensor(inputs.ellipse_phantom(n, 4, 700 + 10 * rep + i)[0], dtype=torch.float32))
                sino.zero_()
            else:
                sino.copy_(torch.tensor(inputs.normal_array((nt, ns), 900 + 10 * rep + i), dtype=torch.float32))
                img.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for plan, img, sino in items:
            if op == "forward":
                assert torch.equal(sino, plan.forward(img))
            else:
                ref = plan.adjoint(sino) if op == "adjoint" else plan.bp_lp(sino)
                assert (img - ref).abs().max().item() <= 1e-6 * ref.abs().max().item()
        _ = torch.ones(1000, device=dev).sum().item()  # eager work between replays


def test_ragged_errors(setup):
    from paper_1506_00014_amd import _lib

    dev, plans = setup
    lib = _lib.load()
    img = torch.zeros(64, 64, device=dev)
    sino = torch.zeros(90, 64, device=dev)
    c_plans = (ctypes.c_void_p * 1)(plans[0]._ptr.value)
    c_imgs = (ctypes.c_void_p * 1)(img.data_ptr())
    c_sinos = (ctypes.c_void_p * 1)(sino.data_ptr())
    out = ctypes.c_void_p()
    bad = (ctypes.c_int32 * 1)(1)  # plan index out of range
    assert lib.rl_batch_create(c_plans, 1, bad, c_imgs, c_sinos, 1, None, ctypes.byref(out)) == _lib.RL_ERR_INVALID_ARG
    ok = (ctypes.c_int32 * 1)(0)
    assert lib.rl_batch_create(c_plans, 1, ok, c_imgs, c_sinos, 1, None, ctypes.byref(out)) == _lib.RL_OK
    need = lib.rl_batch_workspace_bytes(out, 0)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.rl_batch_fwd(out, ctypes.c_void_p(ws.data_ptr()), need - 1, stream) == _lib.RL_ERR_WORKSPACE
    assert lib.rl_batch_fwd(out, ctypes.c_void_p(ws.data_ptr()), need, stream) == _lib.RL_OK
    torch.cuda.synchronize()
    lib.rl_batch_destroy(out)
    empty = ctypes.c_void_p()
    assert lib.rl_batch_create(c_plans, 1, ok, c_imgs, c_sinos, 0, None, ctypes.byref(empty)) == _lib.RL_OK
    assert lib.rl_batch_fwd(empty, None, 0, stream) == _lib.RL_OK  # count 0: no-op
    lib.rl_batch_destroy(empty)


def test_tuning_does_not_change_results(setup):
    """Every value of every launch parameter gives the default's R bitwise and its R# to the FP64
    accumulation order (the tile sums use LDS atomics)."""
    dev, plans = setup
    plan = plans[2]
    n, nt, ns = GEOMS[2]
    x = torch.tensor(inputs.ellipse_phantom(n, 8, 800)[0], dtype=torch.float32, device=dev).expand(3, n, n).contiguous()
    y = torch.tensor(inputs.normal_array((3, nt, ns), 801), dtype=torch.float32, device=dev)
    default = plan.tuning
    r0, b0 = plan.forward(x), plan.adjoint(y)
    try:
        for field, values in (("theta_cols", (1, 2, 3, 8)), ("theta_xcd_order", (0,)), ("prefilter_rows", (32, 96, 1024)),
                              ("fwd_patch_split", (0,)), ("fwd_xcd_order", (0, 1)), ("adj_walk", (0, 1))):
            for v in values:
                plan.tuning = {**default, field: v}
                assert torch.equal(plan.forward(x), r0), (field, v)
                e = ((plan.adjoint(y) - b0).abs().max() / b0.abs().max()).item()
                assert e <= 1e-6, (field, v, e)
        with pytest.raises(Exception):
            plan.tuning = {**default, "prefilter_rows": 100}  # not a multiple of 32
    finally:
        plan.tuning = default


def test_autotune_cache_and_ragged_batch(setup, tmp_path):
    from paper_1506_00014_amd import RaggedBatch

    dev, plans = setup
    cache = tmp_path / "tune.jsonl"
    defaults = [p.tuning for p in plans]
    try:
        items = make_items(dev, plans, 900)
        batch = RaggedBatch(items, tune_cache=cache)
        lines = cache.read_text().splitlines()
        assert len(lines) == len(GEOMS)  # one entry per plan (each for its slice count)
        for ln in lines:
            assert '"key": "gfx950' in ln and "theta_cols" in ln
        batch.forward()
        torch.cuda.synchronize()
        for plan, img, sino in items:
            assert torch.equal(sino, plan.forward(img))
        # a second batch of the same shapes reads the cache and tunes nothing
        RaggedBatch(make_items(dev, plans, 950), tune_cache=cache)
        assert cache.read_text().splitlines() == lines
        # the plan-level call reads it too
        tuned = plans[0].tuning
        plans[0].tuning = defaults[0]
        assert plans[0].autotune(PLAN_OF.count(0), cache=cache) == tuned
    finally:
        for p, d in zip(plans, defaults):
            p.tuning = d
