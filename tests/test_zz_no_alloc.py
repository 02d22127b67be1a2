"""radon_fwd_noalloc (workspace in the library's static device scratch) against radon_fwd (caller
workspace): the same kernels, so the results must agree bit for bit.  Two calls in a row on the
same GPU, the second with a smaller input (fewer and smaller slices), so the second call reuses
scratch the first one filled.  Calls go straight through the C-ABI."""

import ctypes

import numpy as np
import pytest

from paper_1506_00014_amd import RadonPlan, _lib, inputs

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _fwd_both(torch, plan, f):
    lib = _lib.load()
    B = f.shape[0]
    g = plan.geom
    ws = torch.empty(plan.workspace_bytes(B, _lib.RL_OP_FWD), dtype=torch.uint8, device="cuda")
    ref = torch.full((B, g["n_theta"], g["n_s"]), float("nan"), device="cuda")
    out = torch.full_like(ref, float("nan"))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    print(f"radon_fwd / radon_fwd_noalloc: n={g['n']} batch={B}", flush=True)
    _lib.check("radon_fwd", lib.radon_fwd(plan._ptr, _ptr(f), _ptr(ref), B, _ptr(ws), ws.numel(), stream))
    _lib.check("radon_fwd_noalloc", lib.radon_fwd_noalloc(plan._ptr, _ptr(f), _ptr(out), B, stream))
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_matches_radon_fwd_twice_second_smaller():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cases = [(512, 3, 11), (256, 1, 12)]  # (n, batch, seed): the second call is smaller
    for n, B, seed in cases:
        plan = RadonPlan(n, n, n)
        imgs = np.stack([inputs.ellipse_phantom(n, 12, seed + b)[0] for b in range(B)]).astype(np.float32)
        f = torch.tensor(imgs, device="cuda")
        ref, out = _fwd_both(torch, plan, f)
        assert np.isfinite(ref).all()
        assert np.array_equal(ref.view(np.uint32), out.view(np.uint32)), f"n={n} batch={B}: not bitwise equal"
        rel = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        print(f"n={n} batch={B}: bitwise equal (rel L2 {rel:.1e})", flush=True)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lib = _lib.load()
    plan = RadonPlan(2048, 2048, 2048)
    need = plan.workspace_bytes(2, _lib.RL_OP_FWD)
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    f = torch.zeros(2, 2048, 2048, device="cuda")
    g = torch.zeros(2, 2048, 2048, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.radon_fwd_noalloc(plan._ptr, _ptr(f), _ptr(g), 2, stream)
    assert st == _lib.RL_ERR_WORKSPACE
    assert b"static scratch" in lib.rl_last_error()
    assert lib.radon_fwd_noalloc(None, _ptr(f), _ptr(g), 1, stream) == _lib.RL_ERR_INVALID_ARG
    assert lib.radon_fwd_noalloc(plan._ptr, _ptr(f), _ptr(g), 0, stream) == _lib.RL_OK
