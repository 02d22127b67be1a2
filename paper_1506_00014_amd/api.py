"""PyTorch binding of the C-ABI: plans, the three operators, and autograd.

Only argument marshalling happens here: tensors are checked, a workspace is taken from
torch's caching allocator, and the C entry points are called on the current HIP stream.
Every step of R, R# and FBP runs in the library's HIP kernels.  There is no fallback:
without the built library, or without a gfx950 device, the calls raise.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import _lib


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class RadonPlan:
    """A geometry and its device tables (sec. 3 of the paper: grids, kernel coefficients).

    n, n_theta, n_s: image side, number of angles on [0, pi), detector bins on [-1, 1].
    m: angular partitions (beta = pi/m); n_rho, k_theta, r_dec: FFT lengths and fine
    angular oversampling (default: the smallest values meeting the paper's bounds).
    dec_filter: theta low-pass of Algorithm 1 step 4 (0 cubic B-spline, 1 box of one coarse
    cell); q_theta: coarse lattice spacing Delta theta / q_theta (1 or 2); smooth: default FFT
    lengths among 2^a 3^b instead of powers of two.
    """

    def __init__(self, n, n_theta, n_s, m=4, n_rho=None, k_theta=None, r_dec=None, device=None, dec_filter=0,
                 q_theta=1, smooth=False):
        lib = _lib.load()
        g = _lib.geom_default(n, n_theta, n_s, m, q_theta, 1 if smooth else 0)
        g.dec_filter = dec_filter
        if n_rho is not None:
            g.n_rho = n_rho
        if k_theta is not None:
            g.k_theta = k_theta
        if r_dec is not None:
            g.r_dec = r_dec
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._ptr = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check("rl_plan_create", lib.rl_plan_create(ctypes.byref(g), ctypes.byref(self._ptr)))
        self.geom = g.as_dict()
        self._lib = lib

    def __del__(self):
        ptr = getattr(self, "_ptr", None)
        if ptr is not None and ptr.value:
            self._lib.rl_plan_destroy(ptr)
            self._ptr = None

    # ------------------------------------------------------------------ helpers
    @property
    def w_S(self):
        return (math.pi / self.geom["n_theta"]) * (2.0 / self.geom["n_s"])

    @property
    def w_X(self):
        return (2.0 / self.geom["n"]) ** 2

    def workspace_bytes(self, batch, op):
        return int(self._lib.rl_workspace_bytes(self._ptr, batch, op))

    def fine_samples(self):
        """In-D fine log-polar samples of one slice over all partitions (interpolations per R)."""
        out = ctypes.c_int64()
        _lib.check("rl_plan_samples", self._lib.rl_plan_samples(self._ptr, ctypes.byref(out)))
        return int(out.value)

    def _check_in(self, x, shape_tail, name):
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if x.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
        if tuple(x.shape[-2:]) != shape_tail:
            raise ValueError(f"{name} must end in {shape_tail}, got {tuple(x.shape)}")
        if x.device != self.device:
            raise ValueError(f"{name} is on {x.device}, the plan on {self.device}")
        return x.contiguous()

    def _run(self, fname, x, out_tail, op, ws=None, extra=()):
        lead = x.shape[:-2]
        batch = int(math.prod(lead)) if lead else 1
        out = torch.empty(*lead, *out_tail, dtype=torch.float32, device=x.device)
        if batch == 0:
            return out
        need = self.workspace_bytes(batch, op)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=x.device)
        f = getattr(self._lib, fname)
        with torch.cuda.device(self.device):
            st = f(self._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch, *extra,
                   ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), _stream_ptr(self.device))
        _lib.check(fname, st)
        return out

    # ------------------------------------------------------------------ operators
    def forward(self, img, ws=None):
        """R f: [..., n, n] -> [..., n_theta, n_s]."""
        g = self.geom
        img = self._check_in(img, (g["n"], g["n"]), "img")
        return self._run("radon_fwd", img, (g["n_theta"], g["n_s"]), _lib.RL_OP_FWD, ws)

    def adjoint(self, sino, ws=None):
        """R# g (exact weighted transpose): [..., n_theta, n_s] -> [..., n, n]."""
        g = self.geom
        sino = self._check_in(sino, (g["n_theta"], g["n_s"]), "sino")
        return self._run("radon_adj", sino, (g["n"], g["n"]), _lib.RL_OP_ADJ, ws)

    def transpose(self, sino, ws=None):
        """R^T g = (w_X / w_S) R# g: [..., n_theta, n_s] -> [..., n, n]."""
        g = self.geom
        sino = self._check_in(sino, (g["n_theta"], g["n_s"]), "sino")
        return self._run("radon_transpose", sino, (g["n"], g["n"]), _lib.RL_OP_ADJ, ws)

    def adjoint_transpose(self, img, ws=None):
        """(R#)^T f = (w_S / w_X) R f: [..., n, n] -> [..., n_theta, n_s]."""
        g = self.geom
        img = self._check_in(img, (g["n"], g["n"]), "img")
        return self._run("radon_adj_transpose", img, (g["n_theta"], g["n_s"]), _lib.RL_OP_FWD, ws)

    def fbp(self, sino, ws=None, filter="ramlak"):
        """R# W g, W the "ramlak", "cosine" or "shepp-logan" filter: [..., n_theta, n_s] -> [..., n, n]."""
        if filter not in _lib.FILTERS:
            raise ValueError(f"unknown filter {filter!r}; one of {sorted(_lib.FILTERS)}")
        g = self.geom
        sino = self._check_in(sino, (g["n_theta"], g["n_s"]), "sino")
        return self._run("fbp", sino, (g["n"], g["n"]), _lib.RL_OP_FBP, ws, extra=(_lib.FILTERS[filter],))

    def bp_lp(self, sino, ws=None):
        """R# g by the paper's Algorithm 2 (radon_bp_lp): [..., n_theta, n_s] -> [..., n, n]."""
        g = self.geom
        sino = self._check_in(sino, (g["n_theta"], g["n_s"]), "sino")
        return self._run("radon_bp_lp", sino, (g["n"], g["n"]), _lib.RL_OP_BP_LP, ws)

    def fbp_lp(self, sino, ws=None, filter="ramlak"):
        """FBP through Algorithm 2 (fbp_lp): the filter of fbp, then bp_lp."""
        if filter not in _lib.FILTERS:
            raise ValueError(f"unknown filter {filter!r}; one of {sorted(_lib.FILTERS)}")
        g = self.geom
        sino = self._check_in(sino, (g["n_theta"], g["n_s"]), "sino")
        return self._run("fbp_lp", sino, (g["n"], g["n"]), _lib.RL_OP_FBP_LP, ws, extra=(_lib.FILTERS[filter],))

    def em_norm(self, ws=None):
        """R# chi_C, the normalisation of the EM step: [n, n] (rl_em_norm)."""
        g = self.geom
        out = torch.empty(g["n"], g["n"], dtype=torch.float32, device=self.device)
        need = self.workspace_bytes(1, _lib.RL_OP_EM)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            st = self._lib.rl_em_norm(self._ptr, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                      ctypes.c_size_t(ws.numel()), _stream_ptr(self.device))
        _lib.check("rl_em_norm", st)
        return out

    def em(self, sino, img, iters, norm=None, ws=None):
        """`iters` EM steps (rl_em) from the start image `img` for the data `sino`:
        [..., n_theta, n_s], [..., n, n] -> a new [..., n, n] tensor."""
        g = self.geom
        sino = self._check_in(sino, (g["n_theta"], g["n_s"]), "sino")
        f = self._check_in(img, (g["n"], g["n"]), "img").clone()
        if sino.shape[:-2] != f.shape[:-2]:
            raise ValueError("sino and img must have the same leading shape")
        if norm is None:
            norm = self.em_norm()
        norm = self._check_in(norm, (g["n"], g["n"]), "norm")
        lead = f.shape[:-2]
        batch = int(math.prod(lead)) if lead else 1
        if batch == 0 or iters == 0:
            return f
        need = self.workspace_bytes(batch, _lib.RL_OP_EM)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            st = self._lib.rl_em(self._ptr, ctypes.c_void_p(sino.data_ptr()), ctypes.c_void_p(norm.data_ptr()),
                                 ctypes.c_void_p(f.data_ptr()), batch, int(iters), ctypes.c_void_p(ws.data_ptr()),
                                 ctypes.c_size_t(ws.numel()), _stream_ptr(self.device))
        _lib.check("rl_em", st)
        return f

    def debug_stage(self, stage, img):
        """Intermediate of the forward chain for one slice (see rl_debug_stage)."""
        g = self.geom
        img = self._check_in(img, (g["n"], g["n"]), "img")
        n_own = None
        if stage == _lib.RL_STAGE_PREFILTER:
            shape = (g["n"], g["n"])
        elif stage == _lib.RL_STAGE_KERNEL:
            shape = (g["n_rho"] // 2 + 1, g["k_theta"] // 2 + 1, 2)
        else:
            n_own = self.n_own()
            rows = n_own + 4 if stage == _lib.RL_STAGE_LOGPOLAR else n_own
            shape = (g["m"], rows, g["n_rho"])
        out = torch.empty(*shape, dtype=torch.float32, device=img.device)
        need = self.workspace_bytes(1, _lib.RL_OP_FWD)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=img.device)
        with torch.cuda.device(self.device):
            st = self._lib.rl_debug_stage(self._ptr, stage, ctypes.c_void_p(img.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_size_t(out.numel() * 4),
                                          ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                          _stream_ptr(self.device))
        _lib.check("rl_debug_stage", st)
        return out

    @property
    def tuning(self):
        """The plan's execution-only launch parameters (rl_plan_get_tuning) as a dict."""
        t = _lib.RlTune()
        _lib.check("rl_plan_get_tuning", self._lib.rl_plan_get_tuning(self._ptr, ctypes.byref(t)))
        return t.as_dict()

    @tuning.setter
    def tuning(self, values):
        t = _lib.RlTune(**{**self.tuning, **values})
        _lib.check("rl_plan_set_tuning", self._lib.rl_plan_set_tuning(self._ptr, ctypes.byref(t)))

    def autotune(self, batch, cache=None):
        """Choose the launch parameters for `batch` slices by timing (rl_plan_autotune); `cache` is
        an optional JSON-lines file read first and appended to.  Returns the chosen parameters."""
        need = int(self._lib.rl_tune_workspace_bytes(self._ptr, batch))
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            st = self._lib.rl_plan_autotune(self._ptr, int(batch), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(need),
                                            _stream_ptr(self.device), None if cache is None else str(cache).encode())
        _lib.check("rl_plan_autotune", st)
        return self.tuning

    def n_own(self):
        """Largest number of sinogram rows one partition owns (rl_plan_rows)."""
        return self.rows_per_partition()[0]

    def rows_per_partition(self):
        """(n_own, [rows owned by each partition]) from the library (rl_plan_rows)."""
        n_own = ctypes.c_int32()
        rows = (ctypes.c_int32 * self.geom["m"])()
        _lib.check("rl_plan_rows", self._lib.rl_plan_rows(self._ptr, ctypes.byref(n_own), rows))
        return int(n_own.value), [int(x) for x in rows]


# ---------------------------------------------------------------------- functional API
def radon_fwd(plan: RadonPlan, img, ws=None):
    return plan.forward(img, ws)


def radon_adj(plan: RadonPlan, sino, ws=None):
    return plan.adjoint(sino, ws)


def radon_transpose(plan: RadonPlan, sino, ws=None):
    return plan.transpose(sino, ws)


def fbp(plan: RadonPlan, sino, ws=None, filter="ramlak"):
    return plan.fbp(sino, ws, filter=filter)


def radon_bp_lp(plan: RadonPlan, sino, ws=None):
    return plan.bp_lp(sino, ws)


def fbp_lp(plan: RadonPlan, sino, ws=None, filter="ramlak"):
    return plan.fbp_lp(sino, ws, filter=filter)


class RadonFn(torch.autograd.Function):
    """g = R f with the hand-written backward dL/df = R^T dL/dg (the radon_transpose kernels)."""

    @staticmethod
    def forward(ctx, img, plan):
        ctx.plan = plan
        return plan.forward(img)

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.transpose(grad.contiguous()), None


def radon(img, plan):
    """Differentiable R f."""
    return RadonFn.apply(img, plan)


class RadonAdjFn(torch.autograd.Function):
    """f = R# g with the hand-written backward dL/dg = (R#)^T dL/df = (w_S / w_X) R dL/df (the
    radon_adj_transpose kernels)."""

    @staticmethod
    def forward(ctx, sino, plan):
        ctx.plan = plan
        return plan.adjoint(sino)

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.adjoint_transpose(grad.contiguous()), None


def back_project(sino, plan):
    """Differentiable R# g."""
    return RadonAdjFn.apply(sino, plan)


class RaggedBatch:
    """A fixed set of slices of possibly different geometries, transformed together.

    items: list of (plan, image, sinogram) with image [n][n] and sinogram [n_theta][n_s]
    float32 CUDA tensors of that plan (contiguous).  forward() writes every sinogram from its
    image (R), adjoint() every image from its sinogram (R#), bp_lp() every image by Algorithm 2
    (plans with q_theta 1), each as one batched call per plan (the plans' calls concurrent),
    enqueued on the current stream; none allocates, so each can be captured in a CUDA (HIP)
    graph and replayed after the tensors' contents change.  The tensors must stay alive.
    tune_cache: optional autotuner cache file; each plan's launch parameters for its slice count
    come from it or are tuned and appended (rl_batch_create).
    """

    def __init__(self, items, tune_cache=None):
        lib = _lib.load()
        plans, index = [], {}
        plan_of, imgs, sinos = [], [], []
        for plan, img, sino in items:
            g = plan.geom
            plan._check_in(img, (g["n"], g["n"]), "image")
            plan._check_in(sino, (g["n_theta"], g["n_s"]), "sinogram")
            if img.dim() != 2 or sino.dim() != 2 or not img.is_contiguous() or not sino.is_contiguous():
                raise ValueError("ragged batch buffers must be contiguous 2-D tensors")
            if id(plan) not in index:
                index[id(plan)] = len(plans)
                plans.append(plan)
            plan_of.append(index[id(plan)])
            imgs.append(img)
            sinos.append(sino)
        n = len(imgs)
        self._keep = (plans, imgs, sinos)
        self.device = plans[0].device if plans else torch.device("cuda", torch.cuda.current_device())
        c_plans = (ctypes.c_void_p * max(1, len(plans)))(*[p._ptr.value for p in plans])
        c_of = (ctypes.c_int32 * max(1, n))(*plan_of)
        c_imgs = (ctypes.c_void_p * max(1, n))(*[t.data_ptr() for t in imgs])
        c_sinos = (ctypes.c_void_p * max(1, n))(*[t.data_ptr() for t in sinos])
        self._ptr = ctypes.c_void_p()
        self._lib = lib
        with torch.cuda.device(self.device):
            cache = None if tune_cache is None else str(tune_cache).encode()
            _lib.check("rl_batch_create", lib.rl_batch_create(c_plans, len(plans), c_of, c_imgs, c_sinos, n, cache,
                                                              ctypes.byref(self._ptr)))
            # R and R#, and Algorithm 2 if every plan allows it (q_theta 1)
            ops = [_lib.RL_OP_FWD, _lib.RL_OP_ADJ]
            if all(p.geom["q_theta"] == 1 for p in plans):
                ops.append(_lib.RL_OP_BP_LP)
            nbytes = max(int(lib.rl_batch_workspace_bytes(self._ptr, op)) for op in ops)
            self._ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)

    def __del__(self):
        ptr = getattr(self, "_ptr", None)
        if ptr is not None and ptr.value:
            self._lib.rl_batch_destroy(ptr)
            self._ptr = None

    def _run(self, fn, name):
        with torch.cuda.device(self.device):
            _lib.check(name, fn(self._ptr, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                _stream_ptr(self.device)))

    def forward(self):
        self._run(self._lib.rl_batch_fwd, "rl_batch_fwd")

    def adjoint(self):
        self._run(self._lib.rl_batch_adj, "rl_batch_adj")

    def bp_lp(self):
        """Every image from its sinogram by the paper's fast back-projection (Algorithm 2)."""
        self._run(self._lib.rl_batch_bp_lp, "rl_batch_bp_lp")

