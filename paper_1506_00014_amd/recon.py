"""Least-squares reconstruction by autograd on the library's R (sec. 7 of the paper reconstructs
iteratively from R and R#; here the iteration is gradient descent on ||R f - g||^2).

The gradient is what torch's autograd returns through RadonFn, whose backward is the library's
R^T (radon_transpose); the transforms run in the HIP kernels, the update f <- f - grad / lam is
an elementwise torch operation on the batch.  The step 1 / lam uses lam = 2 ||R^T R||, the
Lipschitz constant of the gradient, with ||R^T R|| estimated by power iteration.
"""

from __future__ import annotations

import torch

from .api import RadonFn, RadonPlan


def power_iteration(plan: RadonPlan, iters: int = 20, seed: int = 502, v0: torch.Tensor | None = None,
                    ws=None) -> float:
    """Largest eigenvalue of R^T R (= ||R||_2^2) by `iters` power steps from v0 (default a
    seeded N(0, 1) image); returns the Rayleigh quotient ||R v||^2 / ||v||^2 of the last iterate."""
    n = plan.geom["n"]
    if v0 is None:
        gen = torch.Generator(device=plan.device)
        gen.manual_seed(seed)
        v = torch.randn(n, n, generator=gen, device=plan.device, dtype=torch.float32)
    else:
        v = v0.to(device=plan.device, dtype=torch.float32).clone()
    v /= v.norm()
    est = 0.0
    for _ in range(iters):
        rv = plan.forward(v, ws)
        est = float(rv.double().pow(2).sum().item() / v.double().pow(2).sum().item())
        w = plan.transpose(rv, ws)
        v = w / w.norm()
    return est


def least_squares_gd(plan: RadonPlan, g: torch.Tensor, steps: int, lam: float, f0: torch.Tensor | None = None,
                     callback=None) -> torch.Tensor:
    """`steps` steps of f <- f - grad L(f) / lam, L(f) = ||R f - g||^2 summed over the batch, the
    gradient by autograd through RadonFn.  g: [..., n_theta, n_s]; returns f: [..., n, n]
    (f0, default zeros).  callback(k, loss) is called with the loss before step k if given."""
    n = plan.geom["n"]
    f = torch.zeros(*g.shape[:-2], n, n, device=g.device, dtype=torch.float32) if f0 is None else f0.clone()
    for k in range(steps):
        f.requires_grad_(True)
        loss = (RadonFn.apply(f, plan) - g).pow(2).sum()
        loss.backward()
        if callback is not None:
            callback(k, loss.detach())
        with torch.no_grad():
            f = f - f.grad / lam
    return f.detach()
