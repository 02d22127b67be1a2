"""Plain FP64 CPU oracle of the log-polar Radon transform and back-projection.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
constants with the HIP path: every quantity (geometry, B-spline weights, the
log-polar kernel table, masks, ownership) is recomputed here from the paper's
definitions, in FP64, with numpy.

Modules
  geometry  grids, partition constants, ownership, supports, masks
            (paper sec. 2 eq. aconst/Tdef/Radon_tm/Radon_all_pb; sec. 3 eq.
            Xgrid/Polargrid/vrho/Lopolargrid_f/Lopolargrid_polar)
  bspline   cubic B-spline, its Fourier series, periodic prefilter Q, 4-tap
            weights (sec. 4 eq. Bcoeff/Bhat/Bsplineinterp/Qfrecursive/wsumn)
  kernel    Fourier coefficients of the log-polar kernel zeta (sec. 3,
            eq. exprcoef1) by composite Gauss-Legendre quadrature, and the
            multiplier H = zeta_hat / (B_hat_rho * D_hat_theta)
  radon     Algorithm 1 (fast Radon transform) step by step, its exact
            weighted transpose (the back-projection), and FBP (eq. FBP, ramp)
  bp        Algorithm 2 (fast back-projection) step by step: sinogram spline
            coefficients, lattice samples, convolution with zeta# (eq.
            exprcoef2), bicubic gather to the image; FBP through it
  em        EM reconstruction step (sec. 7) on radon_fwd / radon_adj
  analytic  closed-form Radon transforms (disc, Gaussian, ellipse) used as pins
  brute     brute-force line integrals of the spline interpolant (pin)
  closed_form  the paper's closed form for P(mu, alpha, beta) (eq.
            P_closed_form, appendix) evaluated with mpmath (pin of the kernel)

Parity status of each function is stated in its module docstring.
"""

from .geometry import Geometry, make_geometry  # noqa: F401
from .radon import radon_fwd, radon_adj, fbp, ramp_filter  # noqa: F401
