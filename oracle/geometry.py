"""Discretisation geometry of the log-polar Radon transform (oracle, FP64).

Test infrastructure only (see the package docstring).

Paper passages followed
  * partition constants a_R, a_r: sec. 2, eq. (aconst)
  * partitions beta = pi/M, coordinate change T_m: sec. 2, eq. (Tdef),
    eq. (Radon_tm); ownership m = [theta/beta mod M]: eq. (Radon_all_pb)
  * disc D = T_m(unit disc): sec. 2, eq. (circle_D)
  * Cartesian grid X: sec. 3, eq. (Xgrid); polar grid Sigma: eq. (Polargrid)
  * rho sampling bound: sec. 3, eq. (vrho); fine angular step: the bound on
    Delta theta_lp just before eq. (Lopolargrid_f)
  * fine log-polar grid Omega_lp: eq. (Lopolargrid_f); coarse grid Omega_p:
    eq. (Lopolargrid_polar)

Readings taken where the text is silent or garbled (all mirrored, but not
shared, by the HIP path):
  * the object lives in the unit disc; Delta x = 2/N, Delta s = 2/N_s, nodes
    x = -1 + i*Delta x, s = -1 + k*Delta s, theta_j = j*pi/N_theta;
  * rho_q = (q - N_rho + 1) * Delta rho, q in [0, N_rho), so rho in (log a_r, 0];
  * ownership uses round-half-up, computed exactly in integers; the rows the
    rounding assigns to m = M belong to partition 0 with theta' = theta - pi and
    s -> -s (each line appears twice in the parametrisation);
  * each partition's coarse lattice has spacing Delta theta_c = Delta theta /
    q_theta (q_theta = 1: the sinogram's), the lattice rows of its owned rows
    plus HALO rows on each side (the reach of the decimation filter) form the
    support; the theta-FFT length is k_theta >= 2*q_theta*ceil(N_theta/M);
  * fine angular rows sit at Delta theta_c / r_dec, aligned with the coarse rows;
  * accuracy variants (Algorithm 1 step 4 leaves the theta low-pass open; the
    coarse grid Omega_p of eq. Lopolargrid_polar has the sinogram's spacing):
    q_theta = 2 puts the coarse lattice at Delta theta_c = Delta theta / 2 (every
    other lattice row lies on a sinogram row; the rows between are convolved
    like the others but never evaluated), and dec_filter selects the low-pass
    (kernel.decimation_taps).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

HALO = 2  # coarse rows on each side of the owned rows (decimation filter reach)


def rho_bound(n: int, m: int) -> int:
    """Smallest N_rho allowed by sec. 3 eq. (vrho): ceil(log a_r / log(1 - 2 a_R / N))."""
    a_R, a_r = partition_constants(m)
    return int(math.ceil(math.log(a_r) / math.log(1.0 - 2.0 * a_R / n)))


def r_bound(n: int, n_theta: int, m: int, q_theta: int = 1) -> int:
    """Smallest fine oversampling r with Delta theta_c / r <= 2 a_R / N (sec. 3, before
    eq. Lopolargrid_f), Delta theta_c = Delta theta / q_theta the coarse lattice spacing."""
    a_R, _ = partition_constants(m)
    return int(math.ceil((math.pi / (n_theta * q_theta)) / (2.0 * a_R / n) - 1e-12))


def partition_constants(m: int):
    """a_R and a_r of sec. 2 eq. (aconst) for beta = pi / M."""
    beta = math.pi / m
    sh = math.sin(beta / 2.0)
    ch = math.cos(beta / 2.0)
    return sh / (1.0 + sh), (ch - sh) / (1.0 + sh)


def _next_pow2(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


@dataclass(frozen=True)
class Geometry:
    """All parameters that fix the discrete operator."""

    n: int
    n_theta: int
    n_s: int
    m: int
    n_rho: int
    k_theta: int
    r_dec: int
    dec_filter: int = 0  # theta low-pass of step 4: 0 cubic B-spline, 1 box (kernel.decimation_taps)
    q_theta: int = 1     # coarse lattice spacing Delta theta / q_theta (1 or 2)

    # ---------------------------------------------------------------- constants
    @property
    def beta(self) -> float:
        return math.pi / self.m

    @property
    def a_R(self) -> float:
        return partition_constants(self.m)[0]

    @property
    def a_r(self) -> float:
        return partition_constants(self.m)[1]

    @property
    def L(self) -> float:
        """Period in rho: -log a_r."""
        return -math.log(self.a_r)

    @property
    def d_rho(self) -> float:
        return self.L / self.n_rho

    @property
    def dx(self) -> float:
        return 2.0 / self.n

    @property
    def ds(self) -> float:
        return 2.0 / self.n_s

    @property
    def dtheta(self) -> float:
        return math.pi / self.n_theta

    @property
    def dtheta_c(self) -> float:
        """Spacing of the coarse log-polar lattice Omega_p in theta'."""
        return self.dtheta / self.q_theta

    @property
    def w_X(self) -> float:
        """Quadrature weight of the image grid."""
        return self.dx * self.dx

    @property
    def w_S(self) -> float:
        """Quadrature weight of the sinogram grid."""
        return self.dtheta * self.ds

    # ------------------------------------------------------------------- grids
    def x_nodes(self) -> np.ndarray:
        return -1.0 + self.dx * np.arange(self.n)

    def s_nodes(self) -> np.ndarray:
        return -1.0 + self.ds * np.arange(self.n_s)

    def theta_nodes(self) -> np.ndarray:
        return self.dtheta * np.arange(self.n_theta)

    def rho_nodes(self) -> np.ndarray:
        return (np.arange(self.n_rho) - self.n_rho + 1) * self.d_rho

    # --------------------------------------------------------------- ownership
    def owner(self, j: int):
        """Partition of sinogram row j, the wrap flag, and the integer numerator
        nu with theta'_j = pi * nu / (N_theta * M)  (eq. Radon_all_pb, round half up)."""
        M, Nt = self.m, self.n_theta
        mm = (2 * j * M + Nt) // (2 * Nt)
        nu = j * M - mm * Nt
        if mm == M:
            return 0, True, nu
        return mm, False, nu

    def partition_rows(self, p: int):
        """Rows owned by partition p, sorted by theta': list of (j, wrap, nu)."""
        rows = []
        for j in range(self.n_theta):
            mm, wrap, nu = self.owner(j)
            if mm == p:
                rows.append((j, wrap, nu))
        rows.sort(key=lambda r: r[2])
        for a, b in zip(rows, rows[1:]):
            assert b[2] - a[2] == self.m, "owned rows must be contiguous in theta'"
        return rows

    @property
    def n_own(self) -> int:
        return max(len(self.partition_rows(p)) for p in range(self.m))

    def n_lat(self, n_rows: int) -> int:
        """Lattice rows spanned by n_rows consecutive owned sinogram rows."""
        return self.q_theta * (n_rows - 1) + 1 if n_rows > 0 else 0

    @property
    def n_sup(self) -> int:
        return self.n_lat(self.n_own) + 2 * HALO

    def n_sup_p(self, p: int) -> int:
        """Support rows of partition p: the lattice rows of its owned rows plus HALO on each side."""
        return self.n_lat(len(self.partition_rows(p))) + 2 * HALO

    def lattice_row(self, pos: int) -> int:
        """Lattice row of a partition's pos-th owned sinogram row."""
        return HALO + self.q_theta * pos

    def phi0(self, p: int) -> float:
        """Angle theta' of support row 0 of partition p (HALO lattice rows below the first owned row)."""
        rows = self.partition_rows(p)
        return math.pi * rows[0][2] / (self.n_theta * self.m) - HALO * self.dtheta_c

    def fine_rows(self, p: int) -> np.ndarray:
        """Fine row indices t (phi_t = phi0 + t*dtheta_c/r) that feed partition p's support rows."""
        r = self.r_dec
        return np.arange(-(2 * r - 1), r * (self.n_sup_p(p) - 1) + 2 * r)

    def fine_phi(self, p: int, t) -> np.ndarray:
        return self.phi0(p) + np.asarray(t, dtype=np.float64) * (self.dtheta_c / self.r_dec)

    def d_interval(self, phi):
        """Interval (e_lo, e_hi) of e^rho where the ray of angle phi meets D (eq. circle_D).

        Returns NaNs where the ray misses D (|phi| >= beta/2)."""
        a_R = self.a_R
        phi = np.asarray(phi, dtype=np.float64)
        disc = a_R * a_R - (1.0 - a_R) ** 2 * np.sin(phi) ** 2
        with np.errstate(invalid="ignore"):
            root = np.sqrt(disc)
        c = (1.0 - a_R) * np.cos(phi)
        lo = np.where(disc > 0, c - root, np.nan)
        hi = np.where(disc > 0, c + root, np.nan)
        return lo, hi

    def validate(self):
        if self.n < 8 or self.n % 2:
            raise ValueError("n must be even and >= 8")
        if self.m < 3:
            raise ValueError("m must be >= 3 (a_r = 0 at M = 2)")
        if self.n_theta < self.m or self.n_s < 2:
            raise ValueError("need n_theta >= m and n_s >= 2")
        if self.n_rho < rho_bound(self.n, self.m):
            raise ValueError("n_rho below the sampling bound of eq. (vrho)")
        if self.q_theta not in (1, 2):
            raise ValueError("q_theta must be 1 or 2")
        if self.dec_filter not in (0, 1):
            raise ValueError("dec_filter must be 0 (cubic B-spline) or 1 (box)")
        if (self.k_theta < 2 * self.q_theta * math.ceil(self.n_theta / self.m)
                or self.k_theta < self.n_sup):
            raise ValueError("k_theta must be >= 2*q_theta*ceil(n_theta/m) and hold the support rows")
        if self.r_dec < 1:
            raise ValueError("r_dec must be >= 1")
        return self


def make_geometry(n, n_theta, n_s, m=4, n_rho=None, k_theta=None, r_dec=None, dec_filter=0,
                  q_theta=1) -> Geometry:
    """Geometry with the default choices: power-of-two FFT lengths at or above the
    paper's bounds, K = 2*q_theta*ceil(N_theta/M) rounded up, r at the fine-angle bound."""
    if n_rho is None:
        n_rho = _next_pow2(rho_bound(n, m))
    if k_theta is None:
        k_theta = _next_pow2(2 * q_theta * int(math.ceil(n_theta / m)))
    if r_dec is None:
        r_dec = r_bound(n, n_theta, m, q_theta)
    g = Geometry(n, n_theta, n_s, m, n_rho, k_theta, r_dec, dec_filter, q_theta)
    if g.k_theta < g.n_sup:
        g = Geometry(n, n_theta, n_s, m, n_rho, _next_pow2(g.n_sup), r_dec, dec_filter, q_theta)
    return g.validate()
