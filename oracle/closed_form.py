"""The paper's closed form of P(mu, alpha, beta) = int_{-beta}^{beta} e^{i mu t} cos(t)^alpha dt
(sec. 3 eq. P_closed_form, derived in the appendix), evaluated with mpmath.

Test infrastructure only (see the package docstring).  Used solely as a pin of
the quadrature in kernel.py: zeta_hat(k_theta, k_rho) = P(mu, alpha, beta) with
mu = -2 pi k_theta / P_theta and alpha = -2 pi i k_rho / L - 1 (sec. 3, the text
after eq. Pfor).  The form has a pole at alpha = -1 (k_rho = 0) and loses digits
to cancellation in double precision, so it is evaluated at 30+ digits and never
at k_rho = 0.
"""

from __future__ import annotations

import mpmath as mp


def P_closed(mu, alpha, beta, dps=30):
    with mp.workdps(dps):
        mu = mp.mpf(mu)
        al = mp.mpc(alpha)
        be = mp.mpf(beta)
        cb = mp.cos(be)
        half = mp.mpf(1) / 2
        t0 = (mp.gamma((al + 1) / 2) * mp.gamma(half) * mp.gamma((al + 2) / 2)
              / (mp.gamma((al + mu) / 2 + 1) * mp.gamma((al - mu) / 2 + 1)))
        a1, a2 = al / 2 + mu / 2 + 1, al / 2 - mu / 2 + 1
        t1 = (2 * mu * cb ** (al + 2) * mp.sin(mu * be) / ((al + 1) * (al + 2))
              * mp.hyp3f2(1, a1, a2, (al + 3) / 2, al / 2 + 2, cb ** 2))
        t2 = (2 * cb ** (al + 1) * mp.cos(be * mu) * mp.sin(be) / (al + 1)
              * mp.hyp3f2(1, a1, a2, (al + 3) / 2, al / 2 + 1, cb ** 2))
        return complex(t0 + t1 - t2)


def h_term(mu, alpha, beta, dps=30):
    """h(mu, alpha, beta) of the appendix recursion (eq. hdefin)."""
    with mp.workdps(dps):
        mu, al, be = mp.mpf(mu), mp.mpc(alpha), mp.mpf(beta)
        cb = mp.cos(be)
        return complex(2 / (al * (al - 1)) * (mu * cb ** al * mp.sin(mu * be)
                                              - al * cb ** (al - 1) * mp.cos(mu * be) * mp.sin(be)))


def P_quad(mu, alpha, beta, dps=30):
    """Direct mpmath quadrature of the defining integral (eq. Pfor)."""
    with mp.workdps(dps):
        f = lambda t: mp.exp(1j * mp.mpf(mu) * t) * mp.cos(t) ** mp.mpc(alpha)
        return complex(mp.quad(f, [-mp.mpf(beta), 0, mp.mpf(beta)]))
