"""Runs of the smooth 2D problems of Sec. 5.2 with a fixed streaming speed
and a whole number of steps reaching the end time (no shortened last step:
at omega = 2 the non-equilibrium part is not damped, and a step of another
speed spoils the second order)."""
import math

import numpy as np


def lam0(P):
    """max(|u|, |v|) + c over the initial state (Euler, 2D)."""
    r, mx, my, e = P.U0
    u, v = mx / r, my / r
    p = (P.gamma - 1.0) * (e - 0.5 * r * (u * u + v * v))
    c = np.sqrt(P.gamma * p / r)
    return float(max((np.abs(u) + c).max(), (np.abs(v) + c).max()))


def fixed_xi(P):
    """The problem with xi = (sqrt(5/2) for the centered set) max|lambda_0| / nu,
    raised so that T is reached in a whole number of steps; returns (P, t_end)."""
    f = math.sqrt(2.5) if getattr(P, "eq_set", "weighted") == "centered" else 1.0
    dx = (P.hi[0] - P.lo[0]) / P.n[0]
    xi = f * lam0(P) / P.nu
    steps = int(math.ceil(P.T * xi / dx))
    xi = steps * dx / P.T
    return P.with_(xi_mode="fixed", xi=xi, T=math.inf, max_steps=steps), steps * dx / xi
