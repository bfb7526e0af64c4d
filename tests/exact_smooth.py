"""Exact solutions of the smooth 2D Euler problems of Sec. 5.2 (test
reference only): the sinusoidal entropy wave and the isentropic vortex, both
translated by (u, v) = (1, 1) on their periodic domains."""
import numpy as np

from paper_2608_04283_amd import inputs as I


def entropy_wave_density(P, t):
    X, Y = I.grid2(P.n[0], P.n[1], P.lo, P.hi)
    return (1.0 + 0.1 * np.sin(2 * np.pi * (X + Y - 2.0 * t))).reshape(-1)


def vortex_state(P, t, eps=5.0):
    """Conserved state of the vortex at time t (centre at (t, t), wrapped)."""
    X, Y = I.grid2(P.n[0], P.n[1], P.lo, P.hi)
    L = P.hi[0] - P.lo[0]
    dx = (X - t - P.lo[0]) % L + P.lo[0]
    dy = (Y - t - P.lo[1]) % L + P.lo[1]
    g = P.gamma
    r2 = dx * dx + dy * dy
    Tt = 1.0 - (g - 1.0) * eps * eps / (8.0 * g * np.pi ** 2) * np.exp(1.0 - r2)
    rho = Tt ** (1.0 / (g - 1.0))
    e = eps / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    return I.euler_state(rho, 1.0 - e * dy, rho ** g, g, v=1.0 + e * dx)


def l2(a, b):
    return float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))
