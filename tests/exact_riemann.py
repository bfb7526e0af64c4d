"""Exact Riemann solutions used to pin the oracle (test helper, written from
the textbook theory of the shallow water and Euler Riemann problems; it shares
nothing with the oracle or the HIP path).

* Shallow water: star depth from f_L(h) + f_R(h) + u_R - u_L = 0 with the
  rarefaction branch 2(sqrt(g h) - sqrt(g h_K)) and the shock branch
  (h - h_K) sqrt(g (h + h_K) / (2 h h_K)).
* Euler: star pressure from Toro's pressure function (shock branch
  (p - p_K) sqrt(A_K / (p + B_K)), rarefaction branch
  2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1)), then sampling.
"""
from __future__ import annotations

import numpy as np


def _newton(fun, dfun, x0, lo=1e-14, tol=1e-15, maxit=200):
    x = x0
    for _ in range(maxit):
        fx = fun(x)
        x_new = max(lo, x - fx / dfun(x))
        if abs(x_new - x) <= tol * max(1.0, abs(x)):
            return x_new
        x = x_new
    return x


class ShallowWaterRiemann:
    def __init__(self, hL, uL, hR, uR, g=9.81):
        self.hL, self.uL, self.hR, self.uR, self.g = hL, uL, hR, uR, g
        g = self.g

        def fK(h, hK):
            if h <= hK:
                return 2.0 * (np.sqrt(g * h) - np.sqrt(g * hK))
            return (h - hK) * np.sqrt(0.5 * g * (h + hK) / (h * hK))

        def dfK(h, hK):
            if h <= hK:
                return np.sqrt(g / h)
            s = np.sqrt(0.5 * g * (h + hK) / (h * hK))
            return s - (h - hK) * g * hK / (4.0 * h * h * hK * s)

        fun = lambda h: fK(h, hL) + fK(h, hR) + uR - uL
        dfun = lambda h: dfK(h, hL) + dfK(h, hR)
        self.hs = _newton(fun, dfun, 0.5 * (hL + hR))
        self.us = 0.5 * (uL + uR) + 0.5 * (fK(self.hs, hR) - fK(self.hs, hL))
        cL, cR, cs = np.sqrt(g * hL), np.sqrt(g * hR), np.sqrt(g * self.hs)
        self.cL, self.cR, self.cs = cL, cR, cs
        # left wave
        if self.hs > hL:
            self.SL = uL - cL * np.sqrt(0.5 * self.hs * (self.hs + hL)) / hL
            self.left_shock = True
        else:
            self.left_shock = False
            self.headL, self.tailL = uL - cL, self.us - cs
        if self.hs > hR:
            self.SR = uR + cR * np.sqrt(0.5 * self.hs * (self.hs + hR)) / hR
            self.right_shock = True
        else:
            self.right_shock = False
            self.headR, self.tailR = uR + cR, self.us + cs

    def sample(self, s):
        """(h, u) at similarity coordinate s = (x - x0)/t."""
        s = np.asarray(s, dtype=np.float64)
        h = np.empty_like(s)
        u = np.empty_like(s)
        g = self.g
        for i, si in np.ndenumerate(s):
            if si <= self.us:
                if self.left_shock:
                    hv, uv = (self.hL, self.uL) if si < self.SL else (self.hs, self.us)
                else:
                    if si <= self.headL:
                        hv, uv = self.hL, self.uL
                    elif si >= self.tailL:
                        hv, uv = self.hs, self.us
                    else:
                        uv = (self.uL + 2.0 * self.cL + 2.0 * si) / 3.0
                        cv = (self.uL + 2.0 * self.cL - si) / 3.0
                        hv = cv * cv / g
            else:
                if self.right_shock:
                    hv, uv = (self.hR, self.uR) if si > self.SR else (self.hs, self.us)
                else:
                    if si >= self.headR:
                        hv, uv = self.hR, self.uR
                    elif si <= self.tailR:
                        hv, uv = self.hs, self.us
                    else:
                        uv = (self.uR - 2.0 * self.cR + 2.0 * si) / 3.0
                        cv = (-self.uR + 2.0 * self.cR + si) / 3.0
                        hv = cv * cv / g
            h[i], u[i] = hv, uv
        return h, u


class EulerRiemann:
    def __init__(self, rL, uL, pL, rR, uR, pR, gamma=1.4):
        self.WL = (rL, uL, pL)
        self.WR = (rR, uR, pR)
        self.g = gamma
        g = gamma
        cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
        self.cL, self.cR = cL, cR

        def fK(p, rK, pK, cK):
            if p > pK:
                A, B = 2.0 / ((g + 1.0) * rK), (g - 1.0) / (g + 1.0) * pK
                return (p - pK) * np.sqrt(A / (p + B))
            return 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)

        def dfK(p, rK, pK, cK):
            if p > pK:
                A, B = 2.0 / ((g + 1.0) * rK), (g - 1.0) / (g + 1.0) * pK
                return np.sqrt(A / (B + p)) * (1.0 - (p - pK) / (2.0 * (B + p)))
            return (p / pK) ** (-(g + 1.0) / (2.0 * g)) / (rK * cK)

        fun = lambda p: fK(p, rL, pL, cL) + fK(p, rR, pR, cR) + uR - uL
        dfun = lambda p: dfK(p, rL, pL, cL) + dfK(p, rR, pR, cR)
        self.ps = _newton(fun, dfun, 0.5 * (pL + pR))
        self.us = 0.5 * (uL + uR) + 0.5 * (fK(self.ps, rR, pR, cR) - fK(self.ps, rL, pL, cL))
        ps = self.ps
        gm = (g - 1.0) / (g + 1.0)
        if ps > pL:
            self.rsL = rL * (ps / pL + gm) / (gm * ps / pL + 1.0)
        else:
            self.rsL = rL * (ps / pL) ** (1.0 / g)
        if ps > pR:
            self.rsR = rR * (ps / pR + gm) / (gm * ps / pR + 1.0)
        else:
            self.rsR = rR * (ps / pR) ** (1.0 / g)

    def shock_speed_right(self):
        rR, uR, pR = self.WR
        g = self.g
        return uR + self.cR * np.sqrt((g + 1.0) / (2.0 * g) * self.ps / pR + (g - 1.0) / (2.0 * g))

    def sample(self, s):
        """(rho, u, p) at s = (x - x0)/t."""
        s = np.asarray(s, dtype=np.float64)
        g = self.g
        rL, uL, pL = self.WL
        rR, uR, pR = self.WR
        cL, cR, ps, us = self.cL, self.cR, self.ps, self.us
        out = np.empty((3,) + s.shape)
        for i, si in np.ndenumerate(s):
            if si <= us:
                if ps > pL:
                    SL = uL - cL * np.sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g))
                    W = (rL, uL, pL) if si < SL else (self.rsL, us, ps)
                else:
                    csL = cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
                    if si <= uL - cL:
                        W = (rL, uL, pL)
                    elif si >= us - csL:
                        W = (self.rsL, us, ps)
                    else:
                        fac = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cL) * (uL - si)
                        W = (rL * fac ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * uL + si),
                             pL * fac ** (2.0 * g / (g - 1.0)))
            else:
                if ps > pR:
                    SR = self.shock_speed_right()
                    W = (rR, uR, pR) if si > SR else (self.rsR, us, ps)
                else:
                    csR = cR * (ps / pR) ** ((g - 1.0) / (2.0 * g))
                    if si >= uR + cR:
                        W = (rR, uR, pR)
                    elif si <= us + csR:
                        W = (self.rsR, us, ps)
                    else:
                        fac = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cR) * (uR - si)
                        W = (rR * fac ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * uR + si),
                             pR * fac ** (2.0 * g / (g - 1.0)))
            out[(slice(None),) + i] = W
        return out

    def conserved(self, s):
        r, u, p = self.sample(s)
        return np.stack([r, r * u, p / (self.g - 1.0) + 0.5 * r * u * u])


def cell_average_exact(sampler, x_edges, t, x0, sub=16):
    """Cell averages of an exact solution by midpoint sub-sampling of each cell."""
    nx = len(x_edges) - 1
    fr = (np.arange(sub) + 0.5) / sub
    xs = x_edges[:-1, None] + (x_edges[1:] - x_edges[:-1])[:, None] * fr[None, :]
    vals = sampler((xs - x0) / t)
    return vals.reshape(vals.shape[0], nx, sub).mean(axis=-1)
