"""Shared test helpers: run a Problem on the oracle or on the HIP path and
compare per field."""
import math

import numpy as np


def eq_params(P):
    """(c, k, nu) the oracle runs for a problem's equilibrium set: the
    centered set of Sec. 2.2 is c = 1/3 (1D) or 1/5 (2D) with k = 0 and its
    streaming speed xi = sqrt(3/2 | 5/2) max|lambda| / eta (Sec. 2.3), i.e. the
    CFL rule with nu = eta / sqrt(3/2 | 5/2); the discontinuous set is c = 0
    with step weights (k = inf)."""
    s = getattr(P, "eq_set", "weighted")
    if s == "centered":
        return (1.0 / 3.0 if P.dim == 1 else 0.2), 0.0, P.nu / math.sqrt(1.5 if P.dim == 1 else 2.5)
    if s == "discontinuous":
        return 0.0, math.inf, P.nu
    return P.c, P.k, P.nu


def oracle_config(O, P, **kw):
    c, k, nu = eq_params(P)
    d = dict(system=P.system, dim=P.dim, n=P.n if P.dim == 2 else (P.n[0], 1), lo=P.lo, hi=P.hi, g=P.g,
             gamma=P.gamma, ch_factor=P.ch_factor, adv=P.adv, xi_mode=P.xi_mode, nu=nu, xi=P.xi,
             omega=P.omega, c=c, k=k, bc=P.bc, T=P.T, max_steps=P.max_steps,
             alpha_norm=getattr(P, "alpha_norm", "global"))
    d.update(kw)
    return O.make_config(**d)


def run_oracle(O, P, **kw):
    return O.run(oracle_config(O, P, **kw), P.U0)


def rel_l1(a, b, small=1e-3):
    """Per-field sum|a-b| / sum|b|. Fields whose L1 norm in b is below `small`
    times the largest field's (identically zero, like w and B_z, or zero up to
    rounding in exact arithmetic, like the cleaning potential psi here) are
    measured against the largest field's L1 norm instead."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.abs(a - b).sum(axis=1)
    den = np.abs(b).sum(axis=1)
    big = den.max()
    den = np.where(den <= small * big, big, den)
    return num / den


def steps_bound(P):
    if P.max_steps < 2**62:
        return int(P.max_steps)
    return 10_000_000
