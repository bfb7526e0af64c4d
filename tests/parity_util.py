"""Shared test helpers: run a Problem on the oracle or on the HIP path and
compare per field."""
import math

import numpy as np


def oracle_config(O, P, **kw):
    d = dict(system=P.system, dim=P.dim, n=P.n if P.dim == 2 else (P.n[0], 1), lo=P.lo, hi=P.hi, g=P.g,
             gamma=P.gamma, ch_factor=P.ch_factor, adv=P.adv, xi_mode=P.xi_mode, nu=P.nu, xi=P.xi,
             omega=P.omega, c=P.c, k=P.k, bc=P.bc, T=P.T, max_steps=P.max_steps,
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
