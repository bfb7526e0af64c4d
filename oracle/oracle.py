"""ctypes wrapper of the plain FP64 CPU oracle (oracle/vklb_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg. The product package never imports it, and it
imports nothing from the product package.

Every function here marshals arguments; all arithmetic happens in the C++
oracle, which follows the paper step by step (see the header of
vklb_oracle.cpp for the section each part follows).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vklb_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle_vklb.so")

SW, EULER, MHD, LINEAR = 0, 1, 2, 3
PERIODIC, ZERO_GRADIENT, CHARACTERISTIC = 0, 1, 2
XI_CFL, XI_FIXED = 0, 1

_SYS = {"sw": SW, "shallow_water": SW, "euler": EULER, "mhd": MHD, "linear": LINEAR}
_BC = {"periodic": PERIODIC, "zero_gradient": ZERO_GRADIENT, "outflow": ZERO_GRADIENT, "characteristic": CHARACTERISTIC}


class OrConfig(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int64 * 2),
        ("lo", ctypes.c_double * 2),
        ("hi", ctypes.c_double * 2),
        ("g", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("ch_factor", ctypes.c_double),
        ("adv", ctypes.c_double * 2),
        ("xi_mode", ctypes.c_int),
        ("nu", ctypes.c_double),
        ("xi_fixed", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("c", ctypes.c_double),
        ("k", ctypes.c_double),
        ("alpha_norm", ctypes.c_int),
        ("bc", ctypes.c_int * 2),
        ("T", ctypes.c_double),
        ("max_steps", ctypes.c_int64),
        ("cluster_tol", ctypes.c_double),
        ("threads", ctypes.c_int),
    ]


class OrResult(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("steps", ctypes.c_int64),
        ("xi", ctypes.c_double),
        ("ch", ctypes.c_double),
        ("status", ctypes.c_int),
        ("fail_step", ctypes.c_int64),
        ("fail_cell", ctypes.c_int64),
        ("totals", ctypes.c_double * 9),
        ("threads_used", ctypes.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (IEEE semantics: no fast-math, no -march)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(OrConfig)
        L.or_nvars.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_nvars.restype = ctypes.c_int
        for name in ("or_flux", "or_eigenvalues", "or_jacobian"):
            fn = getattr(L, name)
            fn.argtypes = [cp, ctypes.c_int, dp, ctypes.c_double, dp]
            fn.restype = None
        L.or_split.argtypes = [cp, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_split.restype = ctypes.c_int
        L.or_feq.argtypes = [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.or_feq.restype = ctypes.c_int
        L.or_global_lambda.argtypes = [cp, dp, ctypes.c_int64, dp]
        L.or_global_lambda.restype = ctypes.c_double
        L.or_fast_speed.argtypes = [cp, ctypes.c_int, dp]
        L.or_fast_speed.restype = ctypes.c_double
        L.or_char.argtypes = [cp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        L.or_char.restype = ctypes.c_int
        L.or_run.argtypes = [cp, dp, dp, dp, dp, ctypes.c_int64, ctypes.POINTER(OrResult)]
        L.or_run.restype = ctypes.c_int
        _lib = L
    return _lib


def nvars(system: str, dim: int) -> int:
    return lib().or_nvars(_SYS[system], dim)


def nvel(dim: int) -> int:
    return 3 if dim == 1 else 5


def make_config(system="euler", dim=1, n=(64, 1), lo=(0.0, 0.0), hi=(1.0, 1.0), g=9.81, gamma=1.4,
                ch_factor=6.0, adv=(1.0, 0.0), xi_mode="cfl", nu=0.9, xi=0.0, omega=1.0, c=0.05,
                k=2.0, alpha_norm="global", bc=("zero_gradient", "zero_gradient"), T=math.inf, max_steps=2**62,
                cluster_tol=1e-9, threads=0) -> OrConfig:
    cf = OrConfig()
    cf.kind = _SYS[system]
    cf.dim = dim
    n = tuple(n) if not isinstance(n, int) else (n, 1)
    cf.n[0] = int(n[0])
    cf.n[1] = int(n[1]) if dim == 2 else 1
    cf.lo[0], cf.lo[1] = lo
    cf.hi[0], cf.hi[1] = hi
    if dim == 2:
        dx = (hi[0] - lo[0]) / n[0]
        dy = (hi[1] - lo[1]) / n[1]
        if abs(dx - dy) > 1e-12 * dx:
            raise ValueError("the D2Q5 lattice needs dx == dy")
    cf.g, cf.gamma, cf.ch_factor = g, gamma, ch_factor
    cf.adv[0], cf.adv[1] = adv
    cf.xi_mode = XI_CFL if xi_mode == "cfl" else XI_FIXED
    cf.nu, cf.xi_fixed = nu, xi
    cf.omega, cf.c, cf.k = omega, c, k
    cf.alpha_norm = {"global": 0, "local": 1}[alpha_norm]
    if isinstance(bc, str):
        bc = (bc, bc)
    cf.bc[0], cf.bc[1] = _BC[bc[0]], _BC[bc[1]]
    cf.T = T
    cf.max_steps = int(max_steps)
    cf.cluster_tol = cluster_tol
    cf.threads = threads
    return cf


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x, p):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(p))
    return a


def flux(cf: OrConfig, d: int, U, ch: float = 0.0):
    p = lib().or_nvars(cf.kind, cf.dim)
    U = _vec(U, p)
    F = np.zeros(p)
    lib().or_flux(ctypes.byref(cf), d, _dp(U), ch, _dp(F))
    return F


def eigenvalues(cf: OrConfig, d: int, U, ch: float = 0.0):
    p = lib().or_nvars(cf.kind, cf.dim)
    U = _vec(U, p)
    lam = np.zeros(p)
    lib().or_eigenvalues(ctypes.byref(cf), d, _dp(U), ch, _dp(lam))
    return lam


def jacobian(cf: OrConfig, d: int, U, ch: float = 0.0):
    p = lib().or_nvars(cf.kind, cf.dim)
    U = _vec(U, p)
    A = np.zeros(p * p)
    lib().or_jacobian(ctypes.byref(cf), d, _dp(U), ch, _dp(A))
    return A.reshape(p, p)


def _local_lam(cf, U, ch):
    return max(float(np.max(np.abs(eigenvalues(cf, d, U, ch)))) for d in range(cf.dim))


def split(cf: OrConfig, d: int, U, ch: float = 0.0, lam: float = None):
    """Weighted partial fluxes (F+, F-) of F^(d)(U); lam normalizes the sigmoid
    (default: the state's own max |lambda| over directions)."""
    p = lib().or_nvars(cf.kind, cf.dim)
    U = _vec(U, p)
    if lam is None:
        lam = _local_lam(cf, U, ch)
    Fp, Fm = np.zeros(p), np.zeros(p)
    st = lib().or_split(ctypes.byref(cf), d, _dp(U), ch, lam, _dp(Fp), _dp(Fm))
    if st != 0:
        raise RuntimeError("oracle split failed")
    return Fp, Fm


def feq(cf: OrConfig, U, xi: float, ch: float = 0.0, lam: float = None):
    """Equilibrium populations, shape (Q, p)."""
    p = lib().or_nvars(cf.kind, cf.dim)
    Q = nvel(cf.dim)
    U = _vec(U, p)
    if lam is None:
        lam = _local_lam(cf, U, ch)
    out = np.zeros(Q * p)
    st = lib().or_feq(ctypes.byref(cf), _dp(U), xi, ch, lam, _dp(out))
    if st != 0:
        raise RuntimeError("oracle feq failed")
    return out.reshape(Q, p)


def global_lambda(cf: OrConfig, U):
    """(Lambda, c_h) of a state array U (SoA [var][cell])."""
    p = lib().or_nvars(cf.kind, cf.dim)
    U = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(p, -1))
    ch = ctypes.c_double(0.0)
    lam = lib().or_global_lambda(ctypes.byref(cf), _dp(U), U.shape[1], ctypes.byref(ch))
    return lam, ch.value


def fast_speed(cf: OrConfig, d: int, U):
    p = lib().or_nvars(cf.kind, cf.dim)
    U = _vec(U, p)
    return lib().or_fast_speed(ctypes.byref(cf), d, _dp(U))


def char_correction(cf: OrConfig, Ub, dU, ch: float = 0.0, right: bool = True):
    """P (Lambda dW)' of the characteristic boundary (Sec. 3.3) at a node with
    state Ub for the one-sided increment dU: U_b^{n+1} = U_b - out / xi."""
    p = lib().or_nvars(cf.kind, cf.dim)
    Ub, dU = _vec(Ub, p), _vec(dU, p)
    out = np.zeros(p)
    if lib().or_char(ctypes.byref(cf), _dp(Ub), _dp(dU), ch, 1 if right else 0, _dp(out)) != 0:
        raise RuntimeError("oracle char_correction failed")
    return out


def run(cf: OrConfig, U0, want_f: bool = False, want_xi: bool = False) -> dict:
    """Run the full method from U0 (SoA [var][cell]); returns U, t, steps, ..."""
    p = lib().or_nvars(cf.kind, cf.dim)
    Q = nvel(cf.dim)
    ncell = int(cf.n[0]) * (int(cf.n[1]) if cf.dim == 2 else 1)
    U0 = np.ascontiguousarray(np.asarray(U0, dtype=np.float64).reshape(p, ncell))
    Uout = np.zeros((p, ncell))
    fout = np.zeros((Q, p, ncell)) if want_f else None
    cap = min(int(cf.max_steps), 10_000_000)
    xih = np.zeros(cap) if want_xi else None
    res = OrResult()
    lib().or_run(ctypes.byref(cf), _dp(U0), _dp(Uout), _dp(fout) if want_f else None,
                 _dp(xih) if want_xi else None, cap, ctypes.byref(res))
    out = {
        "U": Uout,
        "t": res.t,
        "steps": int(res.steps),
        "xi": res.xi,
        "ch": res.ch,
        "status": int(res.status),
        "fail_step": int(res.fail_step),
        "fail_cell": int(res.fail_cell),
        "totals": np.array(res.totals[:p]),
        "threads": int(res.threads_used),
    }
    if want_f:
        out["f"] = fout
    if want_xi:
        out["xi_hist"] = xih[: min(out["steps"], cap)]
    return out
