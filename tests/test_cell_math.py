"""The per-cell arithmetic of the HIP path (paper_2608_04283_amd/csrc/vklb_cell.hpp),
compiled for the host, against the oracle on random states (no GPU).

The two sides reach the split by different routes: the oracle takes the
paper's route (Jacobian, null-space eigenvectors, P^-1 F, weights), the HIP
path uses closed forms per system. Agreement to rounding pins the closed forms.
"""
import ctypes
import math
import os

import numpy as np
import pytest

from paper_2608_04283_amd import inputs as I
from test_oracle_cell import rand_state, cfg, ch_for

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CC = os.path.join(ROOT, "paper_2608_04283_amd", "_cellcheck.so")
KIND = {"sw": 0, "euler": 1, "mhd": 2, "linear": 3}


@pytest.fixture(scope="module")
def cc():
    if not os.path.exists(CC):
        from paper_2608_04283_amd import build
        build.build_cellcheck()
    L = ctypes.CDLL(CC)
    dp = ctypes.POINTER(ctypes.c_double)
    L.vklb_cc_split.argtypes = [ctypes.c_int] * 4 + [dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
    L.vklb_cc_feq.argtypes = [ctypes.c_int] * 3 + [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    L.vklb_cc_speeds.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp, dp]
    L.vklb_cc_char.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def prm(g=9.81, gamma=1.4, k=2.0, c=0.05, local=False):
    kinf = 1.0 if math.isinf(k) else 0.0
    return np.array([g, gamma, 6.0, 0.7, -0.3, 1.0, c, 0.0 if kinf else k, kinf, 1.0 if local else 0.0])


def cc_split(cc, prec, system, dim, d, U, pr, Lam, ch):
    p = len(U)
    F, D = np.zeros(p), np.zeros(p)
    U = np.ascontiguousarray(U, dtype=np.float64)
    r = cc.vklb_cc_split(prec, KIND[system], dim, d, _p(U), _p(pr), Lam, ch, _p(F), _p(D))
    assert r == p
    return F, D


SYSTEMS = [("sw", 1), ("sw", 2), ("euler", 1), ("euler", 2), ("mhd", 1), ("mhd", 2)]


@pytest.mark.parametrize("system,dim", SYSTEMS)
@pytest.mark.parametrize("k", [2.0, 0.7, math.inf])
@pytest.mark.parametrize("norm", ["global", "local"])
def test_split_matches_oracle_fp64(oracle, cc, system, dim, k, norm):
    O = oracle
    rng = np.random.default_rng(21)
    gamma = 2.0 if system == "mhd" else 1.4
    cf = cfg(O, system, dim, k=k, alpha_norm=norm)
    pr = prm(gamma=gamma, k=k, local=(norm == "local"))
    for _ in range(25):
        U = rand_state(system, dim, rng)
        ch = ch_for(O, cf, U)
        Lam = 1.3 * max(np.max(np.abs(O.eigenvalues(cf, d, U, ch))) for d in range(dim))
        for d in range(dim):
            Fo = O.flux(cf, d, U, ch)
            Fpo, Fmo = O.split(cf, d, U, ch, lam=Lam)
            F, D = cc_split(cc, 8, system, dim, d, U, pr, Lam, ch)
            sc = np.max(np.abs(Fo)) + 1.0
            assert np.max(np.abs(F - Fo)) < 1e-14 * sc
            assert np.max(np.abs((0.5 * F + D) - Fpo)) < 2e-12 * sc
            assert np.max(np.abs((0.5 * F - D) - Fmo)) < 2e-12 * sc


@pytest.mark.parametrize("deg", ["bt0", "bt_small", "triple", "bx0"])
def test_mhd_split_degenerate_matches_oracle(oracle, cc, deg):
    O = oracle
    rng = np.random.default_rng(22)
    for dim in (1, 2):
        cf = cfg(O, "mhd", dim)
        pr = prm(gamma=2.0)
        for _ in range(10):
            U = rand_state("mhd", dim, rng, degenerate=deg)
            ch = ch_for(O, cf, U)
            Lam = max(np.max(np.abs(O.eigenvalues(cf, d, U, ch))) for d in range(dim))
            for d in range(dim):
                Fpo, _ = O.split(cf, d, U, ch, lam=Lam)
                F, D = cc_split(cc, 8, "mhd", dim, d, U, pr, Lam, ch)
                sc = np.max(np.abs(F)) + 1.0
                assert np.max(np.abs((0.5 * F + D) - Fpo)) < 1e-8 * sc


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_split_fp32_close_to_oracle(oracle, cc, system, dim):
    O = oracle
    rng = np.random.default_rng(23)
    gamma = 2.0 if system == "mhd" else 1.4
    cf = cfg(O, system, dim)
    pr = prm(gamma=gamma)
    for _ in range(25):
        U = rand_state(system, dim, rng)
        ch = ch_for(O, cf, U)
        Lam = max(np.max(np.abs(O.eigenvalues(cf, d, U, ch))) for d in range(dim))
        for d in range(dim):
            Fpo, _ = O.split(cf, d, U, ch, lam=Lam)
            F, D = cc_split(cc, 4, system, dim, d, U, pr, Lam, ch)
            sc = np.max(np.abs(F)) + 1.0
            assert np.max(np.abs((0.5 * F + D) - Fpo)) < 3e-5 * sc


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_feq_and_speeds_match_oracle(oracle, cc, system, dim):
    O = oracle
    rng = np.random.default_rng(24)
    gamma = 2.0 if system == "mhd" else 1.4
    cf = cfg(O, system, dim)
    pr = prm(gamma=gamma)
    Q = 3 if dim == 1 else 5
    for _ in range(10):
        U = np.ascontiguousarray(rand_state(system, dim, rng))
        ch = ch_for(O, cf, U)
        Lam = max(np.max(np.abs(O.eigenvalues(cf, d, U, ch))) for d in range(dim))
        xi = Lam / 0.9
        fo = O.feq(cf, U, xi, ch, lam=Lam)
        out = np.zeros(Q * len(U))
        cc.vklb_cc_feq(8, KIND[system], dim, _p(U), _p(pr), xi, Lam, ch, _p(out))
        assert np.allclose(out.reshape(Q, -1), fo, rtol=1e-12, atol=1e-12 * np.max(np.abs(U)))
        lam, cfm = np.zeros(1), np.zeros(1)
        cc.vklb_cc_speeds(8, KIND[system], dim, _p(U), _p(pr), _p(lam), _p(cfm))
        lam_o, _ = O.global_lambda(cf, U.reshape(-1, 1))
        if system == "mhd":
            cf_o = max(O.fast_speed(cf, d, U) for d in range(dim))
            assert abs(cfm[0] - cf_o) < 1e-13 * cf_o
            # the seven-wave max, without the cleaning pair
            seven = max(abs(U[1 + d] / U[0]) + O.fast_speed(cf, d, U) for d in range(dim))
            assert abs(lam[0] - seven) < 1e-13 * seven
        else:
            assert abs(lam[0] - lam_o) < 1e-13 * lam_o


@pytest.mark.parametrize("deg", [None, "bt0", "bt_small", "triple", "triple_near", "bx0"])
def test_mhd_split_fp32_at_degenerate_states(oracle, cc, deg):
    """The FP32 MHD split (FP64 eigenstructure only near the triple point,
    where the fast and slow speeds meet) stays within 1e-6 of the oracle at
    and near every degenerate state: transverse field zero or tiny (fast or
    slow = Alfven), the triple point, normal field zero."""
    O = oracle
    rng = np.random.default_rng(25)
    for dim in (1, 2):
        cf = cfg(O, "mhd", dim)
        pr = prm(gamma=2.0)
        for _ in range(25):
            U = rand_state("mhd", dim, rng, degenerate=deg)
            ch = ch_for(O, cf, U)
            Lam = max(np.max(np.abs(O.eigenvalues(cf, d, U, ch))) for d in range(dim))
            for d in range(dim):
                Fpo, _ = O.split(cf, d, U, ch, lam=Lam)
                F, D = cc_split(cc, 4, "mhd", dim, d, U, pr, Lam, ch)
                assert np.max(np.abs((0.5 * F + D) - Fpo)) < 1e-6 * (np.max(np.abs(F)) + 1.0)


@pytest.mark.parametrize("system", ["sw", "euler", "linear"])
@pytest.mark.parametrize("right", [True, False])
def test_characteristic_correction_matches_oracle(oracle, cc, system, right):
    """The closed-form characteristic boundary corrections (textbook left and
    right eigenvectors) equal the oracle's eigenvector route: FP64 to 1e-12,
    FP32 to 1e-6, relative to |A| |dU|."""
    O = oracle
    rng = np.random.default_rng(77)
    cf = cfg(O, system, 1) if system != "linear" else O.make_config(system="linear", dim=1, n=(8, 1), adv=(0.7, 0.0))
    pr = prm(gamma=1.4)
    if system == "linear":
        pr[3] = 0.7 if right else -0.7
        cf = O.make_config(system="linear", dim=1, n=(8, 1), adv=(pr[3], 0.0))
    for _ in range(20):
        U = rand_state(system, 1, rng) if system != "linear" else np.array([rng.uniform(0.5, 2.0)])
        # near-sonic states too: u close to +-c
        if system == "euler" and _ % 4 == 0:
            rho, p = U[0], 0.4 * (U[2] - 0.5 * U[1] ** 2 / U[0])
            c = math.sqrt(1.4 * p / rho)
            U = I.euler_state(np.array([rho]), c * (1 + 1e-3 * rng.normal()), p, 1.4)[:, 0]
        dU = rng.normal(size=U.shape) * 0.1
        ref = O.char_correction(cf, U, dU, 0.0, right=right)
        scale = np.max(np.abs(O.jacobian(cf, 0, U, 0.0))) * np.max(np.abs(dU)) + 1e-300
        for prec, tol in ((8, 1e-12), (4, 1e-6)):
            out = np.zeros(len(U))
            Uc = np.ascontiguousarray(U, dtype=np.float64)
            dc = np.ascontiguousarray(dU, dtype=np.float64)
            r = cc.vklb_cc_char(prec, KIND[system], _p(Uc), _p(dc), _p(pr), 0.0, 1 if right else 0, _p(out))
            assert r == len(U)
            assert np.max(np.abs(out - ref)) < tol * scale, (system, prec, out, ref)


@pytest.mark.parametrize("right", [True, False])
def test_mhd_characteristic_correction_matches_oracle(oracle, cc, right):
    """The MHD characteristic correction (primitive Roe-Balsara eigenvectors,
    the cleaning pair and their coupling by divided differences of g) equals
    the oracle's route (eigenvectors as null vectors of the Jacobian, LU) at
    random states, at states where speeds coincide exactly (transverse or
    normal field zero) and near the triple point; it is computed in FP64 in
    both precisions, so FP32 differs only by the rounding of its inputs."""
    O = oracle
    rng = np.random.default_rng(78)
    cf = cfg(O, "mhd", 1)
    pr = prm(gamma=2.0)
    for i in range(40):
        deg = (None, "bt0", "bx0", "triple_near", None)[i % 5]
        U = rand_state("mhd", 1, rng, degenerate=deg)
        ch = ch_for(O, cf, U)
        dU = rng.normal(size=U.shape) * 0.1
        ref = O.char_correction(cf, U, dU, ch, right=right)
        scale = np.max(np.abs(O.jacobian(cf, 0, U, ch))) * np.max(np.abs(dU))
        for prec, tol in ((8, 1e-10 if deg == "triple_near" else 1e-12), (4, 1e-6)):
            out = np.zeros(len(U))
            Uc = np.ascontiguousarray(U, dtype=np.float64)
            dc = np.ascontiguousarray(dU, dtype=np.float64)
            r = cc.vklb_cc_char(prec, KIND["mhd"], _p(Uc), _p(dc), _p(pr), ch, 1 if right else 0, _p(out))
            assert r == len(U)
            assert np.max(np.abs(out - ref)) < tol * scale, (deg, prec, np.max(np.abs(out - ref)) / scale)
