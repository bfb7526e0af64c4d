"""Pins of the oracle's per-cell arithmetic against facts the paper and the
mathematics fix (no GPU). Each test names the passage it checks.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from paper_2608_04283_amd import inputs as I

SYSTEMS = [("sw", 1), ("sw", 2), ("euler", 1), ("euler", 2), ("mhd", 1), ("mhd", 2)]


def rand_state(system, dim, rng, degenerate=None):
    """A random admissible conserved state (float64 vector)."""
    if system == "sw":
        h = rng.uniform(0.3, 2.0)
        u, v = rng.uniform(-1, 1, 2)
        return I.sw_state(np.array([h]), u, None if dim == 1 else v)[:, 0]
    if system == "euler":
        rho, p = rng.uniform(0.2, 2.0), rng.uniform(0.1, 2.0)
        u, v = rng.uniform(-1, 1, 2)
        return I.euler_state(np.array([rho]), u, p, 1.4, v=None if dim == 1 else v)[:, 0]
    rho, p = rng.uniform(0.3, 2.0), rng.uniform(0.1, 2.0)
    u, v, w = rng.uniform(-1, 1, 3)
    B = rng.uniform(-1.2, 1.2, 3)
    if degenerate == "bt0":          # transverse field -> 0 (Alfven/slow or Alfven/fast coincide)
        B[1:] = 0.0
    elif degenerate == "bt_small":
        B[1:] *= 1e-7
    elif degenerate == "triple":     # b_t = 0 and a^2 = b_x^2: three speeds coincide
        B[1:] = 0.0
        B[0] = math.sqrt(2.0 * p)    # gamma = 2 -> a^2 = 2p/rho = Bx^2/rho
    elif degenerate == "triple_near":  # near the triple point, inside the FP32 path's FP64 band
        B[1:] *= 3e-4
        B[0] = math.sqrt(2.0 * p) * (1.0 + 3e-4)
    elif degenerate == "bx0":        # normal field -> 0: five eigenvalues equal u
        B[0] = 0.0
    psi = rng.uniform(-0.1, 0.1)
    return I.mhd_state(np.array([rho]), u, v, w, p, B[0], B[1], B[2], 2.0, psi=psi)[:, 0]


def cfg(O, system, dim, **kw):
    gamma = 2.0 if system == "mhd" else 1.4
    n = (8,) if dim == 1 else (8, 8)
    return O.make_config(system=system, dim=dim, n=n, gamma=gamma, **kw)


def ch_for(O, cf, U):
    """A cleaning speed of the size the method uses: 6 x the largest fast speed."""
    if cf.kind != O.MHD:
        return 0.0
    return 6.0 * max(O.fast_speed(cf, d, U) for d in range(cf.dim))


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_eigenvalues_match_jacobian_spectrum(oracle, system, dim):
    """Sec. 2.2 / 5.1-5.3: the closed-form characteristic speeds are the
    spectrum of the flux Jacobian. The Jacobian is differentiated from the
    oracle's flux, so a dropped or mistyped flux term moves the spectrum."""
    O = oracle
    rng = np.random.default_rng(1)
    cf = cfg(O, system, dim)
    for _ in range(20):
        U = rand_state(system, dim, rng)
        ch = ch_for(O, cf, U)
        for d in range(dim):
            A = O.jacobian(cf, d, U, ch)
            ev = np.sort(np.linalg.eigvals(A).real)
            lam = np.sort(O.eigenvalues(cf, d, U, ch))
            scale = np.max(np.abs(lam))
            assert np.max(np.abs(ev - lam)) < 1e-7 * scale


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_jacobian_matches_finite_differences(oracle, system, dim):
    O = oracle
    rng = np.random.default_rng(2)
    cf = cfg(O, system, dim)
    U = rand_state(system, dim, rng)
    ch = ch_for(O, cf, U)
    for d in range(dim):
        A = O.jacobian(cf, d, U, ch)
        h = 1e-6
        for j in range(len(U)):
            e = np.zeros_like(U)
            e[j] = h
            col = (O.flux(cf, d, U + e, ch) - O.flux(cf, d, U - e, ch)) / (2 * h)
            assert np.allclose(A[:, j], col, rtol=1e-6, atol=1e-7)


def test_euler_flux_is_homogeneous_of_degree_one(oracle):
    """Sec. 2.2: the Euler flux satisfies F(U) = (dF/dU) U (the paper's
    homogeneity condition); shallow water and MHD do not (Sec. 4.2)."""
    O = oracle
    rng = np.random.default_rng(3)
    for dim in (1, 2):
        cf = cfg(O, "euler", dim)
        for _ in range(10):
            U = rand_state("euler", dim, rng)
            for d in range(dim):
                assert np.allclose(O.jacobian(cf, d, U) @ U, O.flux(cf, d, U), rtol=1e-13, atol=1e-13)
    for system in ("sw", "mhd"):
        cf = cfg(O, system, 1)
        U = rand_state(system, 1, rng)
        ch = ch_for(O, cf, U)
        assert np.max(np.abs(O.jacobian(cf, 0, U, ch) @ U - O.flux(cf, 0, U, ch))) > 1e-3


def test_rankine_hugoniot_of_exact_shocks(oracle):
    """The fluxes satisfy the textbook jump conditions across the exact shocks
    of the dam break and of the Sod tube: F(U_R) - F(U*) = S (U_R - U*)."""
    from exact_riemann import EulerRiemann, ShallowWaterRiemann
    O = oracle
    sw = ShallowWaterRiemann(2.0, 0.0, 1.0, 0.0, 9.81)
    cf = cfg(O, "sw", 1, g=9.81)
    UR = np.array([1.0, 0.0])
    Us = np.array([sw.hs, sw.hs * sw.us])
    jump = O.flux(cf, 0, UR) - O.flux(cf, 0, Us) - sw.SR * (UR - Us)
    assert np.max(np.abs(jump)) < 1e-10
    er = EulerRiemann(1, 0, 1, 0.125, 0, 0.1, 1.4)
    cf = cfg(O, "euler", 1)
    S = er.shock_speed_right()
    UR = np.array([0.125, 0.0, 0.1 / 0.4])
    Us = np.array([er.rsR, er.rsR * er.us, er.ps / 0.4 + 0.5 * er.rsR * er.us ** 2])
    jump = O.flux(cf, 0, UR) - O.flux(cf, 0, Us) - S * (UR - Us)
    assert np.max(np.abs(jump)) < 1e-10


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_split_sums_to_flux_and_k0_halves(oracle, system, dim):
    """Sec. 3.1: F+ + F- = F for the weighted split; alpha(0) = 1/2, so k = 0
    gives F+ = F- = F/2 (the centered limit)."""
    O = oracle
    rng = np.random.default_rng(4)
    for k in (2.0, 0.0, 7.5):
        cf = cfg(O, system, dim, k=k)
        for _ in range(10):
            U = rand_state(system, dim, rng)
            ch = ch_for(O, cf, U)
            for d in range(dim):
                F = O.flux(cf, d, U, ch)
                Fp, Fm = O.split(cf, d, U, ch)
                sc = np.max(np.abs(F)) + 1.0
                assert np.max(np.abs(Fp + Fm - F)) < 1e-11 * sc
                if k == 0.0:
                    assert np.max(np.abs(Fp - F / 2)) < 1e-11 * sc


def steger_warming_weighted(U, gamma, d, k, dim):
    """Closed form of P diag(mu) P^{-1} U for Euler with mu_j = alpha_j lambda_j
    (Steger-Warming flux formula with each eigenvalue scaled by its weight)."""
    rho = U[0]
    vel = U[1:1 + dim] / rho
    E = U[dim + 1]
    p = (gamma - 1.0) * (E - 0.5 * rho * vel @ vel)
    c = math.sqrt(gamma * p / rho)
    un = vel[d]
    lam = np.array([un - c, un, un + c])
    lmax = np.max(np.abs(lam))
    al = 1.0 / (1.0 + np.exp(-k * lam / lmax)) if math.isfinite(k) else (lam >= 0).astype(float)
    mu = al * lam
    H = (E + p) / rho
    e = np.zeros(dim)
    e[d] = 1.0
    v2 = vel @ vel
    ent = np.concatenate([[1.0], vel, [0.5 * v2]])
    am = np.concatenate([[1.0], vel - c * e, [H - un * c]])
    ap = np.concatenate([[1.0], vel + c * e, [H + un * c]])
    return rho / (2 * gamma) * (2 * (gamma - 1) * mu[1] * ent + mu[0] * am + mu[2] * ap)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("k", [2.0, 0.5, math.inf])
def test_euler_split_equals_weighted_steger_warming(oracle, dim, k):
    """Sec. 2.2: for a flux homogeneous of degree one the eigenvector split is
    the Steger-Warming split; the weighted split replaces lambda_j by
    alpha(lambda_j) lambda_j. Independent closed form vs the oracle's
    null-space/LU route."""
    O = oracle
    rng = np.random.default_rng(5)
    cf = cfg(O, "euler", dim, k=k)
    for _ in range(25):
        U = rand_state("euler", dim, rng)
        for d in range(dim):
            lam_max = np.max(np.abs(O.eigenvalues(cf, d, U)))
            Fp, Fm = O.split(cf, d, U, lam=lam_max)
            ref = steger_warming_weighted(U, 1.4, d, k, dim)
            assert np.allclose(Fp, ref, rtol=1e-12, atol=1e-13)


def tanh_split(A, F, lam_max, k):
    """Eigenvector-free form: F+ = 1/2 (I + tanh(k A / (2 lam_max))) F."""
    return 0.5 * (F + sla.tanhm(k * A / (2.0 * lam_max)) @ F)


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_split_equals_matrix_function(oracle, system, dim):
    """The weighted split is P diag(alpha) P^{-1} F = alpha(A) F; with the
    sigmoid, alpha(A) = (I + tanh(k A / (2 max|lambda|)))/2, evaluated here by
    scipy's matrix tanh without any eigenvectors."""
    O = oracle
    rng = np.random.default_rng(6)
    cf = cfg(O, system, dim)
    for _ in range(15):
        U = rand_state(system, dim, rng)
        ch = ch_for(O, cf, U)
        for d in range(dim):
            A = O.jacobian(cf, d, U, ch)
            F = O.flux(cf, d, U, ch)
            lam_max = np.max(np.abs(O.eigenvalues(cf, d, U, ch)))
            ref = tanh_split(A, F, lam_max, 2.0)
            Fp, _ = O.split(cf, d, U, ch, lam=lam_max)
            assert np.max(np.abs(Fp - ref)) < 1e-9 * (np.max(np.abs(F)) + 1)


@pytest.mark.parametrize("deg", ["bt0", "bt_small", "triple", "bx0"])
def test_mhd_split_at_degenerate_states(oracle, deg):
    """Near and at coinciding MHD speeds the split is still the well-defined
    matrix function alpha(A) F (the eigenvectors of a cluster span the same
    space whatever basis is chosen)."""
    O = oracle
    rng = np.random.default_rng(7)
    for dim in (1, 2):
        cf = cfg(O, "mhd", dim)
        for _ in range(8):
            U = rand_state("mhd", dim, rng, degenerate=deg)
            ch = ch_for(O, cf, U)
            A = O.jacobian(cf, 0, U, ch)
            F = O.flux(cf, 0, U, ch)
            lam_max = np.max(np.abs(O.eigenvalues(cf, 0, U, ch)))
            ref = tanh_split(A, F, lam_max, 2.0)
            Fp, Fm = O.split(cf, 0, U, ch, lam=lam_max)
            sc = np.max(np.abs(F)) + 1
            assert np.max(np.abs(Fp - ref)) < 1e-7 * sc
            assert np.max(np.abs(Fp + Fm - F)) < 1e-11 * sc


def test_mhd_split_high_precision(oracle):
    """Brute force on tiny inputs: a 50-digit eigen-decomposition of the 9x9
    MHD-GLM Jacobian reproduces the oracle's weighted split."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    O = oracle
    rng = np.random.default_rng(8)
    cf = cfg(O, "mhd", 2)
    for trial in range(3):
        U = rand_state("mhd", 2, rng)
        ch = ch_for(O, cf, U)
        d = trial % 2
        A = O.jacobian(cf, d, U, ch)
        F = O.flux(cf, d, U, ch)
        Am = mp.matrix([[mp.mpf(float(x)) for x in row] for row in A])
        Fm_ = mp.matrix([mp.mpf(float(x)) for x in F])
        E, ER = mp.eig(Am)
        lam = [mp.re(e) for e in E]
        lmax = max(abs(x) for x in lam)
        P = mp.matrix(9, 9)
        for i in range(9):
            for j in range(9):
                P[i, j] = mp.re(ER[i, j])
        phi = mp.lu_solve(P, Fm_)
        ref = np.zeros(9)
        for i in range(9):
            s = mp.mpf(0)
            for j in range(9):
                s += phi[j] * P[i, j] / (1 + mp.exp(-2 * lam[j] / lmax))
            ref[i] = float(s)
        Fp, _ = O.split(cf, d, U, ch, lam=float(lmax))
        assert np.max(np.abs(Fp - ref)) < 1e-11 * (np.max(np.abs(F)) + 1)


@pytest.mark.parametrize("system,dim", SYSTEMS)
def test_equilibrium_moments(oracle, system, dim):
    """Sec. 2.1 moment constraints: sum_q f_q^eq = U and sum_q v_q^d f_q^eq = F^(d)."""
    O = oracle
    rng = np.random.default_rng(9)
    cf = cfg(O, system, dim)
    vel = np.array([[1, 0, -1]]) if dim == 1 else np.array([[1, -1, 0, 0, 0], [0, 0, 0, 1, -1]])
    for _ in range(10):
        U = rand_state(system, dim, rng)
        ch = ch_for(O, cf, U)
        xi = rng.uniform(2.0, 40.0)
        fe = O.feq(cf, U, xi, ch)
        assert np.allclose(fe.sum(axis=0), U, rtol=1e-13, atol=1e-13)
        for d in range(dim):
            F = O.flux(cf, d, U, ch)
            mom = xi * (vel[d][:, None] * fe).sum(axis=0)
            assert np.allclose(mom, F, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim", [1, 2])
def test_presets_reduce_to_centered_and_discontinuous_sets(oracle, dim):
    """Sec. 3.1 / 3.4: c = 1/3 (1D) or 1/5 (2D) with F+ = F- = F/2 (k = 0) is the
    centered set; c = 0 with the discontinuous split (k = inf) is the
    discontinuous upwind set of Sec. 2.2 / 3.4."""
    O = oracle
    rng = np.random.default_rng(10)
    cc = 1.0 / 3.0 if dim == 1 else 1.0 / 5.0
    cf_c = cfg(O, "euler", dim, c=cc, k=0.0)
    cf_u = cfg(O, "euler", dim, c=0.0, k=math.inf)
    for _ in range(5):
        U = rand_state("euler", dim, rng)
        xi = 5.0
        F = [O.flux(cf_c, d, U) for d in range(dim)]
        fe = O.feq(cf_c, U, xi)
        if dim == 1:
            ref = np.stack([U / 3 + F[0] / (2 * xi), U / 3, U / 3 - F[0] / (2 * xi)])
        else:
            ref = np.stack([U / 5 + F[0] / (2 * xi), U / 5 - F[0] / (2 * xi), U / 5,
                            U / 5 + F[1] / (2 * xi), U / 5 - F[1] / (2 * xi)])
        assert np.allclose(fe, ref, rtol=1e-13, atol=1e-14)
        fe = O.feq(cf_u, U, xi)
        Sp = [steger_warming_weighted(U, 1.4, d, math.inf, dim) for d in range(dim)]
        Sm = [F[d] - Sp[d] for d in range(dim)]
        if dim == 1:
            ref = np.stack([Sp[0] / xi, U - (Sp[0] - Sm[0]) / xi, -Sm[0] / xi])
        else:
            ref = np.stack([Sp[0] / xi, -Sm[0] / xi, U - (Sp[0] + Sp[1] - Sm[0] - Sm[1]) / xi,
                            Sp[1] / xi, -Sm[1] / xi])
        assert np.allclose(fe, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("system,dim", [("euler", 2), ("mhd", 2), ("sw", 1)])
def test_local_and_global_normalization(oracle, system, dim):
    """The sigmoid normalization max_j|lambda_j|: with alpha_norm = local the
    oracle uses the cell's own max over that direction's eigenvalues, with
    the default (global) the value passed in; both agree when they coincide."""
    O = oracle
    rng = np.random.default_rng(12)
    cg = cfg(O, system, dim)
    cl = cfg(O, system, dim, alpha_norm="local")
    U = rand_state(system, dim, rng)
    ch = ch_for(O, cg, U)
    for d in range(dim):
        lam_d = float(np.max(np.abs(O.eigenvalues(cg, d, U, ch))))
        a = O.split(cg, d, U, ch, lam=lam_d)[0]
        b = O.split(cl, d, U, ch, lam=123.0)[0]
        assert np.array_equal(a, b)
        c2 = O.split(cg, d, U, ch, lam=3.0 * lam_d)[0]
        assert np.max(np.abs(c2 - a)) > 1e-6


def test_sw_rest_state_split_jacobian(oracle):
    """Closed form derived by hand from the split of Sec. 2.2 at a shallow
    water state at rest (u = 0, c = sqrt(g h)) with the discontinuous split:
    F+ = h(2u + c)/4 (1, u + c), whose Jacobian in (h, hu) is
    [[3c/8, 1/2], [c^2/2, 3c/4]]."""
    O = oracle
    g, h = 9.81, 1.7
    c = math.sqrt(g * h)
    cf = cfg(O, "sw", 1, g=g, k=math.inf)
    U = np.array([h, 1e-9])
    J = np.zeros((2, 2))
    eps = 1e-6
    for j in range(2):
        e = np.zeros(2)
        e[j] = eps
        J[:, j] = (O.split(cf, 0, U + e)[0] - O.split(cf, 0, U - e)[0]) / (2 * eps)
    ref = np.array([[3 * c / 8, 0.5], [c * c / 2, 3 * c / 4]])
    assert np.allclose(J, ref, rtol=1e-6, atol=1e-6)


def test_mhd_cleaning_pair_is_decoupled(oracle):
    """Sec. 5.3 (with the GLM flux): the (B_d, psi) rows of the Jacobian only
    involve (B_d, psi), with eigenvalues +-c_h."""
    O = oracle
    rng = np.random.default_rng(11)
    cf = cfg(O, "mhd", 2)
    U = rand_state("mhd", 2, rng)
    ch = 3.7
    for d in range(2):
        A = O.jacobian(cf, d, U, ch)
        rows = [5 + d, 8]
        other = [j for j in range(9) if j not in rows]
        assert np.all(A[np.ix_(rows, other)] == 0.0)
        sub = A[np.ix_(rows, rows)]
        assert np.allclose(np.sort(np.linalg.eigvals(sub).real), [-ch, ch])


@pytest.mark.parametrize("deg", [None, "bt0", "bt_small", "triple_near", "bx0"])
def test_fast_speed_is_the_fast_eigenvalue_of_the_jacobian(oracle, deg):
    """Sec. 5.3: the fast magnetosonic speed c_f sets the cleaning speed
    c_h = 6 max c_f, and through it Lambda, xi and every weight of an MHD run.
    The oracle computes it by a formula of its own (fast_speed), apart from
    the closed-form eigenvalues. It must equal the largest eigenvalue of the
    flux Jacobian less u_d (and u_d less the smallest), once the cleaning
    pair +-c_h, put far outside the physical speeds, is set aside. The
    Jacobian comes from complex-step differentiation of the flux, so this
    checks the formula against the system itself, not against itself."""
    O = oracle
    rng = np.random.default_rng(23)
    for dim in (1, 2):
        cf = cfg(O, "mhd", dim)
        for _ in range(20):
            U = rand_state("mhd", dim, rng, degenerate=deg)
            for d in range(dim):
                c_f = O.fast_speed(cf, d, U)
                ch = 1e3 * (c_f + 10.0)
                ev = np.sort(np.linalg.eigvals(O.jacobian(cf, d, U, ch)).real)
                assert ev[0] < -0.9 * ch and ev[-1] > 0.9 * ch
                phys = ev[1:-1]
                ud = U[1 + d] / U[0]
                assert abs(phys[-1] - ud - c_f) <= 1e-12 * c_f, (deg, phys[-1] - ud, c_f)
                assert abs(ud - phys[0] - c_f) <= 1e-12 * c_f, (deg, ud - phys[0], c_f)


def test_fast_speed_textbook_limits(oracle):
    """Sec. 5.3, the fast speed in its textbook limits (mu_0 = 1): no field,
    the sound speed a; field along d only, max(a, |B_d|/sqrt(rho)); field
    across d only, sqrt(a^2 + |B|^2/rho); at the triple point (field along d
    with B_d^2/rho = a^2), where three speeds meet and a numerical eigensolver
    loses half its digits, a itself."""
    O = oracle
    cf = cfg(O, "mhd", 2)
    gamma = 2.0
    rng = np.random.default_rng(29)
    for _ in range(20):
        rho, p = rng.uniform(0.3, 2.0), rng.uniform(0.1, 2.0)
        u, v, w = rng.uniform(-1, 1, 3)
        a = math.sqrt(gamma * p / rho)
        b = rng.uniform(0.2, 1.5)
        cases = [
            ((0.0, 0.0, 0.0), 0, a),
            ((b, 0.0, 0.0), 0, max(a, b / math.sqrt(rho))),
            ((0.0, b, 0.0), 1, max(a, b / math.sqrt(rho))),
            ((0.0, b, 0.7 * b), 0, math.sqrt(a * a + 1.49 * b * b / rho)),
            ((0.6 * b, 0.0, 0.8 * b), 1, math.sqrt(a * a + b * b / rho)),
            ((math.sqrt(gamma * p), 0.0, 0.0), 0, a),
        ]
        for B, d, want in cases:
            U = I.mhd_state(np.array([rho]), u, v, w, p, B[0], B[1], B[2], gamma)[:, 0]
            assert abs(O.fast_speed(cf, d, U) - want) <= 1e-14 * want, (B, d)
