"""Seeded synthetic inputs: initial states and run parameters of the workloads.

This module holds no arithmetic of the method itself. It builds initial
conserved states U0 (structure of arrays, shape (p, cells), float64) from the
problem definitions of the paper's test problems and of the benchmark
workloads, plus the run parameters (CFL number, relaxation, equilibrium
weights, boundaries, end condition). Both the HIP path and the CPU oracle are
fed from here; nothing here calls either of them.

Random draws use splitmix64 (Steele, Lea and Flood 2014): the state advances
by 0x9E3779B97F4A7C15 and each output is mixed by the published finalizer; a
uniform double is (x >> 11) * 2^-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

_M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self, a: float = 0.0, b: float = 1.0) -> float:
        return a + (b - a) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Integer in [lo, hi] inclusive."""
        return lo + int(self.uniform() * (hi - lo + 1)) if hi > lo else lo

    def exponential(self, rate: float) -> float:
        return -math.log(1.0 - self.uniform()) / rate


NVARS = {("sw", 1): 2, ("sw", 2): 3, ("euler", 1): 3, ("euler", 2): 4, ("mhd", 1): 9, ("mhd", 2): 9,
         ("linear", 1): 1, ("linear", 2): 1}


@dataclass
class Problem:
    """A complete run description: system, lattice, grid, method parameters, end condition."""
    name: str
    system: str                 # "sw" | "euler" | "mhd" | "linear"
    dim: int
    n: tuple                    # (nx,) or (nx, ny)
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    g: float = 9.81
    gamma: float = 1.4
    ch_factor: float = 6.0
    adv: tuple = (1.0, 0.0)
    xi_mode: str = "cfl"
    nu: float = 0.9
    xi: float = 0.0
    omega: float = 1.0
    c: float = 0.05
    k: float = 2.0
    alpha_norm: str = "global"    # sigmoid normalized by the global max |lambda| (or "local")
    eq_set: str = "weighted"      # "weighted" (c, k), "centered" or "discontinuous" (presets)
    bc: tuple = ("zero_gradient", "zero_gradient")
    T: float = math.inf
    max_steps: int = 2**62
    seed: int = 0
    U0: np.ndarray = field(default=None, repr=False)

    @property
    def p(self) -> int:
        return NVARS[(self.system, self.dim)]

    @property
    def Q(self) -> int:
        return 3 if self.dim == 1 else 5

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self) -> tuple:
        """Array shape of one field: (nx,) in 1D, (ny, nx) in 2D (x fastest)."""
        return (self.n[0],) if self.dim == 1 else (self.n[1], self.n[0])

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def cell_centres(n: int, lo: float, hi: float) -> np.ndarray:
    """Cell-centred nodes, dx/2 away from the boundary."""
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx


def grid2(nx, ny, lo, hi):
    x = cell_centres(nx, lo[0], hi[0])
    y = cell_centres(ny, lo[1], hi[1])
    X, Y = np.meshgrid(x, y)  # shape (ny, nx), x fastest
    return X, Y


# --- primitive -> conserved (problem definitions are in primitive form) ---------

def sw_state(h, u, v=None):
    h = np.asarray(h, dtype=np.float64)
    if v is None:
        return np.stack([h, h * u]).reshape(2, -1)
    return np.stack([h, h * u, h * v]).reshape(3, -1)


def euler_state(rho, u, p, gamma, v=None):
    rho = np.asarray(rho, dtype=np.float64)
    if v is None:
        E = p / (gamma - 1.0) + 0.5 * rho * u * u
        return np.stack(np.broadcast_arrays(rho, rho * u, E)).reshape(3, -1)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack(np.broadcast_arrays(rho, rho * u, rho * v, E)).reshape(4, -1)


def mhd_state(rho, u, v, w, p, Bx, By, Bz, gamma, psi=0.0):
    rho, u, v, w, p, Bx, By, Bz, psi = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64) for a in
                                                            (rho, u, v, w, p, Bx, By, Bz, psi)])
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w) + 0.5 * (Bx * Bx + By * By + Bz * Bz)
    return np.stack([rho, rho * u, rho * v, rho * w, E, Bx, By, Bz, psi]).reshape(9, -1)


# --- workloads --------------------------------------------------------------------

def dam_break(n=1000, **kw) -> Problem:
    """Shallow water dam break: h = 2 | 1 at x = 0.5 on [0,1], g = 9.81, t = 0.1.

    The speed rule 'xi = 1.2 max(|u| + sqrt(g h))' is the CFL rule with nu = 1/1.2.
    """
    P = Problem(name=f"sw1d_dambreak_n{n}", system="sw", dim=1, n=(n,), g=9.81, nu=1.0 / 1.2, T=0.1,
                bc=("zero_gradient", "zero_gradient"))
    P = P.with_(**kw)
    x = cell_centres(n, P.lo[0], P.hi[0])
    h = np.where(x < 0.5, 2.0, 1.0)
    return P.with_(U0=sw_state(h, np.zeros_like(h)))


def sod(n=65536, **kw) -> Problem:
    """Euler shock tube: (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1) at x = 0.5, gamma = 1.4, t = 0.2."""
    P = Problem(name=f"euler1d_sod_n{n}", system="euler", dim=1, n=(n,), gamma=1.4, nu=0.9, T=0.2)
    P = P.with_(**kw)
    x = cell_centres(n, P.lo[0], P.hi[0])
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return P.with_(U0=euler_state(rho, np.zeros_like(rho), p, P.gamma))


def sw_riemann(which="standard", n=1024, **kw) -> Problem:
    """The shallow water Riemann problems of Sec. 5.1 (g = 1, x0 = 0):

    * standard dam break: h = 3 | 1, hu = 0 | 0 on [-5, 5], t = 2;
    * hydraulic flow: h = 10 | 1, hu = 0 | 0 on [-20, 20], t = 4 (the Froude
      number crosses one inside the rarefaction);
    * compression flow: h = 1 | 1, hu = 1 | -1 on [-2, 2], t = 0.5 (one
      eigenvalue starts at zero everywhere).
    The paper runs them at CFL 0.9, 0.8 and 0.9 respectively."""
    table = {
        "standard": ((-5.0, 5.0), 2.0, (3.0, 1.0), (0.0, 0.0), 0.9),
        "hydraulic": ((-20.0, 20.0), 4.0, (10.0, 1.0), (0.0, 0.0), 0.8),
        "compression": ((-2.0, 2.0), 0.5, (1.0, 1.0), (1.0, -1.0), 0.9),
    }
    (a, b), T, (hl, hr), (ql, qr), nu = table[which]
    P = Problem(name=f"sw1d_{which}_n{n}", system="sw", dim=1, n=(n,), lo=(a, 0.0), hi=(b, 1.0), g=1.0, nu=nu,
                T=T)
    P = P.with_(**kw)
    x = cell_centres(n, P.lo[0], P.hi[0])
    left = x < 0.0
    h = np.where(left, hl, hr)
    hu = np.where(left, ql, qr)
    return P.with_(U0=sw_state(h, hu / h))


def euler_riemann(which="sod", n=1024, **kw) -> Problem:
    """The Euler Riemann problems of Sec. 5.2 (CFL 0.9):

    * Sod: (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1) on [-0.5, 0.5], x0 = 0, t = 0.2, gamma = 1.4;
    * Leblanc: (1, 0, 6.667e-2) | (1e-3, 0, 6.667e-9) on [0, 9], x0 = 3, t = 6, gamma = 5/3
      (eight decades of energy across the jump);
    * sonic point: (1, 0.75, 1) | (0.125, 0.75, 0.1) on [-1, 1], x0 = -0.4, t = 0.5, gamma = 1.4
      (the left rarefaction is transonic)."""
    table = {
        "sod": ((-0.5, 0.5), 0.2, 0.0, (1.0, 0.125), (0.0, 0.0), (1.0, 0.1), 1.4),
        "leblanc": ((0.0, 9.0), 6.0, 3.0, (1.0, 1e-3), (0.0, 0.0), (6.667e-2, 6.667e-9), 5.0 / 3.0),
        "sonic": ((-1.0, 1.0), 0.5, -0.4, (1.0, 0.125), (0.75, 0.75), (1.0, 0.1), 1.4),
    }
    (a, b), T, x0, (rl, rr), (ul, ur), (pl, pr), gamma = table[which]
    P = Problem(name=f"euler1d_{which}_n{n}", system="euler", dim=1, n=(n,), lo=(a, 0.0), hi=(b, 1.0),
                gamma=gamma, nu=0.9, T=T)
    P = P.with_(**kw)
    x = cell_centres(n, P.lo[0], P.hi[0])
    left = x < x0
    return P.with_(U0=euler_state(np.where(left, rl, rr), np.where(left, ul, ur), np.where(left, pl, pr),
                                  P.gamma))


def smooth_wave(n=256, **kw) -> Problem:
    """Periodic Euler density wave rho = 1 + 0.2 sin(2 pi x), u = 1, p = 1; exact solution rho(x - t)."""
    P = Problem(name=f"euler1d_wave_n{n}", system="euler", dim=1, n=(n,), gamma=1.4, nu=0.3, T=1.0,
                bc=("periodic", "periodic"))
    P = P.with_(**kw)
    x = cell_centres(n, P.lo[0], P.hi[0])
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    return P.with_(U0=euler_state(rho, np.ones_like(rho), np.ones_like(rho), P.gamma))


def entropy_wave_2d(n=128, **kw) -> Problem:
    """2D sinusoidal entropy wave (Sec. 5.2): rho = 1 + 0.1 sin(2 pi (x + y)),
    u = v = 1, p = 1 on the periodic [0,1]^2; gamma = 1.4, nu = 0.3, omega = 2,
    T = 1. The exact solution translates rho by t (u + v)."""
    P = Problem(name=f"euler2d_entropy_wave_n{n}", system="euler", dim=2, n=(n, n), gamma=1.4, nu=0.3, omega=2.0,
                T=1.0, bc=("periodic", "periodic"))
    P = P.with_(**kw)
    X, Y = grid2(n, n, P.lo, P.hi)
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * (X + Y))
    one = np.ones_like(rho)
    return P.with_(U0=euler_state(rho, one, one, P.gamma, v=one))


def isentropic_vortex(n=128, eps=5.0, **kw) -> Problem:
    """2D smooth vortex (Sec. 5.2) centred at the origin of the periodic
    [-5,5]^2: T = 1 - (gamma-1) eps^2/(8 gamma pi^2) e^{1-r^2}, rho = T^{1/(gamma-1)},
    (u, v) = (1, 1) + eps/(2 pi) e^{(1-r^2)/2} (-y, x), p = rho^gamma; gamma = 1.4,
    nu = 0.3, omega = 2, T_end = 2. eps = 5: the paper leaves it unstated but
    quotes Mach numbers 0.54 .. 1.97, which eps = 5 reproduces (0.547 .. 1.974)."""
    P = Problem(name=f"euler2d_vortex_n{n}", system="euler", dim=2, n=(n, n), lo=(-5.0, -5.0), hi=(5.0, 5.0),
                gamma=1.4, nu=0.3, omega=2.0, T=2.0, bc=("periodic", "periodic"))
    P = P.with_(**kw)
    X, Y = grid2(n, n, P.lo, P.hi)
    g = P.gamma
    r2 = X * X + Y * Y
    Tt = 1.0 - (g - 1.0) * eps * eps / (8.0 * g * np.pi ** 2) * np.exp(1.0 - r2)
    rho = Tt ** (1.0 / (g - 1.0))
    e = eps / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    return P.with_(U0=euler_state(rho, 1.0 - e * Y, rho ** g, g, v=1.0 + e * X))


def quadrants(n=2048, seed=0, steps=2000, **kw) -> Problem:
    """2D Euler four-quadrant Riemann data on [0,1]^2, gamma = 1.4.

    Quadrants are drawn in the order NE, NW, SW, SE; per quadrant the draw
    order is rho ~ U[0.5,1.5], p ~ U[0.3,1.5], u ~ U[-0.5,0.5], v ~ U[-0.5,0.5].
    """
    P = Problem(name=f"euler2d_quadrants_n{n}_s{seed}", system="euler", dim=2, n=(n, n), gamma=1.4,
                nu=0.4, max_steps=steps, seed=seed)
    P = P.with_(**kw)
    rng = SplitMix64(seed)
    states = []
    for _ in range(4):
        rho = rng.uniform(0.5, 1.5)
        p = rng.uniform(0.3, 1.5)
        u = rng.uniform(-0.5, 0.5)
        v = rng.uniform(-0.5, 0.5)
        states.append((rho, p, u, v))
    X, Y = grid2(n, n, P.lo, P.hi)
    east, north = X >= 0.5, Y >= 0.5
    quad = np.where(north & east, 0, np.where(north, 1, np.where(~east, 2, 3)))
    S = np.array(states)
    rho, p, u, v = (S[quad, i] for i in range(4))
    return P.with_(U0=euler_state(rho, u, p, P.gamma, v=v))


def brio_wu(n=16384, **kw) -> Problem:
    """MHD shock tube: (rho, p, B_y) = (1, 1, 1) | (0.125, 0.1, -1), B_x = 0.75, u = 0, gamma = 2, t = 0.1."""
    P = Problem(name=f"mhd1d_briowu_n{n}", system="mhd", dim=1, n=(n,), gamma=2.0, nu=0.9, T=0.1)
    P = P.with_(**kw)
    x = cell_centres(n, P.lo[0], P.hi[0])
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    By = np.where(left, 1.0, -1.0)
    z = np.zeros_like(rho)
    return P.with_(U0=mhd_state(rho, z, z, z, p, 0.75 + z, By, z, P.gamma))


def orszag_tang(n=1024, steps=1000, gamma=2.0, rho0=None, p0=None, **kw) -> Problem:
    """Periodic 2D MHD vortex: rho = gamma^2, p = gamma, u = (-sin 2pi y, sin 2pi x, 0),
    B = (-sin 2pi y, sin 4pi x, 0), psi = 0 on [0,1]^2."""
    P = Problem(name=f"mhd2d_ot_n{n}", system="mhd", dim=2, n=(n, n), gamma=gamma, nu=0.4,
                max_steps=steps, bc=("periodic", "periodic"))
    P = P.with_(**kw)
    X, Y = grid2(n, n, P.lo, P.hi)
    rho = np.full_like(X, gamma * gamma if rho0 is None else rho0)
    p = np.full_like(X, gamma if p0 is None else p0)
    u = -np.sin(2 * np.pi * Y)
    v = np.sin(2 * np.pi * X)
    Bx = -np.sin(2 * np.pi * Y)
    By = np.sin(4 * np.pi * X)
    z = np.zeros_like(X)
    return P.with_(U0=mhd_state(rho, u, v, z, p, Bx, By, z, gamma))


def orszag_tang_paper(n=2048, **kw) -> Problem:
    """The Orszag-Tang problem as the MHD section of the paper runs it:
    gamma = 5/3 on the periodic [0,1]^2 to T = 0.5 (2048^2 there), with the
    printed u and B of unit amplitude and rho = 25/9, p = 5/3. The paper
    prints rho = 25/(36 pi) and p = 5/(12 pi), the values of the common form
    whose field amplitude is 1/sqrt(4 pi); with unit B they must be scaled by
    4 pi to describe the same flow (read literally they give a low-beta
    problem on which the c = 0 weighted set the paper shows fails early)."""
    P = orszag_tang(n, steps=2**62, gamma=5.0 / 3.0, rho0=25.0 / 9.0, p0=5.0 / 3.0, T=0.5)
    P = P.with_(name=f"mhd2d_ot_paper_n{n}")
    return P.with_(**kw)


def constant_state(system, dim, n, seed=0, **kw) -> Problem:
    """A spatially uniform admissible state drawn from the seed."""
    rng = SplitMix64(seed)
    P = Problem(name=f"{system}{dim}d_const", system=system, dim=dim, n=tuple(n), seed=seed, **kw)
    ncell = P.cells
    one = np.ones(ncell)
    if system == "sw":
        h, u, v = rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
        U0 = sw_state(h * one, u, None if dim == 1 else v)
    elif system == "euler":
        rho, p, u, v = rng.uniform(0.5, 1.5), rng.uniform(0.3, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
        U0 = euler_state(rho * one, u, p, P.gamma, v=None if dim == 1 else v)
    elif system == "mhd":
        vals = [rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                rng.uniform(0.3, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1)]
        U0 = mhd_state(vals[0] * one, vals[1], vals[2], vals[3], vals[4], vals[5], vals[6], vals[7], P.gamma)
    else:
        U0 = rng.uniform(0.5, 1.5) * one.reshape(1, -1)
    return P.with_(U0=U0)


def random_riemann(system, dim, n, seed, **kw) -> Problem:
    """Two-state data with the left state on x < 0.5 (1D) or x + y < 1 (2D).

    SW: h ~ U[0.5,1.5], u, v ~ U[-0.5,0.5], g = 9.81. Euler/MHD: rho ~ U[0.5,1.5],
    p ~ U[0.3,1.5], u, v ~ U[-0.5,0.5]; MHD adds B_x = 0.75, B_y ~ U[-1,1],
    w = B_z = psi = 0. Draw order: left state then right state, fields in the
    order listed.
    """
    rng = SplitMix64(seed)
    gamma = 2.0 if system == "mhd" else 1.4
    nu = 0.9 if dim == 1 else 0.4
    nn = (n,) if dim == 1 else (n, n)
    P = Problem(name=f"{system}{dim}d_riemann_n{n}_s{seed}", system=system, dim=dim, n=nn, gamma=gamma, nu=nu,
                seed=seed)
    P = P.with_(**kw)
    sides = []
    for _ in range(2):
        if system == "sw":
            sides.append([rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)])
        elif system == "euler":
            sides.append([rng.uniform(0.5, 1.5), rng.uniform(0.3, 1.5), rng.uniform(-0.5, 0.5),
                          rng.uniform(-0.5, 0.5)])
        else:
            sides.append([rng.uniform(0.5, 1.5), rng.uniform(0.3, 1.5), rng.uniform(-0.5, 0.5),
                          rng.uniform(-0.5, 0.5), rng.uniform(-1.0, 1.0)])
    if dim == 1:
        x = cell_centres(n, P.lo[0], P.hi[0])
        left = x < 0.5
    else:
        X, Y = grid2(n, n, P.lo, P.hi)
        left = (X + Y) < 1.0
    S = np.array(sides)
    sel = np.where(left, 0, 1)
    col = lambda i: S[sel, i]
    if system == "sw":
        U0 = sw_state(col(0), col(1), None if dim == 1 else col(2))
    elif system == "euler":
        U0 = euler_state(col(0), col(2), col(1), gamma, v=None if dim == 1 else col(3))
    else:
        z = np.zeros(sel.shape)
        U0 = mhd_state(col(0), col(2), col(3), z, col(1), 0.75 + z, col(4), z, gamma)
    return P.with_(U0=U0)


@dataclass
class Request:
    rid: int
    arrival: float
    problem: Problem
    steps: int


def serving_requests(count=2000, seed=1, rate=1.0, n1=(2**10, 2**16), n2=(128, 1024), steps=(500, 5000),
                     materialize=False):
    """Poisson arrivals of mixed solves.

    Per request, in order: system uniform over {sw, euler, mhd}; 1D or 2D with
    probability 1/2; 1D N = round(2^U[10,16]) or 2D n = round(e^U[ln 128, ln 1024]);
    steps uniform in [500, 5000]; then the gap to the next arrival ~ Exp(rate);
    the two-state data use seed*1_000_003 + rid.
    """
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    systems = ("sw", "euler", "mhd")
    for rid in range(count):
        system = systems[min(2, int(rng.uniform() * 3))]
        dim = 1 if rng.uniform() < 0.5 else 2
        if dim == 1:
            n = int(round(2.0 ** rng.uniform(math.log2(n1[0]), math.log2(n1[1]))))
        else:
            n = int(round(math.exp(rng.uniform(math.log(n2[0]), math.log(n2[1])))))
        st = rng.randint(steps[0], steps[1])
        gap = rng.exponential(rate)
        prob_seed = seed * 1_000_003 + rid
        if materialize:
            prob = random_riemann(system, dim, n, prob_seed, max_steps=st)
        else:
            nn = (n,) if dim == 1 else (n, n)
            prob = Problem(name=f"{system}{dim}d_riemann_n{n}_s{prob_seed}", system=system, dim=dim, n=nn,
                           seed=prob_seed, max_steps=st, gamma=2.0 if system == "mhd" else 1.4,
                           nu=0.9 if dim == 1 else 0.4)
        out.append(Request(rid=rid, arrival=t, problem=prob, steps=st))
        t += gap
    return out


def materialize(prob: Problem) -> Problem:
    """Fill U0 of a lazily described serving problem."""
    if prob.U0 is not None:
        return prob
    n = prob.n[0]
    return random_riemann(prob.system, prob.dim, n, prob.seed, max_steps=prob.max_steps)


WORKLOADS = {
    "sw1d_dambreak": lambda: dam_break(1000),
    "euler1d_sod": lambda: sod(65536),
    "euler2d_quadrants": lambda: quadrants(2048, seed=0, steps=2000),
    "mhd1d_briowu": lambda: brio_wu(16384),
    "mhd2d_orszag_tang": lambda: orszag_tang(1024, steps=1000),
}
