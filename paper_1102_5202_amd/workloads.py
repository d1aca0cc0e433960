"""Seeded synthetic initial data (primitive variables) for the standard workloads.

This module holds no arithmetic of the numerical scheme: it only draws seeded
random numbers and writes primitive fields
P = (rho, p, u~x, u~y, u~z, Bx, By, Bz, Phi) as float64 arrays ``[9, nz, ny, nx]``
(structure of arrays, x fastest).  Both the GPU path and the CPU oracle consume
exactly these arrays.  Where a recipe is stated in terms of the spacetime (the
velocity of a rigidly rotating blob, a densitised magnetic field) the given
metric functions of that spacetime are evaluated here, as part of the recipe.

The paper's own workloads (rotating neutron stars imported from the rns code,
Thor reference runs) are not available; these synthetic inputs stand in for
them with the shapes, sizes and value ranges of the paper's tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 11025202

FLAT, ISO_SCHW = 0, 1
SOFT_SQRT, SOFT_MAX = 0, 1
PERIODIC, OUTFLOW = 0, 1


@dataclass
class Workload:
    name: str
    P: np.ndarray                  # [9, nz, ny, nx] float64 primitives
    n: tuple
    lo: tuple
    hi: tuple
    bc: tuple
    gamma: float
    rk_order: int
    dt: float
    nsteps: int
    metric: int = FLAT
    M: float = 0.0
    soft: int = SOFT_SQRT
    r_min: float = 1.0
    rho_atm: float = 1e-12
    p_atm: float = 1e-12
    c_h: float = 1.0
    kappa: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def problem_kwargs(self) -> dict:
        """Keyword arguments shared by the solver and the oracle descriptions."""
        return dict(n=tuple(self.n), lo=tuple(self.lo), hi=tuple(self.hi), bc=tuple(self.bc),
                    metric=self.metric, M=self.M, soft=self.soft, r_min=self.r_min,
                    gamma=self.gamma, rk_order=self.rk_order, c_h=self.c_h, kappa=self.kappa,
                    rho_atm=self.rho_atm, p_atm=self.p_atm)


def cfl_dt(n, lo, hi, cfl: float = 0.4) -> float:
    """Time step for Courant number `cfl` of an unsplit update: the signal speed
    is bounded by 1 and the Courant numbers of the active axes add up."""
    s = sum(n[d] / (hi[d] - lo[d]) for d in range(3) if n[d] > 1)
    return cfl / s


def rng_for(config: int, k: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 1000 * config + k)


def centres(n, lo, hi):
    """Cell-centre coordinate arrays (z, y, x order broadcastable to [nz, ny, nx])."""
    xs = [lo[d] + (np.arange(n[d]) + 0.5) * (hi[d] - lo[d]) / n[d] for d in range(3)]
    return (xs[0][None, None, :], xs[1][None, :, None], xs[2][:, None, None])


def _curl_central(A, dx):
    """Central-difference curl of a vector potential sampled on an extended grid.

    ``A`` has shape [3, nz+2, ny+2, nx+2] (one extra layer on each side); the
    result has shape [3, nz, ny, nx] and its central-difference divergence
    vanishes identically (up to rounding).
    """
    def d(comp, axis):
        a = A[comp]
        h = dx[axis]
        if axis == 0:
            return (a[1:-1, 1:-1, 2:] - a[1:-1, 1:-1, :-2]) / (2 * h)
        if axis == 1:
            return (a[1:-1, 2:, 1:-1] - a[1:-1, :-2, 1:-1]) / (2 * h)
        return (a[2:, 1:-1, 1:-1] - a[:-2, 1:-1, 1:-1]) / (2 * h)
    return np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)])


def _extended_centres(n, lo, hi):
    dx = [(hi[d] - lo[d]) / n[d] for d in range(3)]
    xs = [lo[d] + (np.arange(-1, n[d] + 1) + 0.5) * dx[d] for d in range(3)]
    return (xs[0][None, None, :], xs[1][None, :, None], xs[2][:, None, None]), dx


def _modes(rng, count, kmax):
    """Draw `count` integer wave vectors with 0 < |k|_2 <= kmax."""
    ks = []
    while len(ks) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        nk = float(np.sqrt((k * k).sum()))
        if 0.0 < nk <= kmax:
            ks.append(k)
    return np.array(ks)


# -----------------------------------------------------------------------------
# 1D magnetised Riemann problems (seeded states)

def riemann_states(rng):
    """Left/right states: rho U[0.1,1], p U[0.01,1], v = 0, Bx U[0.3,1] shared,
    By, Bz U[-1,1]; Phi = 0.  Draw order: rhoL, rhoR, pL, pR, Bx, ByL, BzL, ByR, BzR."""
    rhoL, rhoR = rng.uniform(0.1, 1.0, 2)
    pL, pR = rng.uniform(0.01, 1.0, 2)
    bx = rng.uniform(0.3, 1.0)
    byL, bzL, byR, bzR = rng.uniform(-1.0, 1.0, 4)
    L = np.array([rhoL, pL, 0.0, 0.0, 0.0, bx, byL, bzL, 0.0])
    R = np.array([rhoR, pR, 0.0, 0.0, 0.0, bx, byR, bzR, 0.0])
    return L, R


def riemann_1d(L, R, n=400, axis=0, x0=0.5):
    """A 1D Riemann problem on [0,1] along `axis` (other axes have one cell)."""
    shape = [1, 1, 1]
    shape[axis] = n
    P = np.empty((9, shape[2], shape[1], shape[0]))
    x = (np.arange(n) + 0.5) / n
    left = x < x0
    for v in range(9):
        P[v] = np.where(left, L[v], R[v]).reshape((shape[2], shape[1], shape[0]))
    # rotate vector components so that the problem's "x" is along `axis`
    if axis != 0:
        perm = [0, 1, 2]
        perm[0], perm[axis] = perm[axis], perm[0]
        P[2:5] = P[[2 + perm[0], 2 + perm[1], 2 + perm[2]]]
        P[5:8] = P[[5 + perm[0], 5 + perm[1], 5 + perm[2]]]
    return P


def config1(k: int = 0, n: int = 400, axis: int = 0) -> Workload:
    """1D special-relativistic MHD Riemann problem, flat metric, n cells on [0,1],
    Gamma = 5/3, outflow, CFL 0.4 to t = 0.4 (dt = 0.4/n), SSP-RK3."""
    L, R = riemann_states(rng_for(1, k))
    P = riemann_1d(L, R, n=n, axis=axis)
    nn = [1, 1, 1]
    nn[axis] = n
    return Workload(name="riemann1d_%d" % n, P=P, n=tuple(nn), lo=(0.0, 0.0, 0.0),
                    hi=(1.0, 1.0, 1.0), bc=(OUTFLOW,) * 3, gamma=5.0 / 3.0, rk_order=3,
                    dt=0.4 / n, nsteps=n, extra={"L": L, "R": R})


def sod(n=400, axis=0, magnetised=False) -> Workload:
    """Sod test of section 5.1 (Gamma = 5/3; rho_L = 1, p_L = 1, rho_R = 0.125,
    p_R = 0.1, velocities 0); with ``magnetised`` the first Balsara test of the
    same section (Bx = 0.5, By = +1 / -1)."""
    L = np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    R = np.array([0.125, 0.1, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    if magnetised:
        L[5], L[6] = 0.5, 1.0
        R[5], R[6] = 0.5, -1.0
    P = riemann_1d(L, R, n=n, axis=axis)
    nn = [1, 1, 1]
    nn[axis] = n
    return Workload(name="balsara1" if magnetised else "sod", P=P, n=tuple(nn),
                    lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(OUTFLOW,) * 3,
                    gamma=5.0 / 3.0, rk_order=3, dt=0.4 / n, nsteps=n, extra={"L": L, "R": R})


# -----------------------------------------------------------------------------
# 3D periodic flat box

def config2(n: int = 128, k: int = 0, nsteps: int = 100, config_id: int = 2) -> Workload:
    """Periodic flat box [0,1]^3, Gamma = 4/3:
    rho = 1 + 0.1 sum_m a_m cos(2 pi k_m.x + phi_m) over 16 modes (|k| <= 4,
    sum |a_m| = 1); p = 0.1; v = 0.3 V / max|V| with V from 16 modes per
    component, u~ = W v; B = (0.1, 0.05, 0) + central curl of a 16-mode vector
    potential scaled to max|dB| = 0.01; Phi = 0.  SSP-RK2 with CFL 0.4 against
    the light-speed bound summed over the axes: dt = 0.4 / sum_d(1/dx_d).
    ``n`` may be a 3-tuple (the modes stay periodic on the unit box)."""
    rng = rng_for(config_id, k)
    nn = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    X = centres(nn, lo, hi)
    shape = (nn[2], nn[1], nn[0])
    eshape = (nn[2] + 2, nn[1] + 2, nn[0] + 2)
    P = np.zeros((9,) + shape)

    def field(count=16, kmax=4):
        ks = _modes(rng, count, kmax)
        ph = rng.uniform(0.0, 2 * np.pi, count)
        am = rng.uniform(-1.0, 1.0, count)
        return ks, ph, am

    def evaluate(ks, ph, am, Xs):
        f = 0.0
        for m in range(len(am)):
            f = f + am[m] * np.cos(2 * np.pi * (ks[m, 0] * Xs[0] + ks[m, 1] * Xs[1]
                                                + ks[m, 2] * Xs[2]) + ph[m])
        return f

    ks, ph, am = field()
    am = am / np.abs(am).sum()
    P[0] = 1.0 + 0.1 * evaluate(ks, ph, am, X)
    P[1] = 0.1
    V = np.stack([np.broadcast_to(evaluate(*field(), X), shape) for _ in range(3)])
    vmag = np.sqrt((V * V).sum(axis=0))
    v = 0.3 * V / vmag.max()
    W = 1.0 / np.sqrt(1.0 - (v * v).sum(axis=0))
    P[2:5] = W * v
    Xe, dx = _extended_centres(nn, lo, hi)
    A = np.stack([np.broadcast_to(evaluate(*field(), Xe), eshape) for _ in range(3)])
    dB = _curl_central(A, dx)
    dB *= 0.01 / np.abs(dB).max()
    P[5] = 0.1 + dB[0]
    P[6] = 0.05 + dB[1]
    P[7] = dB[2]
    P[8] = 0.0
    return Workload(name="periodic_flat_%dx%dx%d" % nn, P=P, n=nn, lo=lo, hi=hi,
                    bc=(PERIODIC,) * 3, gamma=4.0 / 3.0, rk_order=2, dt=cfl_dt(nn, lo, hi),
                    nsteps=nsteps)


# -----------------------------------------------------------------------------
# 3D curved static spacetime: rotating Gaussian blob

def _iso_schw(X, M=1.0, r_min=1.0, soft=SOFT_SQRT):
    """Lapse and conformal factor^4 of the isotropic Schwarzschild metric with
    the radius softened near the origin (the given spacetime of the workload)."""
    r = np.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)
    rs = np.sqrt(r * r + r_min * r_min) if soft == SOFT_SQRT else np.maximum(r, r_min)
    h = M / (2.0 * rs)
    return (1.0 - h) / (1.0 + h), (1.0 + h) ** 4


def config3(n=192, k: int = 0, nsteps: int = 200, half: float = 20.0, noise: bool = True,
            rho_c: float = 1e-3, width: float = 4.0, omega: float = 0.02, K: float = 100.0,
            beta_plasma: float = 1000.0, rho_atm: float = 1e-10, M: float = 1.0) -> Workload:
    """Static curved spacetime on [-half, half]^3 (G = c = M = 1), isotropic
    Schwarzschild with r_s = sqrt(r^2 + 1); Gamma = 2 polytropic data p = K rho^2
    (K = 100); rho = max(rho_c exp(-r^2/w^2)(1 + 0.01 xi), rho_atm) with xi
    U[-1,1] per cell; rigid rotation with coordinate angular velocity Omega
    about z; poloidal field from A = A_b rho_c exp(-r^2/w^2)(-y, x, 0) through a
    central curl of the densitised field, scaled so that max(B^2/2) =
    max(p)/beta_plasma; outflow; SSP-RK3 with dt = 0.4 / sum_d(1/dx_d) (coordinate
    signal speeds are bounded by alpha/psi^2 <= 1).  ``n`` may be a 3-tuple."""
    nn = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    rng = rng_for(3, k)
    lo, hi = (-half,) * 3, (half,) * 3
    X = centres(nn, lo, hi)
    shape = (nn[2], nn[1], nn[0])
    P = np.zeros((9,) + shape)
    r2 = X[0] ** 2 + X[1] ** 2 + X[2] ** 2
    xi = rng.uniform(-1.0, 1.0, shape) if noise else np.zeros(shape)
    rho = np.maximum(rho_c * np.exp(-r2 / width ** 2) * (1.0 + 0.01 * xi), rho_atm)
    P[0] = rho
    P[1] = K * rho ** 2
    alpha, psi4 = _iso_schw(X, M=M)
    # coordinate velocity u^i/u^t = Omega (-y, x, 0); Eulerian V = v/alpha
    vx = np.broadcast_to(-omega * X[1] / alpha, shape)
    vy = np.broadcast_to(omega * X[0] / alpha, shape)
    W = 1.0 / np.sqrt(1.0 - psi4 * (vx ** 2 + vy ** 2))
    P[2] = W * vx
    P[3] = W * vy
    P[4] = 0.0
    # densitised poloidal field Bd = curl A;  B = Bd / sqrt(-g), sqrt(-g) = alpha psi^6
    Xe, dx = _extended_centres(nn, lo, hi)
    env = rho_c * np.exp(-(Xe[0] ** 2 + Xe[1] ** 2 + Xe[2] ** 2) / width ** 2)
    eshape = (nn[2] + 2, nn[1] + 2, nn[0] + 2)
    A = np.stack([np.broadcast_to(-Xe[1] * env, eshape), np.broadcast_to(Xe[0] * env, eshape),
                  np.zeros(eshape)])
    Bd = _curl_central(A, dx)
    sqrtmg = alpha * psi4 ** 1.5
    B = Bd / sqrtmg
    bmag2 = psi4 * (B * B).sum(axis=0)
    scale = np.sqrt((P[1].max() / beta_plasma) / (0.5 * bmag2.max()))
    P[5:8] = B * scale
    P[8] = 0.0
    return Workload(name="curved_blob_%dx%dx%d" % nn, P=P, n=nn, lo=lo, hi=hi,
                    bc=(OUTFLOW,) * 3, gamma=2.0, rk_order=3, dt=cfl_dt(nn, lo, hi), nsteps=nsteps,
                    metric=ISO_SCHW, M=M, soft=SOFT_SQRT, r_min=1.0, rho_atm=rho_atm,
                    p_atm=K * rho_atm ** 2, extra={"K": K})


# -----------------------------------------------------------------------------
# smooth advected pulse (convergence test input)

def pulse_1d(n: int, v: float = 0.5, amp: float = 0.5, axis: int = 0, p: float = 1.0,
             bx: float = 0.3, gamma: float = 5.0 / 3.0) -> Workload:
    """rho = 1 + amp sin^2(pi x) on periodic [0,1], uniform p and velocity v along
    the axis, uniform field along the axis.  The exact solution is rho(x - v t)."""
    nn = [1, 1, 1]
    nn[axis] = n
    x = (np.arange(n) + 0.5) / n
    P = np.zeros((9, nn[2], nn[1], nn[0]))
    W = 1.0 / np.sqrt(1.0 - v * v)
    P[0] = (1.0 + amp * np.sin(np.pi * x) ** 2).reshape(nn[2], nn[1], nn[0])
    P[1] = p
    P[2 + axis] = W * v
    P[5 + axis] = bx
    return Workload(name="pulse_%d" % n, P=P, n=tuple(nn), lo=(0.0,) * 3, hi=(1.0,) * 3,
                    bc=(PERIODIC,) * 3, gamma=gamma, rk_order=3, dt=0.4 / n, nsteps=0)


# -----------------------------------------------------------------------------
# inputs of the derivative checks

def smooth_box(n=(8, 7, 6), k: int = 0, metric: int = FLAT, rk_order: int = 2,
               lo=None, hi=None, nsteps: int = 2) -> Workload:
    """Smooth data monotone along every axis in every variable (a seeded linear
    profile plus a small quadratic), outflow boundaries, Gamma = 4/3.  The MC
    slopes then stay on their central branch away from the boundary cells, so
    that finite differences of the step converge.  metric ISO_SCHW puts the box
    off the origin at [2,4]x[1,3]x[1.5,3.5] with M = 1."""
    rng = rng_for(40, k)
    nn = tuple(int(v) for v in n)
    if lo is None:
        lo = (2.0, 1.0, 1.5) if metric == ISO_SCHW else (0.0, 0.0, 0.0)
    if hi is None:
        hi = (4.0, 3.0, 3.5) if metric == ISO_SCHW else (1.0, 1.0, 1.0)
    X = centres(nn, lo, hi)
    t = [np.broadcast_to((X[d] - lo[d]) / (hi[d] - lo[d]), (nn[2], nn[1], nn[0])) for d in range(3)]
    base = (1.0, 0.1, 0.05, -0.04, 0.03, 0.1, 0.05, 0.02, 0.01)
    P = np.empty((9, nn[2], nn[1], nn[0]))
    for v in range(9):
        a = rng.uniform(0.5, 1.0, 3) * rng.choice([-1.0, 1.0], 3)
        sc = 0.2 * base[v] if v < 2 else 0.3 * abs(base[v])
        P[v] = base[v] + sc * (a[0] * t[0] + a[1] * t[1] + a[2] * t[2]
                               + 0.1 * (t[0] * t[1] + t[2] * t[2]))
    return Workload(name="smooth_box_%dx%dx%d" % nn, P=P, n=nn, lo=tuple(lo), hi=tuple(hi),
                    bc=(OUTFLOW,) * 3, gamma=4.0 / 3.0, rk_order=rk_order,
                    dt=cfl_dt(nn, lo, hi), nsteps=nsteps, metric=metric,
                    M=1.0 if metric == ISO_SCHW else 0.0)


@dataclass
class Ensemble:
    """Independent 1D problems on [0, 1] along x (flat metric, shared EOS and
    boundary rule): problem b has n[b] cells, time step dt[b] and takes
    steps[b] steps; P[b] is its (9, n[b]) initial primitive array."""
    name: str
    P: list
    n: list
    dt: list
    steps: list
    gamma: float = 5.0 / 3.0
    rk_order: int = 3
    bc: int = OUTFLOW
    rho_atm: float = 1e-12
    p_atm: float = 1e-12

    @property
    def ncell(self) -> int:
        return int(sum(self.n))

    def problem(self, b: int) -> Workload:
        """Problem b as a single-grid workload."""
        n = self.n[b]
        return Workload(name="%s_%d" % (self.name, b), P=self.P[b].reshape(9, 1, 1, n), n=(n, 1, 1),
                        lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(self.bc,) * 3, gamma=self.gamma,
                        rk_order=self.rk_order, dt=self.dt[b], nsteps=self.steps[b],
                        rho_atm=self.rho_atm, p_atm=self.p_atm)


def config5(nprob: int = 256, nmin: int = 200, nmax: int = 4000, k: int = 0,
            t_end: float = 0.4) -> Ensemble:
    """The batched ensemble: nprob magnetised 1D Riemann problems with lengths
    n_b uniform in [nmin, nmax] and states drawn as config1 (one seeded
    stream: all lengths first, then the states of each problem in turn), each
    on [0, 1] with dt_b = 0.4 / n_b (CFL 0.4) to t_end: steps_b = t_end / dt_b."""
    rng = rng_for(5, k)
    ns = [int(v) for v in rng.integers(nmin, nmax + 1, size=nprob)]
    P, dts, steps = [], [], []
    for n in ns:
        L, R = riemann_states(rng)
        P.append(riemann_1d(L, R, n=n).reshape(9, n))
        dt = 0.4 / n
        dts.append(dt)
        steps.append(int(round(t_end / dt)))
    return Ensemble(name="ensemble%d_%d_%d" % (nprob, nmin, nmax), P=P, n=ns, dt=dts, steps=steps)


def config4(n=64, k: int = 0, nsteps: int = 50) -> Workload:
    """The adjoint workload: the periodic flat box of config2 (RK2) run for
    nsteps, with a seeded target density rho_t = 1 + 0.1 sum of 16 other
    Fourier modes (extra["target"]); the loss is sum (rho(T) - rho_t)^2."""
    w = config2(n=n, k=k, nsteps=nsteps)
    rng = rng_for(4, k)
    nn = w.n
    X = centres(nn, w.lo, w.hi)
    ks = _modes(rng, 16, 4)
    ph = rng.uniform(0.0, 2 * np.pi, 16)
    am = rng.uniform(-1.0, 1.0, 16)
    am /= np.abs(am).sum()
    f = 0.0
    for m in range(16):
        f = f + am[m] * np.cos(2 * np.pi * (ks[m, 0] * X[0] + ks[m, 1] * X[1] + ks[m, 2] * X[2])
                               + ph[m])
    w.extra["target"] = np.ascontiguousarray(
        np.broadcast_to(1.0 + 0.1 * f, (nn[2], nn[1], nn[0])))
    w.name = "adjoint_periodic_%dx%dx%d" % nn
    return w


def direction(w: Workload, i: int, k: int = 0) -> np.ndarray:
    """Seeded direction i in primitive space for directional-derivative
    checks: standard normal values scaled per variable by the largest
    magnitude of that variable in w.P.  Variables uniform in w.P are left
    unperturbed: every MC slope of a uniform field sits on the limiter's kink
    (both one-sided differences zero), where the step has no derivative."""
    rng = np.random.default_rng(SEED_BASE + 41000 + 100 * k + i)
    flat = w.P.reshape(9, -1)
    scale = np.abs(flat).max(axis=1)
    scale[flat.max(axis=1) == flat.min(axis=1)] = 0.0
    return rng.standard_normal(w.P.shape) * scale.reshape(9, 1, 1, 1)


def ghosted_centres(n, lo, hi):
    """Cell-centre coordinates including 2 ghost layers on every active axis
    (z, y, x order broadcastable to [nz+4, ny+4, nx+4] for a 3D grid)."""
    xs = []
    for d in range(3):
        g = 2 if n[d] > 1 else 0
        xs.append(lo[d] + (np.arange(-g, n[d] + g) + 0.5) * (hi[d] - lo[d]) / n[d])
    return (xs[0][None, None, :], xs[1][None, :, None], xs[2][:, None, None])


def stored_metric(n, lo, hi, k: int = 0, bc=(OUTFLOW, OUTFLOW, OUTFLOW)):
    """A smooth static, conformally flat metric given on the grid (the input of
    the stored-metric form): lapse alpha = 1 - a exp(-s^2 / w^2) and conformal
    factor psi^4 = (1 + b exp(-s^2 / w^2))^4 with seeded a in [0.05, 0.2],
    b in [0.02, 0.1], a centre c inside the box and width w a third of the
    box; s is the distance to c, measured along a periodic axis of length L as
    (L / pi) sin(pi (x - c) / L) so that the metric is periodic there.  Sampled
    at the cell centres and 2 ghost layers on every active axis; the ghost
    layers of a periodic axis are copies of the opposite interior cells.
    Arrays [z][y][x]."""
    rng = rng_for(60, k)
    a, b = rng.uniform(0.05, 0.2), rng.uniform(0.02, 0.1)
    c = [lo[d] + rng.uniform(0.3, 0.7) * (hi[d] - lo[d]) for d in range(3)]
    w = max(hi[d] - lo[d] for d in range(3) if n[d] > 1) / 3.0
    X = ghosted_centres(n, lo, hi)
    r2 = 0.0
    for d in range(3):
        if n[d] <= 1:
            continue
        L = hi[d] - lo[d]
        s = (L / np.pi) * np.sin(np.pi * (X[d] - c[d]) / L) if bc[d] == PERIODIC else X[d] - c[d]
        r2 = r2 + s * s
    bump = np.exp(-r2 / (w * w))
    shape = tuple(n[d] + (4 if n[d] > 1 else 0) for d in (2, 1, 0))
    out = []
    for f in (1.0 - a * bump, (1.0 + b * bump) ** 4):
        f = np.broadcast_to(f, shape).copy()
        for d in range(3):
            if n[d] > 1 and bc[d] == PERIODIC:
                ax = 2 - d
                idx = (np.arange(-2, n[d] + 2) % n[d]) + 2
                f = np.take(f, idx, axis=ax)
        out.append(np.ascontiguousarray(f))
    return out[0], out[1]


def sampled_isotropic_metric(n, lo, hi, M: float = 1.0, r_min: float = 1.0, soft: int = SOFT_SQRT):
    """The workload's isotropic Schwarzschild metric given on the grid (the
    stored-metric form of the same spacetime): lapse and psi^4 at the cell
    centres and 2 ghost layers on every active axis, arrays [z][y][x]."""
    X = ghosted_centres(n, lo, hi)
    shape = tuple(n[d] + (4 if n[d] > 1 else 0) for d in (2, 1, 0))
    alpha, psi4 = _iso_schw(X, M, r_min, soft)
    return np.broadcast_to(alpha, shape).copy(), np.broadcast_to(psi4, shape).copy()
