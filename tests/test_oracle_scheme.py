"""Scheme-level pins of the CPU oracle (no GPU): properties the discretisation
must have whatever its implementation -- exactness on uniform states,
conservation, symmetry under axis permutation and translation, convergence to
exact solutions (a smoothly advected pulse; the Sod shock tube of section 5.1
against the exact special-relativistic Riemann solution), the static-fluid
balance in the curved metric, and the recovery failure policy."""
import numpy as np
import pytest

from paper_1102_5202_amd import workloads as WL
from tests import exact_riemann as ER


def problem(orc, w, **over):
    kw = w.problem_kwargs()
    kw.update(over)
    return orc.Problem(**kw)


def run(orc, w, nsteps=None, **over):
    pb = problem(orc, w, **over)
    U0 = orc.prim2con(pb, w.P)
    U, P, st = orc.step(pb, U0, w.P, w.dt, w.nsteps if nsteps is None else nsteps)
    return U0, U, P, st


def uniform(n, P0, bc=WL.PERIODIC):
    P = np.empty((9, n[2], n[1], n[0]))
    for v in range(9):
        P[v] = P0[v]
    return WL.Workload(name="uniform", P=P, n=n, lo=(0.0,) * 3, hi=(1.0,) * 3, bc=(bc,) * 3,
                       gamma=5.0 / 3.0, rk_order=3, dt=0.05, nsteps=3)


@pytest.mark.parametrize("bc", [WL.PERIODIC, WL.OUTFLOW])
@pytest.mark.parametrize("rk", [2, 3])
def test_uniform_state_held_bitwise(orc, bc, rk):
    P0 = np.array([0.7, 0.3, 0.4, -0.2, 0.5, 0.3, -0.6, 0.2, 0.0])
    w = uniform((6, 5, 4), P0, bc)
    U0, U, P, st = run(orc, w, rk_order=rk)
    assert np.array_equal(U, U0)
    assert st == {"fail": 0, "atm": 0, "pfloor": 0}
    np.testing.assert_allclose(P, w.P, rtol=1e-14, atol=1e-15)


def test_uniform_state_held_bitwise_with_zero_mass_curved_metric(orc):
    P0 = np.array([0.7, 0.3, 0.4, -0.2, 0.5, 0.3, -0.6, 0.2, 0.0])
    w = uniform((5, 4, 6), P0)
    U0, U, P, st = run(orc, w, metric=orc.ISO_SCHW, M=0.0)
    assert np.array_equal(U, U0)


def test_zero_mass_curved_metric_equals_flat_bitwise(orc):
    w = WL.config2(n=8, nsteps=2)
    _, Uf, Pf, _ = run(orc, w)
    _, Uc, Pc, _ = run(orc, w, metric=orc.ISO_SCHW, M=0.0)
    assert np.array_equal(Uf, Uc) and np.array_equal(Pf, Pc)


def test_periodic_box_conserves_all_totals(orc):
    """All eight MHD totals (mass, energy, momenta, densitised field) are
    conserved to round-off in a periodic flat box; Phi is damped, not conserved."""
    w = WL.config2(n=16, nsteps=3)
    U0, U, P, st = run(orc, w)
    assert st["fail"] == 0 and st["atm"] == 0 and st["pfloor"] == 0
    for v in range(8):
        tot0, tot = U0[v].sum(), U[v].sum()
        scale = np.abs(U0[v]).sum()
        assert abs(tot - tot0) <= 1e-14 * scale * w.nsteps * 2, (v, tot - tot0, scale)
    assert not np.array_equal(U, U0)      # something did happen


def test_1d_normal_field_and_phi_preserved_bitwise(orc):
    w = WL.config1(0, n=200)
    U0, U, P, st = run(orc, w, nsteps=100)
    assert np.array_equal(U[5], U0[5]) and np.all(U[8] == 0.0)
    assert np.array_equal(P[5], w.P[5]) and np.all(P[8] == 0.0)


def test_axis_permutation_symmetry(orc):
    """The same 1D problem along x, y and z gives the same result (to rounding:
    permuting the axes reorders sums such as u~x^2 + u~y^2 + u~z^2)."""
    res = []
    for axis in range(3):
        w = WL.config1(3, n=120, axis=axis)
        _, U, P, _ = run(orc, w, nsteps=60)
        # rotate the vector components back so the problem's axis is "x"
        perm = [0, 1, 2]
        perm[0], perm[axis] = perm[axis], perm[0]
        U = U.reshape(9, -1).copy()
        U[2:5] = U[[2 + perm[0], 2 + perm[1], 2 + perm[2]]]
        U[5:8] = U[[5 + perm[0], 5 + perm[1], 5 + perm[2]]]
        res.append(U)
    for r in res[1:]:
        err = np.abs(r - res[0]).max(axis=1) / np.maximum(np.abs(res[0]).max(axis=1), 1e-300)
        assert np.all(err <= 1e-12), err


def test_translation_invariance_periodic(orc):
    w = WL.config2(n=8, nsteps=2, k=1)
    _, U, _, _ = run(orc, w)
    w2 = WL.config2(n=8, nsteps=2, k=1)
    w2.P = np.roll(w.P, shift=(3, -2, 1), axis=(1, 2, 3))
    _, U2, _, _ = run(orc, w2)
    assert np.array_equal(np.roll(U, shift=(3, -2, 1), axis=(1, 2, 3)), U2)


def test_advected_pulse_converges_at_second_order(orc):
    """rho = 1 + 0.5 sin^2(pi x) advected at v = 0.5 with uniform p and a
    parallel field; exact solution rho(x - v t).  L1 order between N = 64, 128,
    256 at t = 0.4 (CFL 0.4)."""
    errs = []
    for n in (64, 128, 256):
        w = WL.pulse_1d(n)
        _, U, P, _ = run(orc, w, nsteps=n)
        t = n * w.dt
        x = (np.arange(n) + 0.5) / n
        exact = 1.0 + 0.5 * np.sin(np.pi * (x - 0.5 * t)) ** 2
        errs.append(np.abs(P[0].ravel() - exact).mean())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders >= 1.8), (errs, orders)
    assert errs[-1] < 1e-4


def test_sod_converges_to_exact_riemann_solution(orc):
    """Sod test of section 5.1 (B = 0) at t = 0.4 on [0,1]: the L1 density error
    against the exact special-relativistic solution falls at the first-order
    rate expected with a shock and a contact."""
    errs = []
    for n in (100, 200, 400, 800):
        w = WL.sod(n=n)
        _, U, P, st = run(orc, w)
        assert st["fail"] == 0
        x = (np.arange(n) + 0.5) / n
        rho, p, v = ER.sample(x, 0.4, 0.5, 1.0, 1.0, 0.0, 0.125, 0.1, 0.0, 5.0 / 3.0)
        errs.append(np.abs(P[0].ravel() - rho).mean())
        if n == 800:
            W = np.sqrt(1 + P[2].ravel() ** 2)
            assert np.abs(P[2].ravel() / W - v).mean() < 5e-3
            assert np.abs(P[1].ravel() - p).mean() < 3e-3
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 0.6), (errs, orders)
    assert errs[-1] < 4e-3, errs


def test_balsara1_runs_clean_and_keeps_bx(orc):
    """First Balsara test of section 5.1: no recovery failures, Bx exact."""
    w = WL.sod(n=200, magnetised=True)
    U0, U, P, st = run(orc, w)
    assert st == {"fail": 0, "atm": 0, "pfloor": 0}
    assert np.array_equal(U[5], U0[5])
    assert np.all(np.abs(P[2:5]) < 1.0) and P[0].min() > 0.1 and P[1].min() > 0.0


def test_static_fluid_in_curved_metric(orc):
    """Uniform fluid at rest, no field, M = 1: the mass and energy right-hand
    sides vanish exactly; the momentum right-hand side converges at second
    order to the hydrostatic imbalance -sqrt(-g) rho h d_j alpha / alpha."""
    errs = []
    for n in (8, 16, 32):
        lo, hi = (2.0, -3.0, 1.0), (6.0, 1.0, 5.0)
        P = np.zeros((9, n, n, n))
        P[0], P[1] = 1e-3, 1e-4
        w = WL.Workload(name="static", P=P, n=(n, n, n), lo=lo, hi=hi, bc=(WL.OUTFLOW,) * 3,
                        gamma=2.0, rk_order=3, dt=0.0, nsteps=0, metric=WL.ISO_SCHW, M=1.0)
        pb = problem(orc, w)
        R = orc.rhs(pb, P)
        assert np.all(R[0] == 0.0) and np.all(R[1] == 0.0) and np.all(R[5:] == 0.0)
        X = WL.centres(w.n, lo, hi)
        Xb = [np.broadcast_to(c, (n, n, n)) for c in X]
        h = 1e-5
        exact = np.zeros((3, n, n, n))
        r2 = Xb[0] ** 2 + Xb[1] ** 2 + Xb[2] ** 2

        def alpha_of(rr2):
            rs = np.sqrt(rr2 + 1.0)
            return (1 - 0.5 / rs) / (1 + 0.5 / rs)
        a = alpha_of(r2)
        psi6 = (1 + 0.5 / np.sqrt(r2 + 1.0)) ** 6
        for j in range(3):
            xp = [c.copy() for c in Xb]
            xm = [c.copy() for c in Xb]
            xp[j] += h
            xm[j] -= h
            da = (alpha_of(sum(c ** 2 for c in xp)) - alpha_of(sum(c ** 2 for c in xm))) / (2 * h)
            exact[j] = -a * psi6 * (1e-3 + 2.0 * 1e-4) * da / a
        # uniform data makes the zero-gradient ghosts exact: use every cell
        errs.append(np.abs(R[2:5] - exact).max() / np.abs(exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), (errs, orders)


def test_recovery_failure_policy(orc):
    """Unphysical cells are flagged and counted, never silently kept: a
    failure keeps the guess (or falls to the atmosphere when the guess is
    tenuous), densities below the atmosphere are reset, and pressures below
    the floor are raised; the matter part of U is then recomputed."""
    w = WL.config2(n=4)
    pb = problem(orc, w, rho_atm=1e-6, p_atm=1e-8)
    P = w.P.copy()
    U = orc.prim2con(pb, P)
    Ubad = U.copy()
    Ubad[1, 0, 0, 0] = -10.0                       # no physical root
    Ubad[2, 1, 0, 0] = 100.0                       # |S| > E
    Ubad[0, 2, 0, 0] = np.nan
    Pg = P.copy()
    Pg[0, 2, 0, 0] = 5e-6                          # tenuous guess -> atmosphere
    Ubad[:, 3, 0, 0] = orc.prim2con(pb, P)[:, 3, 0, 0] * 0.0
    P2, U2, flags, st = orc.con2prim(pb, Ubad, Pg)
    assert flags[0, 0, 0] & orc.FLAG_FAIL and flags[1, 0, 0] & orc.FLAG_FAIL
    assert flags[2, 0, 0] & orc.FLAG_FAIL and flags[2, 0, 0] & orc.FLAG_ATM
    assert flags[3, 0, 0] & orc.FLAG_FAIL
    assert P2[0, 2, 0, 0] == 1e-6 and P2[1, 2, 0, 0] == 1e-8
    np.testing.assert_array_equal(P2[:5, 0, 0, 0], Pg[:5, 0, 0, 0])
    assert st["fail"] == 4 and st["atm"] >= 1
    # adjusted cells are consistent: U(P) reproduced
    Ure = orc.prim2con(pb, P2)
    for c in [(0, 0, 0), (1, 0, 0), (2, 0, 0)]:
        np.testing.assert_allclose(U2[(slice(0, 5),) + c], Ure[(slice(0, 5),) + c], rtol=1e-14)
    # untouched cells keep their U and recover their P
    mask = flags == 0
    assert mask.sum() == 64 - 4
    np.testing.assert_array_equal(U2[:, mask], Ubad[:, mask])
    np.testing.assert_allclose(P2[:, mask], P[:, mask], rtol=1e-12, atol=1e-14)
    # a pressure below the floor is raised
    P3 = P.copy()
    P3[1, 0, 1, 1] = 1e-12
    U3 = orc.prim2con(pb, P3)
    P4, U4, flags4, st4 = orc.con2prim(pb, U3, P3)
    assert flags4[0, 1, 1] == orc.FLAG_PFLOOR and P4[1, 0, 1, 1] == 1e-8 and st4["pfloor"] == 1


def _cleaning_1d(n, phi0, bx0, kappa, t_end=0.5):
    x = (np.arange(n) + 0.5) / n
    P = np.zeros((9, 1, 1, n))
    P[0], P[1] = 1.0, 1.0
    P[5] = bx0(x)
    P[8] = phi0(x)
    w = WL.Workload(name="clean", P=P, n=(n, 1, 1), lo=(0.0,) * 3, hi=(1.0,) * 3,
                    bc=(WL.PERIODIC,) * 3, gamma=5.0 / 3.0, rk_order=3, dt=0.4 / n,
                    nsteps=int(round(t_end * n / 0.4)), kappa=kappa)
    _, U, P, st = run(orc_mod(), w)
    return x, U, P, st, w.nsteps * w.dt


def orc_mod():
    import oracle
    return oracle


def test_cleaning_pair_matches_dalembert_solution(orc):
    """In 1D flat space the (normal field, Phi) pair obeys the linear system
    d_t Bx + d_x Phi = 0, d_t Phi + c_h^2 d_x Bx = 0 (kappa = 0), decoupled from
    the fluid; Phi +- c_h Bx travel at +-c_h.  Second-order convergence."""
    bx0 = lambda x: 0.2 + 0.05 * np.sin(2 * np.pi * x)
    phi0 = lambda x: 0.02 * np.sin(4 * np.pi * x)
    errs = []
    for n in (64, 128, 256):
        x, U, P, st, t = _cleaning_1d(n, phi0, bx0, 0.0)
        assert st["fail"] == 0
        wp = phi0(x - t) + bx0(x - t)
        wm = phi0(x + t) - bx0(x + t)
        bx_ex, phi_ex = 0.5 * (wp - wm), 0.5 * (wp + wm)
        errs.append(max(np.abs(U[5].ravel() - bx_ex).mean(), np.abs(U[8].ravel() - phi_ex).mean()))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), (errs, orders)


@pytest.mark.parametrize("rk", [2, 3])
def test_cleaning_damping_follows_rk_stability_polynomial(orc, rk):
    """A uniform Phi obeys d_t Phi = -kappa Phi.  Per step SSP-RK2 multiplies it
    by 1 + z + z^2/2 and SSP-RK3 by 1 + z + z^2/2 + z^3/6 (z = -kappa dt): the
    Taylor polynomials of exp(z), which fixes the Runge-Kutta coefficients."""
    n = 32
    for kappa in (0.5, 2.0):
        P = np.zeros((9, 1, 1, n))
        P[0], P[1], P[5], P[8] = 1.0, 1.0, 0.3, 0.1
        w = WL.Workload(name="damp", P=P, n=(n, 1, 1), lo=(0.0,) * 3, hi=(1.0,) * 3,
                        bc=(WL.PERIODIC,) * 3, gamma=5.0 / 3.0, rk_order=rk, dt=0.4 / n,
                        nsteps=80, kappa=kappa)
        _, U, _, _ = run(orc, w)
        z = -kappa * w.dt
        amp = 1 + z + z * z / 2 + (z ** 3 / 6 if rk == 3 else 0.0)
        np.testing.assert_allclose(U[8], 0.1 * amp ** w.nsteps, rtol=1e-13)
        np.testing.assert_allclose(U[8], 0.1 * np.exp(-kappa * w.nsteps * w.dt),
                                   rtol=3e-3 if rk == 2 else 3e-5)
        assert np.all(U[5] == 0.3)


def test_initial_field_is_discretely_divergence_free(orc):
    """Initial fields are central-difference curls: their central divergence is
    at round-off."""
    w = WL.config2(n=16)
    dx = 1.0 / 16
    pb = problem(orc, w)
    U0 = orc.prim2con(pb, w.P)
    d = 0.0
    for comp, ax in ((0, 2), (1, 1), (2, 0)):
        d = d + (np.roll(U0[5 + comp], -1, axis=ax) - np.roll(U0[5 + comp], 1, axis=ax)) / (2 * dx)
    assert np.abs(d).max() <= 1e-13 * np.abs(U0[5:8]).max() / dx


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_outflow_boundary_is_two_zero_gradient_ghosts(orc, axis):
    """Zero-gradient outflow means two ghost cells holding the boundary cell's
    primitives: the outflow right-hand side on n cells equals, bitwise, the
    periodic right-hand side on n + 4 cells padded with those copies."""
    n = 24
    w = WL.config1(5, n=n, axis=axis)
    rng = np.random.default_rng(12)
    P = w.P * (1.0 + 0.2 * rng.uniform(size=w.P.shape))     # a non-trivial profile
    P[5 + axis] = w.P[5 + axis]
    pb = problem(orc, w)
    R = orc.rhs(pb, P)
    ax = 3 - axis                                             # array axis of the problem
    first = np.take(P, [0], axis=ax)
    last = np.take(P, [n - 1], axis=ax)
    E = np.concatenate([first, first, P, last, last], axis=ax)
    h = 1.0 / n
    n2 = list(w.n)
    n2[axis] = n + 4
    lo = [0.0, 0.0, 0.0]
    hi = [1.0, 1.0, 1.0]
    lo[axis], hi[axis] = -2 * h, 1.0 + 2 * h
    pb2 = orc.Problem(**{**w.problem_kwargs(), "n": tuple(n2), "lo": tuple(lo), "hi": tuple(hi),
                         "bc": (WL.PERIODIC,) * 3})
    R2 = orc.rhs(pb2, E)
    inner = np.take(R2, np.arange(2, n + 2), axis=ax)
    assert np.array_equal(R, inner)
