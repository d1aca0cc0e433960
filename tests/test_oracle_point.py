"""Pins of the oracle's point functions against what the physics fixes
(no GPU).  Each check uses a route independent of the oracle's own code:
textbook special-relativistic MHD formulas in the local orthonormal frame of
the normal observer, closed-form characteristic speeds, Christoffel symbols by
finite differences of an independently written metric, properties of the MC
limiter and of the HLLE/cleaning face solver."""
import numpy as np
import pytest

GAMMAS = (4.0 / 3.0, 5.0 / 3.0, 2.0)


# ---- independent formula set: special-relativistic MHD (Valencia form) in the
# orthonormal frame of the normal observer, mapped to coordinate components of
# a static conformally flat metric g = diag(-alpha^2, psi^4, psi^4, psi^4).

def metric_iso(x, y, z, M=1.0, r_min=1.0, soft="sqrt"):
    r = np.sqrt(x * x + y * y + z * z)
    rs = np.sqrt(r * r + r_min * r_min) if soft == "sqrt" else max(r, r_min)
    h = M / (2 * rs)
    return (1 - h) / (1 + h), (1 + h) ** 4


def textbook(P, gamma, alpha=1.0, psi4=1.0, c_h=1.0):
    rho, p = P[0], P[1]
    ut = np.asarray(P[2:5], dtype=float)
    B = np.asarray(P[5:8], dtype=float)
    phi = P[8]
    psi2 = np.sqrt(psi4)
    W = np.sqrt(1.0 + psi4 * ut @ ut)
    v = psi2 * ut / W           # orthonormal-frame 3-velocity of the fluid
    Bh = alpha * psi2 * B       # field seen by the normal observer (alpha B^i), orthonormal
    v2, vB, B2 = v @ v, v @ Bh, Bh @ Bh
    w = rho + gamma / (gamma - 1.0) * p
    b2 = B2 / W ** 2 + vB ** 2
    D = rho * W
    S = (w * W ** 2 + B2) * v - vB * Bh
    E = w * W ** 2 - p + 0.5 * B2 + 0.5 * (v2 * B2 - vB ** 2)
    ptot = p + 0.5 * b2
    sqrtg = psi4 ** 1.5
    sqrtmg = alpha * sqrtg
    U = np.zeros(9)
    U[0] = sqrtg * D
    U[1] = sqrtg * (alpha * E - D)
    U[2:5] = sqrtg * psi2 * S
    U[5:8] = sqrtmg * B
    U[8] = phi
    F = np.zeros((3, 9))
    for i in range(3):
        FD = D * v[i]
        FS = S * v[i] - Bh[i] * (Bh / W ** 2 + vB * v)
        FS[i] += ptot
        FE = S[i]
        F[i, 0] = sqrtmg / psi2 * FD
        F[i, 1] = sqrtmg / psi2 * (alpha * FE - FD)
        F[i, 2:5] = sqrtmg * FS
        for j in range(3):
            F[i, 5 + j] = (phi if j == i else
                           sqrtmg / psi4 * (Bh[j] * v[i] - Bh[i] * v[j]))
        F[i, 8] = c_h ** 2 * sqrtmg * B[i]
    # characteristic speeds: closed form for an isotropic signal speed c
    cs2 = gamma * p / w
    ca2 = b2 / (w + b2)
    c2 = cs2 + ca2 - cs2 * ca2
    lam = np.zeros((3, 2))
    for i in range(3):
        disc = (1 - v2) * (1 - v2 * c2 - v[i] ** 2 * (1 - c2))
        lp = (v[i] * (1 - c2) + np.sqrt(c2 * disc)) / (1 - v2 * c2)
        lm = (v[i] * (1 - c2) - np.sqrt(c2 * disc)) / (1 - v2 * c2)
        lam[i] = (alpha / psi2 * lm, alpha / psi2 * lp)
    return U, F, lam, dict(W=W, b2=b2, w=w)


def random_prim(rng, Wmax=10.0, sigmax=100.0, gamma=5.0 / 3.0, psi4=1.0):
    """Random physical primitives with W <= Wmax and b^2/rho <= sigmax."""
    while True:
        rho = 10 ** rng.uniform(-3, 1)
        p = rho * 10 ** rng.uniform(-3, 1)
        W = 1.0 + (Wmax - 1.0) * rng.uniform() ** 2
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        ut = np.sqrt(W * W - 1.0) * n / np.sqrt(psi4)
        B = rng.normal(size=3)
        P = np.array([rho, p, *ut, *B, rng.normal() * 0.1])
        b2 = textbook(P, gamma, psi4=psi4)[3]["b2"]
        sig = 10 ** rng.uniform(-3, np.log10(sigmax))
        P[5:8] *= np.sqrt(sig * rho / b2)
        return P


POINTS = [(0.3, -1.7, 2.2), (5.0, 1.0, -3.0), (0.0, 0.0, 0.1), (-12.0, 7.0, 9.0)]


def test_flat_cons_flux_speeds_match_textbook(orc):
    rng = np.random.default_rng(1)
    for gamma in GAMMAS:
        for _ in range(200):
            P = random_prim(rng, gamma=gamma)
            U_ref, F_ref, lam_ref, _ = textbook(P, gamma)
            U = orc.point_cons(P, gamma)
            np.testing.assert_allclose(U, U_ref, rtol=1e-12, atol=1e-12 * np.abs(U_ref).max())
            for d in range(3):
                F = orc.point_flux(P, gamma, d)
                np.testing.assert_allclose(F, F_ref[d], rtol=1e-11,
                                           atol=1e-12 * np.abs(F_ref[d]).max())
                lm, lp = orc.point_speeds(P, gamma, d)
                np.testing.assert_allclose([lm, lp], lam_ref[d], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("soft", ["sqrt", "max"])
def test_curved_cons_flux_speeds_match_orthonormal_frame(orc, soft):
    rng = np.random.default_rng(2)
    sk = orc.SOFT_SQRT if soft == "sqrt" else orc.SOFT_MAX
    for (x, y, z) in POINTS:
        alpha, psi4 = metric_iso(x, y, z, soft=soft)
        mk = dict(metric=orc.ISO_SCHW, M=1.0, soft=sk, r_min=1.0)
        for _ in range(60):
            gamma = GAMMAS[rng.integers(3)]
            P = random_prim(rng, gamma=gamma, psi4=psi4)
            U_ref, F_ref, lam_ref, _ = textbook(P, gamma, alpha=alpha, psi4=psi4)
            U = orc.point_cons(P, gamma, x, y, z, **mk)
            np.testing.assert_allclose(U, U_ref, rtol=1e-11, atol=1e-12 * np.abs(U_ref).max())
            for d in range(3):
                F = orc.point_flux(P, gamma, d, 1.0, x, y, z, **mk)
                np.testing.assert_allclose(F, F_ref[d], rtol=1e-10,
                                           atol=1e-12 * np.abs(F_ref[d]).max())
                lm, lp = orc.point_speeds(P, gamma, d, x, y, z, **mk)
                np.testing.assert_allclose([lm, lp], lam_ref[d], rtol=1e-10, atol=1e-13)


def test_speeds_closed_forms(orc):
    """Fluid at rest: +-c. Motion along the direction: relativistic velocity
    addition (v +- c)/(1 +- v c). Motion across it: +-c sqrt((1-v^2)/(1-v^2 c^2))."""
    gamma = 5.0 / 3.0
    for (rho, p) in [(1.0, 1.0), (0.1, 0.01), (2.0, 10.0)]:
        cs = np.sqrt(gamma * p / (rho + gamma / (gamma - 1) * p))
        P = np.array([rho, p, 0, 0, 0, 0, 0, 0, 0.0])
        lm, lp = orc.point_speeds(P, gamma, 0)
        np.testing.assert_allclose([lm, lp], [-cs, cs], rtol=1e-14)
        for v in (0.3, -0.9, 0.99):
            W = 1 / np.sqrt(1 - v * v)
            P = np.array([rho, p, W * v, 0, 0, 0, 0, 0, 0.0])
            lm, lp = orc.point_speeds(P, gamma, 0)
            np.testing.assert_allclose([lm, lp], [(v - cs) / (1 - v * cs), (v + cs) / (1 + v * cs)],
                                       rtol=1e-12)
            lm, lp = orc.point_speeds(P, gamma, 1)
            t = cs * np.sqrt((1 - v * v) / (1 - v * v * cs * cs))
            np.testing.assert_allclose([lm, lp], [-t, t], rtol=1e-12)
    # |lambda| <= 1 in flat space for any physical state
    rng = np.random.default_rng(3)
    for _ in range(300):
        P = random_prim(rng)
        for d in range(3):
            lm, lp = orc.point_speeds(P, gamma, d)
            assert -1.0 <= lm <= lp <= 1.0


@pytest.mark.parametrize("metric", ["flat", "curved"])
def test_prim_cons_prim_round_trip(orc, metric):
    """Recovery inverts the algebraic map to round-off (W <= 10, b^2/rho <= 100).
    Inputs are produced by the independent textbook formulas.  Relative errors
    are <= 1e-13 for W <= 3; beyond, they follow the conditioning of the map
    (1 - v^2 = 1/W^2 cancels W^2 digits; a one-ulp change of U moves rho by the
    same amount), so the bound there is 1e-14 W^2."""
    rng = np.random.default_rng(4)
    pts = [(0.0, 0.0, 0.0)] if metric == "flat" else POINTS
    for (x, y, z) in pts:
        alpha, psi4 = (1.0, 1.0) if metric == "flat" else metric_iso(x, y, z)
        mk = {} if metric == "flat" else dict(metric=orc.ISO_SCHW, M=1.0)
        for _ in range(400 // len(pts)):
            gamma = GAMMAS[rng.integers(3)]
            P = random_prim(rng, gamma=gamma, psi4=psi4)
            U_ref = textbook(P, gamma, alpha=alpha, psi4=psi4)[0]
            P2, ok = orc.point_c2p(U_ref, gamma, x, y, z, **mk)
            assert ok
            W = np.sqrt(1 + psi4 * P[2:5] @ P[2:5])
            bound = 1e-13 if W <= 3.0 else 1e-14 * W * W
            assert abs(P2[0] - P[0]) / P[0] <= bound
            assert np.abs(P2[2:5] - P[2:5]).max() / W <= bound
            assert np.abs(P2[5:8] - P[5:8]).max() <= 1e-15 * np.abs(P[5:8]).max()
            assert P2[8] == P[8]
            # the pressure of a cold, strongly magnetised state is ill conditioned:
            # its error scales with (energy density / p)
            en = (U_ref[1] + U_ref[0]) / U_ref[0]
            assert abs(P2[1] - P[1]) / P[1] <= bound * max(1.0, en * P[0] / P[1])


def test_recovery_fails_without_physical_root(orc):
    gamma = 5.0 / 3.0
    P = np.array([1.0, 1.0, 0.5, 0.0, 0.0, 0.1, 0.2, 0.0, 0.0])
    U = orc.point_cons(P, gamma)
    bad = U.copy()
    bad[1] = -0.5                    # tau < 0 beyond any physical state
    assert not orc.point_c2p(bad, gamma)[1]
    bad = U.copy()
    bad[2] = 10.0 * (U[0] + U[1])    # |S| > E
    assert not orc.point_c2p(bad, gamma)[1]
    bad = U.copy()
    bad[0] = np.nan
    assert not orc.point_c2p(bad, gamma)[1]
    bad = U.copy()
    bad[0] = -1.0
    assert not orc.point_c2p(bad, gamma)[1]


def test_source_equals_christoffel_contraction(orc):
    """sqrt(-g) T^k_l Gamma^l_{mu k} with Christoffel symbols from central finite
    differences of an independently written metric equals the oracle source."""
    rng = np.random.default_rng(5)
    h = 1e-4

    def g4(x):
        a, p4 = metric_iso(*x)
        return np.diag([-a * a, p4, p4, p4])

    for X in POINTS:
        X = np.array(X)
        g = g4(X)
        gi = np.linalg.inv(g)
        dg = np.zeros((4, 4, 4))            # dg[mu] = d_mu g_{ab}, static
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            dg[i + 1] = (-g4(X + 2 * e) + 8 * g4(X + e) - 8 * g4(X - e) + g4(X - 2 * e)) / (12 * h)
        Gam = 0.5 * (np.einsum("ls,msk->lmk", gi, dg) + np.einsum("ls,ksm->lmk", gi, dg)
                     - np.einsum("ls,smk->lmk", gi, dg))
        sqrtmg = np.sqrt(-np.linalg.det(g))
        for _ in range(20):
            P = random_prim(rng, psi4=g[1, 1])
            T = orc.point_stress(P, 5.0 / 3.0, *X, metric=orc.ISO_SCHW, M=1.0)
            src = sqrtmg * np.einsum("kl,lmk->m", T, Gam)
            S = orc.point_source(P, 5.0 / 3.0, 0.7, *X, metric=orc.ISO_SCHW, M=1.0)
            scale = sqrtmg * np.abs(T).max() * np.abs(dg).max()
            np.testing.assert_allclose(S[2:5], src[1:4], rtol=1e-7, atol=1e-9 * scale)
            assert abs(S[1] + src[0]) <= 1e-9 * scale   # tau row: minus the T^t_t row
            assert S[0] == 0.0 and np.all(S[5:8] == 0.0)
            assert S[8] == -0.7 * P[8]


def test_flat_space_source_vanishes(orc):
    rng = np.random.default_rng(6)
    for _ in range(50):
        P = random_prim(rng)
        S = orc.point_source(P, 5.0 / 3.0, 0.0, 1.0, 2.0, 3.0)
        assert np.all(S == 0.0)
        # M = 0 reduces the curved metric bitwise to flat space
        S0 = orc.point_source(P, 5.0 / 3.0, 0.0, 1.0, 2.0, 3.0, metric=orc.ISO_SCHW, M=0.0)
        assert np.all(S0 == 0.0)
        U = orc.point_cons(P, 5.0 / 3.0)
        U0 = orc.point_cons(P, 5.0 / 3.0, 1.0, 2.0, 3.0, metric=orc.ISO_SCHW, M=0.0)
        assert np.array_equal(U, U0)


def test_metric_closed_form(orc):
    for X in POINTS:
        a, p4 = metric_iso(*X)
        G = orc.point_geom(*X, metric=orc.ISO_SCHW, M=1.0)
        np.testing.assert_allclose(G["alpha"], a, rtol=1e-15)
        np.testing.assert_allclose(G["sqrtgamma"], p4 ** 1.5, rtol=1e-14)
        np.testing.assert_allclose(G["sqrtmg"], a * p4 ** 1.5, rtol=1e-14)
        np.testing.assert_allclose(G["g"] @ G["gi"], np.eye(4), atol=1e-14)
        # derivative of the closed form against central differences
        h = 1e-5
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            ap, pp = metric_iso(*(np.array(X) + e))
            am, pm = metric_iso(*(np.array(X) - e))
            np.testing.assert_allclose(G["dg"][i][0, 0], -(ap * ap - am * am) / (2 * h),
                                       rtol=1e-7, atol=1e-12)
            np.testing.assert_allclose(G["dg"][i][1, 1], (pp - pm) / (2 * h), rtol=1e-7, atol=1e-12)


# ---- reconstruction --------------------------------------------------------

def test_mc_exact_on_constant_and_linear(orc):
    for q0, d in [(1.0, 0.0), (1.0, 0.25), (-3.0, -0.5), (0.0, 2.0)]:
        s = orc.mc_slope(q0 - d, q0, q0 + d)
        assert s == d
        assert q0 + 0.5 * s == q0 + 0.5 * d and q0 - 0.5 * s == q0 - 0.5 * d


def test_mc_is_tvd_bounded(orc):
    rng = np.random.default_rng(7)
    for _ in range(5000):
        qm, q0, qp = rng.normal(size=3) * 10 ** rng.uniform(-3, 3, size=3)
        s = orc.mc_slope(qm, q0, qp)
        lo, hi = min(qm, q0, qp), max(qm, q0, qp)
        tol = 4e-16 * max(abs(qm), abs(q0), abs(qp))     # rounding of q0 +- s/2
        assert lo - tol <= q0 + 0.5 * s <= hi + tol
        assert lo - tol <= q0 - 0.5 * s <= hi + tol
        if (q0 - qm) * (qp - q0) <= 0:       # extremum: first order
            assert s == 0.0
        else:                                 # same sign as the data, no larger than 2x either jump
            assert s * (qp - qm) > 0
            assert abs(s) <= 2 * min(abs(q0 - qm), abs(qp - q0)) * (1 + 1e-15)
            assert abs(s) <= 0.5 * abs(qp - qm) * (1 + 1e-15)
        assert orc.mc_slope(-qm, -q0, -qp) == -s
        assert orc.mc_slope(qp, q0, qm) == -s


def test_mc_limits_to_twice_the_one_sided_jump(orc):
    assert orc.mc_slope(0.0, 1.0, 10.0) == 2.0
    assert orc.mc_slope(0.0, 9.0, 9.5) == 1.0      # 2 * right jump
    assert orc.mc_slope(9.0, 10.0, 10.5) == 0.75   # centred slope
    assert orc.mc_slope(0.0, 1.0, 2.5) == 1.25     # centred slope


# ---- face solver ----------------------------------------------------------------

def test_face_flux_consistency(orc):
    """Equal left and right states give the physical flux."""
    rng = np.random.default_rng(8)
    for _ in range(200):
        P = random_prim(rng, Wmax=3.0, sigmax=10.0)
        for d in range(3):
            F = orc.point_face_flux(P, P, 5.0 / 3.0, d)
            Fp = orc.point_flux(P, 5.0 / 3.0, d)
            np.testing.assert_allclose(F, Fp, rtol=1e-13, atol=1e-14 * np.abs(Fp).max())


def test_face_flux_supersonic_upwinding(orc):
    """When every signal moves right the flux is the left state's flux (and vice versa)."""
    rng = np.random.default_rng(9)
    gamma = 5.0 / 3.0
    for _ in range(100):
        for sgn in (1, -1):
            qL = np.array([1.0, 0.01, sgn * 20.0, 0.1, 0.0, 0.0, 0.01, 0.0, 0.0])
            qR = qL.copy()
            qL[0] *= 1 + rng.uniform()
            qR[1] *= 1 + rng.uniform()
            qR[3] = -0.1 * rng.uniform()
            F = orc.point_face_flux(qL, qR, gamma, 0)
            up = qL if sgn > 0 else qR
            Fup = orc.point_flux(up, gamma, 0)
            np.testing.assert_array_equal(F[:5], Fup[:5])
            np.testing.assert_array_equal(F[6:8], Fup[6:8])


def test_face_cleaning_pair_is_exact_linear_riemann_solution(orc):
    """The (normal field, Phi) pair: the characteristic variables Phi +- c_h Bn are
    carried from the left and the right state respectively."""
    rng = np.random.default_rng(10)
    for _ in range(100):
        c_h = rng.uniform(0.5, 2.0)
        qL = np.array([1.0, 1.0, 0.1, 0.0, 0.0, rng.normal(), 0.1, 0.0, rng.normal()])
        qR = np.array([0.5, 0.3, 0.0, 0.1, 0.0, rng.normal(), 0.0, 0.2, rng.normal()])
        F = orc.point_face_flux(qL, qR, 5.0 / 3.0, 0, c_h)
        phis, Bs = F[5], F[8] / c_h ** 2
        np.testing.assert_allclose(phis + c_h * Bs, qL[8] + c_h * qL[5], rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(phis - c_h * Bs, qR[8] - c_h * qR[5], rtol=1e-13, atol=1e-14)


def _below_d_states(rng, gamma, psi4, count):
    """States whose recovery root lies below D (Wc = w W^2 < D = rho W, i.e.
    h W < 1): at rest or slow (W <= 1.01) with a negative pressure large
    enough that h = 1 + gamma/(gamma-1) p/rho < 1/W.  Magnetised."""
    out = []
    while len(out) < count:
        rho = 10 ** rng.uniform(-3, 1)
        slow = len(out) % 2 == 1
        W = 1.0 + (10 ** rng.uniform(-6, -2) if slow else 0.0)
        # h W < 1 needs -p/rho > (gamma-1)/gamma (1 - 1/W); take 2-50x that,
        # floored at 1e-8 (at rest any p < 0 has its root below D)
        need = (gamma - 1.0) / gamma * (1.0 - 1.0 / W)
        p = -rho * max(need * 10 ** rng.uniform(np.log10(2.0), np.log10(50.0)), 1e-8 * 10 ** rng.uniform(0, 3))
        if -p / rho >= 0.5 * (gamma - 1.0) / gamma:
            continue                 # keep h > 0 by a margin
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        ut = np.sqrt(W * W - 1.0) * n / np.sqrt(psi4)
        B = rng.normal(size=3) * np.sqrt(rho) * 10 ** rng.uniform(-2, 0)
        P = np.array([rho, p, *ut, *B, 0.0])
        tb = textbook(P, gamma, psi4=psi4)[3]
        assert tb["w"] * tb["W"] ** 2 < rho * tb["W"]       # the root is below D
        out.append(P)
    return out


@pytest.mark.filterwarnings("ignore:invalid value encountered in sqrt")
@pytest.mark.parametrize("metric", ["flat", "curved"])
def test_recovery_root_below_d_negative_pressure(orc, metric):
    """The bracket's search below Wc = D: conserved states of a fluid at rest or
    nearly so (W <= 1.01) with p < 0, built by the textbook formulas, are
    recovered with their negative pressure (the point recovery accepts roots
    with h W < 1); the error bound is the conditioning of p against the
    energy density, as in the round-trip pin."""
    rng = np.random.default_rng(41)
    pts = [(0.0, 0.0, 0.0)] if metric == "flat" else POINTS
    for (x, y, z) in pts:
        alpha, psi4 = (1.0, 1.0) if metric == "flat" else metric_iso(x, y, z)
        mk = {} if metric == "flat" else dict(metric=orc.ISO_SCHW, M=1.0)
        for gamma in GAMMAS:
            for P in _below_d_states(rng, gamma, psi4, 40 // len(pts) + 2):
                U_ref = textbook(P, gamma, alpha=alpha, psi4=psi4)[0]
                P2, ok = orc.point_c2p(U_ref, gamma, x, y, z, **mk)
                assert ok, P
                W = np.sqrt(1 + psi4 * P[2:5] @ P[2:5])
                assert P2[1] < 0.0
                en = (U_ref[1] + U_ref[0]) / U_ref[0]
                assert abs(P2[1] - P[1]) <= 1e-13 * max(abs(P[1]), en * P[0])
                assert abs(P2[0] - P[0]) <= 1e-13 * P[0]
                assert np.abs(P2[2:5] - P[2:5]).max() <= 1e-13 * max(W - 1.0, 1e-3)
                assert np.abs(P2[5:8] - P[5:8]).max() <= 1e-15 * np.abs(P[5:8]).max()


@pytest.mark.filterwarnings("ignore:invalid value encountered in sqrt")
@pytest.mark.parametrize("metric", ["flat", "curved"])
def test_negative_pressure_root_takes_the_pressure_floor(orc, metric):
    """The cell recovery after a root below D: the pressure is raised to p_atm,
    only the pressure-floor flag is set, density, velocity and field keep their
    recovered values, and the matter part of U is rebuilt from the floored
    primitives (textbook formulas); the field and Phi rows are untouched."""
    rng = np.random.default_rng(43)
    gamma = 5.0 / 3.0
    n = 24
    if metric == "flat":
        kw = dict(n=(n, 1, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                  bc=(orc.OUTFLOW,) * 3, gamma=gamma)
        xs = [((i + 0.5) / n, 0.5, 0.5) for i in range(n)]
        geo = [(1.0, 1.0)] * n
    else:
        kw = dict(n=(n, 1, 1), lo=(-3.0, 0.7, -0.4), hi=(9.0, 1.7, 0.6),
                  bc=(orc.OUTFLOW,) * 3, gamma=gamma, metric=orc.ISO_SCHW, M=1.0)
        xs = [(-3.0 + (i + 0.5) * 0.5, 1.2, 0.1) for i in range(n)]
        geo = [metric_iso(*x) for x in xs]
    pb = orc.Problem(rho_atm=1e-10, p_atm=1e-9, **kw)
    Ps = []
    for i in range(n):
        Ps.append(_below_d_states(rng, gamma, geo[i][1], 1 + i % 2)[-1])
    P = np.array(Ps).T.reshape(9, 1, 1, n).copy()
    U = np.zeros_like(P)
    for i in range(n):
        U[:, 0, 0, i] = textbook(P[:, 0, 0, i], gamma, alpha=geo[i][0], psi4=geo[i][1])[0]
    Pn, Ua, flags, st = orc.con2prim(pb, U, P)
    assert np.all(flags == orc.FLAG_PFLOOR)
    assert st == {"fail": 0, "atm": 0, "pfloor": n}
    assert np.all(Pn[1] == pb.p_atm)
    np.testing.assert_allclose(Pn[0], P[0], rtol=1e-13)
    assert np.abs(Pn[2:5] - P[2:5]).max() <= 1e-15
    np.testing.assert_allclose(Pn[5:8], P[5:8], rtol=1e-15, atol=1e-15 * np.abs(P[5:8]).max())
    for i in range(n):
        Pf = Pn[:, 0, 0, i].copy()
        Uf = textbook(Pf, gamma, alpha=geo[i][0], psi4=geo[i][1])[0]
        np.testing.assert_allclose(Ua[:5, 0, 0, i], Uf[:5], rtol=1e-13,
                                   atol=1e-13 * np.abs(Uf[:5]).max())
        assert np.array_equal(Ua[5:, 0, 0, i], U[5:, 0, 0, i])
        # the rebuilt energy carries the raised pressure: it exceeds the input's
        assert Ua[1, 0, 0, i] > U[1, 0, 0, i]
