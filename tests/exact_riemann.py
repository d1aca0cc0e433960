"""Exact solution of the special-relativistic hydrodynamic Riemann problem with
zero tangential velocity and an ideal-gas EOS (test infrastructure).

Written from the jump conditions and the Riemann invariants, following the
published method of Marti & Mueller (J. Fluid Mech. 1994): the pressure p* of
the intermediate states is found where the velocities behind the left and the
right wave agree.  Behind a shock the state follows from the Taub adiabat and
the relativistic Rankine-Hugoniot mass flux; across a rarefaction the entropy
and the Riemann invariant
    J(+/-) = 1/2 ln((1+v)/(1-v)) +/- 1/sqrt(G-1) ln((sqrt(G-1)+c)/(sqrt(G-1)-c))
are constant.  Used only to pin the CPU oracle.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def _h(rho, p, g):
    return 1.0 + g / (g - 1.0) * p / rho


def _cs(rho, p, g):
    return np.sqrt(g * p / (rho * _h(rho, p, g)))


def _log_c(c, g):
    s = np.sqrt(g - 1.0)
    return np.log((s + c) / (s - c)) / s


def _rapidity(v):
    return 0.5 * np.log((1.0 + v) / (1.0 - v))


def _from_rapidity(r):
    return np.tanh(r)


def _rarefaction_v(pb, rho_a, p_a, v_a, g, side):
    """Velocity behind a rarefaction reaching pressure pb (side -1 = left wave)."""
    rho_b = rho_a * (pb / p_a) ** (1.0 / g)
    ca, cb = _cs(rho_a, p_a, g), _cs(rho_b, pb, g)
    # left wave: J+ constant -> rapidity_b = rapidity_a + logc(a) - logc(b)
    # right wave: J- constant -> rapidity_b = rapidity_a - logc(a) + logc(b)
    if side < 0:
        r = _rapidity(v_a) + _log_c(ca, g) - _log_c(cb, g)
    else:
        r = _rapidity(v_a) - _log_c(ca, g) + _log_c(cb, g)
    return _from_rapidity(r), rho_b


def _shock(pb, rho_a, p_a, v_a, g, side):
    """State behind a shock of strength pb > p_a; returns (v_b, rho_b, V_shock)."""
    ha = _h(rho_a, p_a, g)
    # Taub adiabat h_b^2 - h_a^2 = (h_a/rho_a + h_b/rho_b)(p_b - p_a) with
    # rho_b = g p_b / ((g-1)(h_b - 1)) -> quadratic in h_b
    k = (g - 1.0) / (g * pb)
    A = 1.0 + k * (p_a - pb)
    B = -k * (p_a - pb)
    Cc = ha * (p_a - pb) / rho_a - ha * ha
    hb = (-B + np.sqrt(B * B - 4.0 * A * Cc)) / (2.0 * A)
    rho_b = g * pb / ((g - 1.0) * (hb - 1.0))
    j2 = -(p_a - pb) / (ha / rho_a - hb / rho_b)
    j = np.sqrt(j2) * (1.0 if side > 0 else -1.0)
    Wa = 1.0 / np.sqrt(1.0 - v_a * v_a)
    Vs = (rho_a ** 2 * Wa ** 2 * v_a + j * np.sqrt(j2 + rho_a ** 2 * Wa ** 2 * (1.0 - v_a ** 2))) \
        / (rho_a ** 2 * Wa ** 2 + j2)
    Ws = 1.0 / np.sqrt(1.0 - Vs * Vs)
    vb = (ha * Wa * v_a + Ws * (pb - p_a) / j) / (ha * Wa + (pb - p_a) * (Ws * v_a / j + 1.0 / (rho_a * Wa)))
    return vb, rho_b, Vs


def _v_behind(pb, rho_a, p_a, v_a, g, side):
    if pb > p_a:
        return _shock(pb, rho_a, p_a, v_a, g, side)[0]
    return _rarefaction_v(pb, rho_a, p_a, v_a, g, side)[0]


def solve(rhoL, pL, vL, rhoR, pR, vR, g):
    f = lambda p: _v_behind(p, rhoL, pL, vL, g, -1) - _v_behind(p, rhoR, pR, vR, g, +1)
    lo, hi = 1e-12 * min(pL, pR), 10.0 * max(pL, pR)
    while f(hi) > 0:
        hi *= 10.0
    ps = brentq(f, lo, hi, xtol=1e-15, rtol=1e-14, maxiter=500)
    vs = _v_behind(ps, rhoL, pL, vL, g, -1)
    return ps, vs


def sample(x, t, x0, rhoL, pL, vL, rhoR, pR, vR, g):
    """Density, pressure and velocity of the exact solution at positions x, time t."""
    ps, vs = solve(rhoL, pL, vL, rhoR, pR, vR, g)
    xi = (np.asarray(x) - x0) / t
    rho = np.empty_like(xi)
    p = np.empty_like(xi)
    v = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s < vs:      # left of the contact
            side, ra, pa, va = -1, rhoL, pL, vL
        else:
            side, ra, pa, va = +1, rhoR, pR, vR
        if ps > pa:     # shock
            vb, rb, Vs = _shock(ps, ra, pa, va, g, side)
            ahead = (s < Vs) if side < 0 else (s > Vs)
            if ahead:
                rho[n], p[n], v[n] = ra, pa, va
            else:
                rho[n], p[n], v[n] = rb, ps, vs
        else:           # rarefaction
            vb, rb = _rarefaction_v(ps, ra, pa, va, g, side)
            ca, cb = _cs(ra, pa, g), _cs(rb, ps, g)
            if side < 0:
                head = (va - ca) / (1.0 - va * ca)
                tail = (vb - cb) / (1.0 - vb * cb)
            else:
                head = (va + ca) / (1.0 + va * ca)
                tail = (vb + cb) / (1.0 + vb * cb)
            inside = (head <= s <= tail) if side < 0 else (tail <= s <= head)
            outside = (s < head) if side < 0 else (s > head)
            if outside:
                rho[n], p[n], v[n] = ra, pa, va
            elif inside:
                # self-similar fan: characteristic speed equals xi, invariant fixed
                def g_of(pp):
                    vv, rr = _rarefaction_v(pp, ra, pa, va, g, side)
                    cc = _cs(rr, pp, g)
                    lam = (vv - cc) / (1.0 - vv * cc) if side < 0 else (vv + cc) / (1.0 + vv * cc)
                    return lam - s
                pp = brentq(g_of, ps, pa, xtol=1e-15, rtol=1e-13, maxiter=500)
                vv, rr = _rarefaction_v(pp, ra, pa, va, g, side)
                rho[n], p[n], v[n] = rr, pp, vv
            else:
                rho[n], p[n], v[n] = rb, ps, vs
    return rho, p, v
