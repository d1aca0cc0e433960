"""Differentiable FP64 CPU oracle of the GRMHD step (TEST INFRASTRUCTURE ONLY).

The discretisation of the C oracle (conservation form of eq. 2, section 2.2;
scheme choices of section 3.2: MC-limited TVD reconstruction, HLLE fluxes,
SSP Runge-Kutta, Newton primitive recovery, hyperbolic divergence cleaning),
restated with plain PyTorch CPU operations in float64 so that torch.autograd
gives the exact derivative of the discrete step map.  It serves as the
reference gradient for the hand-written adjoint: every quantity is formed
from its textbook definition through full 4x4 contractions, point by point
(vectorised over cells only), without blocking or fusion.

Reading of the recovery's derivative (the paper motivates inverse problems
but gives no adjoint): the primitives P(U) are the root of U(P) = U, so
dP/dU = (dU/dP)^-1 by the implicit function theorem.  The root itself is
taken from the C oracle (no gradient), and the derivative enters through one
linearised correction P = P* + J^-1 (U - U(P*)) with J = dU/dP at P*
detached: its value is P* up to rounding and its derivative is J^-1.
Atmosphere cells (rho reset to rho_atm) have constant hydrodynamic
primitives and pressure-floor cells a constant pressure; the conserved matter
part of both is rebuilt from the final primitives and the field, as in the
forward step, and that rebuild is differentiated too.  A recovery failure has
no derivative and raises.

Only tests/ may import this module.  The GPU path shares nothing with it.
"""
from __future__ import annotations

import numpy as np
import torch

from . import FLAG_ATM, FLAG_FAIL, FLAG_PFLOOR, ISO_SCHW, OUTFLOW, SOFT_SQRT, Problem, con2prim

DT = torch.float64


# ---------------------------------------------------------------------------
# Geometry: static metric, no shift, gamma_ij = psi^4 delta_ij, given in closed
# form (isotropic Schwarzschild with softened radius, or flat).

def geometry(pb: Problem, x, y, z):
    """Metric quantities at points (x, y, z) (tensors of one shape S): alpha,
    sqrt(gamma), sqrt(-g) of shape S; g_{mu nu}, g^{mu nu} of shape S+(4,4);
    dg[..., mu, k, l] = d_mu g_{kl} of shape S+(4,4,4) (mu = 0 is d_t)."""
    x, y, z = torch.broadcast_tensors(*(torch.as_tensor(v, dtype=DT) for v in (x, y, z)))
    S = x.shape
    zero = torch.zeros(S, dtype=DT)
    if pb.metric == ISO_SCHW:
        r = torch.sqrt(x * x + y * y + z * z)
        if pb.soft == SOFT_SQRT:
            rs = torch.sqrt(r * r + pb.r_min * pb.r_min)
            drs = [x / rs, y / rs, z / rs]
        else:
            inside = r <= pb.r_min
            rs = torch.where(inside, torch.full_like(r, pb.r_min), r)
            safe = torch.where(inside, torch.ones_like(r), r)
            drs = [torch.where(inside, zero, c / safe) for c in (x, y, z)]
        h = pb.M / (2.0 * rs)
        dh = -h / rs
        alpha = (1.0 - h) / (1.0 + h)
        psi4 = (1.0 + h) ** 4
        dalpha = [-2.0 / (1.0 + h) ** 2 * dh * c for c in drs]
        dpsi4 = [4.0 * (1.0 + h) ** 3 * dh * c for c in drs]
    else:
        alpha = torch.ones(S, dtype=DT)
        psi4 = torch.ones(S, dtype=DT)
        dalpha = [zero] * 3
        dpsi4 = [zero] * 3
    g = torch.zeros(S + (4, 4), dtype=DT)
    gi = torch.zeros(S + (4, 4), dtype=DT)
    g[..., 0, 0] = -alpha * alpha
    gi[..., 0, 0] = -1.0 / (alpha * alpha)
    for i in range(1, 4):
        g[..., i, i] = psi4
        gi[..., i, i] = 1.0 / psi4
    dg = torch.zeros(S + (4, 4, 4), dtype=DT)
    for i in range(3):
        dg[..., i + 1, 0, 0] = -2.0 * alpha * dalpha[i]
        for j in range(1, 4):
            dg[..., i + 1, j, j] = dpsi4[i]
    sqrtgamma = psi4 ** 1.5
    return {"alpha": alpha, "sqrtgamma": sqrtgamma, "sqrtmg": alpha * sqrtgamma,
            "g": g, "gi": gi, "dg": dg, "gam": g[..., 1:, 1:]}


# ---------------------------------------------------------------------------
# Fluid and field state from the primitives (variable axis last).

def state(G, gamma, q):
    """q[..., 9] = (rho, p, u~^i, B^i, Phi)."""
    rho, p, ut, B, phi = q[..., 0], q[..., 1], q[..., 2:5], q[..., 5:8], q[..., 8]
    W = torch.sqrt(1.0 + torch.einsum("...ij,...i,...j->...", G["gam"], ut, ut))
    u = torch.cat([(W / G["alpha"])[..., None], ut], dim=-1)          # no shift: u^i = u~^i
    ul = torch.einsum("...mn,...n->...m", G["g"], u)
    b0 = (B * ul[..., 1:]).sum(-1)
    bs = (B + b0[..., None] * ut) / u[..., :1]
    b = torch.cat([b0[..., None], bs], dim=-1)
    bl = torch.einsum("...mn,...n->...m", G["g"], b)
    b2 = (b * bl).sum(-1)
    w = rho + gamma / (gamma - 1.0) * p
    return {"rho": rho, "p": p, "B": B, "phi": phi, "W": W, "u": u, "ul": ul, "b": b, "bl": bl,
            "b2": b2, "w": w}


def stress(s):
    """T^mu_nu = (w + b^2) u^mu u_nu + (p + b^2/2) delta^mu_nu - b^mu b_nu."""
    eye = torch.eye(4, dtype=DT)
    return ((s["w"] + s["b2"])[..., None, None] * s["u"][..., :, None] * s["ul"][..., None, :]
            + (s["p"] + 0.5 * s["b2"])[..., None, None] * eye
            - s["b"][..., :, None] * s["bl"][..., None, :])


def cons(G, s):
    T = stress(s)
    sg = G["sqrtmg"]
    out = [sg * s["rho"] * s["u"][..., 0], -sg * (T[..., 0, 0] + s["rho"] * s["u"][..., 0])]
    out += [sg * T[..., 0, j] for j in range(1, 4)]
    out += [sg * s["B"][..., j] for j in range(3)]
    out += [s["phi"]]
    return torch.stack(out, dim=-1)


def flux(G, s, c_h, d):
    """Physical flux along axis d with the cleaning terms."""
    T = stress(s)
    sg = G["sqrtmg"]
    i = d + 1
    u, b = s["u"], s["b"]
    out = [sg * s["rho"] * u[..., i], -sg * (T[..., i, 0] + s["rho"] * u[..., i])]
    out += [sg * T[..., i, j] for j in range(1, 4)]
    for j in range(3):
        f = sg * (b[..., j + 1] * u[..., i] - b[..., i] * u[..., j + 1])
        if j == d:
            f = f + s["phi"]
        out.append(f)
    out.append(c_h * c_h * sg * s["B"][..., d])
    return torch.stack(out, dim=-1)


def speeds(G, s, gamma, d):
    i = d + 1
    cs2 = gamma * s["p"] / s["w"]
    ca2 = s["b2"] / (s["w"] + s["b2"])
    c2 = cs2 + ca2 - cs2 * ca2
    ut, ui = s["u"][..., 0], s["u"][..., i]
    A = ut * ut - c2 * (G["gi"][..., 0, 0] + ut * ut)
    Bq = ut * ui - c2 * (G["gi"][..., 0, i] + ut * ui)
    Cq = ui * ui - c2 * (G["gi"][..., i, i] + ui * ui)
    disc = torch.clamp(Bq * Bq - A * Cq, min=0.0)
    sq = torch.sqrt(disc)
    l1 = (Bq + sq) / A
    l2 = (Bq - sq) / A
    return torch.minimum(l1, l2), torch.maximum(l1, l2)


def source(G, s, kappa):
    """1/2 sqrt(-g) T^{kl} d_mu g_{kl} in the momentum and energy rows, -kappa Phi."""
    T = stress(s)
    Tuu = torch.einsum("...kn,...nl->...kl", T, G["gi"])
    src = 0.5 * G["sqrtmg"][..., None] * torch.einsum("...kl,...mkl->...m", Tuu, G["dg"])
    zero = torch.zeros_like(s["rho"])
    return torch.stack([zero, -src[..., 0], src[..., 1], src[..., 2], src[..., 3], zero, zero,
                        zero, -kappa * s["phi"]], dim=-1)


# ---------------------------------------------------------------------------
# Reconstruction and interface fluxes.

def minmod3(a, b, c):
    """The argument of least magnitude when all three share a sign, else 0.
    At exact ties of magnitude the derivative follows one argument, in the
    order a, c, b (a kink has no derivative; this is the convention taken)."""
    pos = (a > 0) & (b > 0) & (c > 0)
    neg = (a < 0) & (b < 0) & (c < 0)
    zero = torch.zeros_like(a)
    ma, mb, mc = a.abs(), b.abs(), c.abs()
    take_a = (ma <= mc) & (ma <= mb)
    take_c = ~take_a & (mc <= mb)
    least = torch.where(take_a, a, torch.where(take_c, c, b))
    return torch.where(pos | neg, least, zero)


def mc_slope(qm, q0, qp):
    return minmod3(2.0 * (q0 - qm), 0.5 * (qp - qm), 2.0 * (qp - q0))


def face_flux(G, gamma, c_h, d, qL, qR):
    """HLLE flux with the (normal field, Phi) pair solved exactly first."""
    sg = G["sqrtmg"]
    BnL, BnR = sg * qL[..., 5 + d], sg * qR[..., 5 + d]
    Bs = 0.5 * (BnL + BnR) - (qR[..., 8] - qL[..., 8]) / (2.0 * c_h)
    phis = 0.5 * (qL[..., 8] + qR[..., 8]) - 0.5 * c_h * (BnR - BnL)
    col = torch.arange(9) == 5 + d
    qL = torch.where(col, (Bs / sg)[..., None], qL)
    qR = torch.where(col, (Bs / sg)[..., None], qR)
    sL, sR = state(G, gamma, qL), state(G, gamma, qR)
    FL, FR = flux(G, sL, c_h, d), flux(G, sR, c_h, d)
    UL, UR = cons(G, sL), cons(G, sR)
    lmL, lpL = speeds(G, sL, gamma, d)
    lmR, lpR = speeds(G, sR, gamma, d)
    zero = torch.zeros_like(lmL)
    # extreme speeds; at an exact tie (identical states) the derivative goes
    # through the left state's speed, the convention of a kink taken here
    sl = torch.minimum(zero, torch.where(lmL <= lmR, lmL, lmR))[..., None]
    sr = torch.maximum(zero, torch.where(lpL >= lpR, lpL, lpR))[..., None]
    hll = (sr * FL - sl * FR + sl * sr * (UR - UL)) / torch.where(sr - sl == 0, 1.0, sr - sl)
    F = torch.where(sl == 0, FL, torch.where(sr == 0, FR, hll))
    F = torch.where(col, phis[..., None], F)
    return torch.where(torch.arange(9) == 8, (c_h * c_h * Bs)[..., None], F)


# ---------------------------------------------------------------------------
# Grid operations.  Fields are torch float64 [9, nz, ny, nx].

def _axis(d):
    return 3 - d          # tensor axis of spatial direction d in [9, nz, ny, nx]


def _centres(pb, d):
    n = pb.n[d]
    dx = (pb.hi[d] - pb.lo[d]) / n
    return pb.lo[d] + (torch.arange(n, dtype=DT) + 0.5) * dx


def _points(pb, face_dir=None):
    xs = []
    for d in range(3):
        if d == face_dir:
            dx = (pb.hi[d] - pb.lo[d]) / pb.n[d]
            xs.append(pb.lo[d] + torch.arange(pb.n[d] + 1, dtype=DT) * dx)
        else:
            xs.append(_centres(pb, d))
    Z, Y, X = torch.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X, Y, Z


def _ghost_index(n, bc, lo, hi):
    idx = torch.arange(lo, hi)
    if bc == OUTFLOW:
        return idx.clamp(0, n - 1)
    return idx % n


def rhs(pb: Problem, P):
    """Right-hand side -sum_d dF_d/dx_d + sources at the primitives P."""
    Pl = P.movedim(0, -1)                                      # [nz, ny, nx, 9]
    R = torch.zeros_like(Pl)
    for d in range(3):
        n = pb.n[d]
        if n == 1:
            continue
        ax = _axis(d) - 1                                      # axis of Pl
        dx = (pb.hi[d] - pb.lo[d]) / n
        # cells f-2 .. f+1 around face f (f = 0 .. n), ghosts by the boundary rule
        q = [Pl.index_select(ax, _ghost_index(n, pb.bc[d], s - 2, n + s - 1)) for s in range(4)]
        qL = q[1] + 0.5 * mc_slope(q[0], q[1], q[2])
        qR = q[2] - 0.5 * mc_slope(q[1], q[2], q[3])
        G = geometry(pb, *_points(pb, d))
        F = face_flux(G, pb.gamma, pb.c_h, d, qL, qR)
        hi_ = F.narrow(ax, 1, n)
        lo_ = F.narrow(ax, 0, n)
        R = R - (hi_ - lo_) / dx
    G = geometry(pb, *_points(pb))
    R = R + source(G, state(G, pb.gamma, Pl), pb.kappa)
    return R.movedim(-1, 0)


def prim2con(pb: Problem, P):
    G = geometry(pb, *_points(pb))
    Pl = P.movedim(0, -1)
    return cons(G, state(G, pb.gamma, Pl)).movedim(-1, 0)


def cons_jacobian(pb: Problem, P):
    """dU/dP per cell, [nz, ny, nx, 9, 9] (row: conserved, column: primitive)."""
    G = geometry(pb, *_points(pb))
    Pl = P.detach().movedim(0, -1)
    cols = []
    for j in range(9):
        t = torch.zeros_like(Pl)
        t[..., j] = 1.0
        _, jv = torch.func.jvp(lambda q: cons(G, state(G, pb.gamma, q)), (Pl,), (t,))
        cols.append(jv)
    return torch.stack(cols, dim=-1)


def recover(pb: Problem, U, Pguess):
    """Primitives of U and U with the floored cells' matter part rebuilt,
    differentiable through the implicit relation U(P) = U.  Atmosphere cells
    take constant hydrodynamic primitives; pressure-floor cells keep the
    root's rho and u~ and take the constant floor pressure; both rebuild
    their conserved matter part from the final primitives and the field."""
    Ps, Uadj, flags, st = con2prim(pb, U.detach().numpy(), np.ascontiguousarray(
        Pguess.detach().numpy()))
    if (flags & FLAG_FAIL).any():
        raise ValueError("recovery failure: derivative not defined")
    Pd = torch.from_numpy(Ps)
    atm = torch.from_numpy((flags & FLAG_ATM) != 0)
    pfl = torch.from_numpy((flags & FLAG_PFLOOR) != 0) & ~atm
    G = geometry(pb, *_points(pb))
    # U(P) is affine in p at fixed (rho, u~, B), so in a pressure-floor cell
    # the correction below restores the root's pressure exactly before the
    # floor is applied again; its derivative is J^-1 as everywhere else
    J = cons_jacobian(pb, Pd)
    r = (U - prim2con(pb, Pd)).movedim(0, -1)
    r = torch.where(atm[..., None], torch.zeros_like(r), r)
    P = Pd + torch.linalg.solve(J, r.unsqueeze(-1)).squeeze(-1).movedim(-1, 0)
    field = torch.cat([U[5:8] / G["sqrtmg"], U[8:9]], dim=0)
    hydro = torch.tensor([pb.rho_atm, pb.p_atm, 0.0, 0.0, 0.0], dtype=DT)
    Patm = torch.cat([hydro.view(5, 1, 1, 1).expand(5, *U.shape[1:]), field], dim=0)
    P = torch.where(atm, Patm, P)
    pcol = (torch.arange(9) == 1).view(9, 1, 1, 1)
    P = torch.where(pfl & pcol, torch.full_like(P, pb.p_atm), P)
    reb = atm | pfl
    if reb.any():
        Ur = prim2con(pb, P)
        U = torch.where(reb & (torch.arange(9) < 5).view(9, 1, 1, 1), Ur, U)
    return P, U


def primitives_of(pb: Problem, U, Pguess):
    """The primitives of U at the start of a step, P^n = P(U^n): the value
    of the C oracle's recovery (floors included; U itself is not rebuilt,
    the state is taken as it stands) with the derivative of the exact
    inverse, dP/dU = (dU/dP)^-1 at that value, in every cell."""
    Ps, _, flags, _ = con2prim(pb, U.detach().numpy(), np.ascontiguousarray(Pguess.detach().numpy()))
    if (flags & FLAG_FAIL).any():
        raise ValueError("recovery failure: derivative not defined")
    Pd = torch.from_numpy(Ps)
    J = cons_jacobian(pb, Pd)
    dU = (U - U.detach()).movedim(0, -1)
    return Pd + torch.linalg.solve(J, dU.unsqueeze(-1)).squeeze(-1).movedim(-1, 0)


RK = {2: ((0.0, 1.0), (0.5, 0.5)), 3: ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))}


def step(pb: Problem, U, P, dt, nsteps=1):
    """nsteps SSP-RK steps from (U, P) with P the primitives of U; each
    stage uses the primitives of the previous recovery, as the forward scheme
    does.  Differentiable in both U and P."""
    for _ in range(nsteps):
        Un = U
        for a, b in RK[pb.rk_order]:
            U = U + a * (Un - U) + b * (dt * rhs(pb, P))
            P, U = recover(pb, U, P)
    return U, P
