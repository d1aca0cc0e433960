// grmhd_adjoint.h -- reverse-mode (adjoint) versions of the point physics in
// grmhd_device.h, FP64 only.
//
// Each *_rev function takes the forward inputs (recomputed by the caller),
// the cotangent of the forward output, and ACCUMULATES (+=) the cotangents of
// the inputs.  Branches (MC limiter, HLLE signal-speed min/max and upwind
// cases) take the derivative of the branch the forward evaluation took.
#pragma once

#include "grmhd_device.h"

namespace grmhd {

// Cotangents of the fluid-frame quantities of one state.
struct KinBar {
    double W, bt, b[3], b2, w, wtot, ptot;
};

__device__ __forceinline__ KinBar kin_zero()
{
    KinBar k;
    k.W = k.bt = k.b2 = k.w = k.wtot = k.ptot = 0.0;
    k.b[0] = k.b[1] = k.b[2] = 0.0;
    return k;
}

// Reverse of kinematics(): kb -> qb (primitives 0..7).
__device__ __forceinline__ void kinematics_rev(const double* q, const Kin<double>& k, const GeoT<double>& g,
                                               double gfac, KinBar kb, double* qb)
{
    const double u[3] = {q[2], q[3], q[4]};
    const double B[3] = {q[5], q[6], q[7]};
    const double f = g.alpha / k.W;
    // ptot = p + b2/2, wtot = w + b2, w = rho + gfac p
    qb[1] += kb.ptot;
    kb.b2 += 0.5 * kb.ptot;
    kb.w += kb.wtot;
    kb.b2 += kb.wtot;
    qb[0] += kb.w;
    qb[1] += gfac * kb.w;
    // b2 = (psi4 |B|^2 + bt^2) f^2
    const double BB = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double fb = kb.b2 * (g.psi4 * BB + k.bt * k.bt) * 2.0 * f;
    const double c2 = kb.b2 * f * f;
    kb.bt += c2 * 2.0 * k.bt;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        qb[5 + i] += c2 * 2.0 * g.psi4 * B[i];
    // b^i = (B^i + bt u^i) f
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        qb[5 + i] += kb.b[i] * f;
        kb.bt += kb.b[i] * u[i] * f;
        qb[2 + i] += kb.b[i] * k.bt * f;
        fb += kb.b[i] * (B[i] + k.bt * u[i]);
    }
    // bt = psi4 B.u
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        qb[5 + i] += kb.bt * g.psi4 * u[i];
        qb[2 + i] += kb.bt * g.psi4 * B[i];
    }
    // f = alpha / W, W = sqrt(1 + psi4 |u|^2)
    const double Wb = kb.W - fb * f / k.W;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        qb[2 + i] += Wb * g.psi4 * u[i] / k.W;
}

// Reverse of speeds<D>(): (lmb, lpb) -> qb, kb.
template <int D>
__device__ __forceinline__ void speeds_rev(const double* q, const Kin<double>& k, const GeoT<double>& g,
                                           double gamma, double lmb, double lpb, double* qb, KinBar& kb)
{
    const double inv = 1.0 / k.wtot;
    const double c2 = (k.b2 + gamma * q[1]) * inv;
    const double a = (k.w - gamma * q[1]) * inv;
    const double qi = q[2 + D];
    const double den = k.W * k.W * a + c2;
    const double disc = c2 * (den * g.ipsi4 - qi * qi * a);
    const double s = sqrt(fmax(disc, 0.0));
    const double t = g.alpha / den;
    const double m = k.W * qi * a;
    const double mb = (lpb + lmb) * t;
    const double sb = (lpb - lmb) * t;
    const double tb = lpb * (m + s) + lmb * (m - s);
    double denb = -tb * t / den;
    const double discb = disc > 0.0 ? sb / (2.0 * s) : 0.0;
    double c2b = discb * (den * g.ipsi4 - qi * qi * a);
    denb += discb * c2 * g.ipsi4;
    double qib = -discb * c2 * 2.0 * qi * a;
    double ab = -discb * c2 * qi * qi;
    kb.W += mb * qi * a;
    qib += mb * k.W * a;
    ab += mb * k.W * qi;
    kb.W += denb * 2.0 * k.W * a;
    ab += denb * k.W * k.W;
    c2b += denb;
    kb.w += ab * inv;
    qb[1] += (c2b - ab) * gamma * inv;
    kb.b2 += c2b * inv;
    const double invb = ab * (k.w - gamma * q[1]) + c2b * (k.b2 + gamma * q[1]);
    kb.wtot -= invb * inv * inv;
    qb[2 + D] += qib;
}

// Reverse of flux_comp<D>(v, ...) with cotangent c.
template <int D>
__device__ __forceinline__ void flux_comp_rev(int v, const double* q, const Kin<double>& k,
                                              const GeoT<double>& g, double c, double* qb, KinBar& kb)
{
    const double uD = q[2 + D];
    const double cs = c * g.sqrtmg;
    switch (v) {
    case 0:
        qb[0] += cs * uD;
        qb[2 + D] += cs * q[0];
        break;
    case 1:
        kb.wtot += cs * g.alpha * k.W * uD;
        kb.W += cs * k.wtot * g.alpha * uD;
        qb[0] -= cs * uD;
        qb[2 + D] += cs * (k.wtot * g.alpha * k.W - q[0]);
        kb.bt -= cs * g.alpha * g.alpha * k.b[D];
        kb.b[D] -= cs * g.alpha * g.alpha * k.bt;
        break;
    case 2:
    case 3:
    case 4: {
        const int j = v - 2;
        const double cp = cs * g.psi4;
        kb.wtot += cp * uD * q[2 + j];
        qb[2 + D] += cp * k.wtot * q[2 + j];
        qb[2 + j] += cp * k.wtot * uD;
        kb.b[D] -= cp * k.b[j];
        kb.b[j] -= cp * k.b[D];
        if (j == D)
            kb.ptot += cs;
        break;
    }
    default: {
        const int j = v - 5;
        kb.b[j] += cs * uD;
        qb[2 + D] += cs * k.b[j];
        kb.b[D] -= cs * q[2 + j];
        qb[2 + j] -= cs * k.b[D];
    }
    }
}

// Reverse of cons_comp(v, ...) with cotangent c.
__device__ __forceinline__ void cons_comp_rev(int v, const double* q, const Kin<double>& k,
                                              const GeoT<double>& g, double c, double* qb, KinBar& kb)
{
    switch (v) {
    case 0:
        qb[0] += c * g.sqrtg * k.W;
        kb.W += c * g.sqrtg * q[0];
        break;
    case 1:
        kb.wtot += c * g.sqrtmg * k.W * k.W;
        kb.W += c * (2.0 * g.sqrtmg * k.wtot * k.W - g.sqrtg * q[0]);
        kb.ptot -= c * g.sqrtmg;
        kb.bt -= 2.0 * c * g.sqrtmg * g.alpha * g.alpha * k.bt;
        qb[0] -= c * g.sqrtg * k.W;
        break;
    case 2:
    case 3:
    case 4: {
        const int j = v - 2;
        const double cp = c * g.psi4;
        kb.wtot += cp * g.sqrtg * k.W * q[2 + j];
        kb.W += cp * g.sqrtg * k.wtot * q[2 + j];
        qb[2 + j] += cp * g.sqrtg * k.wtot * k.W;
        kb.bt -= cp * g.sqrtmg * k.b[j];
        kb.b[j] -= cp * g.sqrtmg * k.bt;
        break;
    }
    default:
        qb[v] += c * g.sqrtmg;
    }
}

// Derivative of the MC slope with respect to (qm, q0, qp) on the branch the
// forward evaluation takes.
__device__ __forceinline__ void mc_slope_grad(double qm, double q0, double qp, double& dm, double& d0,
                                              double& dp)
{
    const double dl = q0 - qm, dr = qp - q0, dc = 0.5 * (qp - qm);
    dm = d0 = dp = 0.0;
    if (!(dl * dr > 0.0))
        return;
    const double al = 2.0 * fabs(dl), ar = 2.0 * fabs(dr), ac = fabs(dc);
    if (al <= ar && al <= ac) {          // 2 dl
        dm = -2.0;
        d0 = 2.0;
    } else if (ar <= ac) {               // 2 dr
        d0 = -2.0;
        dp = 2.0;
    } else {                             // (qp - qm) / 2
        dm = -0.5;
        dp = 0.5;
    }
}

// The 5x8 block d(D, tau, S)/d(rho, p, u~, B) of the conserved variables at
// one point, row r in J[r][0..7].
__device__ __forceinline__ void cons_jacobian(const double* q, const GeoT<double>& g, double gfac,
                                              double J[5][8])
{
    const Kin<double> k = kinematics(q, g, gfac);
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        double row[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        KinBar kb = kin_zero();
        cons_comp_rev(r, q, k, g, 1.0, row, kb);
        kinematics_rev(q, k, g, gfac, kb, row);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            J[r][c] = row[c];
    }
}

// Solve A^T x = y for the 5x5 block A = J[0..4][0..4]: Gaussian elimination
// with partial pivoting on the transposed matrix, the pivot row found by
// successive conditional swaps so that every index is a compile-time
// constant (the matrix stays in registers).  Returns false if singular.
__device__ __forceinline__ bool solve5_transposed(const double J[5][8], const double* y, double* x)
{
    double M[5][6];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
#pragma unroll
        for (int c = 0; c < 5; ++c)
            M[r][c] = J[c][r];
        M[r][5] = y[r];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
#pragma unroll
        for (int r = c + 1; r < 5; ++r) {
            const bool sw = fabs(M[r][c]) > fabs(M[c][c]);
#pragma unroll
            for (int e = c; e < 6; ++e) {
                const double a = M[c][e], b = M[r][e];
                M[c][e] = sw ? b : a;
                M[r][e] = sw ? a : b;
            }
        }
        if (!(fabs(M[c][c]) > 0.0))
            return false;
        const double inv = 1.0 / M[c][c];
#pragma unroll
        for (int r = c + 1; r < 5; ++r) {
            const double f = M[r][c] * inv;
#pragma unroll
            for (int e = c; e < 6; ++e)
                M[r][e] -= f * M[c][e];
        }
    }
#pragma unroll
    for (int r = 4; r >= 0; --r) {
        double s = M[r][5];
#pragma unroll
        for (int e = r + 1; e < 5; ++e)
            s -= M[r][e] * x[e];
        x[r] = s / M[r][r];
    }
    return true;
}

// y (cotangent of the primitives) -> x = (dU/dP)^-T y (cotangent of the
// conserved variables) at the primitives q.  With the block structure of
// dU/dP: the matter block A^T, then the field (U_B = sqrt(-g) B), then Phi.
__device__ __forceinline__ bool cons_jacobian_solve_t(const double J[5][8], double sqrtmg, const double* y,
                                                      double* x)
{
    if (!solve5_transposed(J, y, x))
        return false;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double s = y[5 + j];
#pragma unroll
        for (int r = 0; r < 5; ++r)
            s -= J[r][5 + j] * x[r];
        x[5 + j] = s / sqrtmg;
    }
    x[8] = y[8];
    return true;
}

}  // namespace grmhd
