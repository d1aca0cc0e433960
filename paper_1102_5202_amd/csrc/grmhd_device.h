// grmhd_device.h -- device-side physics of the GRMHD substep for gfx950.
//
// Static metric without shift, gamma_ij = psi^4 delta_ij (FLAT: alpha = psi = 1),
// so every 4-tensor contraction collapses to a few scalar products.  Formulas
// follow eq. 2 of the paper (conserved variables, fluxes, Christoffel source)
// and the 3+1 primitive recovery of Noble et al. (2006) named in section 3.2.
#pragma once

#include <hip/hip_runtime.h>

namespace grmhd {

enum { FLAT = 0, ISO = 1, STORED = 2 };

// Per-launch constants (passed by value as a kernel argument).
struct Dev {
    int n[3];        // interior cells
    int g[3];        // ghost width per axis (2, or 3 with PPM, on active axes; 0 otherwise)
    int act[3];      // axis active (n > 1)
    int bc[3];       // 0 periodic, 1 outflow
    int px, py, pz;  // dimensions of the ghosted primitive cache (px is the pitch)
    long long sv;    // per-variable stride of the cache
    long long N;     // interior cell count
    long long nf[3]; // face count per direction
    double lo[3], dx[3], idx[3];
    // metric
    double M, rmin, rmin2;
    int soft;        // 0 sqrt(r^2 + r_min^2), 1 max(r, r_min)
    // equation of state and scheme
    double gamma, gk, gfac;   // gamma, (gamma-1)/gamma, gamma/(gamma-1)
    double c_h, ic_h, c_h2, kappa;
    double rho_atm, p_atm, tol;
    int maxit;
    int c2p1d;       // recovery: 0 Newton on (Wc, v^2), 1 Newton on Wc alone
    int ppm;         // reconstruction: 0 MC (2 ghosts), 1 PPM (3 ghosts)
    int ct;          // divergence control: 0 cleaning (Phi), 1 flux-CT (Phi carried)
    int nt;          // grid past the last-level cache: the kernel instances that
                     // stream once-touched arrays with nontemporal accesses
    // stored metric: at cell centres [8][N] (alpha, psi^4, d_x,y,z alpha,
    // d_x,y,z psi^4), at the faces of axis a [2][nf[a]] (alpha, psi^4)
    const double* mc;
    const double* mf[3];
};

// Geometry at one point.
struct Geo {
    double alpha, psi4, ipsi4, sqrtg, sqrtmg, isqrtmg;
};

// 1/r_s at a point (r_s the softened radius); varying is false where r_s is
// constant (MAX softening inside r_min: derivatives vanish).
__device__ __forceinline__ double soft_iradius(const Dev& d, double r2, bool& varying)
{
    if (d.soft == 0) {
        varying = true;
        return rsqrt(r2 + d.rmin2);
    }
    varying = r2 > d.rmin2;
    return rsqrt(varying ? r2 : d.rmin2);
}

// The isotropic metric from h = M / (2 r_s) < 1: alpha = (1-h)/(1+h),
// psi = 1 + h, with one division for 1/(1+h) and 1/(1-h).
__device__ __forceinline__ Geo geo_from_h(double h, double& i1h)
{
    Geo g;
    const double q = 1.0 / ((1.0 - h) * (1.0 + h));
    i1h = (1.0 - h) * q;                  // 1 / (1 + h)
    const double im1h = (1.0 + h) * q;    // 1 / (1 - h)
    const double psi = 1.0 + h;
    const double psi2 = psi * psi;
    const double i2 = i1h * i1h;
    g.alpha = (1.0 - h) * i1h;
    g.psi4 = psi2 * psi2;
    g.ipsi4 = i2 * i2;
    g.sqrtg = g.psi4 * psi2;
    g.sqrtmg = g.alpha * g.sqrtg;
    g.isqrtmg = im1h * i1h * g.ipsi4;     // 1 / ((1 - h) (1 + h)^5)
    return g;
}

// The geometry of a static, conformally flat metric from its lapse and psi^4.
__device__ __forceinline__ Geo geo_from_ap(double alpha, double psi4)
{
    Geo g;
    g.alpha = alpha;
    g.psi4 = psi4;
    g.ipsi4 = 1.0 / psi4;
    g.sqrtg = psi4 * sqrt(psi4);
    g.sqrtmg = alpha * g.sqrtg;
    g.isqrtmg = 1.0 / g.sqrtmg;
    return g;
}

template <int KIND>
__device__ __forceinline__ Geo geo_at(const Dev& d, double x, double y, double z)
{
    if (KIND == FLAT) {
        Geo g;
        g.alpha = g.psi4 = g.ipsi4 = g.sqrtg = g.sqrtmg = g.isqrtmg = 1.0;
        return g;
    }
    bool vary;
    const double irs = soft_iradius(d, x * x + y * y + z * z, vary);
    double i1h;
    return geo_from_h(0.5 * d.M * irs, i1h);
}

// Geometry plus the radial derivative factors at a cell centre:
// d_j alpha = ka * x_j and d_j psi^4 = kp * x_j.
template <int KIND>
__device__ __forceinline__ Geo geo_deriv(const Dev& d, double x, double y, double z, double& ka,
                                         double& kp)
{
    if (KIND == FLAT) {
        Geo g;
        g.alpha = g.psi4 = g.ipsi4 = g.sqrtg = g.sqrtmg = g.isqrtmg = 1.0;
        ka = kp = 0.0;
        return g;
    }
    bool vary;
    const double irs = soft_iradius(d, x * x + y * y + z * z, vary);
    const double h = 0.5 * d.M * irs;
    double i1h;
    const Geo g = geo_from_h(h, i1h);
    const double psi = 1.0 + h;
    const double hr2 = vary ? h * irs * irs : 0.0;
    // d alpha/d r_s = 2 h / (r_s (1+h)^2), d psi^4/d r_s = -4 psi^3 h / r_s, d r_s/d x_j = x_j / r_s
    ka = 2.0 * hr2 * i1h * i1h;
    kp = -4.0 * psi * psi * psi * hr2;
    return g;
}

// Geometry at face f of axis D (position x, y, z) and at the centre of cell c
// (position x, y, z): closed form, or the stored values.
template <int D, int KIND>
__device__ __forceinline__ Geo face_geo(const Dev& d, double x, double y, double z, long long f)
{
    if (KIND == STORED)
        return geo_from_ap(d.mf[D][f], d.mf[D][d.nf[D] + f]);
    return geo_at<KIND>(d, x, y, z);
}

template <int KIND>
__device__ __forceinline__ Geo cell_geo(const Dev& d, double x, double y, double z, long long c)
{
    if (KIND == STORED)
        return geo_from_ap(d.mc[c], d.mc[d.N + c]);
    return geo_at<KIND>(d, x, y, z);
}

// The face physics below is written for a scalar type T: double for the FP64
// path, float for the mixed-precision path (reconstruction, face physics,
// HLLE and sources in FP32; the metric is evaluated in FP64 and rounded once;
// the Runge-Kutta accumulation and the recovery stay in FP64).  Every literal
// is a T so that no expression silently promotes to double.
template <typename T>
struct GeoT {
    T alpha, psi4, ipsi4, sqrtg, sqrtmg, isqrtmg;
};

template <typename T>
__device__ __forceinline__ GeoT<T> geo_cast(const Geo& g)
{
    GeoT<T> r;
    r.alpha = (T)g.alpha;
    r.psi4 = (T)g.psi4;
    r.ipsi4 = (T)g.ipsi4;
    r.sqrtg = (T)g.sqrtg;
    r.sqrtmg = (T)g.sqrtmg;
    r.isqrtmg = (T)g.isqrtmg;
    return r;
}

// Fluid-frame quantities of one state (W, b^mu, enthalpies).
template <typename T>
struct Kin {
    T W, bt, b[3], b2, w, wtot, ptot;
};

template <typename T>
__device__ __forceinline__ Kin<T> kinematics(const T* q, const GeoT<T>& g, T gfac)
{
    Kin<T> k;
    T u0 = q[2], u1 = q[3], u2 = q[4];
    T B0 = q[5], B1 = q[6], B2 = q[7];
    k.W = sqrt(T(1) + g.psi4 * (u0 * u0 + u1 * u1 + u2 * u2));
    T f = g.alpha / k.W;                      // 1/u^t
    k.bt = g.psi4 * (B0 * u0 + B1 * u1 + B2 * u2); // b^t = B^i u_i
    k.b[0] = (B0 + k.bt * u0) * f;                 // b^i = (B^i + b^t u^i)/u^t
    k.b[1] = (B1 + k.bt * u1) * f;
    k.b[2] = (B2 + k.bt * u2) * f;
    k.b2 = (g.psi4 * (B0 * B0 + B1 * B1 + B2 * B2) + k.bt * k.bt) * f * f;
    k.w = q[0] + gfac * q[1];
    k.wtot = k.w + k.b2;
    k.ptot = q[1] + T(0.5) * k.b2;
    return k;
}

// Extreme signal speeds along axis D: the dispersion relation with the
// isotropic fast speed c^2 = (gamma p + b^2)/(w + b^2), solved in closed form.
template <int D, typename T>
__device__ __forceinline__ void speeds(const T* q, const Kin<T>& k, const GeoT<T>& g, T gamma, T& lm,
                                       T& lp)
{
    T inv = T(1) / k.wtot;
    T c2 = (k.b2 + gamma * q[1]) * inv;
    T a = (k.w - gamma * q[1]) * inv;         // 1 - c^2
    T qi = q[2 + D];
    T den = k.W * k.W * a + c2;
    T disc = c2 * (den * g.ipsi4 - qi * qi * a);
    T s = sqrt(fmax(disc, T(0)));
    T t = g.alpha / den;
    T m = k.W * qi * a;
    lp = (m + s) * t;
    lm = (m - s) * t;
}

// Component v (0..7, not the normal field) of the physical flux along D.
template <int D, typename T>
__device__ __forceinline__ T flux_comp(int v, const T* q, const Kin<T>& k, const GeoT<T>& g)
{
    T uD = q[2 + D];
    switch (v) {
    case 0:
        return g.sqrtmg * q[0] * uD;
    case 1:
        return g.sqrtmg * ((k.wtot * g.alpha * k.W - q[0]) * uD - g.alpha * g.alpha * k.bt * k.b[D]);
    case 2:
    case 3:
    case 4: {
        int j = v - 2;
        T t = g.psi4 * (k.wtot * uD * q[2 + j] - k.b[D] * k.b[j]);
        if (j == D)
            t += k.ptot;
        return g.sqrtmg * t;
    }
    default: {
        int j = v - 5;
        return g.sqrtmg * (k.b[j] * uD - k.b[D] * q[2 + j]);
    }
    }
}

// Component v (0..7) of the conserved variables.
template <typename T>
__device__ __forceinline__ T cons_comp(int v, const T* q, const Kin<T>& k, const GeoT<T>& g)
{
    switch (v) {
    case 0:
        return g.sqrtg * q[0] * k.W;
    case 1:
        return g.sqrtmg * (k.wtot * k.W * k.W - k.ptot - g.alpha * g.alpha * k.bt * k.bt)
               - g.sqrtg * q[0] * k.W;
    case 2:
    case 3:
    case 4: {
        int j = v - 2;
        return g.psi4 * (g.sqrtg * k.wtot * k.W * q[2 + j] - g.sqrtmg * k.bt * k.b[j]);
    }
    default:
        return g.sqrtmg * q[v];
    }
}

// MC-limited slope: minmod(2 dq-, (dq- + dq+)/2, 2 dq+).
template <typename T>
__device__ __forceinline__ T mc_slope(T qm, T q0, T qp)
{
    T dl = q0 - qm, dr = qp - q0, dc = T(0.5) * (qp - qm);
    T s = fmin(fmin(T(2) * fabs(dl), T(2) * fabs(dr)), fabs(dc));
    return (dl * dr > T(0)) ? copysign(s, dc) : T(0);
}

// Half the MC slope, the offset of the face values from the cell value:
// minmod(dq-, (dq- + dq+)/4, dq+), the same number as 0.5 * mc_slope (the
// factors of two are exact) in fewer operations.
template <typename T>
__device__ __forceinline__ T mc_hslope(T qm, T q0, T qp)
{
    const T dl = q0 - qm, dr = qp - q0, dq = qp - qm;
    const T h = fmin(fmin(fabs(dl), fabs(dr)), T(0.25) * fabs(dq));
    return (dl * dr > T(0)) ? copysign(h, dq) : T(0);
}

// PPM edge values (Colella & Woodward's piecewise parabolic method, the
// alternative reconstruction of section 3.2) of the middle cell of a0..a4:
// interface values from the four nearest cells with MC-limited slopes, then
// the monotonicity constraints (flat at a local extremum; an edge moved to
// 3 q - 2 other where the parabola would peak inside the cell).
template <typename T>
__device__ __forceinline__ void ppm_edges(T a0, T a1, T a2, T a3, T a4, T& aL, T& aR)
{
    const T sm = mc_slope(a0, a1, a2), s0 = mc_slope(a1, a2, a3), sp = mc_slope(a2, a3, a4);
    T l = T(0.5) * (a1 + a2) - (s0 - sm) / T(6);
    T r = T(0.5) * (a2 + a3) - (sp - s0) / T(6);
    if ((r - a2) * (a2 - l) <= T(0)) {
        l = a2;
        r = a2;
    } else {
        const T dlr = r - l, m6 = T(6) * (a2 - T(0.5) * (l + r));
        if (dlr * m6 > dlr * dlr)
            l = T(3) * a2 - T(2) * r;
        else if (-dlr * dlr > dlr * m6)
            r = T(3) * a2 - T(2) * l;
    }
    aL = l;
    aR = r;
}

// A class test, not arithmetic: with FMA contraction "x - x" may be evaluated
// as fma(a, b, -x) for x = a*b, which is the rounding error of the product.
__device__ __forceinline__ bool finite(double x)
{
    return __builtin_isfinite(x);
}

// ---------------------------------------------------------------------------
// Face solver: from the reconstructed left/right primitives at a face along D
// and the metric there, the 9 components Fo of the numerical flux: exact
// (Bd^n, Phi) cleaning pair, then HLLE on the rest.  The metric is
// conformally flat, so a face of axis D is also a face of axis 0 with the
// vector components cycled (D, D+1, D+2) -> (0, 1, 2).
template <int D, typename T>
__device__ __forceinline__ void face_solve(T* qL, T* qR, const GeoT<T>& g, const Dev& d, T* Fo)
{
    const T half = T(0.5), ch = (T)d.c_h, ich = (T)d.ic_h;

    // cleaning pair: exact solution of the linear (Bd^n, Phi) Riemann problem
    T BnL = g.sqrtmg * qL[5 + D], BnR = g.sqrtmg * qR[5 + D];
    // with flux-CT Phi plays no part: the mean of the reconstructed normal
    // fields
    T Bs = d.ct ? half * (BnL + BnR) : half * (BnL + BnR) - half * ich * (qR[8] - qL[8]);
    T phs = half * (qL[8] + qR[8]) - half * ch * (BnR - BnL);
    qL[5 + D] = qR[5 + D] = Bs * g.isqrtmg;

    const T gfac = (T)d.gfac, gam = (T)d.gamma;
    Kin<T> kL = kinematics(qL, g, gfac);
    Kin<T> kR = kinematics(qR, g, gfac);
    T lmL, lpL, lmR, lpR;
    speeds<D>(qL, kL, g, gam, lmL, lpL);
    speeds<D>(qR, kR, g, gam, lmR, lpR);
    T sl = fmin(T(0), fmin(lmL, lmR));
    T sr = fmax(T(0), fmax(lpL, lpR));
    T cL, cR, cU;
    if (sl == T(0)) {
        cL = T(1);
        cR = T(0);
        cU = T(0);
    } else if (sr == T(0)) {
        cL = T(0);
        cR = T(1);
        cU = T(0);
    } else {
        T inv = T(1) / (sr - sl);
        cL = sr * inv;
        cR = -sl * inv;
        cU = sl * sr * inv;
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        if (v == 5 + D)
            continue;
        T fl = flux_comp<D>(v, qL, kL, g);
        T fr = flux_comp<D>(v, qR, kR, g);
        T o = cL * fl + cR * fr;
        if (cU != T(0))
            o += cU * (cons_comp(v, qR, kR, g) - cons_comp(v, qL, kL, g));
        Fo[v] = o;
    }
    // flux-CT: no normal-field flux and no Phi flux (the transverse field
    // fluxes are replaced once the edge values are known)
    Fo[5 + D] = d.ct ? T(0) : phs;
    Fo[8] = d.ct ? T(0) : (T)d.c_h2 * Bs;
}

// The face solver at face f of axis D (position x, y, z) with the metric there.
template <int D, int KIND, typename T>
__device__ __forceinline__ void face_flux(T* qL, T* qR, double x, double y, double z, long long f,
                                          const Dev& d, T* Fo)
{
    face_solve<D>(qL, qR, geo_cast<T>(face_geo<D, KIND>(d, x, y, z, f)), d, Fo);
}


// ---------------------------------------------------------------------------
// Metric sources at a cell centre (x, y, z) with primitives q, added to R:
// 1/2 sqrt(-g) [T^tt d_j g_tt + sum_k T^kk d_j g_kk] on the momenta (d_j g_tt =
// -2 alpha d_j alpha), zero on mass and energy (static metric), -kappa Phi on
// the cleaning scalar.  The source is evaluated in T; the centre geometry is
// returned in g (double, for the recovery).
template <int KIND, typename T>
__device__ __forceinline__ void add_sources(const Dev& d, double x, double y, double z, long long c,
                                            const T* q, Geo& g, double* R)
{
    if (KIND == STORED) {
        // the stored derivatives d_j alpha, d_j psi^4 along each axis
        g = geo_from_ap(d.mc[c], d.mc[d.N + c]);
        const GeoT<T> gt = geo_cast<T>(g);
        Kin<T> kk = kinematics(q, gt, (T)d.gfac);
        T ia2 = T(1) / (gt.alpha * gt.alpha);
        T Ttt = (kk.wtot * kk.W * kk.W - kk.ptot) * ia2 - kk.bt * kk.bt;
        T uu = q[2] * q[2] + q[3] * q[3] + q[4] * q[4];
        T bb = kk.b[0] * kk.b[0] + kk.b[1] * kk.b[1] + kk.b[2] * kk.b[2];
        T Tkk = kk.wtot * uu + T(3) * kk.ptot * gt.ipsi4 - bb;
        T h = T(0.5) * gt.sqrtmg;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            R[2 + j] += (double)(h * (-T(2) * gt.alpha * Ttt * (T)d.mc[(2 + j) * d.N + c]
                                      + Tkk * (T)d.mc[(5 + j) * d.N + c]));
        if (!d.ct)
            R[8] -= d.kappa * (double)q[8];
        return;
    }
    double ka, kp;
    g = geo_deriv<KIND>(d, x, y, z, ka, kp);
    if (KIND != FLAT) {
        const GeoT<T> gt = geo_cast<T>(g);
        Kin<T> kk = kinematics(q, gt, (T)d.gfac);
        T ia2 = T(1) / (gt.alpha * gt.alpha);
        T Ttt = (kk.wtot * kk.W * kk.W - kk.ptot) * ia2 - kk.bt * kk.bt;
        T uu = q[2] * q[2] + q[3] * q[3] + q[4] * q[4];
        T bb = kk.b[0] * kk.b[0] + kk.b[1] * kk.b[1] + kk.b[2] * kk.b[2];
        T Tkk = kk.wtot * uu + T(3) * kk.ptot * gt.ipsi4 - bb;
        T K = T(0.5) * gt.sqrtmg * (-T(2) * gt.alpha * Ttt * (T)ka + Tkk * (T)kp);
        R[2] += (double)(K * (T)x);
        R[3] += (double)(K * (T)y);
        R[4] += (double)(K * (T)z);
    }
    if (!d.ct)
        R[8] -= d.kappa * (double)q[8];   // flux-CT carries Phi unchanged
}

// ---------------------------------------------------------------------------
// Primitive recovery (section 2.2; the 2D_W equations of Noble et al. 2006 in
// the unknowns Wc = rho h W^2 and v^2).

struct C2P {
    double D, Qn, Qt2, Bc2, QB2;
};

// Newton-Raphson on the two residuals, warm-started.  Converged when the
// relative step in Wc falls below tol, after one more step (which takes the
// iterate to its rounding limit, so that the root does not depend on the
// guess in its last bits); the final point must then satisfy both equations
// to 1e-10 of their scales with v^2 inside (0, 1) unclamped.  Returns true
// on acceptance; iters counts the iterations.
__device__ __forceinline__ bool c2p_newton2d(const C2P& c, double gk, double tol, int maxit,
                                             double& Wc, double& v2, int& iters)
{
    const double vmax = 1.0 - 1e-16;
    int extra = -1;
    bool clamped = false;
    for (int it = 0; it < maxit; ++it) {
        iters = it + 1;
        double bw = c.Bc2 + Wc;
        double iW = 1.0 / Wc;
        double iW2 = iW * iW;
        double is = rsqrt(1.0 - v2);          // 1 / sqrt(1 - v^2) = W
        double s = (1.0 - v2) * is;
        // residuals
        double r1 = v2 * bw * bw - c.QB2 * (c.Bc2 + 2.0 * Wc) * iW2 - c.Qt2;
        double p = gk * (Wc * (1.0 - v2) - c.D * s);
        double r2 = -0.5 * c.Bc2 * (1.0 + v2) + 0.5 * c.QB2 * iW2 - Wc + p - c.Qn;
        // Jacobian
        double a11 = 2.0 * v2 * bw + 2.0 * c.QB2 * bw * iW2 * iW;
        double a12 = bw * bw;
        double a21 = -c.QB2 * iW2 * iW - 1.0 + gk * (1.0 - v2);
        double a22 = -0.5 * c.Bc2 + gk * (-Wc + 0.5 * c.D * is);
        double idet = 1.0 / (a11 * a22 - a12 * a21);
        double dW = (r1 * a22 - a12 * r2) * idet;
        double dv = (a11 * r2 - a21 * r1) * idet;
        double Wn = Wc - dW;
        double vn = v2 - dv;
        if (!(Wn > 0.0))
            Wn = 0.5 * Wc;
        clamped = !(vn < vmax);
        vn = fmin(fmax(vn, 0.0), vmax);
        double step = fabs(Wn - Wc);
        Wc = Wn;
        v2 = vn;
        if (!finite(Wc) || !finite(v2))
            return false;
        if (extra == 0)
            break;
        if (step <= tol * Wc)
            extra = 0;   // converged: one more step takes the iterate to its rounding limit
    }
    if (extra != 0 || clamped || !(Wc > 0.0))
        return false;
    double bw = c.Bc2 + Wc;
    double iW2 = 1.0 / (Wc * Wc);
    double s = sqrt(1.0 - v2);
    double t1 = v2 * bw * bw, t2 = c.QB2 * (c.Bc2 + 2.0 * Wc) * iW2;
    double r1 = t1 - t2 - c.Qt2;
    double p = gk * (Wc * (1.0 - v2) - c.D * s);
    double r2 = -0.5 * c.Bc2 * (1.0 + v2) + 0.5 * c.QB2 * iW2 - Wc + p - c.Qn;
    double sc1 = t1 + t2 + c.Qt2;
    double sc2 = c.Bc2 + Wc + fabs(p) + fabs(c.Qn) + 0.5 * c.QB2 * iW2;
    return fabs(r1) <= 1e-10 * sc1 && fabs(r2) <= 1e-10 * sc2;
}

__device__ __forceinline__ void c2p_v2(const C2P& c, double Wc, double& v2, double& dv2)
{
    double bw = c.Bc2 + Wc;
    double ibw = 1.0 / bw;
    double iW = 1.0 / Wc;
    double gq = (c.Bc2 + 2.0 * Wc) * ibw * ibw * iW * iW;
    v2 = c.Qt2 * ibw * ibw + c.QB2 * gq;
    dv2 = -2.0 * c.Qt2 * ibw * ibw * ibw + c.QB2 * gq * (2.0 / (c.Bc2 + 2.0 * Wc) - 2.0 * ibw - 2.0 * iW);
}

__device__ __forceinline__ double c2p_f1d(const C2P& c, double gk, double Wc, double& df)
{
    double v2, dv2;
    c2p_v2(c, Wc, v2, dv2);
    double s = sqrt(1.0 - v2);
    double p = gk * (Wc * (1.0 - v2) - c.D * s);
    double dp = gk * ((1.0 - v2) + (-Wc + 0.5 * c.D / s) * dv2);
    double iW = 1.0 / Wc;
    df = -0.5 * c.Bc2 * dv2 - c.QB2 * iW * iW * iW - 1.0 + dp;
    return -0.5 * c.Bc2 * (1.0 + v2) + 0.5 * c.QB2 * iW * iW - Wc + p - c.Qn;
}

// Recovery with one unknown: v^2(Wc) eliminated through the momentum
// equation, Newton on the energy equation's residual in Wc, warm-started from
// the guess's Wc.  Accepted as the 2D iteration is: the relative step below
// tol, then one more step, with v^2 in [0, 1) and the residual below 1e-10
// of its scale.
__device__ __forceinline__ bool c2p_newton1d(const C2P& c, double gk, double tol, int maxit, double& Wc,
                                             double& v2, int& iters)
{
    int extra = -1;
    for (int it = 0; it < maxit; ++it) {
        iters = it + 1;
        double dv2;
        c2p_v2(c, Wc, v2, dv2);
        if (!(v2 >= 0.0 && v2 < 1.0))
            return false;
        double df;
        const double f = c2p_f1d(c, gk, Wc, df);
        double Wn = Wc - f / df;
        if (!(Wn > 0.0))
            Wn = 0.5 * Wc;
        const double step = fabs(Wn - Wc);
        Wc = Wn;
        if (!finite(Wc))
            return false;
        if (extra == 0)
            break;
        if (step <= tol * Wc)
            extra = 0;   // converged: one more step takes the iterate to its rounding limit
    }
    if (extra != 0 || !(Wc > 0.0))
        return false;
    double dv2;
    c2p_v2(c, Wc, v2, dv2);
    if (!(v2 >= 0.0 && v2 < 1.0))
        return false;
    double df;
    const double f = c2p_f1d(c, gk, Wc, df);
    const double p = gk * (Wc * (1.0 - v2) - c.D * sqrt(1.0 - v2));
    const double sc = c.Bc2 + Wc + fabs(p) + fabs(c.Qn) + 0.5 * c.QB2 / (Wc * Wc);
    return fabs(f) <= 1e-10 * sc;
}

// Bracketed solve in Wc alone (v^2 eliminated): used when the 2D iteration
// is not accepted.  The bracket starts at the smallest Wc with v^2 < 1 (v^2
// falls with Wc; f falls with Wc), searched above D when v^2(D) >= 1 and
// below D only when f(D) <= 0; Newton steps are kept inside the bracket.
struct WV {
    double Wc, v2;   // Wc < 0 flags a failure
};

// All inputs by value and the result returned by value, so that nothing of
// the caller's state has its address taken (it stays in registers).
__device__ __noinline__ WV c2p_bracketed(double D, double Qn, double Qt2, double Bc2, double QB2,
                                         double gk)
{
    C2P c;
    c.D = D;
    c.Qn = Qn;
    c.Qt2 = Qt2;
    c.Bc2 = Bc2;
    c.QB2 = QB2;
    const WV fail = {-1.0, 0.0};
    double lo = c.D, v2, dv2, df;
    c2p_v2(c, lo, v2, dv2);
    if (!(v2 < 1.0)) {
        double a = lo, b = 2.0 * lo;
        int it = 0;
        for (; it < 1100; ++it) {
            c2p_v2(c, b, v2, dv2);
            if (v2 < 1.0)
                break;
            a = b;
            b *= 2.0;
        }
        if (!(v2 < 1.0))
            return fail;
        for (it = 0; it < 120; ++it) {
            double m = 0.5 * (a + b);
            if (!(m > a && m < b))
                break;
            c2p_v2(c, m, v2, dv2);
            if (v2 < 1.0)
                b = m;
            else
                a = m;
        }
        lo = b;
    } else if (!(c2p_f1d(c, gk, lo, df) > 0.0)) {
        double a = 0.5 * lo, b = lo;
        bool found = false;
        for (int it = 0; it < 700; ++it) {
            c2p_v2(c, a, v2, dv2);
            if (!(v2 < 1.0)) {
                found = true;
                break;
            }
            b = a;
            a *= 0.5;
        }
        for (int it = 0; found && it < 120; ++it) {
            double m = 0.5 * (a + b);
            if (!(m > a && m < b))
                break;
            c2p_v2(c, m, v2, dv2);
            if (v2 < 1.0)
                b = m;
            else
                a = m;
        }
        lo = b;
    }
    if (!(c2p_f1d(c, gk, lo, df) > 0.0))
        return fail;
    double hi = 2.0 * lo;
    for (int it = 0; it < 1100 && c2p_f1d(c, gk, hi, df) >= 0.0; ++it) {
        lo = hi;
        hi *= 2.0;
    }
    if (!(c2p_f1d(c, gk, hi, df) < 0.0))
        return fail;
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 300; ++it) {
        double f = c2p_f1d(c, gk, x, df);
        if (f == 0.0)
            break;
        if (f > 0.0)
            lo = x;
        else
            hi = x;
        double xn = x - f / df;
        if (!(xn > lo && xn < hi))
            xn = 0.5 * (lo + hi);
        bool done = fabs(xn - x) <= 1e-14 * x || hi - lo <= 4e-16 * hi;
        x = xn;
        if (done) {
            f = c2p_f1d(c, gk, x, df);
            xn = x - f / df;
            if (f != 0.0 && xn > lo && xn < hi)
                x = xn;
            break;
        }
    }
    c2p_v2(c, x, v2, dv2);
    if (!(v2 >= 0.0 && v2 < 1.0) || !finite(x))
        return fail;
    WV r = {x, v2};
    return r;
}

enum { FLAG_FAIL = 1, FLAG_ATM = 2, FLAG_PFLOOR = 4, FLAG_FALLBACK = 8 };

// Recovery plus the atmosphere/floor policy for one cell.  u is the conserved
// state (its matter part is rewritten where a floor fired), qg the guess (the
// previous primitives of the cell), p the output primitives.  Returns flags.
__device__ __forceinline__ int recover_cell(const Dev& d, const Geo& g, double* u, const double* qg,
                                            double* p, int& iters)
{
    int flags = 0;
    iters = 0;
    bool ok = true;
#pragma unroll
    for (int v = 0; v < 9; ++v)
        ok = ok && finite(u[v]);
    ok = ok && u[0] > 0.0;
    double Bc[3], Q[3];
    C2P c;
    double isg = g.alpha * g.isqrtmg;   // 1 / sqrt(gamma) = alpha / sqrt(-g)
    c.D = u[0] * isg;
    c.Qn = -(u[1] + u[0]) * g.isqrtmg;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Q[i] = u[2 + i] * isg;
        Bc[i] = g.alpha * (u[5 + i] * g.isqrtmg);
    }
    c.Qt2 = g.ipsi4 * (Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
    c.Bc2 = g.psi4 * (Bc[0] * Bc[0] + Bc[1] * Bc[1] + Bc[2] * Bc[2]);
    double QB = Q[0] * Bc[0] + Q[1] * Bc[1] + Q[2] * Bc[2];
    c.QB2 = QB * QB;

    double Wc = 0.0, v2 = 0.0;
    if (ok) {
        // warm start from the guess primitives
        double uu = g.psi4 * (qg[2] * qg[2] + qg[3] * qg[3] + qg[4] * qg[4]);
        double Wg2 = 1.0 + uu;
        Wc = (qg[0] + d.gfac * qg[1]) * Wg2;
        v2 = uu / Wg2;
        bool guess_ok = finite(Wc) && Wc > 0.0 && finite(v2);
        bool conv = guess_ok && (d.c2p1d ? c2p_newton1d(c, d.gk, d.tol, d.maxit, Wc, v2, iters)
                                         : c2p_newton2d(c, d.gk, d.tol, d.maxit, Wc, v2, iters));
        if (!conv) {
            flags |= FLAG_FALLBACK;
            WV r = c2p_bracketed(c.D, c.Qn, c.Qt2, c.Bc2, c.QB2, d.gk);
            ok = r.Wc > 0.0;
            Wc = r.Wc;
            v2 = r.v2;
        }
    }
    if (ok) {
        double W = rsqrt(1.0 - v2);
        double s = (1.0 - v2) * W;
        p[0] = c.D * s;
        p[1] = d.gk * (Wc * (1.0 - v2) - c.D * s);
        double iq = 1.0 / (Wc * (Wc + c.Bc2));
        double f = W * Wc * iq;                 // W / (Wc + B^2)
        double fq = QB * (Wc + c.Bc2) * iq;     // (Q.B) / Wc
#pragma unroll
        for (int i = 0; i < 3; ++i)
            p[2 + i] = f * (g.ipsi4 * Q[i] + fq * Bc[i]);
#pragma unroll
        for (int v = 0; v < 5; ++v)
            ok = ok && finite(p[v]);
    }
    if (!ok) {
        flags |= FLAG_FAIL;
#pragma unroll
        for (int v = 0; v < 5; ++v)
            p[v] = qg[v];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
        p[5 + i] = u[5 + i] * g.isqrtmg;
    p[8] = u[8];
    // atmosphere: rho below rho_atm by more than a relative 1e-10 (a margin
    // above rounding, so cells sitting at rho_atm are not reset back and forth)
    if (!(p[0] >= (1.0 - 1e-10) * d.rho_atm) || ((flags & FLAG_FAIL) && qg[0] < 10.0 * d.rho_atm)) {
        flags |= FLAG_ATM;
        p[0] = d.rho_atm;
        p[1] = d.p_atm;
        p[2] = p[3] = p[4] = 0.0;
    }
    if (!(p[1] >= d.p_atm)) {
        flags |= FLAG_PFLOOR;
        p[1] = d.p_atm;
    }
    if (flags & (FLAG_FAIL | FLAG_ATM | FLAG_PFLOOR)) {
        GeoT<double> gd = geo_cast<double>(g);
        Kin<double> k = kinematics(p, gd, d.gfac);
#pragma unroll
        for (int v = 0; v < 5; ++v)
            u[v] = cons_comp(v, p, k, gd);
    }
    return flags;
}

}  // namespace grmhd
