// grmhd_adjoint.hip -- reverse (adjoint) kernels of one SSP Runge-Kutta step,
// FP64.
//
// Forward stage s:  U~^(s+1) = U^s + a_s (U^n - U^s) + b_s dt R(P^s),
//                   (P^(s+1), U^(s+1)) = recovery of U~^(s+1) with floors
//                   (a floored cell's conserved matter part is rebuilt).
// Reverse, given the cotangents (Ub, Pb) of (U^(s+1), P^(s+1)), the recovery
// adjoint ((dU/dP)^-T at P^(s+1) by the implicit function theorem, floors as
// constants, the rebuild differentiated) and the RK combination
// (Ub^s = (1 - a_s) Ub~, Ub^n += a_s Ub~, Rb = b_s dt Ub~), then the
// right-hand side's adjoint at P^s:
//   k_adj_rec      the recovery + RK adjoint of the last stage (Pb = 0);
//   k_adj_face     per face of every axis: the flux cotangent (Rb_right - Rb_left)/dx
//                  pulled back through HLLE, the cleaning pair and the face
//                  physics to the reconstructed left/right states;
//   k_adj_gather   per cell and per ghost position: those pulled back
//                  through the MC reconstruction of every axis;
//   k_adj_cell     per cell: plus the ghost positions that copy the cell (the
//                  adjoint of the ghost fill) and the sources' cotangent,
//                  = Pb^s; then the
//                  recovery + RK adjoint of the stage below, or, at the
//                  step's start (P^0 the primitives of U^n),
//                  Ub^n += Unacc + (dU/dP)^-T Pb^0.
// k_adj_final and k_adj_cons serve grmhd_prim_adjoint and grmhd_cons_adjoint.
#include "grmhd_adjoint.h"
#include "grmhd_internal.h"

namespace grmhd {

static constexpr int ABLOCK = 256;

static inline unsigned ablocks(long long n)
{
    return (unsigned)((n + ABLOCK - 1) / ABLOCK);
}

__device__ __forceinline__ long long ghosted(const Dev& d, int i, int j, int k)
{
    return ((long long)(k + d.g[2]) * d.py + (j + d.g[1])) * d.px + (i + d.g[0]);
}

// Interior cell c (x fastest) -> (i, j, k).  The adjoint contexts hold at
// most 2^30 cells, so 32-bit arithmetic suffices.
__device__ __forceinline__ void cell_ijk(const Dev& d, long long c, int& i, int& j, int& k)
{
    const unsigned cu = (unsigned)c, n0 = d.n[0], n1 = d.n[1];
    const unsigned t = cu / n0, kk = t / n1;
    i = (int)(cu - t * n0);
    j = (int)(t - kk * n1);
    k = (int)kk;
}

__device__ __forceinline__ double3 centre(const Dev& d, int i, int j, int k)
{
    return make_double3(d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                        d.lo[2] + (k + 0.5) * d.dx[2]);
}

// ---------------------------------------------------------------------------
// Reverse of the face solver (face_flux of the forward kernels, FP64):
// Fb (9) -> qLb, qRb (9 each, written).
template <int D, int KIND>
__device__ __forceinline__ void face_flux_rev(const double* qL0, const double* qR0, double x, double y,
                                              double z, const Dev& d, const double* Fb, double* qLb,
                                              double* qRb)
{
    const GeoT<double> g = geo_cast<double>(geo_at<KIND>(d, x, y, z));
    double qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        qL[v] = qL0[v];
        qR[v] = qR0[v];
    }
    const double BnL = g.sqrtmg * qL[5 + D], BnR = g.sqrtmg * qR[5 + D];
    const double Bs = 0.5 * (BnL + BnR) - 0.5 * d.ic_h * (qR[8] - qL[8]);
    qL[5 + D] = qR[5 + D] = Bs * g.isqrtmg;
    const Kin<double> kL = kinematics(qL, g, d.gfac);
    const Kin<double> kR = kinematics(qR, g, d.gfac);
    double lmL, lpL, lmR, lpR;
    speeds<D>(qL, kL, g, d.gamma, lmL, lpL);
    speeds<D>(qR, kR, g, d.gamma, lmR, lpR);
    const double sl = fmin(0.0, fmin(lmL, lmR));
    const double sr = fmax(0.0, fmax(lpL, lpR));
    double cL, cR, cU;
    const bool central = !(sl == 0.0) && !(sr == 0.0);
    if (sl == 0.0) {
        cL = 1.0;
        cR = 0.0;
        cU = 0.0;
    } else if (sr == 0.0) {
        cL = 0.0;
        cR = 1.0;
        cU = 0.0;
    } else {
        const double inv = 1.0 / (sr - sl);
        cL = sr * inv;
        cR = -sl * inv;
        cU = sl * sr * inv;
    }

    double aL[9], aR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v)
        aL[v] = aR[v] = 0.0;
    KinBar kLb = kin_zero(), kRb = kin_zero();
    double cLb = 0.0, cRb = 0.0, cUb = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        if (v == 5 + D)
            continue;
        const double c = Fb[v];
        if (central) {
            cLb += c * flux_comp<D>(v, qL, kL, g);
            cRb += c * flux_comp<D>(v, qR, kR, g);
            cUb += c * (cons_comp(v, qR, kR, g) - cons_comp(v, qL, kL, g));
        }
        if (cL != 0.0)
            flux_comp_rev<D>(v, qL, kL, g, cL * c, aL, kLb);
        if (cR != 0.0)
            flux_comp_rev<D>(v, qR, kR, g, cR * c, aR, kRb);
        if (cU != 0.0) {
            cons_comp_rev(v, qR, kR, g, cU * c, aR, kRb);
            cons_comp_rev(v, qL, kL, g, -cU * c, aL, kLb);
        }
    }
    if (central) {
        // cL = sr/(sr-sl), cR = -sl/(sr-sl), cU = sl sr/(sr-sl)
        const double i2 = 1.0 / ((sr - sl) * (sr - sl));
        const double slb = (cLb * sr - cRb * sr + cUb * sr * sr) * i2;
        const double srb = (-cLb * sl + cRb * sl - cUb * sl * sl) * i2;
        // sl = min(0, lmL, lmR) < 0 and sr = max(0, lpL, lpR) > 0 here
        const bool leftmin = lmL <= lmR, leftmax = lpL >= lpR;
        speeds_rev<D>(qL, kL, g, d.gamma, leftmin ? slb : 0.0, leftmax ? srb : 0.0, aL, kLb);
        speeds_rev<D>(qR, kR, g, d.gamma, leftmin ? 0.0 : slb, leftmax ? 0.0 : srb, aR, kRb);
    }
    kinematics_rev(qL, kL, g, d.gfac, kLb, aL);
    kinematics_rev(qR, kR, g, d.gfac, kRb, aR);

    // cleaning pair: Fo[5+D] = phi*, Fo[8] = c_h^2 Bd*, and both states carry
    // B^n = Bd* / sqrt(-g)
    const double phb = Fb[5 + D];
    const double Bsb = d.c_h2 * Fb[8] + (aL[5 + D] + aR[5 + D]) * g.isqrtmg;
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        qLb[v] = aL[v];
        qRb[v] = aR[v];
    }
    qLb[5 + D] = 0.5 * g.sqrtmg * Bsb + 0.5 * d.c_h * g.sqrtmg * phb;
    qRb[5 + D] = 0.5 * g.sqrtmg * Bsb - 0.5 * d.c_h * g.sqrtmg * phb;
    qLb[8] += 0.5 * d.ic_h * Bsb + 0.5 * phb;
    qRb[8] += -0.5 * d.ic_h * Bsb + 0.5 * phb;
}

// Face f along D (one thread).  Face f sits between cells f-1 and f; the
// flux cotangent is (Rb_f - Rb_(f-1)) / dx with out-of-domain cells absent.
template <int D, int KIND>
__device__ __forceinline__ void adj_face(long long f, const double* __restrict__ Pc,
                                         const double* __restrict__ Rb, double* __restrict__ FB, const Dev& d)
{
    const long long nf = d.nf[D];
    if (f >= nf)
        return;
    int m[3] = {d.n[0], d.n[1], d.n[2]};
    m[D] += 1;
    // f < nf < 2^32 (the launch checks it): 32-bit index arithmetic
    const unsigned fu = (unsigned)f, m0 = m[0], m1 = m[1];
    const unsigned t = fu / m0, k = t / m1;
    const int fi[3] = {(int)(fu - t * m0), (int)(t - k * m1), (int)k};
    const int fD = fi[D];
    // The RHS cotangents of the two cells beside the face are loaded whether
    // or not the cells exist (indices clamped into the domain), so that these
    // loads are in flight together with the stencil's; a cell outside the
    // domain then contributes zero.
    const bool hi_in = fD < d.n[D], lo_in = fD > 0;
    int ch[3] = {fi[0], fi[1], fi[2]}, cl[3] = {fi[0], fi[1], fi[2]};
    ch[D] = hi_in ? fD : fD - 1;
    cl[D] = lo_in ? fD - 1 : fD;
    const long long chi = ch[0] + (long long)d.n[0] * (ch[1] + (long long)d.n[1] * ch[2]);
    const long long clo = cl[0] + (long long)d.n[0] * (cl[1] + (long long)d.n[1] * cl[2]);
    double Fb[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const double rh = Rb[v * d.N + chi], rl = Rb[v * d.N + clo];
        double f = 0.0;
        f += (hi_in ? rh : 0.0) * d.idx[D];
        f -= (lo_in ? rl : 0.0) * d.idx[D];
        Fb[v] = f;
    }
    int bi[3] = {fi[0], fi[1], fi[2]};
    bi[D] -= 2;
    const long long base = ghosted(d, bi[0], bi[1], bi[2]);
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)d.px : (long long)d.px * d.py);
    double qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const double* p = Pc + v * d.sv + base;
        const double q0 = p[0], q1 = p[st], q2 = p[2 * st], q3 = p[3 * st];
        qL[v] = q1 + mc_hslope(q0, q1, q2);   // half the MC slope, as the forward kernels take it
        qR[v] = q2 - mc_hslope(q1, q2, q3);
    }
    double pos[3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
        pos[e] = e == D ? d.lo[e] + fi[e] * d.dx[e] : d.lo[e] + (fi[e] + 0.5) * d.dx[e];
    double qLb[9], qRb[9];
    face_flux_rev<D, KIND>(qL, qR, pos[0], pos[1], pos[2], d, Fb, qLb, qRb);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        FB[v * nf + f] = qLb[v];
        FB[(9 + v) * nf + f] = qRb[v];
    }
}

// The faces of every active axis in one launch: workgroups [0, nb0) take x
// faces, the next nb1 y faces, the rest z faces (one launch instead of three
// leaves one partly filled last wave of workgroups instead of three).
//
// Two waves per SIMD are asked for: the curved-metric instance, with every
// load of a face issued up front, would otherwise take 262 registers.
template <int KIND>
__global__ __launch_bounds__(ABLOCK) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_adj_face(const double* __restrict__ Pc, const double* __restrict__ Rb, double* __restrict__ FB0,
                double* __restrict__ FB1, double* __restrict__ FB2, Dev d, unsigned nb0, unsigned nb1)
{
    unsigned b = blockIdx.x;
    if (b < nb0) {
        adj_face<0, KIND>((long long)b * ABLOCK + threadIdx.x, Pc, Rb, FB0, d);
        return;
    }
    b -= nb0;
    if (b < nb1) {
        adj_face<1, KIND>((long long)b * ABLOCK + threadIdx.x, Pc, Rb, FB1, d);
        return;
    }
    b -= nb1;
    adj_face<2, KIND>((long long)b * ABLOCK + threadIdx.x, Pc, Rb, FB2, d);
}

// Cotangent of primitive v at position ci (ci[D] in -2 .. n+1, ghosts of
// axis D included; interior along the other axes) from the faces along D:
// the left/right reconstructed-state cotangents FB (18 rows of nf values)
// pulled back through the MC reconstruction.  Face f sits between cells f-1
// and f; the slope of cell j feeds the left state at face j+1 and the right
// state at face j.
template <int D>
__device__ __forceinline__ double gather_pos_v(const Dev& d, const double* __restrict__ Pc,
                                               const double* __restrict__ FB, const int* ci, int v)
{
    const int i = ci[D], n = d.n[D];
    const long long nf = d.nf[D];
    int fm[3] = {d.n[0], d.n[1], d.n[2]};
    fm[D] += 1;
    // face i along D (i may lie outside 0..n: only used where it exists);
    // neighbouring faces along D are sf apart
    const long long sf = D == 0 ? 1 : (D == 1 ? (long long)fm[0] : (long long)fm[0] * fm[1]);
    int fi0[3] = {ci[0], ci[1], ci[2]};
    fi0[D] = 0;
    const long long fb = fi0[0] + (long long)fm[0] * (fi0[1] + (long long)fm[1] * fi0[2]) + (long long)i * sf;
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)d.px : (long long)d.px * d.py);
    const long long pc = ghosted(d, ci[0], ci[1], ci[2]);
    const bool has_lo = i >= 0 && i <= n;            // face i exists
    const bool has_hi = i + 1 >= 0 && i + 1 <= n;    // face i+1 exists
    const long long f_lo = has_lo ? fb : 0, f_hi = has_hi ? fb + sf : 0;
    const long long f_lm = (i - 1 >= 0 && i - 1 <= n) ? fb - sf : -1;   // face i-1
    const long long f_hp = (i + 2 >= 0 && i + 2 <= n) ? fb + 2 * sf : -1;   // face i+2
    const double* Fl = FB + v * nf;          // left-state cotangents
    const double* Fr = FB + (9 + v) * nf;    // right-state cotangents
    // every load issued up front (absent faces read face 0, stencil taps
    // outside the ghosted line read its last position; neither value is used)
    const long long g_lm = f_lm >= 0 ? f_lm : 0, g_hp = f_hp >= 0 ? f_hp : 0;
    const double* P = Pc + v * d.sv + pc;
    auto tap = [&](int o) -> double {
        const int p = min(max(i + o, -2), n + 1);
        return P[(long long)(p - i) * st];
    };
    const double Fl_lo_v = Fl[f_lo], Fl_hi_v = Fl[f_hi], Fl_hp_v = Fl[g_hp];
    const double Fr_lo_v = Fr[f_lo], Fr_hi_v = Fr[f_hi], Fr_lm_v = Fr[g_lm];
    const double qm2 = tap(-2), qm1 = tap(-1), q00 = P[0], qp1 = tap(1), qp2 = tap(2);
    const double Fl_hi = has_hi ? Fl_hi_v : 0.0, Fr_lo = has_lo ? Fr_lo_v : 0.0;
    double m = Fl_hi + Fr_lo;
    // j = i - 1 (q_i is its qp), j in [-1, n]
    if (i - 1 >= -1 && i - 1 <= n) {
        const double sb = 0.5 * ((has_lo ? Fl_lo_v : 0.0) - (f_lm >= 0 ? Fr_lm_v : 0.0));
        if (sb != 0.0) {
            double dm, d0, dp;
            mc_slope_grad(qm2, qm1, q00, dm, d0, dp);
            m += sb * dp;
        }
    }
    // j = i
    if (i >= -1 && i <= n) {
        const double sb = 0.5 * (Fl_hi - Fr_lo);
        if (sb != 0.0) {
            double dm, d0, dp;
            mc_slope_grad(qm1, q00, qp1, dm, d0, dp);
            m += sb * d0;
        }
    }
    // j = i + 1 (q_i is its qm)
    if (i + 1 >= -1 && i + 1 <= n) {
        const double sb = 0.5 * ((f_hp >= 0 ? Fl_hp_v : 0.0) - (has_hi ? Fr_hi_v : 0.0));
        if (sb != 0.0) {
            double dm, d0, dp;
            mc_slope_grad(q00, qp1, qp2, dm, d0, dp);
            m += sb * dm;
        }
    }
    return m;
}

// Reverse of add_sources() (FP64): Rb (cotangent of R at the cell) -> qb.
template <int KIND>
__device__ __forceinline__ void sources_rev(const Dev& d, double x, double y, double z, const double* q,
                                            const double* Rb, double* qb)
{
    qb[8] -= d.kappa * Rb[8];
    if (KIND == FLAT)
        return;
    double ka, kp;
    const Geo g0 = geo_deriv<KIND>(d, x, y, z, ka, kp);
    const GeoT<double> g = geo_cast<double>(g0);
    const Kin<double> k = kinematics(q, g, d.gfac);
    const double ia2 = 1.0 / (g.alpha * g.alpha);
    const double Kb = Rb[2] * x + Rb[3] * y + Rb[4] * z;
    const double Tttb = Kb * 0.5 * g.sqrtmg * (-2.0 * g.alpha * ka);
    const double Tkkb = Kb * 0.5 * g.sqrtmg * kp;
    KinBar kb = kin_zero();
    // Ttt = (wtot W^2 - ptot)/alpha^2 - bt^2
    kb.wtot += Tttb * k.W * k.W * ia2;
    kb.W += Tttb * 2.0 * k.wtot * k.W * ia2;
    kb.ptot -= Tttb * ia2;
    kb.bt -= 2.0 * Tttb * k.bt;
    // Tkk = wtot |u~|^2 + 3 ptot / psi^4 - |b|^2
    const double uu = q[2] * q[2] + q[3] * q[3] + q[4] * q[4];
    kb.wtot += Tkkb * uu;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        qb[2 + i] += Tkkb * k.wtot * 2.0 * q[2 + i];
        kb.b[i] -= 2.0 * Tkkb * k.b[i];
    }
    kb.ptot += 3.0 * Tkkb * g.ipsi4;
    kinematics_rev(q, k, g, d.gfac, kb, qb);
}

// x = (dU/dP)^-T y at the primitives q of a cell at (x, y, z); false if the
// matter block is singular.
template <int KIND>
__device__ __forceinline__ bool recovery_adjoint(const Dev& d, const double3& x, const double* q,
                                                 const double* y, double* out, double J[5][8],
                                                 GeoT<double>& g)
{
    g = geo_cast<double>(geo_at<KIND>(d, x.x, x.y, x.z));
    cons_jacobian(q, g, d.gfac, J);
    return cons_jacobian_solve_t(J, g.sqrtmg, y, out);
}

// Recovery adjoint of one cell: from the cotangents ub of the recovered
// (and, where a floor fired, rebuilt) conserved state and pb of the
// primitives q = P^(s+1), the cotangent ut of the state before the recovery.
template <int KIND>
__device__ __forceinline__ void rec_adjoint(const Dev& d, const double3& x, const double* q, int fl,
                                            const double* ub, const double* pb, double* ut)
{
    double J[5][8];
    GeoT<double> g;
    if (fl & FLAG_ATM) {
        // hydro primitives constant; B = Bd / sqrt(-g), Phi passed through;
        // the matter part of U rebuilt from (constant hydro, B)
        g = geo_cast<double>(geo_at<KIND>(d, x.x, x.y, x.z));
        cons_jacobian(q, g, d.gfac, J);
#pragma unroll
        for (int e = 5; e < 8; ++e) {
            double s = pb[e];
#pragma unroll
            for (int r = 0; r < 5; ++r)
                s += J[r][e] * ub[r];
            ut[e] = ub[e] + s * g.isqrtmg;
        }
#pragma unroll
        for (int r = 0; r < 5; ++r)
            ut[r] = 0.0;
        ut[8] = ub[8] + pb[8];
    } else if (fl & FLAG_FAIL) {
        // the previous hydro primitives are kept: no derivative through them
        g = geo_cast<double>(geo_at<KIND>(d, x.x, x.y, x.z));
#pragma unroll
        for (int r = 0; r < 5; ++r)
            ut[r] = ub[r];
#pragma unroll
        for (int e = 5; e < 8; ++e)
            ut[e] = ub[e] + pb[e] * g.isqrtmg;
        ut[8] = ub[8] + pb[8];
    } else if (fl & FLAG_PFLOOR) {
        // pressure constant; rho, u~ from the root; matter part rebuilt
        g = geo_cast<double>(geo_at<KIND>(d, x.x, x.y, x.z));
        cons_jacobian(q, g, d.gfac, J);
        double pt[9];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            double s = pb[e];
#pragma unroll
            for (int r = 0; r < 5; ++r)
                s += J[r][e] * ub[r];
            pt[e] = s;
        }
        pt[1] = 0.0;
        pt[8] = pb[8];
        if (!cons_jacobian_solve_t(J, g.sqrtmg, pt, ut)) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                ut[v] = __builtin_nan("");
        }
#pragma unroll
        for (int v = 5; v < 9; ++v)
            ut[v] += ub[v];
    } else {
        if (!recovery_adjoint<KIND>(d, x, q, pb, ut, J, g)) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                ut[v] = __builtin_nan("");
        }
#pragma unroll
        for (int v = 0; v < 9; ++v)
            ut[v] += ub[v];
    }
}

// The last stage's recovery + RK-combination adjoint (the step's output
// cotangent Ub, no primitive cotangent): Ub <- (1 - a) Ub~, Unacc = a Ub~,
// Rb = b dt Ub~ with Ub~ the cotangent before the recovery.
template <int KIND>
__global__ __launch_bounds__(ABLOCK) void k_adj_rec(double* __restrict__ Ub, const double* __restrict__ Pn,
                                                     const unsigned char* __restrict__ flags,
                                                     double* __restrict__ Unacc, double* __restrict__ Rb,
                                                     Dev d, double a, double b, double dt)
{
    const long long c = (long long)blockIdx.x * ABLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    const long long pc = ghosted(d, i, j, k);
    double q[9], ub[9], ut[9];
    const double pb[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        q[v] = Pn[v * d.sv + pc];
        ub[v] = Ub[v * d.N + c];
    }
    rec_adjoint<KIND>(d, centre(d, i, j, k), q, flags[c], ub, pb, ut);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        Ub[v * d.N + c] = (1.0 - a) * ut[v];
        Unacc[v * d.N + c] = a * ut[v];
        Rb[v * d.N + c] = b * dt * ut[v];
    }
}

// Lines along axis D (cells of the other two axes) and the line of a cell.
template <int D>
__device__ __forceinline__ long long lines_of(const Dev& d)
{
    return D == 0 ? (long long)d.n[1] * d.n[2] : (D == 1 ? (long long)d.n[0] * d.n[2] : (long long)d.n[0] * d.n[1]);
}

template <int D>
__device__ __forceinline__ long long line_of(const Dev& d, const int* ci)
{
    return D == 0 ? ci[1] + (long long)d.n[1] * ci[2]
                  : (D == 1 ? ci[0] + (long long)d.n[0] * ci[2] : ci[0] + (long long)d.n[0] * ci[1]);
}

// The ghost positions of axis D, 4 per line (slots 0..3 = positions -2, -1,
// n, n+1): the pull-back of the faces along D there, variable v, into G
// (layout [9][4][lines]); the cell kernel adds each to the interior cell the
// ghost fill copies into that position.
template <int D>
__device__ __forceinline__ void gather_ghost(const Dev& d, const double* __restrict__ Pc,
                                             const double* __restrict__ FB, double* __restrict__ G,
                                             unsigned t, unsigned lines, int v)
{
    const int slot = (int)(t / lines);
    const unsigned line = t - slot * lines;
    int ci[3];
    const int a = D == 0 ? 1 : 0, b = D == 2 ? 1 : 2;   // the two other axes
    const unsigned na = d.n[a], lb = line / na;
    ci[a] = (int)(line - lb * na);
    ci[b] = (int)lb;
    ci[D] = slot < 2 ? slot - 2 : d.n[D] + slot - 2;
    G[(long long)(v * 4 + slot) * lines + line] = gather_pos_v<D>(d, Pc, FB, ci, v);
}

// One thread per position and primitive variable v (v the grid's y index,
// positions along x, so a wave reads consecutive cells of one variable; the
// positions, fewer than 2^32, are counted in 32 bits): positions
// [0, N) are the interior cells, whose cotangent from the face-state
// cotangents of every active axis (FB0/1/2, 18 rows of nf values each)
// pulled back through the MC reconstruction goes to MU (dense [9][N]); then,
// per active axis, 4 positions per line for its ghost slots (into G0/1/2).
// A thread does one variable's loads and slopes, so the many independent
// threads hide the latency of the scattered loads.
__global__ __launch_bounds__(ABLOCK) void k_adj_gather(const double* __restrict__ Pc,
                                                        const double* __restrict__ FB0,
                                                        const double* __restrict__ FB1,
                                                        const double* __restrict__ FB2,
                                                        double* __restrict__ MU, double* __restrict__ G0,
                                                        double* __restrict__ G1, double* __restrict__ G2, Dev d,
                                                        unsigned npos)
{
    unsigned t = blockIdx.x * ABLOCK + threadIdx.x;
    if (t >= npos)
        return;
    const int v = blockIdx.y;
    if (t < (unsigned)d.N) {
        const unsigned n0 = d.n[0], n1 = d.n[1];
        const unsigned r = t / n0, k = r / n1;
        const int ci[3] = {(int)(t - r * n0), (int)(r - k * n1), (int)k};
        double m = 0.0;
        if (d.act[0])
            m += gather_pos_v<0>(d, Pc, FB0, ci, v);
        if (d.act[1])
            m += gather_pos_v<1>(d, Pc, FB1, ci, v);
        if (d.act[2])
            m += gather_pos_v<2>(d, Pc, FB2, ci, v);
        MU[v * d.N + t] = m;
        return;
    }
    t -= (unsigned)d.N;
    if (d.act[0]) {
        const unsigned lines = (unsigned)lines_of<0>(d);
        if (t < 4 * lines) {
            gather_ghost<0>(d, Pc, FB0, G0, t, lines, v);
            return;
        }
        t -= 4 * lines;
    }
    if (d.act[1]) {
        const unsigned lines = (unsigned)lines_of<1>(d);
        if (t < 4 * lines) {
            gather_ghost<1>(d, Pc, FB1, G1, t, lines, v);
            return;
        }
        t -= 4 * lines;
    }
    if (d.act[2]) {
        const unsigned lines = (unsigned)lines_of<2>(d);
        if (t < 4 * lines)
            gather_ghost<2>(d, Pc, FB2, G2, t, lines, v);
    }
}

// The ghost slots of axis D that copy the interior cell ci (the adjoint of
// the ghost fill: periodic images, or the zero-gradient copies beside the
// first and last cells), added to pb.
template <int D>
__device__ __forceinline__ void fold_ghosts(const Dev& d, const double* __restrict__ G, const int* ci, double* pb)
{
    const int i = ci[D], n = d.n[D];
    const long long lines = lines_of<D>(d), line = line_of<D>(d, ci);
    int sl[2], ns = 0;
    if (d.bc[D] == 0) {   // periodic: position n+i, or i-n
        if (i < 2)
            sl[ns++] = i + 2;
        if (i >= n - 2)
            sl[ns++] = i - n + 2;
    } else if (i == 0) {
        sl[ns++] = 0;
        sl[ns++] = 1;
    } else if (i == n - 1) {
        sl[ns++] = 2;
        sl[ns++] = 3;
    }
    for (int e = 0; e < ns; ++e)
#pragma unroll
        for (int v = 0; v < 9; ++v)
            pb[v] += G[(v * 4 + sl[e]) * lines + line];
}

// Per interior cell, after the gather of stage s: Pb^s = MU (the faces'
// pull-back at the cell) + G at the ghost positions that copy the cell + the
// sources' cotangent at P^s; then, for s > 0, the recovery +
// RK adjoint of stage s-1 (whose output is U^s, P^s; flags of that recovery in
// fprev, coefficients a, b): Ub <- (1 - a) Ub~, Unacc += a Ub~,
// Rb = b dt Ub~; for s = 0 (fprev null) the step's input cotangent
// Ub <- Ub + Unacc + (dU/dP)^-T Pb^0.
//
// Two waves per SIMD are asked for: the curved-metric instance would otherwise
// take 266 registers and run one wave per SIMD; held to 256 it spills 10 and
// runs its step adjoint 5 % faster.
template <int KIND>
__global__ __launch_bounds__(ABLOCK) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_adj_cell(const double* __restrict__ Pc, const double* __restrict__ MU, const double* __restrict__ G0,
                const double* __restrict__ G1, const double* __restrict__ G2, double* __restrict__ Rb,
                double* __restrict__ Ub, double* __restrict__ Unacc, const unsigned char* __restrict__ fprev,
                Dev d, double a, double b, double dt)
{
    const long long c = (long long)blockIdx.x * ABLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    const long long pc = ghosted(d, i, j, k);
    const bool any = d.act[0] || d.act[1] || d.act[2];
    double pb[9], q[9], rb[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        pb[v] = any ? MU[v * d.N + c] : 0.0;
        q[v] = Pc[v * d.sv + pc];
        rb[v] = Rb[v * d.N + c];
    }
    const int ci[3] = {i, j, k};
    if (d.act[0])
        fold_ghosts<0>(d, G0, ci, pb);
    if (d.act[1])
        fold_ghosts<1>(d, G1, ci, pb);
    if (d.act[2])
        fold_ghosts<2>(d, G2, ci, pb);
    const double3 x = centre(d, i, j, k);
    sources_rev<KIND>(d, x.x, x.y, x.z, q, rb, pb);
    double ub[9], ut[9];
#pragma unroll
    for (int v = 0; v < 9; ++v)
        ub[v] = Ub[v * d.N + c];
    if (fprev) {
        rec_adjoint<KIND>(d, x, q, fprev[c], ub, pb, ut);
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            Ub[v * d.N + c] = (1.0 - a) * ut[v];
            Unacc[v * d.N + c] += a * ut[v];
            Rb[v * d.N + c] = b * dt * ut[v];
        }
    } else {
        double J[5][8];
        GeoT<double> g;
        if (!recovery_adjoint<KIND>(d, x, q, pb, ut, J, g)) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                ut[v] = __builtin_nan("");
        }
#pragma unroll
        for (int v = 0; v < 9; ++v)
            Ub[v * d.N + c] = ub[v] + Unacc[v * d.N + c] + ut[v];
    }
}

// Ubar = Ub + Unacc + (dU/dP)^-T Pb at P^0 (the step's first primitives).
// With Ub = Unacc = null: Ubar = (dU/dP)^-T Pb (adjoint of the recovery).
template <int KIND>
__global__ __launch_bounds__(ABLOCK) void k_adj_final(const double* __restrict__ Ub,
                                                       const double* __restrict__ Pb,
                                                       const double* __restrict__ P0,
                                                       const double* __restrict__ Unacc,
                                                       double* __restrict__ Ubar, Dev d)
{
    const long long c = (long long)blockIdx.x * ABLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    const long long pc = ghosted(d, i, j, k);
    double q[9], pb[9], ut[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        q[v] = P0[v * d.sv + pc];
        pb[v] = Pb[v * d.N + c];
    }
    double J[5][8];
    GeoT<double> g;
    if (!recovery_adjoint<KIND>(d, centre(d, i, j, k), q, pb, ut, J, g)) {
#pragma unroll
        for (int v = 0; v < 9; ++v)
            ut[v] = __builtin_nan("");
    }
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        double s = ut[v];
        if (Ub)
            s += Ub[v * d.N + c] + Unacc[v * d.N + c];
        Ubar[v * d.N + c] = s;
    }
}

// Pbar = (dU/dP)^T Ubar at the primitives P (dense interior arrays).
template <int KIND>
__global__ __launch_bounds__(ABLOCK) void k_adj_cons(const double* __restrict__ P,
                                                      const double* __restrict__ Ubar,
                                                      double* __restrict__ Pbar, Dev d)
{
    const long long c = (long long)blockIdx.x * ABLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    double q[9], ub[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        q[v] = P[v * d.N + c];
        ub[v] = Ubar[v * d.N + c];
    }
    const double3 x = centre(d, i, j, k);
    const GeoT<double> g = geo_cast<double>(geo_at<KIND>(d, x.x, x.y, x.z));
    double J[5][8];
    cons_jacobian(q, g, d.gfac, J);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        double s = e >= 5 ? g.sqrtmg * ub[e] : 0.0;
#pragma unroll
        for (int r = 0; r < 5; ++r)
            s += J[r][e] * ub[r];
        Pbar[e * d.N + c] = s;
    }
    Pbar[8 * d.N + c] = ub[8];
}

// ---------------------------------------------------------------------------
// Launchers

hipError_t launch_adj_rec(int kind, double* Ub, const double* Pn, const unsigned char* flags, double* Unacc,
                          double* Rb, const Dev& d, double a, double b, double dt, hipStream_t s)
{
    if (kind == FLAT)
        hipLaunchKernelGGL((k_adj_rec<FLAT>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, Ub, Pn, flags, Unacc, Rb, d,
                           a, b, dt);
    else
        hipLaunchKernelGGL((k_adj_rec<ISO>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, Ub, Pn, flags, Unacc, Rb, d,
                           a, b, dt);
    return hipGetLastError();
}

hipError_t launch_adj_gather(const double* Pc, const double* const* FB, double* MU, double* const* G, const Dev& d,
                             hipStream_t s)
{
    long long npos = d.N;
    for (int a = 0; a < 3; ++a)
        if (d.act[a])
            npos += 4 * (d.N / d.n[a]);
    if (npos > 0xffffffffLL - ABLOCK)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_gather, dim3(ablocks(npos), 9), dim3(ABLOCK), 0, s, Pc, FB[0], FB[1], FB[2], MU, G[0],
                       G[1], G[2], d, (unsigned)npos);
    return hipGetLastError();
}

hipError_t launch_adj_cell(int kind, const double* Pc, const double* MU, const double* const* G, double* Rb,
                           double* Ub, double* Unacc, const unsigned char* fprev, const Dev& d, double a, double b,
                           double dt, hipStream_t s)
{
    if (kind == FLAT)
        hipLaunchKernelGGL((k_adj_cell<FLAT>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, Pc, MU, G[0], G[1], G[2], Rb,
                           Ub, Unacc, fprev, d, a, b, dt);
    else
        hipLaunchKernelGGL((k_adj_cell<ISO>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, Pc, MU, G[0], G[1], G[2], Rb,
                           Ub, Unacc, fprev, d, a, b, dt);
    return hipGetLastError();
}

hipError_t launch_adj_face(int kind, const double* Pc, const double* Rb, double* const* FB, const Dev& d,
                           hipStream_t s)
{
    unsigned nb[3];
    for (int a = 0; a < 3; ++a) {
        if (d.nf[a] > 0xffffffffLL - ABLOCK)
            return hipErrorInvalidValue;
        nb[a] = d.act[a] ? ablocks(d.nf[a]) : 0;
    }
    const unsigned total = nb[0] + nb[1] + nb[2];
    if (total == 0)
        return hipSuccess;
    if (kind == FLAT)
        hipLaunchKernelGGL((k_adj_face<FLAT>), dim3(total), dim3(ABLOCK), 0, s, Pc, Rb, FB[0], FB[1], FB[2], d,
                           nb[0], nb[1]);
    else
        hipLaunchKernelGGL((k_adj_face<ISO>), dim3(total), dim3(ABLOCK), 0, s, Pc, Rb, FB[0], FB[1], FB[2], d,
                           nb[0], nb[1]);
    return hipGetLastError();
}

hipError_t launch_adj_final(int kind, const double* Ub, const double* Pb, const double* P0, const double* Unacc,
                            double* Ubar, const Dev& d, hipStream_t s)
{
    if (kind == FLAT)
        hipLaunchKernelGGL((k_adj_final<FLAT>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, Ub, Pb, P0, Unacc, Ubar,
                           d);
    else
        hipLaunchKernelGGL((k_adj_final<ISO>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, Ub, Pb, P0, Unacc, Ubar, d);
    return hipGetLastError();
}

hipError_t launch_adj_cons(int kind, const double* P, const double* Ubar, double* Pbar, const Dev& d,
                           hipStream_t s)
{
    if (kind == FLAT)
        hipLaunchKernelGGL((k_adj_cons<FLAT>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, P, Ubar, Pbar, d);
    else
        hipLaunchKernelGGL((k_adj_cons<ISO>), dim3(ablocks(d.N)), dim3(ABLOCK), 0, s, P, Ubar, Pbar, d);
    return hipGetLastError();
}

}  // namespace grmhd
