// grmhd_kernels.hip -- HIP kernels of the GRMHD substep (gfx950, wave64).
//
// One substep (section 2.2 of the paper) is
//   k_ghosts  : ghost zones of the primitive cache (periodic / zero-gradient)
//   k_flux_x, k_flux_march<D>: per face along axis D: MC reconstruction of the
//               9 primitives,
//               exact (normal field, Phi) cleaning pair, face physics of both
//               states, HLLE flux (section 3.2)
//   k_update  : per cell: flux differences + metric sources (eq. 2), SSP
//               Runge-Kutta combination, Newton recovery of the primitives
//               with the atmosphere/floor policy, status counters
// Threads are mapped linearly over faces (cells), x fastest, so every load
// and store of the structure-of-arrays buffers is coalesced and no lane idles.
#include "grmhd_device.h"
#include "grmhd_internal.h"

namespace grmhd {

static constexpr int BLOCK = 256;
static constexpr int NXCD = 8;   // accelerator complexes (each with its own L2)

// Workgroups are dispatched round-robin over the XCDs: physical block b runs on
// XCD b mod 8.  Give each XCD a contiguous range of logical blocks instead, so
// that neighbouring rows (the y stencil, the second y face of a cell) are read
// through the same L2.  A bijection on [0, gridDim.x).
__device__ __forceinline__ long long xcd_block()
{
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb / NXCD, r = nb % NXCD, x = b % NXCD;
    return (long long)(x * q + (x < r ? x : r) + b / NXCD);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_fill(double* __restrict__ p, long long n, double v)
{
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n)
        p[t] = v;
}

__global__ __launch_bounds__(BLOCK) void k_zero_counters(unsigned long long* cnt)
{
    for (int t = threadIdx.x; t < CNT_WORDS * CNT_SLOTS; t += BLOCK)
        cnt[t] = 0ull;
}

// Ghost fill: one thread per ghost cell of the three face slabs (no edges or
// corners: the stencil is a cross).  Segment a covers axis a: 2*g layers times
// the interior extent of the other two axes.
__global__ __launch_bounds__(BLOCK) void k_ghosts(double* __restrict__ Pc, Dev d, long long s0,
                                                 long long s1, long long s2)
{
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int a;
    if (t < s0)
        a = 0;
    else if (t < s0 + s1) {
        a = 1;
        t -= s0;
    } else if (t < s0 + s1 + s2) {
        a = 2;
        t -= s0 + s1;
    } else
        return;
    int b = (a + 1) % 3, c = (a + 2) % 3;
    int nb = d.n[b], na = d.n[a];
    int layer = (int)(t % (2 * d.g[a]));
    long long r = t / (2 * d.g[a]);
    int ib = (int)(r % nb);
    int ic = (int)(r / nb);
    // ghost index along a: -g..-1 then n..n+g-1
    int ia = layer < d.g[a] ? layer - d.g[a] : na + (layer - d.g[a]);
    int src;
    if (d.bc[a] == 0)
        src = ((ia % na) + na) % na;
    else
        src = ia < 0 ? 0 : na - 1;
    int I[3], S[3];
    I[a] = ia;
    I[b] = ib;
    I[c] = ic;
    S[a] = src;
    S[b] = ib;
    S[c] = ic;
    long long dst = ((long long)(I[2] + d.g[2]) * d.py + (I[1] + d.g[1])) * d.px + (I[0] + d.g[0]);
    long long sp = ((long long)(S[2] + d.g[2]) * d.py + (S[1] + d.g[1])) * d.px + (S[0] + d.g[0]);
#pragma unroll
    for (int v = 0; v < 9; ++v)
        Pc[v * d.sv + dst] = Pc[v * d.sv + sp];
}

// ---------------------------------------------------------------------------
// Face solver: from the reconstructed left/right primitives at a face along D
// (positions x, y, z), the 9 components Fo of the numerical flux: exact
// (Bd^n, Phi) cleaning pair, then HLLE on the rest.
template <int D, int KIND>
__device__ __forceinline__ void face_flux(double* qL, double* qR, double x, double y, double z,
                                          const Dev& d, double* Fo)
{
    Geo g = geo_at<KIND>(d, x, y, z);

    // cleaning pair: exact solution of the linear (Bd^n, Phi) Riemann problem
    double BnL = g.sqrtmg * qL[5 + D], BnR = g.sqrtmg * qR[5 + D];
    double Bs = 0.5 * (BnL + BnR) - 0.5 * d.ic_h * (qR[8] - qL[8]);
    double phs = 0.5 * (qL[8] + qR[8]) - 0.5 * d.c_h * (BnR - BnL);
    qL[5 + D] = qR[5 + D] = Bs * g.isqrtmg;

    Kin kL = kinematics(qL, g, d.gfac);
    Kin kR = kinematics(qR, g, d.gfac);
    double lmL, lpL, lmR, lpR;
    speeds<D>(qL, kL, g, d.gamma, lmL, lpL);
    speeds<D>(qR, kR, g, d.gamma, lmR, lpR);
    double sl = fmin(0.0, fmin(lmL, lmR));
    double sr = fmax(0.0, fmax(lpL, lpR));
    double cL, cR, cU;
    if (sl == 0.0) {
        cL = 1.0;
        cR = 0.0;
        cU = 0.0;
    } else if (sr == 0.0) {
        cL = 0.0;
        cR = 1.0;
        cU = 0.0;
    } else {
        double inv = 1.0 / (sr - sl);
        cL = sr * inv;
        cR = -sl * inv;
        cU = sl * sr * inv;
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        if (v == 5 + D)
            continue;
        double fl = flux_comp<D>(v, qL, kL, g);
        double fr = flux_comp<D>(v, qR, kR, g);
        double o = cL * fl + cR * fr;
        if (cU != 0.0)
            o += cU * (cons_comp(v, qR, kR, g) - cons_comp(v, qL, kL, g));
        Fo[v] = o;
    }
    Fo[5 + D] = phs;
    Fo[8] = d.c_h2 * Bs;
}

template <int D, int KIND>
__device__ __forceinline__ void face_store(double* qL, double* qR, double x, double y, double z,
                                           const Dev& d, double* __restrict__ F, long long NF,
                                           long long f)
{
    double Fo[9];
    face_flux<D, KIND>(qL, qR, x, y, z, d, Fo);
#pragma unroll
    for (int v = 0; v < 9; ++v)
        F[v * NF + f] = Fo[v];
}

// x faces: one thread per face (the x stencil of a wave shares cache lines).
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_flux_x(const double* __restrict__ Pc, double* __restrict__ F,
                                                 Dev d)
{
    long long f = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (f >= d.nf[0])
        return;
    const int nfx = d.n[0] + 1;
    int i = (int)(f % nfx);
    long long t = f / nfx;
    int j = (int)(t % d.n[1]);
    int k = (int)(t / d.n[1]);
    // cell i-2 in ghosted coordinates
    long long base = ((long long)(k + d.g[2]) * d.py + (j + d.g[1])) * d.px + i + d.g[0] - 2;
    double qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const double* p = Pc + v * d.sv + base;
        double q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
        qL[v] = q1 + 0.5 * mc_slope(q0, q1, q2);
        qR[v] = q2 - 0.5 * mc_slope(q1, q2, q3);
    }
    face_store<0, KIND>(qL, qR, d.lo[0] + i * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                        d.lo[2] + (k + 0.5) * d.dx[2], d, F, d.nf[0], f);
}

// y or z faces: a thread marches along D over a segment of up to SEG faces at
// fixed (i, other transverse index).  Moving from face f-1/2 to f+1/2 it keeps
// q_f, q_{f+1} and the MC slope of cell f, so each face loads one new cell
// (9 values instead of 36) and computes one slope instead of two.
template <int D, int KIND, int SEG>
__global__ __launch_bounds__(BLOCK) void k_flux_march(const double* __restrict__ Pc,
                                                     double* __restrict__ F, Dev d)
{
    constexpr int O = D == 1 ? 2 : 1;          // the other transverse axis
    const int nfD = d.n[D] + 1;
    const int nseg = (nfD + SEG - 1) / SEG;
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= (long long)d.n[0] * d.n[O] * nseg)
        return;
    int i = (int)(t % d.n[0]);
    long long r = t / d.n[0];
    int a = (int)(r % d.n[O]);
    int seg = (int)(r / d.n[O]);
    int f0 = seg * SEG;
    int f1 = min(f0 + SEG, nfD);
    const long long st = D == 1 ? (long long)d.px : (long long)d.px * d.py;
    // ghosted address of cell (f0 - 2) along D
    const int gi = i + d.g[0];
    const int gj = D == 1 ? f0 - 2 + d.g[1] : a + d.g[1];
    const int gk = D == 2 ? f0 - 2 + d.g[2] : a + d.g[2];
    long long base = ((long long)gk * d.py + gj) * d.px + gi;
    const long long NF = d.nf[D];
    // face f index stride along D in the face array
    const long long fstr = D == 1 ? (long long)d.n[0] : (long long)d.n[0] * d.n[1];
    long long fidx = D == 1 ? i + (long long)d.n[0] * ((long long)f0 + (long long)(d.n[1] + 1) * a)
                            : i + (long long)d.n[0] * (a + (long long)d.n[1] * f0);
    double qb[9], qc[9], sc[9];      // cells f-1 and f, slope of cell f... set up below
    {
        double qa[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            const double* p = Pc + v * d.sv + base;
            qa[v] = p[0];
            qb[v] = p[st];
            qc[v] = p[2 * st];
        }
        // carried state for face f0: (q_{f-1}, q_f) and the slope of cell f-1
#pragma unroll
        for (int v = 0; v < 9; ++v)
            sc[v] = mc_slope(qa[v], qb[v], qc[v]);
    }
    double xyz[3];
    xyz[0] = d.lo[0] + (i + 0.5) * d.dx[0];
    xyz[O] = d.lo[O] + (a + 0.5) * d.dx[O];
    for (int f = f0; f < f1; ++f) {
        // cell f+1 is 3 cells above cell f-2
        const long long pf = base + (long long)(f - f0 + 3) * st;
        double qL[9], qR[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            double qd = Pc[v * d.sv + pf];
            double sn = mc_slope(qb[v], qc[v], qd);   // slope of cell f
            qL[v] = qb[v] + 0.5 * sc[v];               // cell f-1, right face
            qR[v] = qc[v] - 0.5 * sn;                  // cell f, left face
            sc[v] = sn;
            qb[v] = qc[v];
            qc[v] = qd;
        }
        xyz[D] = d.lo[D] + f * d.dx[D];
        face_store<D, KIND>(qL, qR, xyz[0], xyz[1], xyz[2], d, F, NF, fidx);
        fidx += fstr;
    }
}

// ---------------------------------------------------------------------------
// Metric sources at a cell centre (x, y, z) with primitives q, added to R:
// 1/2 sqrt(-g) [T^tt d_j g_tt + sum_k T^kk d_j g_kk] on the momenta (d_j g_tt =
// -2 alpha d_j alpha), zero on mass and energy (static metric), -kappa Phi on
// the cleaning scalar.  Returns the centre geometry in g.
template <int KIND>
__device__ __forceinline__ void add_sources(const Dev& d, double x, double y, double z,
                                            const double* q, Geo& g, double* R)
{
    double ka, kp;
    g = geo_deriv<KIND>(d, x, y, z, ka, kp);
    if (KIND != FLAT) {
        Kin kk = kinematics(q, g, d.gfac);
        double ia2 = 1.0 / (g.alpha * g.alpha);
        double Ttt = (kk.wtot * kk.W * kk.W - kk.ptot) * ia2 - kk.bt * kk.bt;
        double uu = q[2] * q[2] + q[3] * q[3] + q[4] * q[4];
        double bb = kk.b[0] * kk.b[0] + kk.b[1] * kk.b[1] + kk.b[2] * kk.b[2];
        double Tkk = kk.wtot * uu + 3.0 * kk.ptot * g.ipsi4 - bb;
        double K = 0.5 * g.sqrtmg * (-2.0 * g.alpha * Ttt * ka + Tkk * kp);
        R[2] += K * x;
        R[3] += K * y;
        R[4] += K * z;
    }
    R[8] -= d.kappa * q[8];
}

// Flux differences + sources for cell c (i,j,k); q are its primitives.
template <int KIND>
__device__ __forceinline__ void rhs_cell(const Dev& d, const double* __restrict__ Fx,
                                         const double* __restrict__ Fy,
                                         const double* __restrict__ Fz, long long c, int i, int j,
                                         int k, const double* q, Geo& g, double* R)
{
#pragma unroll
    for (int v = 0; v < 9; ++v)
        R[v] = 0.0;
    if (d.act[0]) {
        long long f = i + (long long)(d.n[0] + 1) * (j + (long long)d.n[1] * k);
#pragma unroll
        for (int v = 0; v < 9; ++v)
            R[v] -= (Fx[v * d.nf[0] + f + 1] - Fx[v * d.nf[0] + f]) * d.idx[0];
    }
    if (d.act[1]) {
        long long f = i + (long long)d.n[0] * (j + (long long)(d.n[1] + 1) * k);
#pragma unroll
        for (int v = 0; v < 9; ++v)
            R[v] -= (Fy[v * d.nf[1] + f + d.n[0]] - Fy[v * d.nf[1] + f]) * d.idx[1];
    }
    if (d.act[2]) {
        long long nxy = (long long)d.n[0] * d.n[1];
#pragma unroll
        for (int v = 0; v < 9; ++v)
            R[v] -= (Fz[v * d.nf[2] + c + nxy] - Fz[v * d.nf[2] + c]) * d.idx[2];
    }
    add_sources<KIND>(d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                      d.lo[2] + (k + 0.5) * d.dx[2], q, g, R);
}

__device__ __forceinline__ long long cache_index(const Dev& d, int i, int j, int k)
{
    return ((long long)(k + d.g[2]) * d.py + (j + d.g[1])) * d.px + (i + d.g[0]);
}

__device__ __forceinline__ void count_flags(unsigned long long* cnt_base, int flags, int iters)
{
    unsigned long long* cnt = cnt_base + (size_t)(blockIdx.x % CNT_SLOTS) * CNT_WORDS;
    // one atomic per wave and counter
    unsigned long long mf = __ballot((flags & FLAG_FAIL) != 0);
    unsigned long long ma = __ballot((flags & FLAG_ATM) != 0);
    unsigned long long mp = __ballot((flags & FLAG_PFLOOR) != 0);
    unsigned long long mb = __ballot((flags & FLAG_FALLBACK) != 0);
    unsigned long long act = __ballot(1);
    int lane = __lane_id();
    int leader = __ffsll((long long)act) - 1;
    int itmax = iters;
    for (int o = 32; o > 0; o >>= 1)
        itmax = max(itmax, __shfl_xor(itmax, o));
    if (lane == leader) {
        if (mf)
            atomicAdd(&cnt[CNT_FAIL], (unsigned long long)__popcll(mf));
        if (ma)
            atomicAdd(&cnt[CNT_ATM], (unsigned long long)__popcll(ma));
        if (mp)
            atomicAdd(&cnt[CNT_PFLOOR], (unsigned long long)__popcll(mp));
        if (mb)
            atomicAdd(&cnt[CNT_FALLBACK], (unsigned long long)__popcll(mb));
        // no returning atomic here: waiting on one would also wait for the
        // wave's outstanding result stores before it can retire
        atomicMax(&cnt[CNT_MAXIT], (unsigned long long)itmax);
    }
}

// Flux differences, sources, Runge-Kutta combination
//   U^(s+1) = U^(s) + a (U^n - U^(s)) + b dt R,
// and recovery of the primitives (in place in the cache), for every cell.
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_update(const double* __restrict__ Fx,
                                                 const double* __restrict__ Fy,
                                                 const double* __restrict__ Fz,
                                                 double* __restrict__ Pc,
                                                 const double* Un, const double* Us, double* Uout,
                                                 Dev d, double dt, double a, double b,
                                                 unsigned long long* __restrict__ cnt)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    bool live = c < d.N;
    int flags = 0, iters = 0;
    if (live) {
        int i = (int)(c % d.n[0]);
        long long t = c / d.n[0];
        int j = (int)(t % d.n[1]);
        int k = (int)(t / d.n[1]);
        long long pc = cache_index(d, i, j, k);
        double q[9], R[9], u[9], p[9];
#pragma unroll
        for (int v = 0; v < 9; ++v)
            q[v] = Pc[v * d.sv + pc];
        Geo g;
        rhs_cell<KIND>(d, Fx, Fy, Fz, c, i, j, k, q, g, R);
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            double un = Un[v * d.N + c], us = Us[v * d.N + c];
            u[v] = us + a * (un - us) + b * (dt * R[v]);
        }
        flags = recover_cell(d, g, u, q, p, iters);
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            Uout[v * d.N + c] = u[v];
            Pc[v * d.sv + pc] = p[v];
        }
    }
    count_flags(cnt, flags, iters);
}

// Per-thread counts (summed over the cells a thread updated) reduced over the
// wave, one atomic per wave and counter into the block's slot.
__device__ __forceinline__ void count_sums(unsigned long long* cnt_base, int nf, int na, int np,
                                           int nb, int itmax)
{
    unsigned long long* cnt = cnt_base + (size_t)(blockIdx.x % CNT_SLOTS) * CNT_WORDS;
    for (int o = 32; o > 0; o >>= 1) {
        nf += __shfl_xor(nf, o);
        na += __shfl_xor(na, o);
        np += __shfl_xor(np, o);
        nb += __shfl_xor(nb, o);
        itmax = max(itmax, __shfl_xor(itmax, o));
    }
    unsigned long long act = __ballot(1);
    if (__lane_id() == __ffsll((long long)act) - 1) {
        if (nf)
            atomicAdd(&cnt[CNT_FAIL], (unsigned long long)nf);
        if (na)
            atomicAdd(&cnt[CNT_ATM], (unsigned long long)na);
        if (np)
            atomicAdd(&cnt[CNT_PFLOOR], (unsigned long long)np);
        if (nb)
            atomicAdd(&cnt[CNT_FALLBACK], (unsigned long long)nb);
        atomicMax(&cnt[CNT_MAXIT], (unsigned long long)itmax);
    }
}

// z faces and the cell update fused (3D grids).  A thread owns cells
// k0..k1-1 of the column (i, j), computes the z faces k0-1/2 .. k1-1/2 in
// order (one face per cell plus one) keeping the previous face flux in
// registers, and for each cell forms R from that z flux difference and the
// x/y face fluxes, adds the sources, combines the RK stage and recovers the
// primitives, written to the other primitive cache Pn (segments of one column
// overlap by two cells, so the cache read here cannot be updated in place).
template <int KIND, int SEG>
__global__ __launch_bounds__(BLOCK) void k_update_zmarch(
    const double* __restrict__ Fx, const double* __restrict__ Fy, const double* __restrict__ Pc,
    double* __restrict__ Pn, const double* Un, const double* Us, double* Uout, Dev d, double dt,
    double a, double b, unsigned long long* __restrict__ cnt)
{
    const int nz = d.n[2];
    const int nseg = (nz + SEG - 1) / SEG;
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int nfail = 0, natm = 0, npf = 0, nfb = 0, itmax = 0;
    if (t < (long long)d.n[0] * d.n[1] * nseg) {
        const int i = (int)(t % d.n[0]);
        const long long r = t / d.n[0];
        const int j = (int)(r % d.n[1]);
        const int seg = (int)(r / d.n[1]);
        const int k0 = seg * SEG;
        const int k1 = min(k0 + SEG, nz);
        const long long st = (long long)d.px * d.py;
        const long long col = (long long)(j + d.g[1]) * d.px + i + d.g[0];
        // ghosted address of cell k0 - 2
        const long long base = col + (long long)(k0 - 2 + d.g[2]) * st;
        const double x = d.lo[0] + (i + 0.5) * d.dx[0];
        const double y = d.lo[1] + (j + 0.5) * d.dx[1];
        double qb[9], qc[9], sc[9], Fp[9];
        {
            double qa[9], qL[9], qR[9];
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                const double* p = Pc + v * d.sv + base;
                qa[v] = p[0];
                qb[v] = p[st];
                qc[v] = p[2 * st];
            }
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                double qd = Pc[v * d.sv + base + 3 * st];
                double s0 = mc_slope(qa[v], qb[v], qc[v]);   // cell k0-1
                double s1 = mc_slope(qb[v], qc[v], qd);      // cell k0
                qL[v] = qb[v] + 0.5 * s0;
                qR[v] = qc[v] - 0.5 * s1;
                sc[v] = s1;
                qb[v] = qc[v];
                qc[v] = qd;
            }
            face_flux<2, KIND>(qL, qR, x, y, d.lo[2] + k0 * d.dx[2], d, Fp);
        }
        // window now: qb = q_k0, qc = q_{k0+1}, sc = slope of cell k0
        for (int k = k0; k < k1; ++k) {
            double q[9], qL[9], qR[9], Fc[9];
            const long long pnext = base + (long long)(k - k0 + 4) * st;   // cell k+2
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                double qd = Pc[v * d.sv + pnext];
                double sn = mc_slope(qb[v], qc[v], qd);      // cell k+1
                q[v] = qb[v];
                qL[v] = qb[v] + 0.5 * sc[v];
                qR[v] = qc[v] - 0.5 * sn;
                sc[v] = sn;
                qb[v] = qc[v];
                qc[v] = qd;
            }
            const double z = d.lo[2] + (k + 0.5) * d.dx[2];
            face_flux<2, KIND>(qL, qR, x, y, z + 0.5 * d.dx[2], d, Fc);
            const long long c = i + (long long)d.n[0] * (j + (long long)d.n[1] * k);
            double R[9], u[9], p[9];
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                R[v] = -(Fc[v] - Fp[v]) * d.idx[2];
                Fp[v] = Fc[v];
            }
            if (d.act[0]) {
                long long f = i + (long long)(d.n[0] + 1) * (j + (long long)d.n[1] * k);
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    R[v] -= (Fx[v * d.nf[0] + f + 1] - Fx[v * d.nf[0] + f]) * d.idx[0];
            }
            if (d.act[1]) {
                long long f = i + (long long)d.n[0] * (j + (long long)(d.n[1] + 1) * k);
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    R[v] -= (Fy[v * d.nf[1] + f + d.n[0]] - Fy[v * d.nf[1] + f]) * d.idx[1];
            }
            Geo g;
            add_sources<KIND>(d, x, y, z, q, g, R);
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                double un = Un[v * d.N + c], us = Us[v * d.N + c];
                u[v] = us + a * (un - us) + b * (dt * R[v]);
            }
            int iters = 0;
            int flags = recover_cell(d, g, u, q, p, iters);
            nfail += (flags & FLAG_FAIL) != 0;
            natm += (flags & FLAG_ATM) != 0;
            npf += (flags & FLAG_PFLOOR) != 0;
            nfb += (flags & FLAG_FALLBACK) != 0;
            itmax = max(itmax, iters);
            const long long pc = col + (long long)(k + d.g[2]) * st;
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                Uout[v * d.N + c] = u[v];
                Pn[v * d.sv + pc] = p[v];
            }
        }
    }
    count_sums(cnt, nfail, natm, npf, nfb, itmax);
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_rhs(const double* __restrict__ Fx,
                                              const double* __restrict__ Fy,
                                              const double* __restrict__ Fz,
                                              const double* __restrict__ Pc, double* __restrict__ R,
                                              Dev d)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i = (int)(c % d.n[0]);
    long long t = c / d.n[0];
    int j = (int)(t % d.n[1]);
    int k = (int)(t / d.n[1]);
    long long pc = cache_index(d, i, j, k);
    double q[9], r[9];
#pragma unroll
    for (int v = 0; v < 9; ++v)
        q[v] = Pc[v * d.sv + pc];
    Geo g;
    rhs_cell<KIND>(d, Fx, Fy, Fz, c, i, j, k, q, g, r);
#pragma unroll
    for (int v = 0; v < 9; ++v)
        R[v * d.N + c] = r[v];
}

// Primitive -> conserved at cell centres; also loads P into the cache.
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_cons(const double* __restrict__ P, double* __restrict__ U,
                                               double* __restrict__ Pc, Dev d)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i = (int)(c % d.n[0]);
    long long t = c / d.n[0];
    int j = (int)(t % d.n[1]);
    int k = (int)(t / d.n[1]);
    long long pc = cache_index(d, i, j, k);
    double q[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        q[v] = P[v * d.N + c];
        Pc[v * d.sv + pc] = q[v];
    }
    if (U) {
        Geo g = geo_at<KIND>(d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                             d.lo[2] + (k + 0.5) * d.dx[2]);
        Kin kk = kinematics(q, g, d.gfac);
#pragma unroll
        for (int v = 0; v < 8; ++v)
            U[v * d.N + c] = cons_comp(v, q, kk, g);
        U[8 * d.N + c] = q[8];
    }
}

// Conserved -> primitive (recovery + floors) with the cache as the guess.
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_prim(const double* __restrict__ U, double* __restrict__ P,
                                               double* __restrict__ Pc, Dev d,
                                               unsigned long long* __restrict__ cnt)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int flags = 0, iters = 0;
    if (c < d.N) {
        int i = (int)(c % d.n[0]);
        long long t = c / d.n[0];
        int j = (int)(t % d.n[1]);
        int k = (int)(t / d.n[1]);
        long long pc = cache_index(d, i, j, k);
        double q[9], u[9], p[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            q[v] = Pc[v * d.sv + pc];
            u[v] = U[v * d.N + c];
        }
        Geo g = geo_at<KIND>(d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                             d.lo[2] + (k + 0.5) * d.dx[2]);
        flags = recover_cell(d, g, u, q, p, iters);
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            P[v * d.N + c] = p[v];
            Pc[v * d.sv + pc] = p[v];
        }
    }
    count_flags(cnt, flags, iters);
}

// ---------------------------------------------------------------------------
// Launchers

static inline unsigned blocks_for(long long n)
{
    return (unsigned)((n + BLOCK - 1) / BLOCK);
}

hipError_t launch_fill(double* p, long long n, double v, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_zero_counters(unsigned long long* cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(BLOCK), 0, s, cnt);
    return hipGetLastError();
}

hipError_t launch_ghosts(double* Pc, const Dev& d, hipStream_t s)
{
    long long seg[3];
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        seg[a] = d.act[a] ? 2LL * d.g[a] * d.n[b] * d.n[c] : 0;
    }
    long long tot = seg[0] + seg[1] + seg[2];
    if (tot > 0)
        hipLaunchKernelGGL(k_ghosts, dim3(blocks_for(tot)), dim3(BLOCK), 0, s, Pc, d, seg[0], seg[1],
                           seg[2]);
    return hipGetLastError();
}

static constexpr int MARCH_SEG = 8;

template <int KIND>
static hipError_t launch_flux_k(int dir, const double* Pc, double* F, const Dev& d, hipStream_t s)
{
    if (dir == 0) {
        hipLaunchKernelGGL(k_flux_x<KIND>, dim3(blocks_for(d.nf[0])), dim3(BLOCK), 0, s, Pc, F, d);
    } else {
        const int o = dir == 1 ? 2 : 1;
        long long nseg = (d.n[dir] + 1 + MARCH_SEG - 1) / MARCH_SEG;
        unsigned nb = blocks_for((long long)d.n[0] * d.n[o] * nseg);
        if (dir == 1)
            hipLaunchKernelGGL((k_flux_march<1, KIND, MARCH_SEG>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        else
            hipLaunchKernelGGL((k_flux_march<2, KIND, MARCH_SEG>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
    }
    return hipGetLastError();
}

hipError_t launch_flux(int kind, int dir, const double* Pc, double* F, const Dev& d, hipStream_t s)
{
    return kind == FLAT ? launch_flux_k<FLAT>(dir, Pc, F, d, s) : launch_flux_k<ISO>(dir, Pc, F, d, s);
}

hipError_t launch_update(int kind, const double* Fx, const double* Fy, const double* Fz, double* Pc,
                         const double* Un, const double* Us, double* Uout, const Dev& d, double dt,
                         double a, double b, unsigned long long* cnt, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL(k_update<FLAT>, dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Un, Us, Uout, d,
                           dt, a, b, cnt);
    else
        hipLaunchKernelGGL(k_update<ISO>, dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Un, Us, Uout, d,
                           dt, a, b, cnt);
    return hipGetLastError();
}

static constexpr int ZSEG = 8;

hipError_t launch_update_zmarch(int kind, const double* Fx, const double* Fy, const double* Pc,
                                double* Pn, const double* Un, const double* Us, double* Uout,
                                const Dev& d, double dt, double a, double b, unsigned long long* cnt,
                                hipStream_t s)
{
    long long nseg = (d.n[2] + ZSEG - 1) / ZSEG;
    unsigned nb = blocks_for((long long)d.n[0] * d.n[1] * nseg);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_update_zmarch<FLAT, ZSEG>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Pc, Pn, Un,
                           Us, Uout, d, dt, a, b, cnt);
    else
        hipLaunchKernelGGL((k_update_zmarch<ISO, ZSEG>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Pc, Pn, Un,
                           Us, Uout, d, dt, a, b, cnt);
    return hipGetLastError();
}

hipError_t launch_rhs(int kind, const double* Fx, const double* Fy, const double* Fz, const double* Pc,
                      double* R, const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL(k_rhs<FLAT>, dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    else
        hipLaunchKernelGGL(k_rhs<ISO>, dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    return hipGetLastError();
}

hipError_t launch_cons(int kind, const double* P, double* U, double* Pc, const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL(k_cons<FLAT>, dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    else
        hipLaunchKernelGGL(k_cons<ISO>, dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    return hipGetLastError();
}

hipError_t launch_prim(int kind, const double* U, double* P, double* Pc, const Dev& d,
                       unsigned long long* cnt, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL(k_prim<FLAT>, dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    else
        hipLaunchKernelGGL(k_prim<ISO>, dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    return hipGetLastError();
}

}  // namespace grmhd
