// grmhd_kernels.hip -- HIP kernels of the GRMHD substep (gfx950, wave64).
//
// One substep (section 2.2 of the paper) on a 3D grid is four launches:
//   k_ghosts          ghost zones of the primitive cache (periodic / zero-gradient)
//   k_flux_x          per x face: MC reconstruction of the 9 primitives, exact
//                     (normal field, Phi) cleaning pair, face physics of both
//                     states, HLLE flux (section 3.2)
//   k_flux_march<1>   the same for y faces, a thread marching along y
//   k_update_zmarch   a thread marching along z: z faces, flux differences,
//                     metric sources (eq. 2), SSP Runge-Kutta combination,
//                     Newton recovery of the primitives with the
//                     atmosphere/floor policy, status counters
// 1D and 2D grids use the face kernels of every active axis and k_update.
//
// T is the type of the primitive caches, the face fluxes and the face physics:
// double (FP64 path) or float (mixed precision).  The metric is always
// evaluated in double, and the Runge-Kutta accumulation, the conserved
// variables and the recovery are always double.
//
// Threads are mapped over faces (cells), x fastest, so every load and store of
// the structure-of-arrays buffers is coalesced.
#include "grmhd_device.h"
#include "grmhd_internal.h"

namespace grmhd {

static constexpr int BLOCK = 256;
static constexpr int MARCH_SEG = 8;   // faces per thread in the y and z marches

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(T* __restrict__ p, long long n, T v)
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
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ghosts(T* __restrict__ Pc, Dev d, long long s0, long long s1,
                                                 long long s2)
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
template <int D, int KIND, typename T>
__device__ __forceinline__ void face_flux(T* qL, T* qR, double x, double y, double z, const Dev& d,
                                          T* Fo)
{
    const GeoT<T> g = geo_cast<T>(geo_at<KIND>(d, x, y, z));
    const T half = T(0.5), ch = (T)d.c_h, ich = (T)d.ic_h;

    // cleaning pair: exact solution of the linear (Bd^n, Phi) Riemann problem
    T BnL = g.sqrtmg * qL[5 + D], BnR = g.sqrtmg * qR[5 + D];
    T Bs = half * (BnL + BnR) - half * ich * (qR[8] - qL[8]);
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
    Fo[5 + D] = phs;
    Fo[8] = (T)d.c_h2 * Bs;
}

template <int D, int KIND, typename T>
__device__ __forceinline__ void face_store(T* qL, T* qR, double x, double y, double z, const Dev& d,
                                           T* __restrict__ F, long long NF, long long f)
{
    T Fo[9];
    face_flux<D, KIND>(qL, qR, x, y, z, d, Fo);
#pragma unroll
    for (int v = 0; v < 9; ++v)
        F[v * NF + f] = Fo[v];
}

// x faces: one thread per face (the x stencil of a wave shares cache lines).
template <int KIND, typename T>
__global__ __launch_bounds__(BLOCK) void k_flux_x(const T* __restrict__ Pc, T* __restrict__ F, Dev d)
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
    const T half = T(0.5);
    T qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const T* p = Pc + v * d.sv + base;
        T q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
        qL[v] = q1 + half * mc_slope(q0, q1, q2);
        qR[v] = q2 - half * mc_slope(q1, q2, q3);
    }
    face_store<0, KIND>(qL, qR, d.lo[0] + i * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                        d.lo[2] + (k + 0.5) * d.dx[2], d, F, d.nf[0], f);
}

// y or z faces: a thread marches along D over a segment of up to SEG faces at
// fixed (i, other transverse index).  Moving from face f-1/2 to f+1/2 it keeps
// q_f, q_{f+1} and the MC slope of cell f, so each face loads one new cell
// (9 values instead of 36) and computes one slope instead of two.
template <int D, int KIND, int SEG, typename T>
__global__ __launch_bounds__(BLOCK) void k_flux_march(const T* __restrict__ Pc, T* __restrict__ F, Dev d)
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
    // face index and its stride along D in the face array
    const long long fstr = D == 1 ? (long long)d.n[0] : (long long)d.n[0] * d.n[1];
    long long fidx = D == 1 ? i + (long long)d.n[0] * ((long long)f0 + (long long)(d.n[1] + 1) * a)
                            : i + (long long)d.n[0] * (a + (long long)d.n[1] * f0);
    const T half = T(0.5);
    T qb[9], qc[9], sc[9];      // cells f-1 and f, MC slope of cell f-1
    {
        T qa[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            const T* p = Pc + v * d.sv + base;
            qa[v] = p[0];
            qb[v] = p[st];
            qc[v] = p[2 * st];
        }
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
        T qL[9], qR[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            T qd = Pc[v * d.sv + pf];
            T sn = mc_slope(qb[v], qc[v], qd);   // slope of cell f
            qL[v] = qb[v] + half * sc[v];        // cell f-1, right face
            qR[v] = qc[v] - half * sn;           // cell f, left face
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
// the cleaning scalar.  The source is evaluated in T; the centre geometry is
// returned in g (double, for the recovery).
template <int KIND, typename T>
__device__ __forceinline__ void add_sources(const Dev& d, double x, double y, double z, const T* q,
                                            Geo& g, double* R)
{
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
    R[8] -= d.kappa * (double)q[8];
}

// Flux differences + sources for cell c (i,j,k); q are its primitives.
template <int KIND, typename T>
__device__ __forceinline__ void rhs_cell(const Dev& d, const T* __restrict__ Fx, const T* __restrict__ Fy,
                                         const T* __restrict__ Fz, long long c, int i, int j, int k,
                                         const T* q, Geo& g, double* R)
{
#pragma unroll
    for (int v = 0; v < 9; ++v)
        R[v] = 0.0;
    if (d.act[0]) {
        long long f = i + (long long)(d.n[0] + 1) * (j + (long long)d.n[1] * k);
#pragma unroll
        for (int v = 0; v < 9; ++v)
            R[v] -= ((double)Fx[v * d.nf[0] + f + 1] - (double)Fx[v * d.nf[0] + f]) * d.idx[0];
    }
    if (d.act[1]) {
        long long f = i + (long long)d.n[0] * (j + (long long)(d.n[1] + 1) * k);
#pragma unroll
        for (int v = 0; v < 9; ++v)
            R[v] -= ((double)Fy[v * d.nf[1] + f + d.n[0]] - (double)Fy[v * d.nf[1] + f]) * d.idx[1];
    }
    if (d.act[2]) {
        long long nxy = (long long)d.n[0] * d.n[1];
#pragma unroll
        for (int v = 0; v < 9; ++v)
            R[v] -= ((double)Fz[v * d.nf[2] + c + nxy] - (double)Fz[v * d.nf[2] + c]) * d.idx[2];
    }
    add_sources<KIND>(d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                      d.lo[2] + (k + 0.5) * d.dx[2], q, g, R);
}

__device__ __forceinline__ long long cache_index(const Dev& d, int i, int j, int k)
{
    return ((long long)(k + d.g[2]) * d.py + (j + d.g[1])) * d.px + (i + d.g[0]);
}

// Per-thread counts reduced over the wave, one atomic per wave and counter
// into the block's slot (never a returning atomic: waiting on one would also
// wait for the wave's outstanding stores).
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

__device__ __forceinline__ void tally(int flags, int iters, int& nf, int& na, int& np, int& nb, int& itmax)
{
    nf += (flags & FLAG_FAIL) != 0;
    na += (flags & FLAG_ATM) != 0;
    np += (flags & FLAG_PFLOOR) != 0;
    nb += (flags & FLAG_FALLBACK) != 0;
    itmax = max(itmax, iters);
}

// RK combination U^(s+1) = U^(s) + a (U^n - U^(s)) + b dt R and the recovery
// of the primitives for one cell (all in double); q are the cell's current
// primitives (the Newton guess).  Writes U^(s+1) and the new primitives.
template <typename T>
__device__ __forceinline__ int stage_cell(const Dev& d, const Geo& g, const double* R, const T* q,
                                          const double* Un, const double* Us, double* Uout, long long c,
                                          T* Pout, long long pc, double dt, double a, double b,
                                          int& iters)
{
    double u[9], p[9], qg[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        double un = Un[v * d.N + c], us = Us[v * d.N + c];
        u[v] = us + a * (un - us) + b * (dt * R[v]);
        qg[v] = (double)q[v];
    }
    int flags = recover_cell(d, g, u, qg, p, iters);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        Uout[v * d.N + c] = u[v];
        Pout[v * d.sv + pc] = (T)p[v];
    }
    return flags;
}

// 1D/2D update: flux differences, sources, RK combination and recovery of the
// primitives (in place in the cache), for every cell.
template <int KIND, typename T>
__global__ __launch_bounds__(BLOCK) void k_update(const T* __restrict__ Fx, const T* __restrict__ Fy,
                                                 const T* __restrict__ Fz, T* __restrict__ Pc,
                                                 const double* Un, const double* Us, double* Uout, Dev d,
                                                 double dt, double a, double b,
                                                 unsigned long long* __restrict__ cnt)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int nf = 0, na = 0, np = 0, nb = 0, itmax = 0;
    if (c < d.N) {
        int i = (int)(c % d.n[0]);
        long long t = c / d.n[0];
        int j = (int)(t % d.n[1]);
        int k = (int)(t / d.n[1]);
        long long pc = cache_index(d, i, j, k);
        T q[9];
        double R[9];
#pragma unroll
        for (int v = 0; v < 9; ++v)
            q[v] = Pc[v * d.sv + pc];
        Geo g;
        rhs_cell<KIND>(d, Fx, Fy, Fz, c, i, j, k, q, g, R);
        int iters = 0;
        int flags = stage_cell(d, g, R, q, Un, Us, Uout, c, Pc, pc, dt, a, b, iters);
        tally(flags, iters, nf, na, np, nb, itmax);
    }
    count_sums(cnt, nf, na, np, nb, itmax);
}

// z faces and the cell update fused (3D grids).  A thread owns cells
// k0..k1-1 of the column (i, j), computes the z faces k0-1/2 .. k1-1/2 in
// order (one face per cell plus one) keeping the previous face flux in
// registers, and for each cell forms R from that z flux difference and the
// x/y face fluxes, adds the sources, combines the RK stage and recovers the
// primitives, written to the other primitive cache Pn (segments of one column
// overlap by two cells, so the cache read here cannot be updated in place).
template <int KIND, int SEG, typename T>
__global__ __launch_bounds__(BLOCK) void k_update_zmarch(
    const T* __restrict__ Fx, const T* __restrict__ Fy, const T* __restrict__ Pc, T* __restrict__ Pn,
    const double* Un, const double* Us, double* Uout, Dev d, double dt, double a, double b,
    unsigned long long* __restrict__ cnt)
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
        const T half = T(0.5);
        T qb[9], qc[9], sc[9], Fp[9];
        {
            T qa[9], qL[9], qR[9];
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                const T* p = Pc + v * d.sv + base;
                qa[v] = p[0];
                qb[v] = p[st];
                qc[v] = p[2 * st];
            }
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                T qd = Pc[v * d.sv + base + 3 * st];
                T s0 = mc_slope(qa[v], qb[v], qc[v]);   // cell k0-1
                T s1 = mc_slope(qb[v], qc[v], qd);      // cell k0
                qL[v] = qb[v] + half * s0;
                qR[v] = qc[v] - half * s1;
                sc[v] = s1;
                qb[v] = qc[v];
                qc[v] = qd;
            }
            face_flux<2, KIND>(qL, qR, x, y, d.lo[2] + k0 * d.dx[2], d, Fp);
        }
        // window now: qb = q_k0, qc = q_{k0+1}, sc = slope of cell k0
        for (int k = k0; k < k1; ++k) {
            T q[9], qL[9], qR[9], Fc[9];
            const long long pnext = base + (long long)(k - k0 + 4) * st;   // cell k+2
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                T qd = Pc[v * d.sv + pnext];
                T sn = mc_slope(qb[v], qc[v], qd);      // cell k+1
                q[v] = qb[v];
                qL[v] = qb[v] + half * sc[v];
                qR[v] = qc[v] - half * sn;
                sc[v] = sn;
                qb[v] = qc[v];
                qc[v] = qd;
            }
            const double z = d.lo[2] + (k + 0.5) * d.dx[2];
            face_flux<2, KIND>(qL, qR, x, y, z + 0.5 * d.dx[2], d, Fc);
            const long long c = i + (long long)d.n[0] * (j + (long long)d.n[1] * k);
            double R[9];
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                R[v] = -((double)Fc[v] - (double)Fp[v]) * d.idx[2];
                Fp[v] = Fc[v];
            }
            if (d.act[0]) {
                long long f = i + (long long)(d.n[0] + 1) * (j + (long long)d.n[1] * k);
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    R[v] -= ((double)Fx[v * d.nf[0] + f + 1] - (double)Fx[v * d.nf[0] + f]) * d.idx[0];
            }
            if (d.act[1]) {
                long long f = i + (long long)d.n[0] * (j + (long long)(d.n[1] + 1) * k);
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    R[v] -= ((double)Fy[v * d.nf[1] + f + d.n[0]] - (double)Fy[v * d.nf[1] + f]) *
                            d.idx[1];
            }
            Geo g;
            add_sources<KIND>(d, x, y, z, q, g, R);
            int iters = 0;
            const long long pc = col + (long long)(k + d.g[2]) * st;
            int flags = stage_cell(d, g, R, q, Un, Us, Uout, c, Pn, pc, dt, a, b, iters);
            tally(flags, iters, nfail, natm, npf, nfb, itmax);
        }
    }
    count_sums(cnt, nfail, natm, npf, nfb, itmax);
}

template <int KIND, typename T>
__global__ __launch_bounds__(BLOCK) void k_rhs(const T* __restrict__ Fx, const T* __restrict__ Fy,
                                              const T* __restrict__ Fz, const T* __restrict__ Pc,
                                              double* __restrict__ R, Dev d)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= d.N)
        return;
    int i = (int)(c % d.n[0]);
    long long t = c / d.n[0];
    int j = (int)(t % d.n[1]);
    int k = (int)(t / d.n[1]);
    long long pc = cache_index(d, i, j, k);
    T q[9];
    double r[9];
#pragma unroll
    for (int v = 0; v < 9; ++v)
        q[v] = Pc[v * d.sv + pc];
    Geo g;
    rhs_cell<KIND>(d, Fx, Fy, Fz, c, i, j, k, q, g, r);
#pragma unroll
    for (int v = 0; v < 9; ++v)
        R[v * d.N + c] = r[v];
}

// Primitive -> conserved at cell centres (double); also loads P into the cache.
template <int KIND, typename T>
__global__ __launch_bounds__(BLOCK) void k_cons(const double* __restrict__ P, double* __restrict__ U,
                                               T* __restrict__ Pc, Dev d)
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
        Pc[v * d.sv + pc] = (T)q[v];
    }
    if (U) {
        const GeoT<double> g = geo_cast<double>(geo_at<KIND>(
            d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1], d.lo[2] + (k + 0.5) * d.dx[2]));
        Kin<double> kk = kinematics(q, g, d.gfac);
#pragma unroll
        for (int v = 0; v < 8; ++v)
            U[v * d.N + c] = cons_comp(v, q, kk, g);
        U[8 * d.N + c] = q[8];
    }
}

// Conserved -> primitive (recovery + floors, double) with the cache as the guess.
template <int KIND, typename T>
__global__ __launch_bounds__(BLOCK) void k_prim(const double* __restrict__ U, double* __restrict__ P,
                                               T* __restrict__ Pc, Dev d,
                                               unsigned long long* __restrict__ cnt)
{
    long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int nf = 0, na = 0, np = 0, nb = 0, itmax = 0;
    if (c < d.N) {
        int i = (int)(c % d.n[0]);
        long long t = c / d.n[0];
        int j = (int)(t % d.n[1]);
        int k = (int)(t / d.n[1]);
        long long pc = cache_index(d, i, j, k);
        double q[9], u[9], p[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            q[v] = (double)Pc[v * d.sv + pc];
            u[v] = U[v * d.N + c];
        }
        Geo g = geo_at<KIND>(d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                             d.lo[2] + (k + 0.5) * d.dx[2]);
        int iters = 0;
        int flags = recover_cell(d, g, u, q, p, iters);
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            P[v * d.N + c] = p[v];
            Pc[v * d.sv + pc] = (T)p[v];
        }
        tally(flags, iters, nf, na, np, nb, itmax);
    }
    count_sums(cnt, nf, na, np, nb, itmax);
}

// ---------------------------------------------------------------------------
// Launchers (T = double or float)

static inline unsigned blocks_for(long long n)
{
    return (unsigned)((n + BLOCK - 1) / BLOCK);
}

template <typename T>
hipError_t launch_fill(T* p, long long n, double v, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n, (T)v);
    return hipGetLastError();
}

hipError_t launch_zero_counters(unsigned long long* cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(BLOCK), 0, s, cnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ghosts(T* Pc, const Dev& d, hipStream_t s)
{
    long long seg[3];
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        seg[a] = d.act[a] ? 2LL * d.g[a] * d.n[b] * d.n[c] : 0;
    }
    long long tot = seg[0] + seg[1] + seg[2];
    if (tot > 0)
        hipLaunchKernelGGL(k_ghosts<T>, dim3(blocks_for(tot)), dim3(BLOCK), 0, s, Pc, d, seg[0], seg[1],
                           seg[2]);
    return hipGetLastError();
}

template <int KIND, typename T>
static hipError_t launch_flux_k(int dir, const T* Pc, T* F, const Dev& d, hipStream_t s)
{
    if (dir == 0) {
        hipLaunchKernelGGL((k_flux_x<KIND, T>), dim3(blocks_for(d.nf[0])), dim3(BLOCK), 0, s, Pc, F, d);
    } else {
        const int o = dir == 1 ? 2 : 1;
        long long nseg = (d.n[dir] + 1 + MARCH_SEG - 1) / MARCH_SEG;
        unsigned nb = blocks_for((long long)d.n[0] * d.n[o] * nseg);
        if (dir == 1)
            hipLaunchKernelGGL((k_flux_march<1, KIND, MARCH_SEG, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        else
            hipLaunchKernelGGL((k_flux_march<2, KIND, MARCH_SEG, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_flux(int kind, int dir, const T* Pc, T* F, const Dev& d, hipStream_t s)
{
    return kind == FLAT ? launch_flux_k<FLAT>(dir, Pc, F, d, s) : launch_flux_k<ISO>(dir, Pc, F, d, s);
}

template <typename T>
hipError_t launch_update(int kind, const T* Fx, const T* Fy, const T* Fz, T* Pc, const double* Un,
                         const double* Us, double* Uout, const Dev& d, double dt, double a, double b,
                         unsigned long long* cnt, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_update<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Un, Us, Uout, d,
                           dt, a, b, cnt);
    else
        hipLaunchKernelGGL((k_update<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Un, Us, Uout, d,
                           dt, a, b, cnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update_zmarch(int kind, const T* Fx, const T* Fy, const T* Pc, T* Pn, const double* Un,
                                const double* Us, double* Uout, const Dev& d, double dt, double a,
                                double b, unsigned long long* cnt, hipStream_t s)
{
    long long nseg = (d.n[2] + MARCH_SEG - 1) / MARCH_SEG;
    unsigned nb = blocks_for((long long)d.n[0] * d.n[1] * nseg);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_update_zmarch<FLAT, MARCH_SEG, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Pc, Pn,
                           Un, Us, Uout, d, dt, a, b, cnt);
    else
        hipLaunchKernelGGL((k_update_zmarch<ISO, MARCH_SEG, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Pc, Pn,
                           Un, Us, Uout, d, dt, a, b, cnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rhs(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, double* R,
                      const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_rhs<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    else
        hipLaunchKernelGGL((k_rhs<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cons(int kind, const double* P, double* U, T* Pc, const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_cons<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    else
        hipLaunchKernelGGL((k_cons<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prim(int kind, const double* U, double* P, T* Pc, const Dev& d, unsigned long long* cnt,
                       hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_prim<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    else
        hipLaunchKernelGGL((k_prim<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    return hipGetLastError();
}

// explicit instantiations for the two precisions
#define GRMHD_INSTANTIATE(T)                                                                            \
    template hipError_t launch_fill<T>(T*, long long, double, hipStream_t);                             \
    template hipError_t launch_ghosts<T>(T*, const Dev&, hipStream_t);                                  \
    template hipError_t launch_flux<T>(int, int, const T*, T*, const Dev&, hipStream_t);               \
    template hipError_t launch_update<T>(int, const T*, const T*, const T*, T*, const double*,          \
                                         const double*, double*, const Dev&, double, double, double,    \
                                         unsigned long long*, hipStream_t);                             \
    template hipError_t launch_update_zmarch<T>(int, const T*, const T*, const T*, T*, const double*,   \
                                                const double*, double*, const Dev&, double, double,     \
                                                double, unsigned long long*, hipStream_t);              \
    template hipError_t launch_rhs<T>(int, const T*, const T*, const T*, const T*, double*, const Dev&,  \
                                      hipStream_t);                                                     \
    template hipError_t launch_cons<T>(int, const double*, double*, T*, const Dev&, hipStream_t);      \
    template hipError_t launch_prim<T>(int, const double*, double*, T*, const Dev&, unsigned long long*, \
                                       hipStream_t);
GRMHD_INSTANTIATE(double)
GRMHD_INSTANTIATE(float)

}  // namespace grmhd
