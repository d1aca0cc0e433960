// grmhd_kernels.hip -- HIP kernels of the GRMHD substep (gfx950, wave64).
//
// One substep (section 2.2 of the paper) is
//   k_ghosts  : ghost zones of the primitive cache (periodic / zero-gradient)
//   k_flux<D> : per face along axis D: MC reconstruction of the 9 primitives,
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
template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_flux(const double* __restrict__ Pc, double* __restrict__ F,
                                               Dev d)
{
    long long f = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (f >= d.nf[D])
        return;
    const int nfx = d.n[0] + (D == 0), nfy = d.n[1] + (D == 1);
    int i = (int)(f % nfx);
    long long t = f / nfx;
    int j = (int)(t % nfy);
    int k = (int)(t / nfy);
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)d.px : (long long)d.px * d.py);
    // cell f-2 along D, in ghosted coordinates
    long long base = ((long long)(k + d.g[2]) * d.py + (j + d.g[1])) * d.px + (i + d.g[0]) - 2 * st;

    double qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const double* p = Pc + v * d.sv + base;
        double q0 = p[0], q1 = p[st], q2 = p[2 * st], q3 = p[3 * st];
        qL[v] = q1 + 0.5 * mc_slope(q0, q1, q2);
        qR[v] = q2 - 0.5 * mc_slope(q1, q2, q3);
    }
    double x = d.lo[0] + (D == 0 ? (double)i : i + 0.5) * d.dx[0];
    double y = d.lo[1] + (D == 1 ? (double)j : j + 0.5) * d.dx[1];
    double z = d.lo[2] + (D == 2 ? (double)k : k + 0.5) * d.dx[2];
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
    const long long NF = d.nf[D];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        if (v == 5 + D)
            continue;
        double fl = flux_comp<D>(v, qL, kL, g);
        double fr = flux_comp<D>(v, qR, kR, g);
        double o = cL * fl + cR * fr;
        if (cU != 0.0)
            o += cU * (cons_comp(v, qR, kR, g) - cons_comp(v, qL, kL, g));
        F[v * NF + f] = o;
    }
    F[(5 + D) * NF + f] = phs;
    F[8 * NF + f] = d.c_h2 * Bs;
}

// ---------------------------------------------------------------------------
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
    double x = d.lo[0] + (i + 0.5) * d.dx[0];
    double y = d.lo[1] + (j + 0.5) * d.dx[1];
    double z = d.lo[2] + (k + 0.5) * d.dx[2];
    double ka, kp;
    g = geo_deriv<KIND>(d, x, y, z, ka, kp);
    if (KIND != FLAT) {
        // 1/2 sqrt(-g) [T^tt d_j g_tt + sum_k T^kk d_j g_kk], d_j g_tt = -2 alpha d_j alpha
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

template <int KIND>
static hipError_t launch_flux_k(int dir, const double* Pc, double* F, const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.nf[dir]);
    if (dir == 0)
        hipLaunchKernelGGL((k_flux<0, KIND>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
    else if (dir == 1)
        hipLaunchKernelGGL((k_flux<1, KIND>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
    else
        hipLaunchKernelGGL((k_flux<2, KIND>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
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
