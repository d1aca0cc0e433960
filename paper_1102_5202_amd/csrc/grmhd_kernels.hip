// grmhd_kernels.hip -- HIP kernels of the GRMHD substep (gfx950, wave64).
//
// One substep (section 2.2 of the paper) on a 3D grid is one launch of
// k_substep: per tile of z columns and plane, the primitives staged in LDS,
// MC reconstruction of the 9 primitives, exact (normal field, Phi) cleaning
// pair, face physics of both states and HLLE flux (section 3.2) for the x and
// y faces from LDS and for the z faces from a register window, then per cell
// the flux differences, metric sources (eq. 2), SSP Runge-Kutta combination,
// Newton recovery of the primitives with the atmosphere/floor policy and the
// status counters.  Every kernel that writes primitives also writes their
// ghost images, so the ghost pass k_ghosts runs only for caches filled
// otherwise.  1D and 2D grids, PPM (k_flux_ppm) and flux-CT (k_ct_edges,
// k_ct_faces) use face kernels per active axis (k_flux_x, k_flux_march) and the
// cell kernel k_update.  Also here: the stored metric's set-up (k_metric), the
// single-kernel maps (k_cons, k_prim, k_rhs) and the batched 1D ensemble
// (k_batch_*).
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
static constexpr int MARCH_SEG = 8;   // faces per thread in the z face march (flux-CT)
static constexpr unsigned MIN_BLOCKS = 1024;   // 4 workgroups per CU: enough to fill the GPU
// the fused substep kernel: tile of TX x TY columns, SUB_SEG planes per workgroup
static constexpr int SUB_TX = 32, SUB_TY = 8, SUB_SEG = 8;
static constexpr long long SUB_MIN_BLOCKS = 1024;

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
// corners: the stencil is a cross).  The kernels that write a cache fill its
// ghost images themselves; this one remains for caches written otherwise.  Segment a covers axis a: 2*g layers times
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

__device__ __forceinline__ long long cache_index(const Dev& d, int i, int j, int k)
{
    return ((long long)(k + d.g[2]) * d.py + (j + d.g[1])) * d.px + (i + d.g[0]);
}

template <int D, int KIND, bool NT, typename T>
__device__ __forceinline__ void face_store(T* qL, T* qR, double x, double y, double z, const Dev& d,
                                           T* __restrict__ F, long long NF, long long f)
{
    T Fo[9];
    face_flux<D, KIND>(qL, qR, x, y, z, f, d, Fo);
    // the face records are read back by another kernel, not by this one: on
    // large grids (NT) nontemporal stores
    if constexpr (NT) {
#pragma unroll
        for (int v = 0; v < 9; ++v)
            __builtin_nontemporal_store(Fo[v], &F[v * NF + f]);
    } else {
#pragma unroll
        for (int v = 0; v < 9; ++v)
            F[v * NF + f] = Fo[v];
    }
}

// x faces: one thread per face (the x stencil of a wave shares cache lines).
template <int KIND, bool NT, typename T>
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
    T qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const T* p = Pc + v * d.sv + base;
        T q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
        qL[v] = q1 + mc_hslope(q0, q1, q2);
        qR[v] = q2 - mc_hslope(q1, q2, q3);
    }
    face_store<0, KIND, NT>(qL, qR, d.lo[0] + i * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                        d.lo[2] + (k + 0.5) * d.dx[2], d, F, d.nf[0], f);
}

// y or z faces: a thread marches along D over a segment of up to SEG faces at
// fixed (i, other transverse index).  Moving from face f-1/2 to f+1/2 it keeps
// q_f, q_{f+1} and the MC slope of cell f, so each face loads one new cell
// (9 values instead of 36) and computes one slope instead of two.
template <int D, int KIND, int SEG, bool NT, typename T>
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
    T qb[9], qc[9], sc[9];      // cells f-1 and f, half MC slope of cell f-1
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
            sc[v] = mc_hslope(qa[v], qb[v], qc[v]);
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
            T sn = mc_hslope(qb[v], qc[v], qd);   // half slope of cell f
            qL[v] = qb[v] + sc[v];                // cell f-1, right face
            qR[v] = qc[v] - sn;                   // cell f, left face
            sc[v] = sn;
            qb[v] = qc[v];
            qc[v] = qd;
        }
        xyz[D] = d.lo[D] + f * d.dx[D];
        face_store<D, KIND, NT>(qL, qR, xyz[0], xyz[1], xyz[2], d, F, NF, fidx);
        fidx += fstr;
    }
}

// Faces along D with PPM reconstruction: one thread per face, the six cells
// f-3 .. f+2 along D; the left state is the right edge of cell f-1, the
// right state the left edge of cell f.  Needs 3 ghost layers.
template <int D, int KIND, bool NT, typename T>
__global__ __launch_bounds__(BLOCK) void k_flux_ppm(const T* __restrict__ Pc, T* __restrict__ F, Dev d)
{
    const long long NF = d.nf[D];
    const long long f = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (f >= NF)
        return;
    int m[3] = {d.n[0], d.n[1], d.n[2]};
    m[D] += 1;
    int fi[3];
    fi[0] = (int)(f % m[0]);
    const long long t = f / m[0];
    fi[1] = (int)(t % m[1]);
    fi[2] = (int)(t / m[1]);
    int ci[3] = {fi[0], fi[1], fi[2]};
    ci[D] -= 3;
    const long long base = cache_index(d, ci[0], ci[1], ci[2]);
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)d.px : (long long)d.px * d.py);
    T qL[9], qR[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const T* p = Pc + v * d.sv + base;
        const T a0 = p[0], a1 = p[st], a2 = p[2 * st], a3 = p[3 * st], a4 = p[4 * st], a5 = p[5 * st];
        T e;
        ppm_edges(a0, a1, a2, a3, a4, e, qL[v]);
        ppm_edges(a1, a2, a3, a4, a5, qR[v], e);
    }
    double pos[3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
        pos[e] = e == D ? d.lo[e] + fi[e] * d.dx[e] : d.lo[e] + (fi[e] + 0.5) * d.dx[e];
    face_store<D, KIND, NT>(qL, qR, pos[0], pos[1], pos[2], d, F, NF, f);
}

// ---------------------------------------------------------------------------
// Flux-CT (Toth 2000).  For every pair (a, b) of active axes (a < b; e the
// third), the edge value at a-face fa, b-face fb, cell ce along e:
//   W_ab = 1/4 [F^b(Bd^a) at the two b-faces beside the edge
//               - F^a(Bd^b) at the two a-faces beside it],
// face neighbours across a boundary mapped like cells (periodic wrap,
// outflow clamp); edge arrays [ce][fb][fa].  Then every face of an active
// axis a gets, for each active partner b, F^a(Bd^b) = -1/2 (W_ab at its two
// edges) when a < b and +1/2 when a > b; its normal-field and Phi fluxes
// vanish.  The cell update keeps the corner-centred divergence of Bd.

__device__ __forceinline__ int ct_map(int c, int n, int bc)
{
    return c < 0 ? (bc == 0 ? c + n : 0) : (c >= n ? (bc == 0 ? c - n : n - 1) : c);
}

__device__ __forceinline__ long long face_index(const Dev& d, int dir, int i, int j, int k)
{
    const long long nf0 = d.n[0] + (dir == 0), nf1 = d.n[1] + (dir == 1);
    return ((long long)k * nf1 + j) * nf0 + i;
}

// Edge values of the pair p = (a, b) sit at (face a, face b, cell e): extents
// n + 1 along a and b, n along e.  Every pair is stored x fastest, so that a
// wave of consecutive edges or faces reads and writes consecutive addresses.
__device__ __forceinline__ long long edge_index(const Dev& d, int a, int b, int i, int j, int k)
{
    const long long e0 = d.n[0] + (a == 0 || b == 0), e1 = d.n[1] + (a == 1 || b == 1);
    return ((long long)k * e1 + j) * e0 + i;
}

template <typename T>
struct CtArgs {
    T* F[3];          // face fluxes of the three axes ([9][nf])
    T* W[3];          // edge values of the pairs (x,y), (x,z), (y,z)
    long long nW[3];  // edges per pair (0: a partner inactive)
};

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ct_edges(CtArgs<T> A, Dev d)
{
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int p = 0;
    while (p < 3 && t >= A.nW[p]) {
        t -= A.nW[p];
        ++p;
    }
    if (p == 3)
        return;
    const int a = p == 2 ? 1 : 0, b = p == 0 ? 1 : 2;
    const int na = d.n[a], nb = d.n[b];
    const int e0 = d.n[0] + (a == 0), e1 = d.n[1] + (a == 1 || b == 1);
    int ix[3];
    ix[0] = (int)(t % e0);
    const long long r = t / e0;
    ix[1] = (int)(r % e1);
    ix[2] = (int)(r / e1);
    const int fa = ix[a], fb = ix[b];
    const long long NFa = d.nf[a], NFb = d.nf[b];
    T s = T(0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        ix[a] = fa;
        ix[b] = ct_map(fb - 1 + q, nb, d.bc[b]);
        s -= A.F[a][(5 + b) * NFa + face_index(d, a, ix[0], ix[1], ix[2])];
        ix[a] = ct_map(fa - 1 + q, na, d.bc[a]);
        ix[b] = fb;
        s += A.F[b][(5 + a) * NFb + face_index(d, b, ix[0], ix[1], ix[2])];
    }
    A.W[p][t] = T(0.25) * s;
}

// The normal-field and Phi rows of every face flux are zero under flux-CT
// (the face kernels write them so); this kernel replaces the transverse rows.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ct_faces(CtArgs<T> A, Dev d)
{
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int a = 0;
    while (a < 3 && (!d.act[a] || t >= d.nf[a])) {
        if (d.act[a])
            t -= d.nf[a];
        ++a;
    }
    if (a == 3)
        return;
    const long long NF = d.nf[a];
    const int m0 = d.n[0] + (a == 0), m1 = d.n[1] + (a == 1);
    int ix[3];
    ix[0] = (int)(t % m0);
    const long long r = t / m0;
    ix[1] = (int)(r % m1);
    ix[2] = (int)(r / m1);
    T* F = A.F[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == a || !d.act[b])
            continue;
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        const int p = lo == 0 ? (hi == 1 ? 0 : 1) : 2;
        int eh[3] = {ix[0], ix[1], ix[2]};
        eh[b] += 1;
        const long long w0 = edge_index(d, lo, hi, ix[0], ix[1], ix[2]);
        const long long w1 = edge_index(d, lo, hi, eh[0], eh[1], eh[2]);
        const T sign = a < b ? T(-0.5) : T(0.5);
        F[(5 + b) * NF + t] = sign * (A.W[p][w0] + A.W[p][w1]);
    }
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
                      d.lo[2] + (k + 0.5) * d.dx[2], c, q, g, R);
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

// Store the primitives of cell (i, j, k) at cache position pc, and at the
// ghost positions whose boundary rule copies this cell, so that the cache
// leaves the kernel with its ghost slabs filled (only the face slabs are
// ghosts: every stencil is 1D).  Periodic: the cell is the image of ghost
// idx + n when idx < g and of ghost idx - n when idx >= n - g.  Outflow
// (zero gradient): the first and last cells fill both ghost layers beside
// them.  Active axes have n >= g, so these are all the images.
template <typename T>
__device__ __forceinline__ void store_prim(const Dev& d, T* __restrict__ P, long long pc, int i, int j,
                                           int k, const double* p)
{
#pragma unroll
    for (int v = 0; v < 9; ++v)
        P[v * d.sv + pc] = (T)p[v];
    const int idx[3] = {i, j, k};
    const long long stride[3] = {1, d.px, (long long)d.px * d.py};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!d.act[a])
            continue;
        const int n = d.n[a], g = d.g[a];
        const long long st = stride[a];
        if (d.bc[a] == 0) {
            if (idx[a] < g) {
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    P[v * d.sv + pc + n * st] = (T)p[v];
            }
            if (idx[a] >= n - g) {
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    P[v * d.sv + pc - n * st] = (T)p[v];
            }
        } else if (idx[a] == 0 || idx[a] == n - 1) {
            const long long s1 = idx[a] == 0 ? -st : st;
            for (int e = 1; e <= g; ++e)
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    P[v * d.sv + pc + e * s1] = (T)p[v];
        }
    }
}

// The stage inputs of cell c: U^n and U^s.  U^n, U^s and U^(s+1) are touched
// once per cell and substep: on large grids (NT) nontemporal accesses keep them
// from displacing the face records and primitives that neighbouring
// workgroups read again.
template <bool NT, typename TS>
__device__ __forceinline__ void stage_load(const Dev& d, const double* Un, const TS* Us, long long c, double* un,
                                           double* us)
{
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        if constexpr (NT) {
            un[v] = __builtin_nontemporal_load(&Un[v * d.N + c]);
            us[v] = (double)__builtin_nontemporal_load(&Us[v * d.N + c]);
        } else {
            un[v] = Un[v * d.N + c];
            us[v] = (double)Us[v * d.N + c];
        }
    }
}

// Runge-Kutta combination U^(s+1) = U^s + a (U^n - U^s) + b dt R and recovery
// of the primitives for one cell (all in double) from its stage inputs un, us;
// q are the cell's current primitives (the Newton guess).  Writes U^(s+1) and
// the new primitives (with their ghost images).  TO is the type of the stage
// state written: double, or float for the intermediate stages of the mixed
// path.  fout (may be null) receives the cell's recovery flags.
template <bool NT, typename T, typename TO>
__device__ __forceinline__ int stage_finish(const Dev& d, const Geo& g, const double* R, const T* q,
                                            const double* un, const double* us, TO* Uout, long long c, T* Pout,
                                            long long pc, int i, int j, int k, double dt, double a, double b,
                                            unsigned char* fout, int& iters)
{
    double u[9], p[9], qg[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        u[v] = us[v] + a * (un[v] - us[v]) + b * (dt * R[v]);
        qg[v] = (double)q[v];
    }
    int flags = recover_cell(d, g, u, qg, p, iters);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        if constexpr (NT)
            __builtin_nontemporal_store((TO)u[v], &Uout[v * d.N + c]);
        else
            Uout[v * d.N + c] = (TO)u[v];
    }
    store_prim(d, Pout, pc, i, j, k, p);
    if (fout)
        fout[c] = (unsigned char)flags;
    return flags;
}

// stage_load then stage_finish.  TS is the type of the stage state read.
template <bool NT, typename T, typename TS, typename TO>
__device__ __forceinline__ int stage_cell(const Dev& d, const Geo& g, const double* R, const T* q,
                                          const double* Un, const TS* Us, TO* Uout, long long c,
                                          T* Pout, long long pc, int i, int j, int k, double dt,
                                          double a, double b, unsigned char* fout, int& iters)
{
    double un[9], us[9];
    stage_load<NT>(d, Un, Us, c, un, us);
    return stage_finish<NT>(d, g, R, q, un, us, Uout, c, Pout, pc, i, j, k, dt, a, b, fout, iters);
}

// 1D/2D update: flux differences, sources, RK combination and recovery of the
// primitives for every cell.  The cell's primitives are read from Pc and the
// new ones written to Pn (which may be Pc: each thread reads only its own cell).
template <int KIND, bool NT, typename T, typename TS, typename TO>
__global__ __launch_bounds__(BLOCK) void k_update(const T* __restrict__ Fx, const T* __restrict__ Fy,
                                                 const T* __restrict__ Fz, const T* Pc, T* Pn,
                                                 const double* Un, const TS* Us, TO* Uout, Dev d,
                                                 double dt, double a, double b,
                                                 unsigned long long* __restrict__ cnt,
                                                 unsigned char* __restrict__ fout)
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
        int flags = stage_cell<NT>(d, g, R, q, Un, Us, Uout, c, Pn, pc, i, j, k, dt, a, b, fout, iters);
        tally(flags, iters, nf, na, np, nb, itmax);
    }
    count_sums(cnt, nf, na, np, nb, itmax);
}

// ---------------------------------------------------------------------------
// The whole substep of a 3D grid in one kernel (MC reconstruction, cleaning).
// A workgroup owns a TX x TY tile of z columns and a segment of SEG planes and
// walks the planes upwards.  For plane k it
//   (1) stages the primitives of the tile and of a 2-cell halo in x and y (the
//       cross-shaped stencil, no corners) in LDS: each thread writes its own
//       cell from its z window, the halo cells come from the cache in HBM;
//   (2) solves the tile's x faces (TX + 1 per row) and y faces (TY + 1 per
//       column) from LDS into LDS, one face of each axis per thread plus the
//       tile's last row and column of faces;
//   (3) per cell: the z face above the cell from the thread's register
//       window (one new cell and one half slope per plane), the
//       flux differences of the three axes, the sources, the Runge-Kutta
//       combination and the recovery, the new primitives (with their ghost
//       images) going to another cache.
// The x and y face fluxes never leave the chip, and every primitive of the
// cache is read from HBM once per substep, plus the halo rows and columns
// shared with the neighbouring tiles.
template <int TX, int TY>
struct Tile {
    static constexpr int NT = TX * TY;          // threads: one column each
    static constexpr int W = TX + 4;            // LDS row of a staged plane
    static constexpr int PLANE = (TY + 4) * W;  // staged positions per variable
    static constexpr int NFX = (TX + 1) * TY;   // x faces of the tile
    static constexpr int NFY = TX * (TY + 1);   // y faces of the tile
    static constexpr int NH = 4 * (TX + TY);    // halo positions
    static_assert(NH <= NT - 64, "one halo position per thread, the last wave free");
    static_assert(TX + TY <= 64 && NT % 64 == 0, "the tile's last faces in one wave");
};

// An x (dir 0) or y (dir 1) face of the tile, dir per lane, solved as a face
// of axis 0 with the vector components cycled (the metric is conformally
// flat): MC states from the four staged cells at sP + base + m * stride
// (m = 0..3, the face between the 2nd and the 3rd), the face solver, the flux
// into sF.
template <int KIND, int PLANE, typename T>
__device__ __forceinline__ void tile_face(const T* sP, int dir, int base, int stride, double fx, double fy,
                                          double fz, long long fglob, const Dev& d, T* sF, int nslot, int slot)
{
    int vo[9];   // variable v of the cycled frame is variable vo[v] of the grid
    vo[0] = 0;
    vo[1] = 1;
    vo[8] = 8;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int c = dir == 0 ? m : (m == 2 ? 0 : m + 1);
        vo[2 + m] = 2 + c;
        vo[5 + m] = 5 + c;
    }
    T qL[9], qR[9], Fo[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        const T* p = sP + vo[v] * PLANE + base;
        const T q0 = p[0], q1 = p[stride], q2 = p[2 * stride], q3 = p[3 * stride];
        qL[v] = q1 + mc_hslope(q0, q1, q2);
        qR[v] = q2 - mc_hslope(q1, q2, q3);
    }
    Geo g;
    if (KIND == STORED) {
        const double* mf = dir == 0 ? d.mf[0] : d.mf[1];
        const long long nf = dir == 0 ? d.nf[0] : d.nf[1];
        g = geo_from_ap(mf[fglob], mf[nf + fglob]);
    } else {
        g = geo_at<KIND>(d, fx, fy, fz);
    }
    face_solve<0>(qL, qR, geo_cast<T>(g), d, Fo);
#pragma unroll
    for (int v = 0; v < 9; ++v)
        sF[vo[v] * nslot + slot] = Fo[v];
}

template <int KIND, int TX, int TY, int SEG, bool NT, typename T, typename TS, typename TO>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_substep(
    const T* __restrict__ Pc, T* __restrict__ Pn, const double* Un, const TS* Us, TO* Uout, Dev d, double dt,
    double a, double b, unsigned long long* __restrict__ cnt, unsigned char* __restrict__ fout, int ntx, int ntiles)
{
    using G = Tile<TX, TY>;
    // With a float cache the staged planes and the face fluxes are double
    // buffered (70.8 KB of LDS, still two workgroups per CU): the faces of
    // plane k + 1 and the update of plane k then share one barrier interval.
    // With a double cache that would take 141.7 KB, one workgroup per CU, so
    // each plane has its staging, faces and update between two barriers.
    constexpr bool DB = sizeof(T) < sizeof(double);
    constexpr int NB = DB ? 2 : 1;
    __shared__ T sP[NB][9 * G::PLANE];
    __shared__ T sFx[NB][9 * G::NFX];
    __shared__ T sFy[NB][9 * G::NFY];

    const int t = threadIdx.x;
    const int tx = t % TX, ty = t / TX;
    const unsigned nbk = gridDim.x;
    const unsigned item = (nbk % 8 == 0) ? (blockIdx.x % 8) * (nbk / 8) + blockIdx.x / 8 : blockIdx.x;
    const int tile = (int)(item % (unsigned)ntiles);
    const int seg = (int)(item / (unsigned)ntiles);
    const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
    const int i = i0 + tx, j = j0 + ty;
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const bool act = i < nx && j < ny;
    const bool ax = d.act[0], ay = d.act[1];   // an axis of one cell has no faces
    const int k0 = seg * SEG;
    const int k1 = min(k0 + SEG, nz);
    const long long st = (long long)d.px * d.py;
    // cache address of (i, j, k = 0); cell k adds k * st
    const long long col = (long long)(j + d.g[1]) * d.px + i + d.g[0] + (long long)d.g[2] * st;
    const double x = d.lo[0] + (i + 0.5) * d.dx[0];
    const double y = d.lo[1] + (j + 0.5) * d.dx[1];
    int nfail = 0, natm = 0, npf = 0, nfb = 0, itmax = 0;

    // The cell this thread stages from HBM each plane: a halo position
    // (threads t < NH), or its own position when it is a ghost cell that a
    // face near the domain's edge reads (ragged tiles); -1: none.
    int hslot = -1;
    long long hoff = 0;
    if (t < G::NH) {
        int hx, hy;
        if (t < 2 * TX) {
            hx = t % TX;
            hy = -2 + t / TX;
        } else if (t < 4 * TX) {
            hx = (t - 2 * TX) % TX;
            hy = TY + (t - 2 * TX) / TX;
        } else if (t < 4 * TX + 2 * TY) {
            hx = -2 + (t - 4 * TX) % 2;
            hy = (t - 4 * TX) / 2;
        } else {
            hx = TX + (t - 4 * TX - 2 * TY) % 2;
            hy = (t - 4 * TX - 2 * TY) / 2;
        }
        const int gi = i0 + hx, gj = j0 + hy;
        // rows below/above: an interior column; columns left/right: an interior row
        const bool need =
            (hy < 0 || hy >= TY) ? (ay && gi < nx && gj < ny + 2) : (ax && gj < ny && gi < nx + 2);
        if (need) {
            hslot = (hy + 2) * G::W + hx + 2;
            hoff = (long long)(j0 + hy + d.g[1]) * d.px + i0 + hx + d.g[0] + (long long)d.g[2] * st;
        }
    }
    const bool own_ghost = !act && ((ax && i < nx + 2 && j < ny) || (ay && i < nx && j < ny + 2));
    const int oslot = (ty + 2) * G::W + tx + 2;

    // z window of the thread's column: qb = q_k, qc = q_(k+1), sc = half slope of
    // cell k, Fp = the flux through the face below cell k
    T qb[9], qc[9], sc[9], Fp[9];
    if (act) {
        const long long base = col + (long long)(k0 - 2) * st;
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
            T s0 = mc_hslope(qa[v], qb[v], qc[v]);   // cell k0-1
            T s1 = mc_hslope(qb[v], qc[v], qd);      // cell k0
            qL[v] = qb[v] + s0;
            qR[v] = qc[v] - s1;
            sc[v] = s1;
            qb[v] = qc[v];
            qc[v] = qd;
        }
        face_flux<2, KIND>(qL, qR, x, y, d.lo[2] + k0 * d.dx[2],
                           i + (long long)nx * (j + (long long)ny * k0), d, Fp);
    }

    // Staging of plane k into buffer pb: the own cell (own: its value from the
    // window) and the halo cell (hv: loaded ahead with a float cache).
    T hv[9];
    auto halo_load = [&](int k) {
        if (hslot >= 0) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                hv[v] = Pc[v * d.sv + hoff + (long long)k * st];
        }
    };
    auto stage = [&](int k, int pb, const T* own, bool hv_loaded) {
        T* P = sP[pb];
        if (act) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                P[v * G::PLANE + oslot] = own[v];
        } else if (own_ghost) {
            const long long o = col + (long long)k * st;
#pragma unroll
            for (int v = 0; v < 9; ++v)
                P[v * G::PLANE + oslot] = Pc[v * d.sv + o];
        }
        if (hslot >= 0) {
            if (!hv_loaded)
                halo_load(k);
#pragma unroll
            for (int v = 0; v < 9; ++v)
                P[v * G::PLANE + hslot] = hv[v];
        }
    };

    // The faces of plane k from staged buffer pb into face buffer fb: every
    // thread the x face left of its cell and the y face below it; the last
    // wave, which stages no halo cells, also the tile's last face of each
    // row and column.  One face solver serves both axes (a loop, not
    // unrolled, keeps one copy of its code).
    auto faces = [&](int k, int pb, int fb) {
        const double zc = d.lo[2] + (k + 0.5) * d.dx[2];
        const int ntask = t >= G::NT - 64 ? 3 : 2;
#pragma nounroll
        for (int task = 0; task < ntask; ++task) {
            int dir = task, xs = tx, ys = ty;
            if (task == 2) {
                const int l = t - (G::NT - 64);
                dir = l < TY ? 0 : 1;
                xs = l < TY ? TX : l - TY;
                ys = l < TY ? l : TY;
                if (l >= TX + TY)
                    continue;
            }
            const int fi = i0 + xs, fj = j0 + ys;
            if (dir == 0 ? !(ax && fi <= nx && fj < ny) : !(ay && fj <= ny && fi < nx))
                continue;
            const double fx = d.lo[0] + (dir == 0 ? fi : fi + 0.5) * d.dx[0];
            const double fy = d.lo[1] + (dir == 0 ? fj + 0.5 : fj) * d.dx[1];
            const long long fglob = dir == 0 ? fi + (long long)(nx + 1) * (fj + (long long)ny * k)
                                             : fi + (long long)nx * (fj + (long long)(ny + 1) * k);
            tile_face<KIND, G::PLANE>(sP[pb], dir, dir == 0 ? (ys + 2) * G::W + xs : ys * G::W + xs + 2,
                                      dir == 0 ? 1 : G::W, fx, fy, zc, fglob, d, dir == 0 ? sFx[fb] : sFy[fb],
                                      dir == 0 ? G::NFX : G::NFY, dir == 0 ? ys * (TX + 1) + xs : ys * TX + xs);
        }
    };

    // The update of plane k (x and y fluxes in face buffer fb): the z face
    // above the cell from the window (which moves up one plane), the flux
    // differences, sources, RK combination and recovery.  With a float
    // cache the stage inputs are loaded first, so that the z face covers
    // their latency, and the halo cell of plane kh is loaded before the
    // recovery; a double cache has no registers to spare for either.
    auto update = [&](int k, int fb, int kh) {
        constexpr bool early = sizeof(T) < sizeof(double);
        if (!act) {
            if (early && kh >= 0)
                halo_load(kh);
            return;
        }
        const long long c = i + (long long)nx * (j + (long long)ny * k);
        double un[9], us[9];
        if constexpr (early)
            stage_load<NT>(d, Un, Us, c, un, us);
        T qd[9];
#pragma unroll
        for (int v = 0; v < 9; ++v)
            qd[v] = Pc[v * d.sv + col + (long long)(k + 2) * st];
        T q[9], qL[9], qR[9], Fc[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            T sn = mc_hslope(qb[v], qc[v], qd[v]);   // cell k+1
            q[v] = qb[v];
            qL[v] = qb[v] + sc[v];
            qR[v] = qc[v] - sn;
            sc[v] = sn;
            qb[v] = qc[v];
            qc[v] = qd[v];
        }
        const double zc = d.lo[2] + (k + 0.5) * d.dx[2];
        face_flux<2, KIND>(qL, qR, x, y, zc + 0.5 * d.dx[2], i + (long long)nx * (j + (long long)ny * (k + 1)), d,
                           Fc);
        if constexpr (!early)
            stage_load<NT>(d, Un, Us, c, un, us);
        double R[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            R[v] = -((double)Fc[v] - (double)Fp[v]) * d.idx[2];
            Fp[v] = Fc[v];
        }
        const int fx = ty * (TX + 1) + tx, fy = ty * TX + tx;
        if (ax) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                R[v] -= ((double)sFx[fb][v * G::NFX + fx + 1] - (double)sFx[fb][v * G::NFX + fx]) * d.idx[0];
        }
        if (ay) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
                R[v] -= ((double)sFy[fb][v * G::NFY + fy + TX] - (double)sFy[fb][v * G::NFY + fy]) * d.idx[1];
        }
        Geo g;
        add_sources<KIND>(d, x, y, zc, c, q, g, R);
        if (early && kh >= 0)
            halo_load(kh);
        int iters = 0;
        int flags = stage_finish<NT>(d, g, R, q, un, us, Uout, c, Pn, col + (long long)k * st, i, j, k, dt, a, b,
                                     fout, iters);
        tally(flags, iters, nfail, natm, npf, nfb, itmax);
    };

    if constexpr (DB) {
        // prologue: planes k0 and k0 + 1 staged, the faces of k0 solved
        stage(k0, 0, qb, false);
        __syncthreads();
        faces(k0, 0, 0);
        if (k0 + 1 < k1)
            stage(k0 + 1, 1, qc, false);
        __syncthreads();
        // plane k: the faces of k + 1, the update of k, the staging of k + 2
        // (into the buffer plane k used; its own cell is the window's qc once
        // the update has moved the window up)
        for (int k = k0; k < k1; ++k) {
            const int cur = (k - k0) & 1, nxt = cur ^ 1;
            if (k + 1 < k1)
                faces(k + 1, nxt, nxt);
            update(k, cur, k + 2 < k1 ? k + 2 : -1);   // also loads the halo cell of k + 2
            if (k + 2 < k1)
                stage(k + 2, cur, qc, true);
            __syncthreads();
        }
    } else {
        for (int k = k0; k < k1; ++k) {
            stage(k, 0, qb, false);
            __syncthreads();
            faces(k, 0, 0);
            __syncthreads();
            update(k, 0, -1);
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
    for (int v = 0; v < 9; ++v)
        q[v] = P[v * d.N + c];
    store_prim(d, Pc, pc, i, j, k, q);
    if (U) {
        const GeoT<double> g = geo_cast<double>(cell_geo<KIND>(
            d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1], d.lo[2] + (k + 0.5) * d.dx[2], c));
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
        Geo g = cell_geo<KIND>(d, d.lo[0] + (i + 0.5) * d.dx[0], d.lo[1] + (j + 0.5) * d.dx[1],
                               d.lo[2] + (k + 0.5) * d.dx[2], c);
        int iters = 0;
        int flags = recover_cell(d, g, u, q, p, iters);
#pragma unroll
        for (int v = 0; v < 9; ++v)
            P[v * d.N + c] = p[v];
        store_prim(d, Pc, pc, i, j, k, p);
        tally(flags, iters, nf, na, np, nb, itmax);
    }
    count_sums(cnt, nf, na, np, nb, itmax);
}


// ---------------------------------------------------------------------------
// Batched ensemble of independent 1D problems (flat metric, along x).
//
// Every problem b has n_b cells, its own dx and dt, and a step budget.  The
// packed arrays hold problem b's 9 x n_b values from element 9 * off_b on,
// variable-major.  The primitive row of a problem (9 rows of n_b + 4 values,
// two ghosts each side) lives in global memory between calls and, during the
// evolve kernel, in LDS when it fits.
//
// k_batch_evolve: one persistent workgroup per problem runs all its steps.
// Thread t owns the contiguous cells [t*ch, (t+1)*ch) with ch = ceil(n/NT);
// per substep it marches over them computing each face once (the
// previous face flux stays in registers), forms the flux difference and the
// source, combines the Runge-Kutta stage (U^n from U, the intermediate stage
// state in Us) and recovers the primitives, written to the next row.  A
// barrier ends the substep (with the row in LDS, after a copy of the own
// cells from the global staging row back into LDS and a second barrier).

__device__ __forceinline__ int batch_find(const BatchProb* __restrict__ probs, int nprob, long long c)
{
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].off <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Primitive value and its ghost images in a ghosted row of pitch n + 4.
template <typename T>
__device__ __forceinline__ void row_store(T* __restrict__ row, int pitch, int n, int bc, int c, const double* p)
{
#pragma unroll
    for (int v = 0; v < 9; ++v)
        row[v * pitch + c + 2] = (T)p[v];
    int o[2], no = 0;
    if (bc == 0) {
        if (c < 2)
            o[no++] = c + n;
        if (c >= n - 2)
            o[no++] = c - n;
    } else if (c == 0) {
        o[no++] = -1;
        o[no++] = -2;
    } else if (c == n - 1) {
        o[no++] = n;
        o[no++] = n + 1;
    }
    for (int e = 0; e < no; ++e)
#pragma unroll
        for (int v = 0; v < 9; ++v)
            row[v * pitch + o[e] + 2] = (T)p[v];
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_batch_cons(const BatchProb* __restrict__ probs, int nprob,
                                                     long long ncell, const double* __restrict__ P,
                                                     double* __restrict__ U, T* __restrict__ Prow, Dev d)
{
    const long long g = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (g >= ncell)
        return;
    const int b = batch_find(probs, nprob, g);
    const BatchProb pr = probs[b];
    const int c = (int)(g - pr.off);
    double q[9];
#pragma unroll
    for (int v = 0; v < 9; ++v)
        q[v] = P[9 * pr.off + (long long)v * pr.n + c];
    row_store(Prow + pr.poff, pr.n + 4, pr.n, d.bc[0], c, q);
    if (U) {
        const GeoT<double> gt = geo_cast<double>(geo_at<FLAT>(d, 0.0, 0.0, 0.0));
        const Kin<double> kk = kinematics(q, gt, d.gfac);
#pragma unroll
        for (int v = 0; v < 8; ++v)
            U[9 * pr.off + (long long)v * pr.n + c] = cons_comp(v, q, kk, gt);
        U[9 * pr.off + 8LL * pr.n + c] = q[8];
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_batch_prim(const BatchProb* __restrict__ probs, int nprob,
                                                     long long ncell, const double* __restrict__ U,
                                                     double* __restrict__ P, T* __restrict__ Prow, Dev d,
                                                     unsigned long long* __restrict__ cnt)
{
    const long long g = (long long)blockIdx.x * BLOCK + threadIdx.x;
    int nf = 0, na = 0, np = 0, nb = 0, itmax = 0;
    if (g < ncell) {
        const int b = batch_find(probs, nprob, g);
        const BatchProb pr = probs[b];
        const int c = (int)(g - pr.off);
        const int pitch = pr.n + 4;
        double u[9], q[9], p[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            u[v] = U[9 * pr.off + (long long)v * pr.n + c];
            q[v] = (double)Prow[pr.poff + v * pitch + c + 2];
        }
        const Geo geo = geo_at<FLAT>(d, 0.0, 0.0, 0.0);
        int iters = 0;
        const int flags = recover_cell(d, geo, u, q, p, iters);
#pragma unroll
        for (int v = 0; v < 9; ++v)
            P[9 * pr.off + (long long)v * pr.n + c] = p[v];
        row_store(Prow + pr.poff, pitch, pr.n, d.bc[0], c, p);
        tally(flags, iters, nf, na, np, nb, itmax);
    }
    count_sums(cnt, nf, na, np, nb, itmax);
}

// The workgroup's start (taken on entry) and end on the GPU's constant-rate
// clock, into span[2 b], span[2 b + 1] for workgroup b, once all of its
// threads are done: the host derives how busy the workgroup slots were.
__device__ __forceinline__ void span_record(unsigned long long* span, unsigned long long t_start)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        span[2 * blockIdx.x] = t_start;
        span[2 * blockIdx.x + 1] = wall_clock64();
    }
}

template <typename T, int NT, bool LDS>
__global__ __launch_bounds__(NT) void k_batch_evolve(BatchProb* __restrict__ probs, const int* __restrict__ order,
                                                     double* __restrict__ U, T* __restrict__ Us,
                                                     T* __restrict__ Prow, T* __restrict__ Pnext, Dev d, int ns,
                                                     int max_steps, unsigned long long* __restrict__ cnt,
                                                     unsigned long long* __restrict__ span)
{
    const unsigned long long t_start = wall_clock64();
    extern __shared__ unsigned char smem[];
    const int b = order[blockIdx.x];
    const BatchProb pr = probs[b];
    const int n = pr.n, pitch = n + 4;
    // LDS: the row lives in LDS and new values go through the global row
    // Pnext (own cells only).  Global: the rows Prow and Pnext alternate.
    T* cur = LDS ? (T*)smem : Prow + pr.poff;
    T* nxt = Pnext + pr.poff;
    if (LDS) {
        for (int e = threadIdx.x; e < 9 * pitch; e += NT)
            cur[e] = Prow[pr.poff + e];
        __syncthreads();
    }
    const int nsteps = min(max_steps, pr.steps - pr.done);
    const int ch = (n + NT - 1) / NT;
    const int c0 = min((int)threadIdx.x * ch, n), c1 = min(c0 + ch, n);
    double* Ub = U + 9 * pr.off;
    T* Usb = Us + 9 * pr.off;
    const Geo geo = geo_at<FLAT>(d, 0.0, 0.0, 0.0);
    int nfail = 0, natm = 0, npf = 0, nfb = 0, itmax = 0;
    for (int step = 0; step < nsteps; ++step) {
        for (int s = 0; s < ns; ++s) {
            const double a = ns == 3 ? (s == 0 ? 0.0 : (s == 1 ? 0.75 : 1.0 / 3.0)) : (s == 0 ? 0.0 : 0.5);
            const double bb = ns == 3 ? (s == 0 ? 1.0 : (s == 1 ? 0.25 : 2.0 / 3.0)) : (s == 0 ? 1.0 : 0.5);
            T Fp[9];
            if (c0 < c1) {
                // face c0 - 1/2 from cells c0-2 .. c0+1 (row index + 2)
                T qL[9], qR[9];
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    const T* r = cur + v * pitch + c0;
                    const T q0 = r[0], q1 = r[1], q2 = r[2], q3 = r[3];
                    qL[v] = q1 + mc_hslope(q0, q1, q2);
                    qR[v] = q2 - mc_hslope(q1, q2, q3);
                }
                face_flux<0, FLAT>(qL, qR, 0.0, 0.0, 0.0, 0, d, Fp);
            }
            for (int c = c0; c < c1; ++c) {
                T qL[9], qR[9], Fc[9], q[9];
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    const T* r = cur + v * pitch + c + 1;      // cells c-1 .. c+2
                    const T q0 = r[0], q1 = r[1], q2 = r[2], q3 = r[3];
                    q[v] = q1;
                    qL[v] = q1 + mc_hslope(q0, q1, q2);
                    qR[v] = q2 - mc_hslope(q1, q2, q3);
                }
                face_flux<0, FLAT>(qL, qR, 0.0, 0.0, 0.0, 0, d, Fc);
                double R[9];
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    R[v] = -((double)Fc[v] - (double)Fp[v]) * pr.idx;
                    Fp[v] = Fc[v];
                }
                R[8] -= d.kappa * (double)q[8];
                double u[9], qg[9], p[9];
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    const double un = Ub[(long long)v * n + c];
                    const double us = s == 0 ? un : (double)Usb[(long long)v * n + c];
                    u[v] = us + a * (un - us) + bb * (pr.dt * R[v]);
                    qg[v] = (double)q[v];
                }
                int iters = 0;
                const int flags = recover_cell(d, geo, u, qg, p, iters);
                tally(flags, iters, nfail, natm, npf, nfb, itmax);
                if (s == ns - 1) {
#pragma unroll
                    for (int v = 0; v < 9; ++v)
                        Ub[(long long)v * n + c] = u[v];
                } else {
#pragma unroll
                    for (int v = 0; v < 9; ++v)
                        Usb[(long long)v * n + c] = (T)u[v];
                }
                if (LDS) {
#pragma unroll
                    for (int v = 0; v < 9; ++v)
                        nxt[v * pitch + c + 2] = (T)p[v];
                } else {
                    row_store(nxt, pitch, n, d.bc[0], c, p);
                }
            }
            __syncthreads();
            if (LDS) {
                // own cells only: this thread wrote them, so no fence is needed
                for (int c = c0; c < c1; ++c) {
                    double p[9];
#pragma unroll
                    for (int v = 0; v < 9; ++v)
                        p[v] = (double)nxt[v * pitch + c + 2];
                    row_store(cur, pitch, n, d.bc[0], c, p);
                }
                __syncthreads();
            } else {
                T* t = cur;
                cur = nxt;
                nxt = t;
            }
        }
    }
    if (LDS) {
        for (int e = threadIdx.x; e < 9 * pitch; e += NT)
            Prow[pr.poff + e] = cur[e];
    } else if (cur != Prow + pr.poff) {
        // an odd number of substeps left the row in Pnext (every write to it
        // is behind the last barrier)
        for (int e = threadIdx.x; e < 9 * pitch; e += NT)
            Prow[pr.poff + e] = cur[e];
    }
    if (threadIdx.x == 0)
        probs[b].done = pr.done + nsteps;
    count_sums(cnt, nfail, natm, npf, nfb, itmax);
    span_record(span, t_start);
}

// k_batch_split: a problem's cells divided among several workgroups (parts)
// that run at the same time, the rows in HBM.  A part walks its segment in
// chunks of NT - 1 cells, one cell per thread (consecutive cells on
// consecutive threads, so that row accesses are coalesced), the chunk's face
// fluxes exchanged through LDS.  The two cells beside a segment's ends come
// from the neighbouring parts through the rows.  Parts
// may sit on different XCDs, whose L2 caches are not kept coherent for this
// memory, so the values that cross parts (each segment's two end cells at
// either end and their ghost images) are stored and loaded with system-scope
// accesses, which bypass the non-coherent caches, while the rest of the row
// stays cached: after a substep the threads that wrote such values wait for
// their stores, and one thread publishes the part's count of completed
// substeps in flags; before the next substep one thread waits until both
// neighbours have completed the current one (which also tells them this part
// no longer reads the row they are about to overwrite).  Waits are bounded:
// past the limit the part counts a stall (CNT_STALL) and stops instead of
// hanging, so that a launch whose parts are not all resident ends.
static constexpr int SPLIT_SPIN = 1 << 22;   // polls of the flags before a part gives up

template <typename T>
__device__ __forceinline__ T sys_load(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Thread 0 polls until the flags of parts l and r (-1: none) reach target;
// the result is shared through LDS.  Returns false on a stall.
__device__ __forceinline__ bool split_wait(int* flags, int l, int r, int target, int* s_ok)
{
    if (threadIdx.x == 0) {
        int ok = 1;
        for (int it = 0;; ++it) {
            const int fl = l >= 0 ? sys_load(&flags[l]) : target;
            const int fr = r >= 0 ? sys_load(&flags[r]) : target;
            if (fl >= target && fr >= target)
                break;
            if (it >= SPLIT_SPIN) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *s_ok = ok;
    }
    __syncthreads();
    // the same for every thread: read once, as a uniform value
    return __builtin_amdgcn_readfirstlane(*s_ok) != 0;
}

// row_store with system-scope stores (values other parts read).
template <typename T>
__device__ __forceinline__ void row_store_sys(T* __restrict__ row, int pitch, int n, int bc, int c, const double* p)
{
#pragma unroll
    for (int v = 0; v < 9; ++v)
        __hip_atomic_store(&row[v * pitch + c + 2], (T)p[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    int o[2], no = 0;
    if (bc == 0) {
        if (c < 2)
            o[no++] = c + n;
        if (c >= n - 2)
            o[no++] = c - n;
    } else if (c == 0) {
        o[no++] = -1;
        o[no++] = -2;
    } else if (c == n - 1) {
        o[no++] = n;
        o[no++] = n + 1;
    }
    for (int e = 0; e < no; ++e)
#pragma unroll
        for (int v = 0; v < 9; ++v)
            __hip_atomic_store(&row[v * pitch + o[e] + 2], (T)p[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A record the whole workgroup reads at one address, moved into scalar
// registers word by word (the records of a later part are loaded after
// stores to the same array, so the compiler would keep them per lane).
template <typename S>
__device__ __forceinline__ S uniform_load(const S* p)
{
    static_assert(sizeof(S) % 4 == 0, "whole words");
    S r;
    const int* src = (const int*)p;
    int* dst = (int*)&r;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / 4); ++k)
        dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return r;
}

// Workgroup w runs the parts runs[w].x .. runs[w].x + runs[w].y - 1 one
// after another: a segment of a split problem (a run of one), or several
// small problems packed whole (no neighbours, so no waits).  The register
// budget of 3 waves per SIMD with a double cache, 4 with a float cache (some
// spills either way: measured faster than fewer, larger-register waves)
// keeps more parts resident.
template <typename T>
constexpr int split_waves()
{
    return sizeof(T) == sizeof(double) ? 3 : 4;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(split_waves<T>(), split_waves<T>())))
void k_batch_split(
    BatchProb* __restrict__ probs, const BatchPart* __restrict__ parts, const int2* __restrict__ runs, int* flags,
    double* __restrict__ U, T* __restrict__ Us, T* Prow, T* Pnext, Dev d, int ns, int max_steps,
    unsigned long long* __restrict__ cnt, unsigned long long* __restrict__ span)
{
    const unsigned long long t_start = wall_clock64();
    __shared__ int s_ok;
    // face fluxes of a chunk of cells, double buffered: sF[b][v][f]
    __shared__ T sF[2][9 * NT];
    const int2 run = runs[blockIdx.x];
    int nfail = 0, natm = 0, npf = 0, nfb = 0, itmax = 0;
    bool stalled = false;
    for (int part = run.x; part < run.x + run.y && !stalled; ++part) {
        const BatchPart pt = uniform_load(&parts[part]);
        const BatchProb pr = uniform_load(&probs[pt.b]);
        const int n = pr.n, pitch = n + 4;
        const int nsteps = min(max_steps, pr.steps - pr.done);
        const int base = pr.done * ns;   // substeps every part of the problem had completed
        const int nsub = nsteps * ns;
        // cells within two of either end of the segment (and those beyond it,
        // the neighbours' and the ghost images) are written and read with
        // system-scope accesses; the rest of the row with plain ones
        auto edge = [&](int x) { return x < pt.c0 + 2 || x >= pt.c1 - 2; };
        auto rd = [&](const T* r, int x) { return edge(x) ? sys_load(r + x + 2) : r[x + 2]; };
        const int t = threadIdx.x;
        double* Ub = U + 9 * pr.off;
        T* Usb = Us + 9 * pr.off;
        T* cur = Prow + pr.poff;
        T* nxt = Pnext + pr.poff;
        const Geo geo = geo_at<FLAT>(d, 0.0, 0.0, 0.0);
        for (int i = 0; i < nsub && !stalled; ++i) {
            if (i > 0 && !split_wait(flags, pt.left, pt.right, base + i, &s_ok)) {
                stalled = true;
                break;
            }
            const int s = i % ns;
            const double a = ns == 3 ? (s == 0 ? 0.0 : (s == 1 ? 0.75 : 1.0 / 3.0)) : (s == 0 ? 0.0 : 0.5);
            const double bb = ns == 3 ? (s == 0 ? 1.0 : (s == 1 ? 0.25 : 2.0 / 3.0)) : (s == 0 ? 1.0 : 0.5);
            // the segment in chunks of NT - 1 cells, consecutive cells on
            // consecutive threads (coalesced rows): thread t solves the face
            // left of cell base + t (NT faces per chunk, the last one the
            // right face of the chunk's last cell), then updates that cell
            bool wrote_edge = false;
            int chunk = 0;
            for (int cb = pt.c0; cb < pt.c1; cb += NT - 1, ++chunk) {
                const int cend = min(cb + NT - 1, pt.c1);   // cells [cb, cend), faces [cb, cend]
                const int c = cb + t;
                T* F = sF[chunk & 1];
                T q[9];
                if (c <= cend) {
                    // face c - 1/2 from cells c-2 .. c+1 (row index + 2)
                    T qL[9], qR[9], Fc[9];
    #pragma unroll
                    for (int v = 0; v < 9; ++v) {
                        const T* r = cur + v * pitch;
                        const T q0 = rd(r, c - 2), q1 = rd(r, c - 1), q2 = rd(r, c), q3 = rd(r, c + 1);
                        q[v] = q2;
                        qL[v] = q1 + mc_hslope(q0, q1, q2);
                        qR[v] = q2 - mc_hslope(q1, q2, q3);
                    }
                    face_flux<0, FLAT>(qL, qR, 0.0, 0.0, 0.0, 0, d, Fc);
    #pragma unroll
                    for (int v = 0; v < 9; ++v)
                        F[v * NT + t] = Fc[v];
                }
                __syncthreads();
                if (c < cend) {
                    double R[9];
    #pragma unroll
                    for (int v = 0; v < 9; ++v)
                        R[v] = -((double)F[v * NT + t + 1] - (double)F[v * NT + t]) * pr.idx;
                    R[8] -= d.kappa * (double)q[8];
                    double u[9], qg[9], p[9];
    #pragma unroll
                    for (int v = 0; v < 9; ++v) {
                        const double un = Ub[(long long)v * n + c];
                        const double us = s == 0 ? un : (double)Usb[(long long)v * n + c];
                        u[v] = us + a * (un - us) + bb * (pr.dt * R[v]);
                        qg[v] = (double)q[v];
                    }
                    int iters = 0;
                    const int fl = recover_cell(d, geo, u, qg, p, iters);
                    tally(fl, iters, nfail, natm, npf, nfb, itmax);
                    if (s == ns - 1) {
    #pragma unroll
                        for (int v = 0; v < 9; ++v)
                            Ub[(long long)v * n + c] = u[v];
                    } else {
    #pragma unroll
                        for (int v = 0; v < 9; ++v)
                            Usb[(long long)v * n + c] = (T)u[v];
                    }
                    if (edge(c)) {
                        row_store_sys(nxt, pitch, n, d.bc[0], c, p);
                        wrote_edge = true;
                    } else {
                        row_store(nxt, pitch, n, d.bc[0], c, p);
                    }
                }
            }
            // publish: the values other parts read have reached memory, then the count
            if (wrote_edge)
                __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(&flags[part], base + i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            T* t = cur;
            cur = nxt;
            nxt = t;
        }
        if (!stalled && (nsub & 1)) {
            // the row ended in Pnext: once the neighbours no longer read Prow (they
            // completed every substep), copy the own cells and their ghost images
            if (!split_wait(flags, pt.left, pt.right, base + nsub, &s_ok))
                stalled = true;
            else {
                for (int c = pt.c0 + t; c < pt.c1; c += NT) {
                    double p[9];
    #pragma unroll
                    for (int v = 0; v < 9; ++v)
                        p[v] = (double)rd(cur + v * pitch, c);
                    row_store(Prow + pr.poff, pitch, n, d.bc[0], c, p);
                }
            }
        }
        // the problem's first part records the steps once every part has taken them
        if (!stalled && part == pt.first) {
            for (int q = 0; q < pt.count && !stalled; ++q)
                if (!split_wait(flags, pt.first + q, -1, base + nsub, &s_ok))
                    stalled = true;
            if (!stalled && threadIdx.x == 0)
                probs[pt.b].done = pr.done + nsteps;
        }
    }
    if (stalled && threadIdx.x == 0)
        atomicAdd(&cnt[(size_t)(blockIdx.x % CNT_SLOTS) * CNT_WORDS + CNT_STALL], 1ull);
    count_sums(cnt, nfail, natm, npf, nfb, itmax);
    span_record(span, t_start);
}

// The device arithmetic the kernels use, on arrays, for checking it against
// correctly rounded results: x / y, sqrt(x), rsqrt(x) (FP64).
__global__ __launch_bounds__(BLOCK) void k_arith(const double* __restrict__ x, const double* __restrict__ y,
                                                double* __restrict__ out, long long n)
{
    const long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= n)
        return;
    const double a = x[t], b = y[t];
    out[t] = a / b;
    out[n + t] = sqrt(a);
    out[2 * n + t] = rsqrt(a);
}

// ---------------------------------------------------------------------------
// Launchers (T = double or float)

static inline unsigned blocks_for(long long n)
{
    return (unsigned)((n + BLOCK - 1) / BLOCK);
}

hipError_t launch_arith(const double* x, const double* y, double* out, long long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_arith, dim3(blocks_for(n)), dim3(BLOCK), 0, s, x, y, out, n);
    return hipGetLastError();
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

template <int KIND, bool NT, typename T>
static hipError_t launch_flux_k(int dir, const T* Pc, T* F, const Dev& d, hipStream_t s)
{
    if (d.ppm) {
        const unsigned nb = blocks_for(d.nf[dir]);
        if (dir == 0)
            hipLaunchKernelGGL((k_flux_ppm<0, KIND, NT, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        else if (dir == 1)
            hipLaunchKernelGGL((k_flux_ppm<1, KIND, NT, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        else
            hipLaunchKernelGGL((k_flux_ppm<2, KIND, NT, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        return hipGetLastError();
    }
    if (dir == 0) {
        hipLaunchKernelGGL((k_flux_x<KIND, NT, T>), dim3(blocks_for(d.nf[0])), dim3(BLOCK), 0, s, Pc, F, d);
    } else {
        const int o = dir == 1 ? 2 : 1;
        // faces per thread along y: 12 (fewer re-read window cells than 8: the
        // y kernel 4 % faster at 192^3, measured) where that still gives
        // MIN_BLOCKS workgroups, else 2 (small grids: the whole GPU busy);
        // 8 along z
        const long long lines = (long long)d.n[0] * d.n[o];
        const bool longy = blocks_for(lines * ((d.n[1] + 1 + 11) / 12)) >= MIN_BLOCKS;
        const int seg = dir == 1 ? (longy ? 12 : 2) : MARCH_SEG;
        long long nseg = (d.n[dir] + 1 + seg - 1) / seg;
        unsigned nb = blocks_for(lines * nseg);
        if (dir == 1 && longy)
            hipLaunchKernelGGL((k_flux_march<1, KIND, 12, NT, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        else if (dir == 1)
            hipLaunchKernelGGL((k_flux_march<1, KIND, 2, NT, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
        else
            hipLaunchKernelGGL((k_flux_march<2, KIND, MARCH_SEG, NT, T>), dim3(nb), dim3(BLOCK), 0, s, Pc, F, d);
    }
    return hipGetLastError();
}

// Stored metric: the caller's lapse and psi^4 at the cell centres with 2
// ghost layers on every active axis (dense [z][y][x]) to the values the
// kernels read: at cell centres the values and the fourth-order central
// differences (a_{i-2} - 8 a_{i-1} + 8 a_{i+1} - a_{i+2}) / (12 dx) (zero
// along an inactive axis); at the faces of every active axis the
// fourth-order interpolation (-a_{f-2} + 9 a_{f-1} + 9 a_f - a_{f+1}) / 16.
__global__ __launch_bounds__(BLOCK) void k_metric(const double* __restrict__ A, const double* __restrict__ Pq,
                                                  double* __restrict__ mc, double* __restrict__ mf0,
                                                  double* __restrict__ mf1, double* __restrict__ mf2, Dev d)
{
    long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    const int g[3] = {d.act[0] ? 2 : 0, d.act[1] ? 2 : 0, d.act[2] ? 2 : 0};
    const long long sx = 1, sy = d.n[0] + 2 * g[0], sz = sy * (d.n[1] + 2 * g[1]);
    const long long st[3] = {sx, sy, sz};
    auto at = [&](int i, int j, int k) { return (long long)(k + g[2]) * sz + (long long)(j + g[1]) * sy + (i + g[0]); };
    if (t < d.N) {
        const int i = (int)(t % d.n[0]);
        const long long r = t / d.n[0];
        const int j = (int)(r % d.n[1]);
        const int k = (int)(r / d.n[1]);
        const long long c = at(i, j, k);
        mc[t] = A[c];
        mc[d.N + t] = Pq[c];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double da = 0.0, dp = 0.0;
            if (d.act[a]) {
                const long long s = st[a];
                da = (A[c - 2 * s] - 8.0 * A[c - s] + 8.0 * A[c + s] - A[c + 2 * s]) / (12.0 * d.dx[a]);
                dp = (Pq[c - 2 * s] - 8.0 * Pq[c - s] + 8.0 * Pq[c + s] - Pq[c + 2 * s]) / (12.0 * d.dx[a]);
            }
            mc[(2 + a) * d.N + t] = da;
            mc[(5 + a) * d.N + t] = dp;
        }
        return;
    }
    t -= d.N;
    double* mf[3] = {mf0, mf1, mf2};
    for (int a = 0; a < 3; ++a) {
        if (!d.act[a])
            continue;
        if (t >= d.nf[a]) {
            t -= d.nf[a];
            continue;
        }
        const int m0 = d.n[0] + (a == 0), m1 = d.n[1] + (a == 1);
        int ix[3];
        ix[0] = (int)(t % m0);
        const long long r = t / m0;
        ix[1] = (int)(r % m1);
        ix[2] = (int)(r / m1);
        const long long c = at(ix[0], ix[1], ix[2]);   // cell f along a
        const long long s = st[a];
        mf[a][t] = (-A[c - 2 * s] + 9.0 * A[c - s] + 9.0 * A[c] - A[c + s]) / 16.0;
        mf[a][d.nf[a] + t] = (-Pq[c - 2 * s] + 9.0 * Pq[c - s] + 9.0 * Pq[c] - Pq[c + s]) / 16.0;
        return;
    }
}

hipError_t launch_metric(const double* alpha, const double* psi4, double* mc, double* const* mf, const Dev& d,
                         hipStream_t s)
{
    const long long total = d.N + d.nf[0] + d.nf[1] + d.nf[2];
    hipLaunchKernelGGL(k_metric, dim3(blocks_for(total)), dim3(BLOCK), 0, s, alpha, psi4, mc, mf[0], mf[1], mf[2],
                       d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ct(T* const* F, T* const* W, const Dev& d, hipStream_t s)
{
    CtArgs<T> A;
    long long edges = 0, faces = 0;
    for (int p = 0; p < 3; ++p) {
        const int a = p == 2 ? 1 : 0, b = p == 0 ? 1 : 2, e = 3 - a - b;
        A.F[p] = F[p];
        A.W[p] = W[p];
        A.nW[p] = d.act[a] && d.act[b] ? (long long)(d.n[a] + 1) * (d.n[b] + 1) * d.n[e] : 0;
        edges += A.nW[p];
        faces += d.act[p] ? d.nf[p] : 0;
    }
    if (edges == 0)
        return hipSuccess;   // one active axis: no transverse flux to replace
    hipLaunchKernelGGL(k_ct_edges<T>, dim3(blocks_for(edges)), dim3(BLOCK), 0, s, A, d);
    hipLaunchKernelGGL(k_ct_faces<T>, dim3(blocks_for(faces)), dim3(BLOCK), 0, s, A, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_flux(int kind, int dir, const T* Pc, T* F, const Dev& d, hipStream_t s)
{
    if (d.nt) {
        if (kind == FLAT)
            return launch_flux_k<FLAT, true>(dir, Pc, F, d, s);
        return kind == ISO ? launch_flux_k<ISO, true>(dir, Pc, F, d, s)
                           : launch_flux_k<STORED, true>(dir, Pc, F, d, s);
    }
    if (kind == FLAT)
        return launch_flux_k<FLAT, false>(dir, Pc, F, d, s);
    return kind == ISO ? launch_flux_k<ISO, false>(dir, Pc, F, d, s) : launch_flux_k<STORED, false>(dir, Pc, F, d, s);
}

template <bool NT, typename T, typename TS, typename TO>
static void launch_update_nt(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, T* Pn, const double* Un,
                             const TS* Us, TO* Uout, const Dev& d, double dt, double a, double b,
                             unsigned long long* cnt, unsigned char* fout, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_update<FLAT, NT, T, TS, TO>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Pn, Un, Us,
                           Uout, d, dt, a, b, cnt, fout);
    else if (kind == ISO)
        hipLaunchKernelGGL((k_update<ISO, NT, T, TS, TO>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Pn, Un, Us,
                           Uout, d, dt, a, b, cnt, fout);
    else
        hipLaunchKernelGGL((k_update<STORED, NT, T, TS, TO>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, Pn, Un,
                           Us, Uout, d, dt, a, b, cnt, fout);
}

template <typename T, typename TS, typename TO>
hipError_t launch_update(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, T* Pn, const double* Un,
                         const TS* Us, TO* Uout, const Dev& d, double dt, double a, double b,
                         unsigned long long* cnt, unsigned char* fout, hipStream_t s)
{
    if (d.nt)
        launch_update_nt<true>(kind, Fx, Fy, Fz, Pc, Pn, Un, Us, Uout, d, dt, a, b, cnt, fout, s);
    else
        launch_update_nt<false>(kind, Fx, Fy, Fz, Pc, Pn, Un, Us, Uout, d, dt, a, b, cnt, fout, s);
    return hipGetLastError();
}

template <bool NT, int SEG, typename T, typename TS, typename TO>
static void launch_substep_nt(int kind, const T* Pc, T* Pn, const double* Un, const TS* Us, TO* Uout, const Dev& d,
                              double dt, double a, double b, unsigned long long* cnt, unsigned char* fout,
                              hipStream_t s)
{
    constexpr int TX = SUB_TX, TY = SUB_TY;
    const int ntx = (d.n[0] + TX - 1) / TX, nty = (d.n[1] + TY - 1) / TY;
    const int ntiles = ntx * nty;
    const long long nseg = (d.n[2] + SEG - 1) / SEG;
    const dim3 grid((unsigned)(ntiles * nseg)), block(TX * TY);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_substep<FLAT, TX, TY, SEG, NT, T, TS, TO>), grid, block, 0, s, Pc, Pn, Un, Us, Uout, d,
                           dt, a, b, cnt, fout, ntx, ntiles);
    else if (kind == ISO)
        hipLaunchKernelGGL((k_substep<ISO, TX, TY, SEG, NT, T, TS, TO>), grid, block, 0, s, Pc, Pn, Un, Us, Uout, d,
                           dt, a, b, cnt, fout, ntx, ntiles);
    else
        hipLaunchKernelGGL((k_substep<STORED, TX, TY, SEG, NT, T, TS, TO>), grid, block, 0, s, Pc, Pn, Un, Us, Uout,
                           d, dt, a, b, cnt, fout, ntx, ntiles);
}

template <typename T, typename TS, typename TO>
hipError_t launch_substep(int kind, const T* Pc, T* Pn, const double* Un, const TS* Us, TO* Uout, const Dev& d,
                          double dt, double a, double b, unsigned long long* cnt, unsigned char* fout, hipStream_t s)
{
    // planes per workgroup: the long segment where it still gives enough
    // workgroups to fill the GPU, else a short one (small grids)
    const long long tiles = (long long)((d.n[0] + SUB_TX - 1) / SUB_TX) * ((d.n[1] + SUB_TY - 1) / SUB_TY);
    const bool lng = tiles * ((d.n[2] + SUB_SEG - 1) / SUB_SEG) >= SUB_MIN_BLOCKS;
    if (d.nt && lng)
        launch_substep_nt<true, SUB_SEG>(kind, Pc, Pn, Un, Us, Uout, d, dt, a, b, cnt, fout, s);
    else if (d.nt)
        launch_substep_nt<true, 2>(kind, Pc, Pn, Un, Us, Uout, d, dt, a, b, cnt, fout, s);
    else if (lng)
        launch_substep_nt<false, SUB_SEG>(kind, Pc, Pn, Un, Us, Uout, d, dt, a, b, cnt, fout, s);
    else
        launch_substep_nt<false, 2>(kind, Pc, Pn, Un, Us, Uout, d, dt, a, b, cnt, fout, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rhs(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, double* R,
                      const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_rhs<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    else if (kind == ISO)
        hipLaunchKernelGGL((k_rhs<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    else
        hipLaunchKernelGGL((k_rhs<STORED, T>), dim3(nb), dim3(BLOCK), 0, s, Fx, Fy, Fz, Pc, R, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cons(int kind, const double* P, double* U, T* Pc, const Dev& d, hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_cons<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    else if (kind == ISO)
        hipLaunchKernelGGL((k_cons<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    else
        hipLaunchKernelGGL((k_cons<STORED, T>), dim3(nb), dim3(BLOCK), 0, s, P, U, Pc, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prim(int kind, const double* U, double* P, T* Pc, const Dev& d, unsigned long long* cnt,
                       hipStream_t s)
{
    unsigned nb = blocks_for(d.N);
    if (kind == FLAT)
        hipLaunchKernelGGL((k_prim<FLAT, T>), dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    else if (kind == ISO)
        hipLaunchKernelGGL((k_prim<ISO, T>), dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    else
        hipLaunchKernelGGL((k_prim<STORED, T>), dim3(nb), dim3(BLOCK), 0, s, U, P, Pc, d, cnt);
    return hipGetLastError();
}


template <typename T>
hipError_t launch_batch_cons(const BatchProb* probs, int nprob, long long ncell, const double* P, double* U,
                             T* Prow, const Dev& d, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch_cons<T>), dim3(blocks_for(ncell)), dim3(BLOCK), 0, s, probs, nprob, ncell, P, U,
                       Prow, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_prim(const BatchProb* probs, int nprob, long long ncell, const double* U, double* P,
                             T* Prow, const Dev& d, unsigned long long* cnt, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch_prim<T>), dim3(blocks_for(ncell)), dim3(BLOCK), 0, s, probs, nprob, ncell, U, P,
                       Prow, d, cnt);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t batch_evolve_k(int lds, size_t lds_bytes, BatchProb* probs, const int* order, int nprob,
                                 double* U, T* Us, T* Prow, T* Pnext, const Dev& d, int ns, int max_steps,
                                 unsigned long long* cnt, unsigned long long* span, hipStream_t s)
{
    if (lds) {
        // (the dynamic LDS size was allowed by allow_batch_lds at set-up)
        hipLaunchKernelGGL((k_batch_evolve<T, NT, true>), dim3(nprob), dim3(NT), lds_bytes, s, probs, order, U,
                           Us, Prow, Pnext, d, ns, max_steps, cnt, span);
    } else
        hipLaunchKernelGGL((k_batch_evolve<T, NT, false>), dim3(nprob), dim3(NT), 0, s, probs, order, U, Us,
                           Prow, Pnext, d, ns, max_steps, cnt, span);
    return hipGetLastError();
}

template <typename T, int NT>
static int evolve_occupancy_k(int lds, size_t lds_bytes)
{
    int nb = 0;
    const hipError_t e =
        lds ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_evolve<T, NT, true>, NT, lds_bytes)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_evolve<T, NT, false>, NT, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

template <typename T>
int batch_evolve_occupancy(int shape, int lds, size_t lds_bytes)
{
    switch (BATCH_THREADS[shape]) {
    case 256:
        return evolve_occupancy_k<T, 256>(lds, lds_bytes);
    case 512:
        return evolve_occupancy_k<T, 512>(lds, lds_bytes);
    default:
        return evolve_occupancy_k<T, 1024>(lds, lds_bytes);
    }
}

// Dynamic LDS beyond the default launch limit must be allowed per kernel, once,
// outside any graph capture: raised for every launch shape of T to at least
// `bytes`, never lowered (other contexts may need more).
template <typename T>
hipError_t allow_batch_lds(size_t bytes)
{
    static size_t allowed = 0;
    if (bytes <= allowed)
        return hipSuccess;
    const void* fn[3] = {(const void*)k_batch_evolve<T, 256, true>, (const void*)k_batch_evolve<T, 512, true>,
                         (const void*)k_batch_evolve<T, 1024, true>};
    for (const void* f : fn) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess)
            return e;
    }
    allowed = bytes;
    return hipSuccess;
}

// Before a split launch: every part's flag at the substeps its problem has
// completed, so that the flags agree with the records whatever ran before
// (another launch shape, a tuning run on copies, a reset).
__global__ __launch_bounds__(BLOCK) void k_split_flags(const BatchProb* __restrict__ probs,
                                                       const BatchPart* __restrict__ parts, int nparts,
                                                       int* __restrict__ flags, int ns)
{
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (p < nparts)
        flags[p] = probs[parts[p].b].done * ns;
}

template <typename T>
hipError_t launch_batch_split(BatchProb* probs, const BatchPart* parts, int nparts, const int2* runs, int nruns,
                              int* flags, double* U, T* Us, T* Prow, T* Pnext, const Dev& d, int rk_order,
                              int max_steps, unsigned long long* cnt, unsigned long long* span, hipStream_t s)
{
    hipLaunchKernelGGL(k_split_flags, dim3(blocks_for(nparts)), dim3(BLOCK), 0, s, probs, parts, nparts, flags,
                       rk_order);
    hipLaunchKernelGGL((k_batch_split<T, BATCH_SPLIT_THREADS>), dim3(nruns), dim3(BATCH_SPLIT_THREADS), 0, s, probs,
                       parts, runs, flags, U, Us, Prow, Pnext, d, rk_order, max_steps, cnt, span);
    return hipGetLastError();
}

template <typename T>
int batch_split_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_split<T, BATCH_SPLIT_THREADS>,
                                                     BATCH_SPLIT_THREADS, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

template <typename T>
hipError_t launch_batch_evolve(int shape, int lds, size_t lds_bytes, BatchProb* probs, const int* order, int nprob,
                               double* U, T* Us, T* Prow, T* Pnext, const Dev& d, int rk_order, int max_steps,
                               unsigned long long* cnt, unsigned long long* span, hipStream_t s)
{
    switch (shape) {
    case 0:
        return batch_evolve_k<T, 256>(lds, lds_bytes, probs, order, nprob, U, Us, Prow, Pnext, d, rk_order,
                                      max_steps, cnt, span, s);
    case 1:
        return batch_evolve_k<T, 512>(lds, lds_bytes, probs, order, nprob, U, Us, Prow, Pnext, d, rk_order,
                                      max_steps, cnt, span, s);
    default:
        return batch_evolve_k<T, 1024>(lds, lds_bytes, probs, order, nprob, U, Us, Prow, Pnext, d, rk_order,
                                       max_steps, cnt, span, s);
    }
}

// explicit instantiations for the two precisions
#define GRMHD_INSTANTIATE_UPDATE(T, TS, TO)                                                             \
    template hipError_t launch_update<T, TS, TO>(int, const T*, const T*, const T*, const T*, T*,       \
                                                 const double*, const TS*, TO*, const Dev&, double,     \
                                                 double, double, unsigned long long*, unsigned char*,   \
                                                 hipStream_t);                                          \
    template hipError_t launch_substep<T, TS, TO>(int, const T*, T*, const double*, const TS*, TO*,     \
                                                  const Dev&, double, double, double, unsigned long long*, \
                                                  unsigned char*, hipStream_t);
#define GRMHD_INSTANTIATE_BATCH(T)                                                                      \
    template hipError_t launch_batch_cons<T>(const BatchProb*, int, long long, const double*, double*, T*,     \
                                             const Dev&, hipStream_t);                                        \
    template hipError_t launch_batch_prim<T>(const BatchProb*, int, long long, const double*, double*, T*,     \
                                             const Dev&, unsigned long long*, hipStream_t);                   \
    template hipError_t allow_batch_lds<T>(size_t);                                                           \
    template hipError_t launch_batch_split<T>(BatchProb*, const BatchPart*, int, const int2*, int, int*, double*, \
                                              T*, T*, T*, const Dev&, int, int, unsigned long long*,              \
                                              unsigned long long*, hipStream_t);                                 \
    template int batch_split_occupancy<T>();                                                                  \
    template int batch_evolve_occupancy<T>(int, int, size_t);                                                 \
    template hipError_t launch_batch_evolve<T>(int, int, size_t, BatchProb*, const int*, int, double*, T*, T*, \
                                               T*, const Dev&, int, int, unsigned long long*, unsigned long long*, \
                                               hipStream_t);
GRMHD_INSTANTIATE_BATCH(double)
GRMHD_INSTANTIATE_BATCH(float)
GRMHD_INSTANTIATE_UPDATE(double, double, double)
GRMHD_INSTANTIATE_UPDATE(float, double, float)
GRMHD_INSTANTIATE_UPDATE(float, float, float)
GRMHD_INSTANTIATE_UPDATE(float, float, double)

#define GRMHD_INSTANTIATE(T)                                                                            \
    template hipError_t launch_fill<T>(T*, long long, double, hipStream_t);                             \
    template hipError_t launch_ghosts<T>(T*, const Dev&, hipStream_t);                                  \
    template hipError_t launch_flux<T>(int, int, const T*, T*, const Dev&, hipStream_t);               \
    template hipError_t launch_ct<T>(T* const*, T* const*, const Dev&, hipStream_t);                   \
    template hipError_t launch_rhs<T>(int, const T*, const T*, const T*, const T*, double*, const Dev&,  \
                                      hipStream_t);                                                     \
    template hipError_t launch_cons<T>(int, const double*, double*, T*, const Dev&, hipStream_t);      \
    template hipError_t launch_prim<T>(int, const double*, double*, T*, const Dev&, unsigned long long*, \
                                       hipStream_t);
GRMHD_INSTANTIATE(double)
GRMHD_INSTANTIATE(float)

}  // namespace grmhd
