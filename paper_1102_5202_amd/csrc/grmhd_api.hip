// grmhd_api.hip -- the C ABI declared in include/grmhd.h.
//
// Host side only: validation, carving the caller's workspace, and enqueuing
// the kernels of grmhd_kernels.hip on the caller's stream.  No device memory
// is allocated or freed here and no call except grmhd_status/grmhd_timing
// synchronises.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>

#include "grmhd.h"
#include "grmhd_internal.h"

using grmhd::Dev;

namespace {

struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};

struct Layout {
    int g[3], px, py, pz;
    long long sv, N, nf[3];
    size_t off_cnt, off_pc[3], off_us, off_f[3];
    // flux-CT: edge values of the axis pairs (x,y), (x,z), (y,z)
    bool ct = false;
    size_t off_w[3] = {0, 0, 0};
    // adjoint part (FP64): stage primitive caches P^0..P^ns, the stages'
    // recovery flags, the recomputed stage state, the U^n cotangent
    // accumulator, the R cotangent, a dense primitive scratch, the ghosted
    // cotangent of the primitives and the face-state cotangents of one axis
    bool adj;
    size_t off_ac[4], off_aflags, off_aus, off_unacc, off_rb, off_pb, off_mu, off_fb[3], off_gmu[3];
    // tape of recorded steps (FP64): per slot the ns+1 stage caches and the
    // ns stages' recovery flags
    int tape = 0;
    size_t off_tape = 0, tape_slot = 0, tape_flags = 0;
    size_t total;
};

size_t round_up(size_t x, size_t a)
{
    return (x + a - 1) / a * a;
}

bool grid_ok(const grmhd_grid* g)
{
    if (!g)
        return false;
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 1 || g->n[d] > (1 << 20))
            return false;
        if (!(g->hi[d] > g->lo[d]) || !std::isfinite(g->lo[d]) || !std::isfinite(g->hi[d]))
            return false;
        if (g->bc[d] != GRMHD_BC_PERIODIC && g->bc[d] != GRMHD_BC_OUTFLOW)
            return false;
    }
    // at most 2^38 cells: workspace sizes stay far inside size_t and every
    // launch inside the 2^31 - 1 workgroups of a grid dimension
    const long long N = (long long)g->n[0] * g->n[1] * g->n[2];
    return N <= (1LL << 38);
}

Layout make_layout(const grmhd_grid* g, size_t esize, bool adjoint = false, int ns = 3, int tape = 0,
                   int ghost = 2, bool ct = false)
{
    Layout L{};
    for (int d = 0; d < 3; ++d)
        L.g[d] = g->n[d] > 1 ? ghost : 0;
    // x pitch rounded to 8 doubles (64 bytes) so rows start aligned
    L.px = (int)round_up((size_t)(g->n[0] + 2 * L.g[0]), 8);
    L.py = g->n[1] + 2 * L.g[1];
    L.pz = g->n[2] + 2 * L.g[2];
    L.sv = (long long)L.px * L.py * L.pz;
    L.N = (long long)g->n[0] * g->n[1] * g->n[2];
    for (int d = 0; d < 3; ++d) {
        long long nf = 1;
        for (int e = 0; e < 3; ++e)
            nf *= g->n[e] + (e == d ? 1 : 0);
        L.nf[d] = g->n[d] > 1 ? nf : 0;
    }
    size_t off = 0;
    L.off_cnt = off;
    off = round_up(off + grmhd::CNT_BYTES, 256);
    for (int b = 0; b < 3; ++b) {
        L.off_pc[b] = off;
        if (b == 0 || g->n[2] > 1)   // the extra caches serve the fused 3D update only
            off = round_up(off + esize * 9 * (size_t)L.sv, 256);
    }
    L.off_us = off;                  // intermediate Runge-Kutta stage state
    off = round_up(off + esize * 9 * (size_t)L.N, 256);
    for (int d = 0; d < 3; ++d) {
        L.off_f[d] = off;
        off = round_up(off + esize * 9 * (size_t)L.nf[d], 256);
    }
    L.ct = ct;
    if (ct) {
        for (int p = 0; p < 3; ++p) {
            const int x = p == 2 ? 1 : 0, y = p == 0 ? 1 : 2, z = 3 - x - y;
            L.off_w[p] = off;
            if (g->n[x] > 1 && g->n[y] > 1)
                off = round_up(off + esize * (size_t)(g->n[x] + 1) * (g->n[y] + 1) * g->n[z], 256);
        }
    }
    L.adj = adjoint;
    if (adjoint) {
        const size_t cache = sizeof(double) * 9 * (size_t)L.sv, dense = sizeof(double) * 9 * (size_t)L.N;
        for (int b = 0; b < 4; ++b) {
            L.off_ac[b] = off;
            if (b <= ns)
                off = round_up(off + cache, 256);
        }
        L.off_aflags = off;
        off = round_up(off + (size_t)ns * L.N, 256);
        size_t* dense_offs[5] = {&L.off_aus, &L.off_unacc, &L.off_rb, &L.off_pb, &L.off_mu};
        for (size_t* o : dense_offs) {
            *o = off;
            off = round_up(off + dense, 256);
        }
        // the left/right face-state cotangents of every active axis, and the
        // primitive cotangents at its ghost positions (4 per line)
        for (int d = 0; d < 3; ++d) {
            L.off_fb[d] = off;
            off = round_up(off + sizeof(double) * 18 * (size_t)L.nf[d], 256);
            L.off_gmu[d] = off;
            if (L.nf[d])
                off = round_up(off + sizeof(double) * 9 * 4 * (size_t)(L.N / g->n[d]), 256);
        }
        if (tape > 0) {
            L.tape = tape;
            L.tape_flags = round_up(cache, 256) * (size_t)(ns + 1);
            L.tape_slot = L.tape_flags + round_up((size_t)ns * L.N, 256);
            L.off_tape = off;
            off += L.tape_slot * (size_t)tape;
        }
    }
    L.total = off;
    return L;
}

// The stored-metric buffer: centre values [8][N], then face values [2][nf]
// of every active axis, each part 256-byte aligned.
size_t metric_layout(const grmhd_grid* g, size_t off_mf[3])
{
    long long N = (long long)g->n[0] * g->n[1] * g->n[2];
    size_t off = round_up(sizeof(double) * 8 * (size_t)N, 256);
    for (int d = 0; d < 3; ++d) {
        long long nf = 0;
        if (g->n[d] > 1) {
            nf = 1;
            for (int e = 0; e < 3; ++e)
                nf *= g->n[e] + (e == d ? 1 : 0);
        }
        if (off_mf)
            off_mf[d] = off;
        off = round_up(off + sizeof(double) * 2 * (size_t)nf, 256);
    }
    return off;
}

bool wants_adjoint(const grmhd_opts* o)
{
    return o && o->adjoint && o->precision == GRMHD_FP64;
}

// Ghost layers of the reconstruction: MC reads 2 cells beside a face, PPM 3.
int ghost_width(const grmhd_opts* o)
{
    return o && o->reconstruction == GRMHD_RECON_PPM ? 3 : 2;
}

// Options that fit the grid: PPM needs 3 cells on every active axis (the
// periodic images of the ghost layers) and has no adjoint; an adjoint context
// holds at most 2^30 cells.
bool opts_fit(const grmhd_grid* g, const grmhd_opts* o)
{
    if (!o)
        return true;   // defaults: MC
    if (o->reconstruction != GRMHD_RECON_MC && o->reconstruction != GRMHD_RECON_PPM)
        return false;
    if (o->divergence != GRMHD_DIV_CLEANING && o->divergence != GRMHD_DIV_FLUXCT)
        return false;
    if (o->divergence == GRMHD_DIV_FLUXCT && o->adjoint)
        return false;
    // the adjoint kernels index cells, faces and ghost positions in 32 bits
    if (o->adjoint && (long long)g->n[0] * g->n[1] * g->n[2] > (1LL << 30))
        return false;
    if (o->reconstruction == GRMHD_RECON_PPM) {
        if (o->adjoint)
            return false;
        for (int d = 0; d < 3; ++d)
            if (g->n[d] > 1 && g->n[d] < 3)
                return false;
    }
    return true;
}

int tape_slots(const grmhd_opts* o)
{
    return wants_adjoint(o) && o->tape_steps > 0 && o->tape_steps <= 4096 ? o->tape_steps : 0;
}

// bytes of one value of the primitive caches and face buffers
size_t elem_size(const grmhd_opts* o)
{
    return o && o->precision == GRMHD_MIXED ? sizeof(float) : sizeof(double);
}

}  // namespace

struct grmhd_ctx {
    Dev d;
    int kind;
    int rk_order;
    hipStream_t stream = nullptr;
    Layout L;
    unsigned char* ws = nullptr;
    // Primitive caches.  Pbuf[0] holds the current primitives between calls.
    // A 3D step rotates through all three (RK3: 0 -> 1 -> 2 -> 0, RK2: 0 -> 1
    // -> 0) so that every substep writes a cache it does not read and the step
    // ends in Pbuf[0] (a captured step can be replayed).
    void* Pbuf[3] = {nullptr, nullptr, nullptr};
    void* Us = nullptr;                     // intermediate stage state (cache type)
    void* F[3] = {nullptr, nullptr, nullptr};
    void* W[3] = {nullptr, nullptr, nullptr};   // flux-CT edge values
    // stored metric: set by grmhd_set_metric (kernels read d.mc, d.mf)
    bool metric_ok = true;
    grmhd_grid grid{};
    // cache b has its ghost slabs filled: every kernel that writes a cache
    // (cons, prim, the updates) writes the ghost images of its cells as well
    bool ghosts_ok[3] = {false, false, false};
    bool mixed = false;                     // float caches and face physics
    // adjoint workspace (FP64)
    bool adj = false;
    bool adj_prepared = false;
    double* Ac[4] = {nullptr, nullptr, nullptr, nullptr};
    unsigned char* Aflags = nullptr;
    double *Aus = nullptr, *Unacc = nullptr, *Rb = nullptr, *Pb = nullptr, *MU = nullptr;
    double* FB[3] = {nullptr, nullptr, nullptr};
    double* GMU[3] = {nullptr, nullptr, nullptr};
    // recorded steps: dt of each slot (NaN: never recorded)
    std::vector<double> tape_dt;
    unsigned long long* cnt = nullptr;
    bool prepared = false;
    bool cache_valid = false;
    int timing = 0;
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> spare;
    double ms[GRMHD_K_COUNT] = {};
    long long launches[GRMHD_K_COUNT] = {};
};

namespace {

hipEvent_t take_event(grmhd_ctx* c)
{
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Run `f` (which enqueues one kernel) bracketed by events when timing is on.
template <class Fn>
int timed(grmhd_ctx* c, int kind, Fn&& f)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        a = take_event(c);
        b = take_event(c);
        if (!a || !b)
            return GRMHD_ERR_HIP;
        if (hipEventRecord(a, c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    }
    if (f() != hipSuccess)
        return GRMHD_ERR_HIP;
    if (c->timing) {
        if (hipEventRecord(b, c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
        c->pending.push_back({kind, a, b});
    }
    return GRMHD_OK;
}

// First enqueuing call: clear the counters and poison the caches with NaN so
// that a read outside the stencil (edges, corners, pitch padding) shows up.
template <typename T>
int prepare_t(grmhd_ctx* c)
{
    if (c->prepared)
        return GRMHD_OK;
    if (grmhd::launch_zero_counters(c->cnt, c->stream) != hipSuccess)
        return GRMHD_ERR_HIP;
    for (int b = 0; b < 3; ++b)
        if (c->d.act[2] || b == 0)
            if (grmhd::launch_fill((T*)c->Pbuf[b], 9 * c->L.sv, std::nan(""), c->stream) != hipSuccess)
                return GRMHD_ERR_HIP;
    c->prepared = true;
    return GRMHD_OK;
}

template <typename T>
T* cache(grmhd_ctx* c, int b = 0)
{
    return (T*)c->Pbuf[b];
}

template <typename T>
T* faces(grmhd_ctx* c, int d)
{
    return (T*)c->F[d];
}

// Ghost fill of cache b (unless the kernel that wrote it filled them) and the
// face fluxes of the active axes up to ndir.
template <typename T>
int fluxes(grmhd_ctx* c, int b, int ndir)
{
    T* P = cache<T>(c, b);
    int rc = GRMHD_OK;
    if (!c->ghosts_ok[b]) {
        rc = timed(c, GRMHD_K_BC, [&] { return grmhd::launch_ghosts(P, c->d, c->stream); });
        if (rc)
            return rc;
        c->ghosts_ok[b] = true;
    }
    for (int dir = 0; dir < ndir; ++dir) {
        if (!c->d.act[dir])
            continue;
        rc = timed(c, GRMHD_K_FLUX_X + dir, [&] {
            return grmhd::launch_flux(c->kind, dir, (const T*)P, faces<T>(c, dir), c->d, c->stream);
        });
        if (rc)
            return rc;
    }
    if (c->d.ct && ndir == 3) {
        T* F[3] = {faces<T>(c, 0), faces<T>(c, 1), faces<T>(c, 2)};
        T* W[3] = {(T*)c->W[0], (T*)c->W[1], (T*)c->W[2]};
        rc = timed(c, GRMHD_K_CT, [&] { return grmhd::launch_ct(F, W, c->d, c->stream); });
        if (rc)
            return rc;
    }
    return GRMHD_OK;
}

template <typename T>
int cons_t(grmhd_ctx* c, const double* P, double* U)
{
    int rc = prepare_t<T>(c);
    if (rc)
        return rc;
    rc = timed(c, GRMHD_K_CONS, [&] { return grmhd::launch_cons(c->kind, P, U, cache<T>(c), c->d, c->stream); });
    if (rc)
        return rc;
    c->cache_valid = true;
    c->ghosts_ok[0] = true;
    return GRMHD_OK;
}

template <typename T>
int prim_t(grmhd_ctx* c, const double* U, double* P)
{
    int rc = prepare_t<T>(c);
    if (rc)
        return rc;
    rc = timed(c, GRMHD_K_PRIM, [&] {
        return grmhd::launch_prim(c->kind, U, P, cache<T>(c), c->d, c->cnt, c->stream);
    });
    if (rc)
        return rc;
    c->cache_valid = true;
    c->ghosts_ok[0] = true;
    return GRMHD_OK;
}

template <typename T>
int rhs_t(grmhd_ctx* c, const double* P, double* R)
{
    int rc = prepare_t<T>(c);
    if (rc)
        return rc;
    rc = timed(c, GRMHD_K_CONS, [&] {
        return grmhd::launch_cons(c->kind, P, (double*)nullptr, cache<T>(c), c->d, c->stream);
    });
    if (rc)
        return rc;
    c->cache_valid = true;
    c->ghosts_ok[0] = true;
    rc = fluxes<T>(c, 0, 3);
    if (rc)
        return rc;
    return timed(c, GRMHD_K_RHS, [&] {
        return grmhd::launch_rhs(c->kind, (const T*)faces<T>(c, 0), (const T*)faces<T>(c, 1),
                                 (const T*)faces<T>(c, 2), (const T*)cache<T>(c), R, c->d, c->stream);
    });
}

// SSP Runge-Kutta stages: U^(s+1) = U^s + a_s (U^n - U^s) + b_s dt R(P^s)
const double RK3A[3] = {0.0, 0.75, 1.0 / 3.0};
const double RK3B[3] = {1.0, 0.25, 2.0 / 3.0};
const double RK2A[2] = {0.0, 0.5};
const double RK2B[2] = {1.0, 0.5};

// One substep's update launch with the stage-state types TS (read) and TO
// (written).
template <typename T, typename TS, typename TO>
int update_stage(grmhd_ctx* c, bool fused, int src, int dst, const double* U, const TS* Us, TO* Uout,
                 double dt, double a, double b)
{
    return timed(c, GRMHD_K_UPDATE, [&] {
        if (fused)
            return grmhd::launch_substep(c->kind, (const T*)cache<T>(c, src), cache<T>(c, dst), U, Us, Uout, c->d,
                                         dt, a, b, c->cnt, (unsigned char*)nullptr, c->stream);
        return grmhd::launch_update(c->kind, (const T*)faces<T>(c, 0), (const T*)faces<T>(c, 1),
                                    (const T*)faces<T>(c, 2), (const T*)cache<T>(c, src), cache<T>(c, dst), U,
                                    Us, Uout, c->d, dt, a, b, c->cnt, (unsigned char*)nullptr, c->stream);
    });
}

template <typename T>
int step_t(grmhd_ctx* c, double* U, double dt)
{
    const int ns = c->rk_order;
    const double* A = ns == 3 ? RK3A : RK2A;
    const double* B = ns == 3 ? RK3B : RK2B;
    // 3D grids with MC and cleaning: one launch of the fused substep kernel
    // (the faces of every axis, the differences, sources, RK combination and
    // recovery), which writes the new primitives to another cache; otherwise
    // (1D, 2D, PPM, flux-CT) the face kernels and then the update in place on
    // the cache (for flux-CT with the face fluxes corrected in between).  The first stage
    // reads U^n as its stage state; the intermediate stage state has the cache
    // type (float in the mixed path); the last stage writes U.
    const bool fused = c->d.act[2] && !c->d.ppm && !c->d.ct;
    T* Us = (T*)c->Us;
    for (int s = 0; s < ns; ++s) {
        const int src = fused ? s : 0;
        const int dst = fused ? (s == ns - 1 ? 0 : s + 1) : 0;
        int rc = fluxes<T>(c, src, fused ? 0 : 3);
        if (rc)
            return rc;
        if (s == 0)
            rc = update_stage<T>(c, fused, src, dst, U, (const double*)U, Us, dt, A[s], B[s]);
        else if (s < ns - 1)
            rc = update_stage<T>(c, fused, src, dst, U, (const T*)Us, Us, dt, A[s], B[s]);
        else
            rc = update_stage<T>(c, fused, src, dst, U, (const T*)Us, U, dt, A[s], B[s]);
        if (rc)
            return rc;
        c->ghosts_ok[dst] = true;
    }
    return GRMHD_OK;
}

double* tape_cache(grmhd_ctx* c, int slot, int b);

// Adjoint: first use fills the stage caches with NaN (their never-written
// edge and corner ghosts included), so that the first recovery of P^0 has no
// valid guess and takes the bracketed solve.
int adj_prepare(grmhd_ctx* c)
{
    int rc = prepare_t<double>(c);
    if (rc)
        return rc;
    if (c->adj_prepared)
        return GRMHD_OK;
    for (int b = 0; b <= c->rk_order; ++b)
        if (grmhd::launch_fill(c->Ac[b], 9 * c->L.sv, std::nan(""), c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    for (int t = 0; t < c->L.tape; ++t)
        for (int b = 0; b <= c->rk_order; ++b)
            if (grmhd::launch_fill(tape_cache(c, t, b), 9 * c->L.sv, std::nan(""), c->stream) != hipSuccess)
                return GRMHD_ERR_HIP;
    c->adj_prepared = true;
    return GRMHD_OK;
}

// Recompute the stages of the step from U: P^0 (recovered, guess = the
// previous call's P^0), then P^(s+1), U^(s+1) and the recovery flags of every
// stage.  The forward caches are not touched.
int adj_recompute(grmhd_ctx* c, const double* U, double dt, const double* A, const double* B)
{
    const int ns = c->rk_order;
    const bool fused = c->d.act[2] && !c->d.ppm && !c->d.ct;
    int rc = timed(c, GRMHD_K_PRIM, [&] {
        return grmhd::launch_prim(c->kind, U, c->Pb, c->Ac[0], c->d, c->cnt, c->stream);
    });
    if (rc)
        return rc;
    for (int s = 0; s < ns; ++s) {
        const double* Ps = c->Ac[s];
        for (int dir = 0; dir < (fused ? 0 : 3); ++dir) {
            if (!c->d.act[dir])
                continue;
            rc = timed(c, GRMHD_K_FLUX_X + dir, [&] {
                return grmhd::launch_flux(c->kind, dir, Ps, (double*)c->F[dir], c->d, c->stream);
            });
            if (rc)
                return rc;
        }
        const double* Us = s == 0 ? U : c->Aus;
        unsigned char* fl = c->Aflags + (size_t)s * c->L.N;
        rc = timed(c, GRMHD_K_UPDATE, [&] {
            if (fused)
                return grmhd::launch_substep(c->kind, Ps, c->Ac[s + 1], U, Us, c->Aus, c->d, dt, A[s], B[s], c->cnt,
                                             fl, c->stream);
            return grmhd::launch_update(c->kind, (const double*)c->F[0], (const double*)c->F[1],
                                        (const double*)c->F[2], Ps, c->Ac[s + 1], U, Us, c->Aus, c->d, dt,
                                        A[s], B[s], c->cnt, fl, c->stream);
        });
        if (rc)
            return rc;
    }
    return GRMHD_OK;
}

// Reverse sweep of one step whose stage primitives P^0..P^ns are Ps[] and
// whose stages' recovery flags are flags[s * N]: Ubar <- (dU^(n+1)/dU^n)^T Ubar.
int reverse_sweep(grmhd_ctx* c, const double* const* Ps, const unsigned char* flags, double* Ubar, double dt)
{
    const int ns = c->rk_order;
    const double* A = ns == 3 ? RK3A : RK2A;
    const double* B = ns == 3 ? RK3B : RK2B;
    // the last stage's recovery + RK adjoint (its output is the step's)
    int rc = timed(c, GRMHD_K_ADJ_REC, [&] {
        return grmhd::launch_adj_rec(c->kind, Ubar, Ps[ns], flags + (size_t)(ns - 1) * c->L.N, c->Unacc, c->Rb,
                                     c->d, A[ns - 1], B[ns - 1], dt, c->stream);
    });
    if (rc)
        return rc;
    for (int s = ns - 1; s >= 0; --s) {
        const bool any = c->d.act[0] || c->d.act[1] || c->d.act[2];
        if (any) {
            rc = timed(c, GRMHD_K_ADJ_FACE, [&] {
                return grmhd::launch_adj_face(c->kind, Ps[s], c->Rb, c->FB, c->d, c->stream);
            });
            if (rc)
                return rc;
            rc = timed(c, GRMHD_K_ADJ_GATHER, [&] {
                return grmhd::launch_adj_gather(Ps[s], c->FB, c->MU, c->GMU, c->d, c->stream);
            });
            if (rc)
                return rc;
        }
        // Pb^s, then the recovery + RK adjoint of stage s-1 (or the step's start)
        const unsigned char* fprev = s > 0 ? flags + (size_t)(s - 1) * c->L.N : nullptr;
        const double a = s > 0 ? A[s - 1] : 0.0, b = s > 0 ? B[s - 1] : 0.0;
        rc = timed(c, GRMHD_K_ADJ_CELL, [&] {
            return grmhd::launch_adj_cell(c->kind, Ps[s], c->MU, c->GMU, c->Rb, Ubar, c->Unacc, fprev, c->d, a,
                                          b, dt, c->stream);
        });
        if (rc)
            return rc;
    }
    return GRMHD_OK;
}

int step_adjoint(grmhd_ctx* c, const double* U, double* Ubar, double dt)
{
    const int ns = c->rk_order;
    int rc = adj_recompute(c, U, dt, ns == 3 ? RK3A : RK2A, ns == 3 ? RK3B : RK2B);
    if (rc)
        return rc;
    return reverse_sweep(c, c->Ac, c->Aflags, Ubar, dt);
}

double* tape_cache(grmhd_ctx* c, int slot, int b)
{
    const size_t cache = round_up(sizeof(double) * 9 * (size_t)c->L.sv, 256);
    return (double*)(c->ws + c->L.off_tape + (size_t)slot * c->L.tape_slot + (size_t)b * cache);
}

unsigned char* tape_flags(grmhd_ctx* c, int slot)
{
    return c->ws + c->L.off_tape + (size_t)slot * c->L.tape_slot + c->L.tape_flags;
}

// One forward step with the kernels, inputs and order of step_t<double> (so
// U and the primitives come out bitwise the same), the stage primitives
// written to the caches of tape slot `slot` instead of the rotating caches
// and the stages' recovery flags kept beside them.  The step's starting
// primitives are copied into the slot first, its final ones back to the
// current cache afterwards.
int step_record(grmhd_ctx* c, double* U, double dt, int slot)
{
    const int ns = c->rk_order;
    const double* A = ns == 3 ? RK3A : RK2A;
    const double* B = ns == 3 ? RK3B : RK2B;
    const bool fused = c->d.act[2] && !c->d.ppm && !c->d.ct;
    const size_t bytes = sizeof(double) * 9 * (size_t)c->L.sv;
    int rc = GRMHD_OK;
    if (!c->ghosts_ok[0]) {
        rc = timed(c, GRMHD_K_BC, [&] { return grmhd::launch_ghosts((double*)c->Pbuf[0], c->d, c->stream); });
        if (rc)
            return rc;
        c->ghosts_ok[0] = true;
    }
    if (hipMemcpyAsync(tape_cache(c, slot, 0), c->Pbuf[0], bytes, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
        return GRMHD_ERR_HIP;
    double* Us = (double*)c->Us;
    unsigned char* fl = tape_flags(c, slot);
    for (int s = 0; s < ns; ++s) {
        const double* Ps = tape_cache(c, slot, s);
        double* Pn = tape_cache(c, slot, s + 1);
        for (int dir = 0; dir < (fused ? 0 : 3); ++dir) {
            if (!c->d.act[dir])
                continue;
            rc = timed(c, GRMHD_K_FLUX_X + dir, [&] {
                return grmhd::launch_flux(c->kind, dir, Ps, (double*)c->F[dir], c->d, c->stream);
            });
            if (rc)
                return rc;
        }
        const double* Uin = s == 0 ? U : Us;
        double* Uo = s == ns - 1 ? U : Us;
        unsigned char* f = fl + (size_t)s * c->L.N;
        rc = timed(c, GRMHD_K_UPDATE, [&] {
            if (fused)
                return grmhd::launch_substep(c->kind, Ps, Pn, U, Uin, Uo, c->d, dt, A[s], B[s], c->cnt, f,
                                             c->stream);
            return grmhd::launch_update(c->kind, (const double*)c->F[0], (const double*)c->F[1],
                                        (const double*)c->F[2], Ps, Pn, U, Uin, Uo, c->d, dt, A[s], B[s],
                                        c->cnt, f, c->stream);
        });
        if (rc)
            return rc;
    }
    if (hipMemcpyAsync(c->Pbuf[0], tape_cache(c, slot, ns), bytes, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
        return GRMHD_ERR_HIP;
    c->ghosts_ok[0] = true;
    c->tape_dt[slot] = dt;
    return GRMHD_OK;
}

int step_adjoint_recorded(grmhd_ctx* c, int slot, double* Ubar)
{
    const double dt = c->tape_dt[slot];
    const double* Ps[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int b = 0; b <= c->rk_order; ++b)
        Ps[b] = tape_cache(c, slot, b);
    return reverse_sweep(c, Ps, tape_flags(c, slot), Ubar, dt);
}

}  // namespace

extern "C" {

size_t grmhd_workspace_bytes(const grmhd_grid* grid, const grmhd_opts* opts)
{
    if (!grid_ok(grid))
        return 0;
    const int ns = opts && opts->rk_order == 2 ? 2 : 3;
    if (!opts_fit(grid, opts))
        return 0;
    return make_layout(grid, elem_size(opts), wants_adjoint(opts), ns, tape_slots(opts), ghost_width(opts),
                       opts && opts->divergence == GRMHD_DIV_FLUXCT)
        .total;
}

}  // extern "C"

namespace {

// Validate the arguments of grmhd_init and fill the (host-side) context c,
// whose workspace is opts->workspace.
int init_ctx(grmhd_ctx* c, const grmhd_metric* metric, const grmhd_grid* grid, const grmhd_eos* eos,
             const grmhd_opts* opts)
{
    if (!grid_ok(grid))
        return GRMHD_ERR_ARG;
    if (metric->kind != GRMHD_METRIC_FLAT && metric->kind != GRMHD_METRIC_ISO_SCHW &&
        metric->kind != GRMHD_METRIC_STORED)
        return GRMHD_ERR_ARG;
    if (metric->kind == GRMHD_METRIC_STORED && opts->adjoint)
        return GRMHD_ERR_ARG;   // the adjoint kernels take the closed-form metrics
    if (metric->kind == GRMHD_METRIC_ISO_SCHW) {
        if (metric->soft != GRMHD_SOFT_SQRT && metric->soft != GRMHD_SOFT_MAX)
            return GRMHD_ERR_ARG;
        if (!(metric->M >= 0.0) || !(metric->r_min > 0.5 * metric->M))
            return GRMHD_ERR_ARG;
    }
    if (eos->kind != GRMHD_EOS_IDEAL || !(eos->gamma > 1.0) || !(eos->gamma <= 2.0))
        return GRMHD_ERR_ARG;
    if (opts->rk_order != 2 && opts->rk_order != 3)
        return GRMHD_ERR_ARG;
    if (opts->precision != GRMHD_FP64 && opts->precision != GRMHD_MIXED)
        return GRMHD_ERR_ARG;
    if (opts->c_h < 0.0 || opts->kappa < 0.0 || !(opts->rho_atm > 0.0))
        return GRMHD_ERR_ARG;
    if (opts->newton_tol < 0.0 || opts->newton_maxit < 0)
        return GRMHD_ERR_ARG;
    if (opts->recovery != GRMHD_RECOVERY_2D && opts->recovery != GRMHD_RECOVERY_1D)
        return GRMHD_ERR_ARG;
    if (opts->adjoint && opts->precision != GRMHD_FP64)
        return GRMHD_ERR_ARG;
    if (opts->tape_steps < 0 || opts->tape_steps > 4096)
        return GRMHD_ERR_ARG;
    if (!opts_fit(grid, opts))
        return GRMHD_ERR_ARG;
    Layout L = make_layout(grid, elem_size(opts), wants_adjoint(opts), opts->rk_order, tape_slots(opts),
                           ghost_width(opts), opts->divergence == GRMHD_DIV_FLUXCT);
    if (!opts->workspace || opts->workspace_bytes < L.total)
        return GRMHD_ERR_WORKSPACE;
    if (((uintptr_t)opts->workspace) % 256 != 0)
        return GRMHD_ERR_WORKSPACE;

    c->L = L;
    c->kind = metric->kind == GRMHD_METRIC_FLAT ? grmhd::FLAT
              : (metric->kind == GRMHD_METRIC_ISO_SCHW ? grmhd::ISO : grmhd::STORED);
    c->metric_ok = c->kind != grmhd::STORED;
    c->grid = *grid;
    c->rk_order = opts->rk_order;
    c->timing = opts->timing;
    c->mixed = opts->precision == GRMHD_MIXED;
    Dev& d = c->d;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = grid->n[a];
        d.g[a] = L.g[a];
        d.act[a] = grid->n[a] > 1;
        d.bc[a] = grid->bc[a] == GRMHD_BC_PERIODIC ? 0 : 1;
        d.lo[a] = grid->lo[a];
        d.dx[a] = (grid->hi[a] - grid->lo[a]) / grid->n[a];
        d.idx[a] = 1.0 / d.dx[a];
        d.nf[a] = L.nf[a];
    }
    d.px = L.px;
    d.py = L.py;
    d.pz = L.pz;
    d.sv = L.sv;
    d.N = L.N;
    d.M = metric->M;
    d.rmin = metric->r_min;
    d.rmin2 = metric->r_min * metric->r_min;
    d.soft = metric->soft == GRMHD_SOFT_SQRT ? 0 : 1;
    d.gamma = eos->gamma;
    d.gk = (eos->gamma - 1.0) / eos->gamma;
    d.gfac = eos->gamma / (eos->gamma - 1.0);
    d.c_h = opts->c_h > 0.0 ? opts->c_h : 1.0;
    d.ic_h = 1.0 / d.c_h;
    d.c_h2 = d.c_h * d.c_h;
    d.kappa = opts->kappa;
    d.rho_atm = opts->rho_atm;
    d.p_atm = opts->p_atm >= 0.0 ? opts->p_atm : eos->K * std::pow(opts->rho_atm, eos->gamma);
    d.tol = opts->newton_tol > 0.0 ? opts->newton_tol : 1e-12;
    d.maxit = opts->newton_maxit > 0 ? opts->newton_maxit : 50;
    d.c2p1d = opts->recovery == GRMHD_RECOVERY_1D;
    d.ppm = opts->reconstruction == GRMHD_RECON_PPM;
    d.ct = opts->divergence == GRMHD_DIV_FLUXCT;
    // Nontemporal accesses for the once-touched arrays pay where a substep's
    // arrays are larger than the 256 MB Infinity Cache (192^3: the update 8 %
    // faster; 128^3: the step 8 %; 96^3: 4 %) and cost where they would fit
    // in it (64^3: a step 7 % slower), measured: on from 2^19 cells (80^3)
    d.nt = d.N >= (1LL << 19);

    c->ws = (unsigned char*)opts->workspace;
    c->cnt = (unsigned long long*)(c->ws + L.off_cnt);
    for (int b = 0; b < 3; ++b)
        c->Pbuf[b] = (void*)(c->ws + L.off_pc[b]);
    c->Us = (void*)(c->ws + L.off_us);
    for (int a = 0; a < 3; ++a)
        c->F[a] = L.nf[a] ? (void*)(c->ws + L.off_f[a]) : nullptr;
    for (int p = 0; p < 3; ++p)
        c->W[p] = L.ct ? (void*)(c->ws + L.off_w[p]) : nullptr;
    if (L.adj) {
        c->adj = true;
        for (int b = 0; b <= c->rk_order; ++b)
            c->Ac[b] = (double*)(c->ws + L.off_ac[b]);
        c->Aflags = c->ws + L.off_aflags;
        c->Aus = (double*)(c->ws + L.off_aus);
        c->Unacc = (double*)(c->ws + L.off_unacc);
        c->Rb = (double*)(c->ws + L.off_rb);
        c->Pb = (double*)(c->ws + L.off_pb);
        c->MU = (double*)(c->ws + L.off_mu);
        for (int a = 0; a < 3; ++a)
            c->FB[a] = L.nf[a] ? (double*)(c->ws + L.off_fb[a]) : nullptr;
        for (int a = 0; a < 3; ++a)
            c->GMU[a] = L.nf[a] ? (double*)(c->ws + L.off_gmu[a]) : nullptr;
        c->tape_dt.assign((size_t)L.tape, std::nan(""));
    }
    return GRMHD_OK;
}

}  // namespace

extern "C" {

int grmhd_init(grmhd_ctx** out, const grmhd_metric* metric, const grmhd_grid* grid,
               const grmhd_eos* eos, const grmhd_opts* opts)
{
    if (!out || !metric || !grid || !eos || !opts)
        return GRMHD_ERR_ARG;
    *out = nullptr;
    grmhd_ctx* c = new (std::nothrow) grmhd_ctx();
    if (!c)
        return GRMHD_ERR_ARG;
    const int rc = init_ctx(c, metric, grid, eos, opts);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return GRMHD_OK;
}

int grmhd_set_stream(grmhd_ctx* c, void* stream)
{
    if (!c)
        return GRMHD_ERR_ARG;
    c->stream = (hipStream_t)stream;
    return GRMHD_OK;
}

int grmhd_cons(grmhd_ctx* c, const double* P, double* U)
{
    if (!c || !P || !U)
        return GRMHD_ERR_ARG;
    if (!c->metric_ok)
        return GRMHD_ERR_STATE;
    return c->mixed ? cons_t<float>(c, P, U) : cons_t<double>(c, P, U);
}

int grmhd_prim(grmhd_ctx* c, const double* U, double* P)
{
    if (!c || !U || !P)
        return GRMHD_ERR_ARG;
    if (!c->metric_ok)
        return GRMHD_ERR_STATE;
    return c->mixed ? prim_t<float>(c, U, P) : prim_t<double>(c, U, P);
}

size_t grmhd_metric_bytes(const grmhd_grid* grid)
{
    if (!grid_ok(grid))
        return 0;
    return metric_layout(grid, nullptr);
}

int grmhd_set_metric(grmhd_ctx* c, const double* alpha, const double* psi4, void* buf, size_t buf_bytes)
{
    if (!c || !alpha || !psi4 || !buf)
        return GRMHD_ERR_ARG;
    if (c->kind != grmhd::STORED)
        return GRMHD_ERR_ARG;
    size_t off_mf[3];
    if (buf_bytes < metric_layout(&c->grid, off_mf) || ((uintptr_t)buf) % 256 != 0)
        return GRMHD_ERR_WORKSPACE;
    unsigned char* b = (unsigned char*)buf;
    c->d.mc = (const double*)b;
    double* mf[3];
    for (int d = 0; d < 3; ++d) {
        mf[d] = c->d.nf[d] ? (double*)(b + off_mf[d]) : nullptr;
        c->d.mf[d] = mf[d];
    }
    if (grmhd::launch_metric(alpha, psi4, (double*)b, mf, c->d, c->stream) != hipSuccess)
        return GRMHD_ERR_HIP;
    c->metric_ok = true;
    return GRMHD_OK;
}

int grmhd_rhs(grmhd_ctx* c, const double* P, double* R)
{
    if (!c || !P || !R)
        return GRMHD_ERR_ARG;
    if (!c->metric_ok)
        return GRMHD_ERR_STATE;
    return c->mixed ? rhs_t<float>(c, P, R) : rhs_t<double>(c, P, R);
}

}  // extern "C"

namespace {

// Scratch of grmhd_rhs_noalloc: one array per GPU (its copy of this
// file-scope device array), its address taken once per device on the first
// call there.  In host code `noalloc_scratch` names a host-side stand-in, not
// device memory: only the address from hipGetSymbolAddress is used.
__device__ __align__(256) unsigned char noalloc_scratch[GRMHD_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch array (nullptr on failure).
void* noalloc_base()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p)
            return nullptr;
        noalloc_ptr[dev] = p;
    }
    return noalloc_ptr[dev];
}

}  // namespace

extern "C" {

int grmhd_rhs_noalloc(const grmhd_metric* metric, const grmhd_grid* grid, const grmhd_eos* eos,
                      const grmhd_opts* opts, const double* P, double* R, void* stream)
{
    if (!metric || !grid || !eos || !opts || !P || !R)
        return GRMHD_ERR_ARG;
    if (metric->kind == GRMHD_METRIC_STORED)
        return GRMHD_ERR_ARG;   // its metric buffer would be a second allocation
    grmhd_opts o = *opts;
    o.timing = 0;
    o.adjoint = 0;
    o.tape_steps = 0;
    if (!grid_ok(grid) || !opts_fit(grid, &o))
        return GRMHD_ERR_ARG;
    const size_t need = grmhd_workspace_bytes(grid, &o);
    if (need == 0)
        return GRMHD_ERR_ARG;
    if (need > GRMHD_NOALLOC_SCRATCH_BYTES)
        return GRMHD_ERR_WORKSPACE;
    void* base = noalloc_base();
    if (!base)
        return GRMHD_ERR_HIP;
    o.workspace = base;
    o.workspace_bytes = GRMHD_NOALLOC_SCRATCH_BYTES;
    // a context on the stack (no timing, no adjoint: nothing of it allocates)
    grmhd_ctx c;
    int rc = init_ctx(&c, metric, grid, eos, &o);
    if (rc)
        return rc;
    c.stream = (hipStream_t)stream;
    return c.mixed ? rhs_t<float>(&c, P, R) : rhs_t<double>(&c, P, R);
}

int grmhd_step(grmhd_ctx* c, double* U, double dt)
{
    if (!c || !U || !std::isfinite(dt))
        return GRMHD_ERR_ARG;
    if (!c->cache_valid)
        return GRMHD_ERR_STATE;
    return c->mixed ? step_t<float>(c, U, dt) : step_t<double>(c, U, dt);
}

int grmhd_step_adjoint(grmhd_ctx* c, const double* U, double* Ubar, double dt)
{
    if (!c || !U || !Ubar || !std::isfinite(dt))
        return GRMHD_ERR_ARG;
    if (!c->adj)
        return GRMHD_ERR_NO_ADJOINT;
    int rc = adj_prepare(c);
    if (rc)
        return rc;
    return step_adjoint(c, U, Ubar, dt);
}

int grmhd_step_record(grmhd_ctx* c, double* U, double dt, int slot)
{
    if (!c || !U || !std::isfinite(dt))
        return GRMHD_ERR_ARG;
    if (!c->adj)
        return GRMHD_ERR_NO_ADJOINT;
    if (slot < 0 || slot >= c->L.tape)
        return GRMHD_ERR_ARG;
    if (!c->cache_valid)
        return GRMHD_ERR_STATE;
    int rc = adj_prepare(c);
    if (rc)
        return rc;
    return step_record(c, U, dt, slot);
}

int grmhd_step_adjoint_recorded(grmhd_ctx* c, int slot, double* Ubar)
{
    if (!c || !Ubar)
        return GRMHD_ERR_ARG;
    if (!c->adj)
        return GRMHD_ERR_NO_ADJOINT;
    if (slot < 0 || slot >= c->L.tape)
        return GRMHD_ERR_ARG;
    if (!std::isfinite(c->tape_dt[slot]))
        return GRMHD_ERR_STATE;
    int rc = adj_prepare(c);
    if (rc)
        return rc;
    return step_adjoint_recorded(c, slot, Ubar);
}

int grmhd_cons_adjoint(grmhd_ctx* c, const double* P, const double* Ubar, double* Pbar)
{
    if (!c || !P || !Ubar || !Pbar)
        return GRMHD_ERR_ARG;
    if (!c->adj)
        return GRMHD_ERR_NO_ADJOINT;
    return timed(c, GRMHD_K_ADJ_REC, [&] { return grmhd::launch_adj_cons(c->kind, P, Ubar, Pbar, c->d, c->stream); });
}

int grmhd_prim_adjoint(grmhd_ctx* c, const double* U, const double* Pbar, double* Ubar)
{
    if (!c || !U || !Pbar || !Ubar)
        return GRMHD_ERR_ARG;
    if (!c->adj)
        return GRMHD_ERR_NO_ADJOINT;
    int rc = adj_prepare(c);
    if (rc)
        return rc;
    rc = timed(c, GRMHD_K_PRIM, [&] {
        return grmhd::launch_prim(c->kind, U, c->Pb, c->Ac[0], c->d, c->cnt, c->stream);
    });
    if (rc)
        return rc;
    return timed(c, GRMHD_K_ADJ_REC, [&] {
        return grmhd::launch_adj_final(c->kind, nullptr, Pbar, c->Ac[0], nullptr, Ubar, c->d, c->stream);
    });
}

int grmhd_status(grmhd_ctx* c, grmhd_stats* st, int reset)
{
    if (!c || !st)
        return GRMHD_ERR_ARG;
    std::vector<unsigned long long> slots(grmhd::CNT_WORDS * grmhd::CNT_SLOTS, 0ull);
    if (c->prepared) {
        if (hipMemcpyAsync(slots.data(), c->cnt, grmhd::CNT_BYTES, hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    }
    unsigned long long h[grmhd::CNT_WORDS] = {};
    for (int s = 0; s < grmhd::CNT_SLOTS; ++s) {
        const unsigned long long* w = &slots[(size_t)s * grmhd::CNT_WORDS];
        for (int i = 0; i < grmhd::CNT_WORDS; ++i)
            h[i] = i == grmhd::CNT_MAXIT ? (w[i] > h[i] ? w[i] : h[i]) : h[i] + w[i];
    }
    st->c2p_fail = (long long)h[grmhd::CNT_FAIL];
    st->atm_hits = (long long)h[grmhd::CNT_ATM];
    st->p_floor_hits = (long long)h[grmhd::CNT_PFLOOR];
    st->fallback_1d = (long long)h[grmhd::CNT_FALLBACK];
    st->max_newton_it = (int)h[grmhd::CNT_MAXIT];
    if (reset && c->prepared) {
        if (grmhd::launch_zero_counters(c->cnt, c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    }
    return GRMHD_OK;
}

int grmhd_timing(grmhd_ctx* c, double* ms, long long* launches, int reset)
{
    if (!c)
        return GRMHD_ERR_ARG;
    if (!c->pending.empty()) {
        if (hipStreamSynchronize(c->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
        for (auto& t : c->pending) {
            float e = 0.0f;
            if (hipEventElapsedTime(&e, t.start, t.stop) != hipSuccess)
                return GRMHD_ERR_HIP;
            c->ms[t.kind] += e;
            c->launches[t.kind] += 1;
            c->spare.push_back(t.start);
            c->spare.push_back(t.stop);
        }
        c->pending.clear();
    }
    for (int k = 0; k < GRMHD_K_COUNT; ++k) {
        if (ms)
            ms[k] = c->ms[k];
        if (launches)
            launches[k] = c->launches[k];
        if (reset) {
            c->ms[k] = 0.0;
            c->launches[k] = 0;
        }
    }
    return GRMHD_OK;
}

int grmhd_free(grmhd_ctx* c)
{
    if (!c)
        return GRMHD_ERR_ARG;
    for (auto& t : c->pending) {
        hipEventDestroy(t.start);
        hipEventDestroy(t.stop);
    }
    for (auto e : c->spare)
        hipEventDestroy(e);
    delete c;
    return GRMHD_OK;
}

int grmhd_device_arith(const double* x, const double* y, double* out, long long n, void* stream)
{
    if (!x || !y || !out || n < 0 || n > (1LL << 38))
        return GRMHD_ERR_ARG;
    return grmhd::launch_arith(x, y, out, n, (hipStream_t)stream) == hipSuccess ? GRMHD_OK : GRMHD_ERR_HIP;
}

const char* grmhd_strerror(int code)
{
    switch (code) {
    case GRMHD_OK:
        return "success";
    case GRMHD_ERR_ARG:
        return "invalid argument";
    case GRMHD_ERR_WORKSPACE:
        return "workspace missing, misaligned or smaller than grmhd_workspace_bytes()";
    case GRMHD_ERR_HIP:
        return "HIP runtime or kernel launch error";
    case GRMHD_ERR_STATE:
        return "primitive cache not initialised: call grmhd_cons or grmhd_prim first";
    case GRMHD_ERR_NO_ADJOINT:
        return "adjoint call on a context created without opts.adjoint (FP64 only)";
    default:
        return "unknown error";
    }
}

}  // extern "C"
