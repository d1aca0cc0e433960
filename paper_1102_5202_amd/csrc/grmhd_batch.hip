// grmhd_batch.hip -- C ABI of the batched ensemble of 1D problems
// (include/grmhd.h, grmhd_batch_*).  Host code: workspace layout, the
// per-problem records, launch-shape selection; the kernels are in
// grmhd_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <new>
#include <numeric>
#include <vector>

#include "grmhd.h"
#include "grmhd_internal.h"

using grmhd::BatchProb;
using grmhd::Dev;

namespace {

constexpr size_t LDS_LIMIT = 160 * 1024;
// Split launch: at most this many workgroups (and split parts beyond one
// per problem), each part at least this many cells.
constexpr int SPLIT_MAX_PARTS = 4096;
constexpr int SPLIT_MIN_CELLS = 64;
// Placement of the primitive rows (grmhd_batch_set_shape's lds argument).
enum { PLACE_HBM = 0, PLACE_LDS = 1, PLACE_SPLIT = 2 };

size_t up(size_t x, size_t a)
{
    return (x + a - 1) / a * a;
}

struct BatchLayout {
    long long ncell = 0, nrow = 0;   // cells in all; elements of all ghosted rows
    int nmax = 0;
    size_t off_cnt, off_probs, off_order, off_probs_t, off_prow, off_pnext, off_us, off_prow_t, off_u_t;
    size_t off_parts, off_flags, off_runs, off_span, total;
};

bool desc_ok(const grmhd_batch_desc* d)
{
    if (!d || d->nprob < 1 || d->nprob > (1 << 20) || !d->n || !d->lo || !d->hi || !d->dt || !d->steps)
        return false;
    if (d->bc != GRMHD_BC_PERIODIC && d->bc != GRMHD_BC_OUTFLOW)
        return false;
    long long cells = 0;
    for (int b = 0; b < d->nprob; ++b) {
        if (d->n[b] < 2 || d->n[b] > (1 << 24) || d->steps[b] < 0)
            return false;
        cells += d->n[b];
        if (!(d->hi[b] > d->lo[b]) || !std::isfinite(d->lo[b]) || !std::isfinite(d->hi[b]))
            return false;
        if (!(d->dt[b] >= 0.0) || !std::isfinite(d->dt[b]))
            return false;
    }
    return cells <= (1LL << 38);   // launches stay inside 2^31 - 1 workgroups
}

BatchLayout batch_layout(const grmhd_batch_desc* d, size_t esize)
{
    BatchLayout L;
    for (int b = 0; b < d->nprob; ++b) {
        L.ncell += d->n[b];
        L.nrow += 9LL * (d->n[b] + 4);
        L.nmax = std::max(L.nmax, d->n[b]);
    }
    size_t off = 0;
    L.off_cnt = off;
    off = up(off + grmhd::CNT_BYTES, 256);
    L.off_probs = off;
    off = up(off + sizeof(BatchProb) * d->nprob, 256);
    L.off_order = off;
    off = up(off + sizeof(int) * d->nprob, 256);
    L.off_probs_t = off;                 // the records used by tuning runs
    off = up(off + sizeof(BatchProb) * d->nprob, 256);
    L.off_prow = off;
    off = up(off + esize * L.nrow, 256);
    L.off_pnext = off;
    off = up(off + esize * L.nrow, 256);
    L.off_us = off;
    off = up(off + esize * 9 * L.ncell, 256);
    L.off_prow_t = off;                  // rows and state of tuning runs
    off = up(off + esize * L.nrow, 256);
    L.off_u_t = off;
    off = up(off + sizeof(double) * 9 * L.ncell, 256);
    // the split launch: its parts (at most one per problem plus the extra
    // parts of split problems), their flags and the workgroups' runs of parts
    const size_t maxparts = (size_t)d->nprob + SPLIT_MAX_PARTS;
    L.off_parts = off;
    off = up(off + sizeof(grmhd::BatchPart) * maxparts, 256);
    L.off_flags = off;
    off = up(off + sizeof(int) * maxparts, 256);
    L.off_runs = off;
    off = up(off + sizeof(int2) * SPLIT_MAX_PARTS, 256);
    L.off_span = off;                    // start and end of every workgroup of the last launch
    off = up(off + 2 * sizeof(unsigned long long) * std::max(d->nprob, SPLIT_MAX_PARTS), 256);
    L.total = off;
    return L;
}

size_t esize_of(const grmhd_opts* o)
{
    return o && o->precision == GRMHD_MIXED ? sizeof(float) : sizeof(double);
}

}  // namespace

struct grmhd_batch {
    Dev d;
    int nprob = 0, rk_order = 3;
    bool mixed = false;
    BatchLayout L;
    unsigned char* ws = nullptr;
    hipStream_t stream = nullptr;
    std::vector<BatchProb> probs;   // host copy (done = 0)
    std::vector<int> order;          // problems by decreasing work, one per workgroup
    bool uploaded = false;
    bool cache_valid = false;
    int shape = 1;                   // index into BATCH_THREADS
    int lds = 0;
    size_t lds_bytes = 0;
    bool lds_ok = false;   // rows fit in LDS and their LDS size is allowed
    std::vector<grmhd::BatchPart> parts;   // the split launch (empty: not available)
    std::vector<int2> runs;                 // its workgroups: runs of consecutive parts
    unsigned long long* cnt = nullptr;
    // the last evolve launch: its workgroups and its shape (for the busy fraction)
    int last_wgs = 0, last_shape = 0, last_lds = 0;
};

namespace {

template <typename T>
T* at(grmhd_batch* b, size_t off)
{
    return (T*)(b->ws + off);
}

// First use: the problem order and zeroed counters; with reset (or on first
// use) the problem records with their step counts at zero.
int upload(grmhd_batch* b, bool reset)
{
    if (reset || !b->uploaded) {
        if (hipMemcpyAsync(at<BatchProb>(b, b->L.off_probs), b->probs.data(), sizeof(BatchProb) * b->nprob,
                           hipMemcpyHostToDevice, b->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    }
    if (!b->uploaded) {
        if (hipMemcpyAsync(at<int>(b, b->L.off_order), b->order.data(), sizeof(int) * b->nprob,
                           hipMemcpyHostToDevice, b->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
        if (!b->parts.empty() &&
            (hipMemcpyAsync(at<grmhd::BatchPart>(b, b->L.off_parts), b->parts.data(),
                            sizeof(grmhd::BatchPart) * b->parts.size(), hipMemcpyHostToDevice,
                            b->stream) != hipSuccess ||
             hipMemcpyAsync(at<int2>(b, b->L.off_runs), b->runs.data(), sizeof(int2) * b->runs.size(),
                            hipMemcpyHostToDevice, b->stream) != hipSuccess))
            return GRMHD_ERR_HIP;
        if (grmhd::launch_zero_counters(b->cnt, b->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
        b->uploaded = true;
    }
    return GRMHD_OK;
}

template <typename T>
int evolve_t(grmhd_batch* b, double* U, int max_steps, size_t off_probs, size_t off_prow)
{
    unsigned long long* span = at<unsigned long long>(b, b->L.off_span);
    b->last_shape = b->shape;
    b->last_lds = b->lds;
    if (b->lds == PLACE_SPLIT) {
        b->last_wgs = (int)b->runs.size();
        const hipError_t e = grmhd::launch_batch_split<T>(
            at<BatchProb>(b, off_probs), at<grmhd::BatchPart>(b, b->L.off_parts), (int)b->parts.size(),
            at<int2>(b, b->L.off_runs), (int)b->runs.size(), at<int>(b, b->L.off_flags), U, at<T>(b, b->L.off_us),
            at<T>(b, off_prow), at<T>(b, b->L.off_pnext), b->d, b->rk_order, max_steps, b->cnt, span, b->stream);
        return e == hipSuccess ? GRMHD_OK : GRMHD_ERR_HIP;
    }
    b->last_wgs = b->nprob;
    const hipError_t e = grmhd::launch_batch_evolve<T>(
        b->shape, b->lds, b->lds_bytes, at<BatchProb>(b, off_probs), at<int>(b, b->L.off_order), b->nprob, U,
        at<T>(b, b->L.off_us), at<T>(b, off_prow), at<T>(b, b->L.off_pnext), b->d, b->rk_order, max_steps, b->cnt,
        span, b->stream);
    return e == hipSuccess ? GRMHD_OK : GRMHD_ERR_HIP;
}

int evolve(grmhd_batch* b, double* U, int max_steps, size_t off_probs, size_t off_prow)
{
    return b->mixed ? evolve_t<float>(b, U, max_steps, off_probs, off_prow)
                    : evolve_t<double>(b, U, max_steps, off_probs, off_prow);
}

// The split launch's plan, for cap resident workgroups: with w the target
// work (cells x steps) of a workgroup, every problem of more work than w is
// split into ceil(work / w) parts (at most one per SPLIT_MIN_CELLS cells),
// each with a workgroup of its own; the smaller problems, largest first, are
// packed whole into shared workgroups of at most w work each (next fit), run
// one after another.  w starts at the mean work per workgroup and grows until
// the workgroups fit in cap.  A split problem's parts are consecutive; with
// periodic ends its first and last part are neighbours.  Returns false when
// no plan fits.
bool split_plan(const std::vector<BatchProb>& probs, int bc, int cap, std::vector<grmhd::BatchPart>& parts,
                std::vector<int2>& runs)
{
    parts.clear();
    runs.clear();
    const int np = (int)probs.size();
    cap = std::min(cap, SPLIT_MAX_PARTS);
    if (cap < 1)
        return false;
    std::vector<double> work(np);
    double total = 0.0;
    for (int b = 0; b < np; ++b) {
        work[b] = (double)probs[b].n * std::max(probs[b].steps, 1);
        total += work[b];
    }
    std::vector<int> bysize(np);
    std::iota(bysize.begin(), bysize.end(), 0);
    std::stable_sort(bysize.begin(), bysize.end(), [&](int x, int y) { return work[x] > work[y]; });
    double w = total / cap;
    std::vector<int> g(np, 0);   // parts of a split problem; 0: packed whole
    bool fits = false;
    for (int tries = 0; tries < 2000 && !fits; ++tries, w *= 1.02) {
        long long nwg = 0;
        double bin = -1.0;   // work in the open shared workgroup (< 0: none)
        for (int b : bysize) {
            if (work[b] > w) {
                g[b] = std::min(std::max(1, probs[b].n / SPLIT_MIN_CELLS), (int)std::ceil(work[b] / w));
                nwg += g[b];
            } else {
                g[b] = 0;
                if (bin < 0.0 || bin + work[b] > w) {
                    ++nwg;
                    bin = 0.0;
                }
                bin += work[b];
            }
        }
        fits = nwg <= cap;
    }
    if (!fits)
        return false;
    double bin = -1.0;
    for (int b : bysize) {
        const int n = probs[b].n, first = (int)parts.size();
        if (g[b] > 0) {
            for (int q = 0; q < g[b]; ++q) {
                grmhd::BatchPart pt{};
                pt.b = b;
                pt.c0 = (int)((long long)n * q / g[b]);
                pt.c1 = (int)((long long)n * (q + 1) / g[b]);
                const bool wrap = bc == 0 && g[b] > 1;
                pt.left = q > 0 ? first + q - 1 : (wrap ? first + g[b] - 1 : -1);
                pt.right = q + 1 < g[b] ? first + q + 1 : (wrap ? first : -1);
                pt.first = first;
                pt.count = g[b];
                parts.push_back(pt);
                runs.push_back(make_int2(first + q, 1));
            }
            continue;
        }
        grmhd::BatchPart pt{};
        pt.b = b;
        pt.c0 = 0;
        pt.c1 = n;
        pt.left = pt.right = -1;
        pt.first = first;
        pt.count = 1;
        parts.push_back(pt);
        if (bin < 0.0 || bin + work[b] > w) {
            runs.push_back(make_int2(first, 0));
            bin = 0.0;
        }
        runs.back().y += 1;
        bin += work[b];
    }
    return (int)runs.size() <= cap;
}

}  // namespace

extern "C" {

size_t grmhd_batch_workspace_bytes(const grmhd_batch_desc* desc, const grmhd_opts* opts)
{
    if (!desc_ok(desc))
        return 0;
    return batch_layout(desc, esize_of(opts)).total;
}

int grmhd_batch_init(grmhd_batch** out, const grmhd_batch_desc* desc, const grmhd_eos* eos, const grmhd_opts* opts)
{
    if (!out || !desc || !eos || !opts)
        return GRMHD_ERR_ARG;
    *out = nullptr;
    if (!desc_ok(desc))
        return GRMHD_ERR_ARG;
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
    if (opts->reconstruction != GRMHD_RECON_MC)
        return GRMHD_ERR_ARG;   // the batched rows carry two ghost cells: MC only
    if (opts->divergence != GRMHD_DIV_CLEANING)
        return GRMHD_ERR_ARG;
    const size_t es = esize_of(opts);
    BatchLayout L = batch_layout(desc, es);
    if (!opts->workspace || opts->workspace_bytes < L.total || ((uintptr_t)opts->workspace) % 256 != 0)
        return GRMHD_ERR_WORKSPACE;
    grmhd_batch* b = new (std::nothrow) grmhd_batch();
    if (!b)
        return GRMHD_ERR_ARG;
    b->L = L;
    b->nprob = desc->nprob;
    b->rk_order = opts->rk_order;
    b->mixed = opts->precision == GRMHD_MIXED;
    b->ws = (unsigned char*)opts->workspace;
    b->cnt = at<unsigned long long>(b, L.off_cnt);
    Dev& d = b->d;
    d = Dev{};
    d.bc[0] = desc->bc == GRMHD_BC_PERIODIC ? 0 : 1;
    d.act[0] = 1;
    d.M = 0.0;
    d.rmin = d.rmin2 = 1.0;
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
    b->probs.resize(b->nprob);
    long long off = 0, poff = 0;
    for (int i = 0; i < b->nprob; ++i) {
        BatchProb& p = b->probs[i];
        p = BatchProb{};
        p.n = desc->n[i];
        p.steps = desc->steps[i];
        p.done = 0;
        p.off = off;
        p.poff = poff;
        p.lo = desc->lo[i];
        p.dx = (desc->hi[i] - desc->lo[i]) / desc->n[i];
        p.idx = 1.0 / p.dx;
        p.dt = desc->dt[i];
        off += p.n;
        poff += 9LL * (p.n + 4);
    }
    // longest-processing-time order: the largest problems start first
    b->order.resize(b->nprob);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (double)b->probs[x].n * b->probs[x].steps > (double)b->probs[y].n * b->probs[y].steps;
    });
    b->lds_bytes = es * 9 * (size_t)(L.nmax + 4);
    b->shape = 1;
    // rows in LDS need their dynamic LDS size allowed once, here, outside any
    // graph capture; where that fails (no device yet) the rows stay in HBM
    if (b->lds_bytes <= LDS_LIMIT) {
        const hipError_t e = b->mixed ? grmhd::allow_batch_lds<float>(b->lds_bytes)
                                      : grmhd::allow_batch_lds<double>(b->lds_bytes);
        if (e != hipSuccess)
            (void)hipGetLastError();   // clear it: launches check the last error
        b->lds_ok = e == hipSuccess;
    }
    b->lds = b->lds_ok ? PLACE_LDS : PLACE_HBM;
    // the split launch needs every part resident at once: its occupancy on
    // this device (where that cannot be asked, there is no split launch)
    int dev = -1, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
        const int occ = b->mixed ? grmhd::batch_split_occupancy<float>() : grmhd::batch_split_occupancy<double>();
        if (occ > 0 && cus > 0 &&
            !split_plan(b->probs, desc->bc == GRMHD_BC_PERIODIC ? 0 : 1, occ * cus, b->parts, b->runs)) {
            b->parts.clear();
            b->runs.clear();
        }
    }
    (void)hipGetLastError();
    *out = b;
    return GRMHD_OK;
}

int grmhd_batch_set_stream(grmhd_batch* b, void* stream)
{
    if (!b)
        return GRMHD_ERR_ARG;
    b->stream = (hipStream_t)stream;
    return GRMHD_OK;
}

int grmhd_batch_cons(grmhd_batch* b, const double* P, double* U)
{
    if (!b || !P)
        return GRMHD_ERR_ARG;
    int rc = upload(b, true);
    if (rc)
        return rc;
    hipError_t e = b->mixed
                       ? grmhd::launch_batch_cons<float>(at<BatchProb>(b, b->L.off_probs), b->nprob, b->L.ncell, P,
                                                         U, at<float>(b, b->L.off_prow), b->d, b->stream)
                       : grmhd::launch_batch_cons<double>(at<BatchProb>(b, b->L.off_probs), b->nprob, b->L.ncell,
                                                          P, U, at<double>(b, b->L.off_prow), b->d, b->stream);
    if (e != hipSuccess)
        return GRMHD_ERR_HIP;
    b->cache_valid = true;
    return GRMHD_OK;
}

int grmhd_batch_evolve(grmhd_batch* b, double* U, int max_steps)
{
    if (!b || !U || max_steps < 0)
        return GRMHD_ERR_ARG;
    if (!b->cache_valid)
        return GRMHD_ERR_STATE;
    return evolve(b, U, max_steps, b->L.off_probs, b->L.off_prow);
}

int grmhd_batch_prim(grmhd_batch* b, const double* U, double* P)
{
    if (!b || !U || !P)
        return GRMHD_ERR_ARG;
    int rc = upload(b, false);
    if (rc)
        return rc;
    hipError_t e = b->mixed ? grmhd::launch_batch_prim<float>(at<BatchProb>(b, b->L.off_probs), b->nprob,
                                                               b->L.ncell, U, P, at<float>(b, b->L.off_prow), b->d,
                                                               b->cnt, b->stream)
                            : grmhd::launch_batch_prim<double>(at<BatchProb>(b, b->L.off_probs), b->nprob,
                                                                b->L.ncell, U, P, at<double>(b, b->L.off_prow), b->d,
                                                                b->cnt, b->stream);
    if (e != hipSuccess)
        return GRMHD_ERR_HIP;
    b->cache_valid = true;
    return GRMHD_OK;
}

int grmhd_batch_tune(grmhd_batch* b, const double* U, int trial_steps, int* threads, int* lds)
{
    if (!b || !U || trial_steps < 1)
        return GRMHD_ERR_ARG;
    if (!b->cache_valid)
        return GRMHD_ERR_STATE;
    const size_t es = b->mixed ? sizeof(float) : sizeof(double);
    double* Ut = at<double>(b, b->L.off_u_t);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return GRMHD_ERR_HIP;
    // The trial records: every problem keeps its step count so far and gets a
    // share of trial_steps in proportion to the steps it has left, so that
    // the problems' work in a trial is in the same proportion as in the run
    // (a shape that balances uneven problems is judged on uneven problems).
    std::vector<BatchProb> tp(b->nprob);
    if (hipMemcpyAsync(tp.data(), at<BatchProb>(b, b->L.off_probs), sizeof(BatchProb) * b->nprob,
                       hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return GRMHD_ERR_HIP;
    }
    int left_max = 0;
    for (const BatchProb& p : tp)
        left_max = std::max(left_max, p.steps - p.done);
    for (BatchProb& p : tp) {
        const int left = p.steps - p.done;
        const int share = left_max > 0 ? (int)std::ceil((double)left * trial_steps / left_max) : 0;
        p.steps = p.done + std::min(left, share);
    }
    const int keep_shape = b->shape, keep_lds = b->lds;
    float best = -1.0f;
    int best_shape = keep_shape, best_lds = keep_lds, rc = GRMHD_OK;
    for (int l = PLACE_HBM; l <= PLACE_SPLIT && rc == GRMHD_OK; ++l) {
        if ((l == PLACE_LDS && !b->lds_ok) || (l == PLACE_SPLIT && b->parts.empty()))
            continue;
        for (int s = 0; s < grmhd::BATCH_SHAPES && rc == GRMHD_OK; ++s) {
            if (l == PLACE_SPLIT && grmhd::BATCH_THREADS[s] != grmhd::BATCH_SPLIT_THREADS)
                continue;
            // fresh copies of the state for every candidate
            if (hipMemcpyAsync(Ut, U, sizeof(double) * 9 * b->L.ncell, hipMemcpyDeviceToDevice, b->stream) !=
                    hipSuccess ||
                hipMemcpyAsync(b->ws + b->L.off_prow_t, b->ws + b->L.off_prow, es * b->L.nrow,
                               hipMemcpyDeviceToDevice, b->stream) != hipSuccess ||
                hipMemcpyAsync(b->ws + b->L.off_probs_t, tp.data(), sizeof(BatchProb) * b->nprob,
                               hipMemcpyHostToDevice, b->stream) != hipSuccess) {
                rc = GRMHD_ERR_HIP;
                break;
            }
            b->shape = s;
            b->lds = l;
            if (hipEventRecord(e0, b->stream) != hipSuccess) {
                rc = GRMHD_ERR_HIP;
                break;
            }
            rc = evolve(b, Ut, INT_MAX, b->L.off_probs_t, b->L.off_prow_t);
            if (rc) {
                if (l == PLACE_LDS) {   // an LDS size the runtime refuses: not a candidate
                    (void)hipGetLastError();
                    rc = GRMHD_OK;
                    continue;
                }
                break;
            }
            float ms = 0.0f;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = GRMHD_ERR_HIP;
                break;
            }
            if (best < 0.0f || ms < best) {
                best = ms;
                best_shape = s;
                best_lds = l;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->shape = rc == GRMHD_OK ? best_shape : keep_shape;
    b->lds = rc == GRMHD_OK ? best_lds : keep_lds;
    if (threads)
        *threads = grmhd::BATCH_THREADS[b->shape];
    if (lds)
        *lds = b->lds;
    return rc;
}

int grmhd_batch_set_shape(grmhd_batch* b, int threads, int lds)
{
    if (!b)
        return GRMHD_ERR_ARG;
    int shape = -1;
    for (int s = 0; s < grmhd::BATCH_SHAPES; ++s)
        if (grmhd::BATCH_THREADS[s] == threads)
            shape = s;
    if (shape < 0 || lds < PLACE_HBM || lds > PLACE_SPLIT || (lds == PLACE_LDS && !b->lds_ok))
        return GRMHD_ERR_ARG;
    if (lds == PLACE_SPLIT && (b->parts.empty() || threads != grmhd::BATCH_SPLIT_THREADS))
        return GRMHD_ERR_ARG;
    b->shape = shape;
    b->lds = lds;
    return GRMHD_OK;
}

int grmhd_batch_status(grmhd_batch* b, grmhd_stats* st, int reset)
{
    if (!b || !st)
        return GRMHD_ERR_ARG;
    std::vector<unsigned long long> slots(grmhd::CNT_WORDS * grmhd::CNT_SLOTS, 0ull);
    if (b->uploaded) {
        if (hipMemcpyAsync(slots.data(), b->cnt, grmhd::CNT_BYTES, hipMemcpyDeviceToHost, b->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
        if (hipStreamSynchronize(b->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    }
    unsigned long long h[grmhd::CNT_WORDS] = {};
    for (int s = 0; s < grmhd::CNT_SLOTS; ++s) {
        const unsigned long long* w = &slots[(size_t)s * grmhd::CNT_WORDS];
        for (int k = 0; k < grmhd::CNT_WORDS; ++k)
            h[k] = k == grmhd::CNT_MAXIT ? std::max(h[k], w[k]) : h[k] + w[k];
    }
    st->c2p_fail = (long long)h[grmhd::CNT_FAIL];
    st->atm_hits = (long long)h[grmhd::CNT_ATM];
    st->p_floor_hits = (long long)h[grmhd::CNT_PFLOOR];
    st->fallback_1d = (long long)h[grmhd::CNT_FALLBACK];
    st->max_newton_it = (int)h[grmhd::CNT_MAXIT];
    const bool stalled = h[grmhd::CNT_STALL] != 0;
    if (reset && b->uploaded) {
        if (grmhd::launch_zero_counters(b->cnt, b->stream) != hipSuccess)
            return GRMHD_ERR_HIP;
    }
    return stalled ? GRMHD_ERR_STATE : GRMHD_OK;
}

int grmhd_batch_busy(grmhd_batch* b, double* busy, int* slots)
{
    if (!b || !busy)
        return GRMHD_ERR_ARG;
    if (b->last_wgs < 1)
        return GRMHD_ERR_STATE;
    int per_cu = 0;
    if (b->last_lds == PLACE_SPLIT)
        per_cu = b->mixed ? grmhd::batch_split_occupancy<float>() : grmhd::batch_split_occupancy<double>();
    else
        per_cu = b->mixed ? grmhd::batch_evolve_occupancy<float>(b->last_shape, b->last_lds, b->lds_bytes)
                          : grmhd::batch_evolve_occupancy<double>(b->last_shape, b->last_lds, b->lds_bytes);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1)
        return GRMHD_ERR_HIP;
    const int nw = b->last_wgs;
    std::vector<unsigned long long> sp(2 * (size_t)nw);
    if (hipStreamSynchronize(b->stream) != hipSuccess ||
        hipMemcpy(sp.data(), at<unsigned long long>(b, b->L.off_span), sizeof(unsigned long long) * sp.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return GRMHD_ERR_HIP;
    unsigned long long t0 = ~0ull, t1 = 0;
    double sum = 0.0;
    for (int w = 0; w < nw; ++w) {
        t0 = std::min(t0, sp[2 * (size_t)w]);
        t1 = std::max(t1, sp[2 * (size_t)w + 1]);
        sum += (double)(sp[2 * (size_t)w + 1] - sp[2 * (size_t)w]);
    }
    const int S = std::min(nw, per_cu * cus);
    if (slots)
        *slots = S;
    *busy = t1 > t0 ? sum / ((double)S * (double)(t1 - t0)) : 0.0;
    return GRMHD_OK;
}

int grmhd_batch_free(grmhd_batch* b)
{
    if (!b)
        return GRMHD_ERR_ARG;
    delete b;
    return GRMHD_OK;
}

}  // extern "C"
