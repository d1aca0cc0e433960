// grmhd_internal.h -- launchers shared by the C ABI and the kernel unit.
#pragma once

#include <hip/hip_runtime.h>

#include "grmhd_device.h"

namespace grmhd {

// Device counters: CNT_SLOTS copies of CNT_WORDS unsigned 64-bit words, one
// 128-byte line per slot.  A wave adds into slot (block index mod CNT_SLOTS),
// so that atomics from different waves rarely meet on one address (atomics on
// a single address serialise in the L2); the host sums (max for MAXIT) the
// slots when it reads them.
enum { CNT_FAIL = 0, CNT_ATM = 1, CNT_PFLOOR = 2, CNT_FALLBACK = 3, CNT_MAXIT = 4, CNT_WORDS = 16 };
enum { CNT_SLOTS = 256 };
static constexpr size_t CNT_BYTES = sizeof(unsigned long long) * CNT_WORDS * CNT_SLOTS;

// Launchers; T (double or float) is the type of the primitive caches and the
// face-flux buffers.  The caller's conserved arrays are always double.
template <typename T>
hipError_t launch_fill(T* p, long long n, double v, hipStream_t s);
hipError_t launch_zero_counters(unsigned long long* cnt, hipStream_t s);
hipError_t launch_arith(const double* x, const double* y, double* out, long long n, hipStream_t s);
template <typename T>
hipError_t launch_ghosts(T* Pc, const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_flux(int kind, int dir, const T* Pc, T* F, const Dev& d, hipStream_t s);
// Stored metric: the caller's ghosted centre arrays to the centre [8][N] and
// face [2][nf] values the kernels read.
hipError_t launch_metric(const double* alpha, const double* psi4, double* mc, double* const* mf, const Dev& d,
                         hipStream_t s);
// Flux-CT: the field fluxes of all active axes (F[3]) replaced from the edge
// values W[3] of the axis pairs (x,y), (x,z), (y,z).
template <typename T>
hipError_t launch_ct(T* const* F, T* const* W, const Dev& d, hipStream_t s);
// TS / TO: types of the stage state read (U^s) and written (U^(s+1)); double,
// or float for the intermediate stages of the mixed-precision path.  U^n is
// always double.  The update kernels read the primitives from Pc and write
// the new ones, with their ghost images, to Pn (Pc == Pn allowed for
// launch_update only); fout (may be null) receives per-cell recovery flags.
template <typename T, typename TS, typename TO>
hipError_t launch_update(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, T* Pn, const double* Un,
                         const TS* Us, TO* Uout, const Dev& d, double dt, double a, double b,
                         unsigned long long* cnt, unsigned char* fout, hipStream_t s);
// The whole substep of a 3D grid (MC, cleaning) in one launch: faces of all
// three axes, flux differences, sources, RK combination and recovery; reads
// the primitives from Pc, writes the new ones (with ghost images) to Pn.
template <typename T, typename TS, typename TO>
hipError_t launch_substep(int kind, const T* Pc, T* Pn, const double* Un, const TS* Us, TO* Uout, const Dev& d,
                          double dt, double a, double b, unsigned long long* cnt, unsigned char* fout,
                          hipStream_t s);
template <typename T>
hipError_t launch_rhs(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, double* R,
                      const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_cons(int kind, const double* P, double* U, T* Pc, const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_prim(int kind, const double* U, double* P, T* Pc, const Dev& d, unsigned long long* cnt,
                       hipStream_t s);

// Batched ensemble of independent 1D problems along x (flat metric).  One
// record per problem, in device memory.
struct BatchProb {
    int n;              // cells
    int steps;          // Runge-Kutta steps to take in all
    int done;           // steps taken so far (advanced by the evolve kernel)
    int pad;
    long long off;      // first cell of the problem in the packed arrays
    long long poff;     // first element of its ghosted primitive row (9 rows of n + 4)
    double lo, dx, idx, dt;
};

// Launch shapes of the batched evolve kernel: threads per workgroup.
static constexpr int BATCH_SHAPES = 3;
static constexpr int BATCH_THREADS[BATCH_SHAPES] = {256, 512, 1024};

// A problem split among several workgroups ("parts") that run at the same
// time: part p owns the cells [c0, c1) of problem b; left and right are the
// parts holding the cells beside c0 and c1 (-1 at the problem's ends); the
// problem's parts are [first, first + count).  A problem too small to split
// is one part holding all of its cells.
struct BatchPart {
    int b, c0, c1, left, right, first, count, pad;
};
static constexpr int BATCH_SPLIT_THREADS = 256;
// Word of the counter block set when a part of a split launch stopped waiting
// for a neighbour (the parts were not all resident at once).
enum { CNT_STALL = 5 };

template <typename T>
hipError_t launch_batch_cons(const BatchProb* probs, int nprob, long long ncell, const double* P, double* U,
                             T* Prow, const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_batch_prim(const BatchProb* probs, int nprob, long long ncell, const double* U, double* P,
                             T* Prow, const Dev& d, unsigned long long* cnt, hipStream_t s);
// shape: index into BATCH_THREADS; lds: keep the primitive rows in LDS (needs
// lds_bytes <= 160 KiB).  order: the problem each workgroup takes.  Pnext is
// a second set of rows (the next substep's, or the staging of the LDS rows).
// Allows k_batch_evolve's LDS variants `bytes` of dynamic LDS (set-up only:
// not a stream operation, so never called while a step may be captured).
template <typename T>
hipError_t allow_batch_lds(size_t bytes);

// The split launch: parts[nparts] as above, flags[nparts] the substeps each
// part has completed (kept across launches, consistent with probs[].done).
// runs[nruns]: workgroup w runs parts runs[w].x .. runs[w].x + runs[w].y - 1
// in turn (a split problem's parts each have a workgroup of their own; small
// whole problems share one).  span: 2 entries per workgroup, its start and
// end on the GPU's constant-rate clock (written by every workgroup).
template <typename T>
hipError_t launch_batch_split(BatchProb* probs, const BatchPart* parts, int nparts, const int2* runs, int nruns,
                              int* flags, double* U, T* Us, T* Prow, T* Pnext, const Dev& d, int rk_order,
                              int max_steps, unsigned long long* cnt, unsigned long long* span, hipStream_t s);
// Resident workgroups of the split launch per CU (0 if unknown).
template <typename T>
int batch_split_occupancy();
// Resident workgroups of an evolve launch shape per CU (0 if unknown).
template <typename T>
int batch_evolve_occupancy(int shape, int lds, size_t lds_bytes);

template <typename T>
hipError_t launch_batch_evolve(int shape, int lds, size_t lds_bytes, BatchProb* probs, const int* order, int nprob,
                               double* U, T* Us, T* Prow, T* Pnext, const Dev& d, int rk_order, int max_steps,
                               unsigned long long* cnt, unsigned long long* span, hipStream_t s);

// Adjoint kernels (FP64; grmhd_adjoint.hip).  FB: the face-state cotangents
// of one axis (18 rows of nf[d] values); MU: a ghosted cotangent of the
// primitives.
hipError_t launch_adj_rec(int kind, double* Ub, const double* Pn, const unsigned char* flags, double* Unacc,
                          double* Rb, const Dev& d, double a, double b, double dt, hipStream_t s);
hipError_t launch_adj_face(int kind, const double* Pc, const double* Rb, double* const* FB, const Dev& d,
                           hipStream_t s);
hipError_t launch_adj_gather(const double* Pc, const double* const* FB, double* MU, double* const* G, const Dev& d,
                             hipStream_t s);
hipError_t launch_adj_cell(int kind, const double* Pc, const double* MU, const double* const* G, double* Rb,
                           double* Ub, double* Unacc, const unsigned char* fprev, const Dev& d, double a, double b,
                           double dt, hipStream_t s);
hipError_t launch_adj_final(int kind, const double* Ub, const double* Pb, const double* P0, const double* Unacc,
                            double* Ubar, const Dev& d, hipStream_t s);
hipError_t launch_adj_cons(int kind, const double* P, const double* Ubar, double* Pbar, const Dev& d,
                           hipStream_t s);

}  // namespace grmhd
