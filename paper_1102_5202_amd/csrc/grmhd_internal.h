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
// face-flux buffers.  Conserved variables and U arrays are always double.
template <typename T>
hipError_t launch_fill(T* p, long long n, double v, hipStream_t s);
hipError_t launch_zero_counters(unsigned long long* cnt, hipStream_t s);
template <typename T>
hipError_t launch_ghosts(T* Pc, const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_flux(int kind, int dir, const T* Pc, T* F, const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_update(int kind, const T* Fx, const T* Fy, const T* Fz, T* Pc, const double* Un,
                         const double* Us, double* Uout, const Dev& d, double dt, double a, double b,
                         unsigned long long* cnt, hipStream_t s);
template <typename T>
hipError_t launch_update_zmarch(int kind, const T* Fx, const T* Fy, const T* Pc, T* Pn, const double* Un,
                                const double* Us, double* Uout, const Dev& d, double dt, double a,
                                double b, unsigned long long* cnt, hipStream_t s);
template <typename T>
hipError_t launch_rhs(int kind, const T* Fx, const T* Fy, const T* Fz, const T* Pc, double* R,
                      const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_cons(int kind, const double* P, double* U, T* Pc, const Dev& d, hipStream_t s);
template <typename T>
hipError_t launch_prim(int kind, const double* U, double* P, T* Pc, const Dev& d, unsigned long long* cnt,
                       hipStream_t s);

}  // namespace grmhd
