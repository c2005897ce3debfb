// Shared device/host helpers for the hcov HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace hc {

struct Bufs {
  double* p[B_COUNT];
};

// Status bits written by kernels (device int status[0]); status[1] holds the
// first failing cluster-order row of a non-SPD pivot (atomicMin), status[2]
// the number of saturated sketches.
enum StatusBits : int {
  STAT_RANK_OVERFLOW = 1,   // a block needed more than the rank capacity
  STAT_SKETCH_SAT = 2,      // a randomised sketch showed no decay
  STAT_NOT_SPD = 4,         // non-positive / non-finite pivot
  STAT_NONFINITE = 8,       // non-finite matrix entry
  STAT_SAT_CAP = 16,        // a sketch saturated at the widest width the plan allows
};

// The buffer table lives in device memory (one per context): a uniform
// index into it is a scalar load, whereas a dynamically indexed
// kernel-argument array would be copied to scratch memory.
__device__ __forceinline__ double* refp(const Bufs* __restrict__ b, const Ref& r) {
  return b->p[r.buf] + r.off;
}

// A pointer read from memory is generic to the compiler, and its loads
// become flat loads, which also count against the LDS wait counter: a wait
// for an LDS read then waits for every global load in flight.  Every buffer
// here is device memory; accesses through gmem(p) are global loads and
// stores.
#define HC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const HC_GLOBAL T* gmem(const T* p) {
  return (const HC_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ HC_GLOBAL T* gmem(T* p) {
  return (HC_GLOBAL T*)p;
}

__device__ __forceinline__ int dimv(const int* __restrict__ dyn, const Dim& d) {
  if (d.slot < 0) return d.maxv;
  int v = dyn[d.slot] + d.add;
  return v < d.maxv ? v : d.maxv;
}

// Matérn parameters of Eq. (3) prepared on the host for one theta.
struct MaternParams {
  double sigma2;
  double inv_ell;
  double nu;
  double nugget;
  double norm;      // sigma2 * 2^(1-nu) / Gamma(nu)
  double mu;        // nu - N, |mu| <= 1/2
  double g1, g2;    // Temme's Gamma_1(mu), Gamma_2(mu)
  double gp, gm;    // Gamma(1+mu), Gamma(1-mu)
  double mupi;      // mu*pi / sin(mu*pi)
  int N;            // round(nu)
  int kind;         // 0 generic, 1: nu=1/2, 2: nu=3/2, 3: nu=5/2
};

}  // namespace hc
