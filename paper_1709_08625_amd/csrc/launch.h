// Host-side launch wrappers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "plan.h"

namespace hc {

struct FillJob {
  int64_t off;
  int64_t r0, c0;
  int32_t p, q;
  int32_t diag;
  int32_t pad;
};
struct AcaJob {
  int64_t off_u, off_v;
  int64_t r0, c0;
  int32_t p, q;
  int32_t rank_slot;
  int32_t cap;         // rank capacity of the block's arenas (<= the launch's kcap)
  int32_t need_slot;   // dyn slot raised to cap + 1 when the approximation stops at cap unconverged
  int32_t pad;
};

// Device copies of the plan arrays and the run-time state a stage needs.
struct LaunchCtx {
  Bufs bufs;            // host copy of the buffer table
  const Bufs* dbufs;    // the same table in device memory (kernels read it)
  int* dyn;
  const GemmJob* gjobs;
  const GemmProd* gprods;
  const GemmTile* gtiles;
  const TsqrSeg* tsegs;
  const TsqrRed* treds;
  const SmallJob* smalls;
  const LeafJob* leafs;
  const TrsmJob* trsms;
  const int4* copy_pairs;   // (rank, sketch width, rank hint, candidate hint) slots per low-rank block
  int n_copy;
  int rmax;
  int oversample;       // sketch columns beyond the assembly rank (ST_COPY_RANK)
  int fixed_rank;       // > 0: every truncation keeps at most this rank
  double eps;
  double tau;
  double* logdet;
  int* status;
};

struct AcaBigState;
struct AcaBigChunk {
  int job;   // index into the large-block job list
  int c0;    // first row / column of the chunk
};
constexpr int ACA_BIG_CHUNK = 2048;   // entries per work-group in a pass
constexpr int ACA_BIG_PREC = 3 + 64;  // partial record length
constexpr int ACA_BIG_STATE_BYTES = 48 + 128 * 4;
// ACA of the large blocks with many work-groups per block (aca_big.hip)
hipError_t run_aca_big(double* U, double* V, int* dyn, const double* loc, const AcaJob* d_jobs, int nj,
                       const AcaBigChunk* d_rows, int nrow, const AcaBigChunk* d_cols, int ncol,
                       const int* d_row_first, const int* d_row_count, const int* d_col_first,
                       const int* d_col_count, AcaBigState* d_state, double* d_part, double* d_acc,
                       int* d_active, const MaternParams& P, double eps_aca, int kcap, int cap_ok, int* status,
                       hipStream_t st);

hipError_t setup_kernel_attributes();
hipError_t launch_stage(const Stage& s, const LaunchCtx& L, hipStream_t st);
hipError_t launch_adopt_hints(const LaunchCtx& L, hipStream_t st);
hipError_t launch_fill(double* D, const double* loc, const FillJob* jobs, int njobs,
                       const MaternParams& P, hipStream_t st);
// cap_ok: reaching the rank capacity is not an error (fixed-rank mode)
hipError_t launch_aca(double* U, double* V, int* dyn, const double* loc, const AcaJob* jobs, int njobs,
                      const MaternParams& P, double eps_aca, int kcap, int cap_ok, int* status, hipStream_t st);
hipError_t launch_permute(const double* in, double* out, const int* perm, int64_t n, int scatter,
                          hipStream_t st);
hipError_t launch_reduce(const double* x, const double* y, int64_t n, int mode, double* part, hipStream_t st,
                         int64_t* nparts);
hipError_t launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t st);
hipError_t launch_exact_matvec(const double* loc, const double* x, double* y, int64_t n, const MaternParams& P,
                               hipStream_t st);
hipError_t launch_probe(const double* h, double* out, int64_t n, const MaternParams& P, hipStream_t st);
hipError_t launch_gaussian(double* out, int64_t n, uint64_t seed, hipStream_t st);
hipError_t launch_fill_value(double* out, int64_t n, double v, hipStream_t st);

}  // namespace hc
