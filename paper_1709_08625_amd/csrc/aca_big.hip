// Partially pivoted ACA for large admissible blocks, spread over many
// work-groups.  The algorithm is the one of the single-work-group kernel
// (Bebendorf 2000: pivot row -> residual row -> column of the largest entry
// -> next row of the largest residual-column entry; stop when
// ||u_k|| ||v_k|| <= eps_aca ||S_k||_F with the exact incremental Frobenius
// norm), executed in lock-step for all large blocks with four launches per
// rank step:
//   row pass   : residual row, partial max |r_j|, ||r||^2, <V_l, r>
//   pivot      : per block, choose j*, or skip a zero row
//   column pass: v = r / r_j*, residual column u, partial max |u_i|,
//                ||u||^2, <U_l, u>
//   update     : per block, norms, stopping test, next pivot row
// Partial results are reduced in a fixed order, so the factors are
// deterministic.
#include <hip/hip_runtime.h>

#include "common.h"
#include "launch.h"
#include "matern.h"

namespace hc {

constexpr int ACH = ACA_BIG_CHUNK;

struct AcaBigState {
  int k;          // current rank
  int istar;      // pivot row of the current step
  int jstar;      // pivot column
  int done;       // 1: finished
  int nused;
  int phase_ok;   // 1: the current row gave a nonzero pivot
  int pending;    // 1: the column written in this step awaits scaling by ipiv
  int pad1;
  double nrm2;
  double ipiv;
  int used[128];
};
static_assert(sizeof(AcaBigState) == ACA_BIG_STATE_BYTES, "state layout");

// partial record per (block, chunk): [0] max |x|, [1] index (as double),
// [2] sum x^2, [3..3+k) dots with previous columns
constexpr int PREC = ACA_BIG_PREC;

__device__ __forceinline__ void wg_argmax_sum(double& best, int& bi, double& ss, double* sh_v, int* sh_i,
                                              double* sh_s) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    double b2 = __shfl_down(best, o);
    int i2 = __shfl_down(bi, o);
    double s2 = __shfl_down(ss, o);
    if (b2 > best || (b2 == best && i2 < bi)) {
      best = b2;
      bi = i2;
    }
    ss += s2;
  }
  if (lane == 0) {
    sh_v[wave] = best;
    sh_i[wave] = bi;
    sh_s[wave] = ss;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) {
      if (sh_v[w] > best || (sh_v[w] == best && sh_i[w] < bi)) {
        best = sh_v[w];
        bi = sh_i[w];
      }
    }
    ss = (sh_s[0] + sh_s[1]) + (sh_s[2] + sh_s[3]);
  }
  __syncthreads();
}

// dots[l] = sum over this WG's entries of X[j + l*ld] * x[j], l < k
__device__ void wg_dots(const double* X, int ld, const double* x, int j0, int j1, int k, double* out,
                        double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int l = 0; l < k; ++l) {
    double s = 0.0;
    for (int j = j0 + tid; j < j1; j += 256) s += X[j + (size_t)l * ld] * x[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (tid == 0) out[l] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_acab_init(AcaBigState* st, int nj) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nj) return;
  AcaBigState& S = st[i];
  S.k = 0;
  S.istar = 0;
  S.jstar = 0;
  S.done = 0;
  S.nused = 0;
  S.phase_ok = 0;
  S.pending = 0;
  S.nrm2 = 0.0;
  S.ipiv = 0.0;
}

// row pass: chunks over the q columns of every active block
__global__ __launch_bounds__(256) void k_acab_row(double* __restrict__ Ub, double* __restrict__ Vb,
                                                  const double2* __restrict__ loc,
                                                  const AcaJob* __restrict__ jobs, AcaBigState* __restrict__ st,
                                                  const AcaBigChunk* __restrict__ chunks, MaternParams P,
                                                  double* __restrict__ part) {
  const AcaBigChunk ch = chunks[blockIdx.x];
  const AcaJob J = jobs[ch.job];
  const AcaBigState& S = st[ch.job];
  if (S.done) return;
  const int k = S.k, i = S.istar, q = J.q;
  double* U = Ub + J.off_u;
  double* V = Vb + J.off_v;
  __shared__ double rowU[64];
  __shared__ double sh_v[4], sh_s[4], sh[4];
  __shared__ int sh_i[4];
  if (threadIdx.x < k) rowU[threadIdx.x] = U[i + (size_t)threadIdx.x * J.p];
  __syncthreads();
  const double2 xi = loc[J.r0 + i];
  double* vk = V + (size_t)k * q;
  const int j0 = ch.c0, j1 = min(ch.c0 + ACH, q);
  double best = -1.0, ss = 0.0;
  int bj = 0x7fffffff;
  for (int j = j0 + threadIdx.x; j < j1; j += 256) {
    double2 y = loc[J.c0 + j];
    double dx = xi.x - y.x, dy = xi.y - y.y;
    double r = matern_eval(sqrt(dx * dx + dy * dy), P);
    for (int l = 0; l < k; ++l) r -= rowU[l] * V[j + (size_t)l * q];
    vk[j] = r;
    double a = fabs(r);
    if (a > best) {
      best = a;
      bj = j;
    }
    ss += r * r;
  }
  wg_argmax_sum(best, bj, ss, sh_v, sh_i, sh_s);
  double* out = part + (size_t)blockIdx.x * PREC;
  if (threadIdx.x == 0) {
    out[0] = best;
    out[1] = double(bj);
    out[2] = ss;
  }
  __syncthreads();
  wg_dots(V, q, vk, j0, j1, k, out + 3, sh);
}

// pivot: one thread per active block reduces its row-pass partials
__global__ void k_acab_pivot(const AcaJob* __restrict__ jobs, AcaBigState* __restrict__ st,
                             const int* __restrict__ row_first, const int* __restrict__ row_count,
                             double* __restrict__ part, double* __restrict__ acc, int nj, int* __restrict__ status) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nj) return;
  AcaBigState& S = st[b];
  S.pending = 0;
  if (S.done) return;
  const int k = S.k;
  double best = -1.0, ss = 0.0;
  int bj = 0x7fffffff;
  double* a = acc + (size_t)b * PREC;
  for (int l = 0; l < k; ++l) a[3 + l] = 0.0;
  for (int c = 0; c < row_count[b]; ++c) {
    const double* pr = part + (size_t)(row_first[b] + c) * PREC;
    int idx = int(pr[1]);
    if (pr[0] > best || (pr[0] == best && idx < bj)) {
      best = pr[0];
      bj = idx;
    }
    ss += pr[2];
    for (int l = 0; l < k; ++l) a[3 + l] += pr[3 + l];
  }
  a[2] = ss;
  if (S.nused < 128) S.used[S.nused] = S.istar;
  S.nused = S.nused < 128 ? S.nused + 1 : 128;
  const AcaJob J = jobs[b];
  if (!(best > 0.0) || !isfinite(best)) {
    if (!isfinite(best)) atomicOr(status, STAT_NONFINITE);
    // zero residual row: next unused row, else stop
    int nxt = -1;
    for (int r = 0; r < J.p && nxt < 0; ++r) {
      bool u = false;
      for (int x = 0; x < S.nused; ++x) u |= (S.used[x] == r);
      if (!u) nxt = r;
    }
    S.phase_ok = 0;
    if (nxt < 0 || !isfinite(best) || S.nused >= J.p) {
      S.done = 1;
    } else {
      S.istar = nxt;
    }
    return;
  }
  S.phase_ok = 1;
  S.jstar = bj;
  const double* Vk = nullptr;
  (void)Vk;
  S.ipiv = 0.0;   // set in the column pass from the stored row value
}

// column pass: v = r / r_j* (scaling the stored row), residual column u
__global__ __launch_bounds__(256) void k_acab_col(double* __restrict__ Ub, double* __restrict__ Vb,
                                                  const double2* __restrict__ loc,
                                                  const AcaJob* __restrict__ jobs, AcaBigState* __restrict__ st,
                                                  const AcaBigChunk* __restrict__ chunks, MaternParams P,
                                                  double* __restrict__ part) {
  const AcaBigChunk ch = chunks[blockIdx.x];
  const AcaJob J = jobs[ch.job];
  const AcaBigState& S = st[ch.job];
  if (S.done || !S.phase_ok) return;
  const int k = S.k, js = S.jstar, p = J.p, q = J.q;
  double* U = Ub + J.off_u;
  double* V = Vb + J.off_v;
  __shared__ double colV[64];
  __shared__ double sh_v[4], sh_s[4], sh[4];
  __shared__ int sh_i[4];
  if (threadIdx.x < k) colV[threadIdx.x] = V[js + (size_t)threadIdx.x * q];
  __syncthreads();
  const double piv = V[js + (size_t)k * q];   // unscaled r_j*
  const double2 yj = loc[J.c0 + js];
  double* uk = U + (size_t)k * p;
  const int i0 = ch.c0, i1 = min(ch.c0 + ACH, p);
  double best = -1.0, ss = 0.0;
  int bi = 0x7fffffff;
  for (int r = i0 + threadIdx.x; r < i1; r += 256) {
    double2 x = loc[J.r0 + r];
    double dx = x.x - yj.x, dy = x.y - yj.y;
    double u = matern_eval(sqrt(dx * dx + dy * dy), P);
    for (int l = 0; l < k; ++l) u -= colV[l] * U[r + (size_t)l * p];
    uk[r] = u;
    double a = fabs(u);
    if (a > best) {
      best = a;
      bi = r;
    }
    ss += u * u;
  }
  wg_argmax_sum(best, bi, ss, sh_v, sh_i, sh_s);
  double* out = part + (size_t)blockIdx.x * PREC;
  if (threadIdx.x == 0) {
    out[0] = best;
    out[1] = double(bi);
    out[2] = ss;
  }
  __syncthreads();
  wg_dots(U, p, uk, i0, i1, k, out + 3, sh);
  (void)piv;
}

// update: norms, stopping test, scaling of v, next pivot row
__global__ void k_acab_update(double* __restrict__ Vb, const AcaJob* __restrict__ jobs,
                              AcaBigState* __restrict__ st, const int* __restrict__ col_first,
                              const int* __restrict__ col_count, const double* __restrict__ part,
                              const double* __restrict__ acc, int nj, double eps_aca, int kcap, int cap_ok,
                              int* __restrict__ dyn, int* __restrict__ status, int* __restrict__ active) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nj) return;
  AcaBigState& S = st[b];
  const AcaJob J = jobs[b];
  if (!S.done && S.phase_ok) {
    const int k = S.k;
    const double piv = Vb[J.off_v + S.jstar + (size_t)k * J.q];
    const double ip = 1.0 / piv;
    const double* a = acc + (size_t)b * PREC;
    double best = -1.0, su = 0.0;
    int bi = 0x7fffffff;
    double cross = 0.0;
    double du[64];
    for (int l = 0; l < k; ++l) du[l] = 0.0;
    for (int c = 0; c < col_count[b]; ++c) {
      const double* pr = part + (size_t)(col_first[b] + c) * PREC;
      int idx = int(pr[1]);
      if (pr[0] > best || (pr[0] == best && idx < bi)) {
        best = pr[0];
        bi = idx;
      }
      su += pr[2];
      for (int l = 0; l < k; ++l) du[l] += pr[3 + l];
    }
    for (int l = 0; l < k; ++l) cross += du[l] * (a[3 + l] * ip);
    const double sv = a[2] * ip * ip;
    const double nuv = su * sv;
    S.nrm2 += nuv + 2.0 * cross;
    S.ipiv = ip;
    S.k = k + 1;
    S.pending = 1;
    bool stop = sqrt(nuv) <= eps_aca * sqrt(fmax(S.nrm2, 0.0));
    const int kmax = min(min(J.p, J.q), min(kcap, J.cap));
    if (S.k >= kmax) {
      if (!stop && kmax < min(J.p, J.q) && !cap_ok) {
        atomicOr(status, STAT_RANK_OVERFLOW);
        if (J.need_slot >= 0) atomicMax(dyn + J.need_slot, kmax + 1);
      }
      stop = true;
    }
    if (!stop) {
      bool isused = false;
      for (int x = 0; x < S.nused; ++x) isused |= (S.used[x] == bi);
      if (isused || !(best > 0.0)) {
        int nxt = -1;
        for (int r = 0; r < J.p && nxt < 0; ++r) {
          bool u = false;
          for (int x = 0; x < S.nused; ++x) u |= (S.used[x] == r);
          if (!u) nxt = r;
        }
        if (nxt < 0)
          stop = true;
        else
          bi = nxt;
      }
    }
    S.istar = bi;
    if (stop) S.done = 1;
  }
  dyn[J.rank_slot] = S.k;
  if (!S.done) atomicAdd(active, 1);
}

// v = r * ipiv for the columns produced in the last step (after update)
__global__ __launch_bounds__(256) void k_acab_scale(double* __restrict__ Vb, const AcaJob* __restrict__ jobs,
                                                    const AcaBigState* __restrict__ st,
                                                    const AcaBigChunk* __restrict__ chunks, int step) {
  const AcaBigChunk ch = chunks[blockIdx.x];
  const AcaJob J = jobs[ch.job];
  const AcaBigState& S = st[ch.job];
  // the column written in this step is k-1 after the update (if it advanced)
  if (!S.pending) return;
  double* vk = Vb + J.off_v + (size_t)(S.k - 1) * J.q;
  const int j1 = min(ch.c0 + ACH, J.q);
  for (int j = ch.c0 + threadIdx.x; j < j1; j += 256) vk[j] *= S.ipiv;
  (void)step;
}

// ------------------------------------------------------------------ driver
hipError_t run_aca_big(double* U, double* V, int* dyn, const double* loc, const AcaJob* d_jobs, int nj,
                       const AcaBigChunk* d_rows, int nrow, const AcaBigChunk* d_cols, int ncol,
                       const int* d_row_first, const int* d_row_count, const int* d_col_first,
                       const int* d_col_count, AcaBigState* d_state, double* d_part, double* d_acc,
                       int* d_active, const MaternParams& P, double eps_aca, int kcap, int cap_ok, int* status,
                       hipStream_t st) {
  if (nj <= 0) return hipSuccess;
  k_acab_init<<<(nj + 255) / 256, 256, 0, st>>>(d_state, nj);
  const int maxsteps = 2 * kcap + 8;   // zero rows may consume extra steps
  for (int s = 0; s < maxsteps; ++s) {
    k_acab_row<<<nrow, 256, 0, st>>>(U, V, (const double2*)loc, d_jobs, d_state, d_rows, P, d_part);
    k_acab_pivot<<<(nj + 127) / 128, 128, 0, st>>>(d_jobs, d_state, d_row_first, d_row_count, d_part, d_acc,
                                                     nj, status);
    k_acab_col<<<ncol, 256, 0, st>>>(U, V, (const double2*)loc, d_jobs, d_state, d_cols, P, d_part);
    hipError_t e = hipMemsetAsync(d_active, 0, 4, st);
    if (e != hipSuccess) return e;
    k_acab_update<<<(nj + 127) / 128, 128, 0, st>>>(V, d_jobs, d_state, d_col_first, d_col_count, d_part, d_acc,
                                                      nj, eps_aca, kcap, cap_ok, dyn, status, d_active);
    k_acab_scale<<<nrow, 256, 0, st>>>(V, d_jobs, d_state, d_rows, s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((s & 3) == 3) {
      int act = 0;
      e = hipMemcpyAsync(&act, d_active, 4, hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      if (act == 0) break;
    }
  }
  return hipGetLastError();
}

}  // namespace hc
