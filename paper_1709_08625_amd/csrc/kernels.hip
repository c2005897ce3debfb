// Batched device kernels of the H-matrix likelihood (gfx950, FP64).
//
//   k_gemm       grouped sum-of-products GEMM over variable-size jobs
//   k_tsqr_seg   Householder R factor of a row segment of a tall matrix
//   k_tsqr_red   R factor of a stack of segment R factors
//   k_small      one-sided Jacobi SVDs of the small R-factor products
//                (recompression and randomised-sketch truncation)
//   k_leaf       dense leaf targets: Schur update in registers, potrf in LDS
//   k_trsm       triangular solves with a diagonal leaf factor
//   k_dense_fill Matérn entries of the dense leaves (+ nugget, Sec. 5.2)
//   k_aca        partially pivoted ACA of admissible blocks
//   small utilities (permutations, reductions)
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "common.h"
#include "matern.h"
#include "launch.h"

namespace hc {

// ------------------------------------------------------------------ GEMM
// One work-group (256 threads) computes a 64 x 64 tile of one job's output:
// C_tile = (zero ? 0 : C_tile) + sum_p alpha_p op(A_p) op(B_p) restricted to
// the tile, accumulating all products of the job in registers (each thread
// owns a 4 x 4 sub-tile).  k is streamed through LDS in chunks of 16.
constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void k_gemm(Bufs bufs, const int* __restrict__ dyn,
                                              const GemmJob* __restrict__ jobs,
                                              const GemmProd* __restrict__ prods,
                                              const GemmTile* __restrict__ tiles, int t0) {
  const GemmTile T = tiles[t0 + blockIdx.x];
  const GemmJob J = jobs[T.job];
  const int m = dimv(dyn, J.m), n = dimv(dyn, J.n);
  const int r0 = T.ti * GT, c0 = T.tj * GT;
  if (r0 >= m || c0 >= n) return;
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

  for (int pi = J.p0; pi < J.p1; ++pi) {
    const GemmProd Pd = prods[pi];
    const int k = dimv(dyn, Pd.k);
    int mi = dimv(dyn, Pd.mi), nj = dimv(dyn, Pd.nj);
    if (k <= 0 || mi <= 0 || nj <= 0) continue;
    // product rows [Pd.i0, Pd.i0+mi) intersect tile rows [r0, r0+GT)
    const int pr0 = Pd.i0, pr1 = min(Pd.i0 + mi, m), pc0 = Pd.j0, pc1 = min(Pd.j0 + nj, n);
    if (pr1 <= r0 || pr0 >= r0 + GT || pc1 <= c0 || pc0 >= c0 + GT) continue;
    const double* __restrict__ A = refp(bufs, Pd.A);
    const double* __restrict__ B = refp(bufs, Pd.B);
    const int lda = Pd.A.ld, ldb = Pd.B.ld;
    const double alpha = Pd.alpha;
    for (int k0 = 0; k0 < k; k0 += GK) {
      // A tile: rows r0..r0+63 (global C rows) -> product row i - pr0
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int e = tid + 256 * r;
        int ii, kk;
        if (Pd.ta == 0) {
          ii = e & 63;
          kk = e >> 6;
        } else {
          ii = e >> 4;
          kk = e & 15;
        }
        int gi = r0 + ii, gk = k0 + kk;
        double v = 0.0;
        if (gi >= pr0 && gi < pr1 && gk < k) {
          int li = gi - pr0;
          v = Pd.ta == 0 ? A[li + (size_t)gk * lda] : A[gk + (size_t)li * lda];
        }
        As[kk][ii] = alpha * v;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int e = tid + 256 * r;
        int jj, kk;
        if (Pd.tb == 0) {
          kk = e & 15;
          jj = e >> 4;
        } else {
          jj = e & 63;
          kk = e >> 6;
        }
        int gj = c0 + jj, gk = k0 + kk;
        double v = 0.0;
        if (gj >= pc0 && gj < pc1 && gk < k) {
          int lj = gj - pc0;
          v = Pd.tb == 0 ? B[gk + (size_t)lj * ldb] : B[lj + (size_t)gk * ldb];
        }
        Bs[kk][jj] = v;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[q] = As[kk][ty * 4 + q];
          b[q] = Bs[kk][tx * 4 + q];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
      }
      __syncthreads();
    }
  }
  double* __restrict__ C = refp(bufs, J.C);
  const int ldc = J.C.ld;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    int gi = r0 + ty * 4 + x;
    if (gi >= m) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      int gj = c0 + tx * 4 + y;
      if (gj >= n) continue;
      size_t o = gi + (size_t)gj * ldc;
      C[o] = J.zero ? acc[x][y] : C[o] + acc[x][y];
    }
  }
}

// ------------------------------------------------------------------ TSQR
// Householder QR in LDS of an mrows x c matrix (col-major, ld = LDM).  On
// exit the upper triangle of the leading c x c block holds R.
constexpr int QR_CH = 64;            // rows added per step
constexpr int QR_CMAX = 96;          // max columns
constexpr int LDM = QR_CH + QR_CMAX; // 160

__device__ void house_qr_lds(double* M, int mrows, int c, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < c && j < mrows; ++j) {
    // norm of column j below the diagonal (wave 0)
    if (wave == 0) {
      double s = 0.0;
      for (int i = j + lane; i < mrows; i += 64) {
        double v = M[i + j * LDM];
        s += v * v;
      }
      for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
      if (lane == 0) {
        double nrm = sqrt(s);
        double a = M[j + j * LDM];
        double alpha = (a >= 0.0) ? -nrm : nrm;
        // v = x - alpha e1 ; v^T v = 2 nrm (nrm + |a|)
        double vtv = 2.0 * nrm * (nrm + fabs(a));
        red[0] = alpha;
        red[1] = (vtv > 0.0) ? 2.0 / vtv : 0.0;
        M[j + j * LDM] = a - alpha;   // v stored in column j
      }
    }
    __syncthreads();
    const double beta = red[1];
    if (beta != 0.0) {
      for (int l = j + 1 + wave; l < c; l += 4) {
        double s = 0.0;
        for (int i = j + lane; i < mrows; i += 64) s += M[i + j * LDM] * M[i + l * LDM];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
        s = __shfl(s, 0);
        s *= beta;
        for (int i = j + lane; i < mrows; i += 64) M[i + l * LDM] -= s * M[i + j * LDM];
      }
    }
    __syncthreads();
    if (tid == 0) M[j + j * LDM] = red[0];
    for (int i = j + 1 + tid; i < mrows; i += 256) M[i + j * LDM] = 0.0;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_tsqr_seg(Bufs bufs, const int* __restrict__ dyn,
                                                  const TsqrSeg* __restrict__ segs, int s0, int rmax) {
  const TsqrSeg S = segs[s0 + blockIdx.x];
  const int c = dimv(dyn, S.cols);
  double* __restrict__ R = refp(bufs, S.R);
  extern __shared__ double smem[];
  double* M = smem;                 // LDM x QR_CMAX
  double* red = smem + LDM * QR_CMAX;
  const int tid = threadIdx.x;
  if (c <= 0) {
    return;
  }
  const double* __restrict__ X = refp(bufs, S.X);
  const int ld = S.X.ld;
  int have = 0;   // rows of R currently held at the top of M
  for (int base = 0; base < S.rows; base += QR_CH) {
    int nr = min(QR_CH, S.rows - base);
    // rows [have, have+nr) <- X[base.., :]
    for (int e = tid; e < nr * c; e += 256) {
      int i = e % nr, l = e / nr;
      M[have + i + l * LDM] = X[(size_t)(base + i) + (size_t)l * ld];
    }
    __syncthreads();
    int mrows = have + nr;
    house_qr_lds(M, mrows, c, red);
    have = min(mrows, c);
    // zero below the kept R rows for the next round (columns c)
    __syncthreads();
  }
  // write R (c x c), rows >= have are zero
  for (int e = tid; e < c * c; e += 256) {
    int i = e % c, l = e / c;
    R[i + (size_t)l * rmax] = (i < have && i <= l) ? M[i + l * LDM] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_tsqr_red(Bufs bufs, const int* __restrict__ dyn,
                                                  const TsqrRed* __restrict__ reds, int r0i, int rmax) {
  const TsqrRed S = reds[r0i + blockIdx.x];
  const int c = dimv(dyn, S.cols);
  double* __restrict__ R = refp(bufs, S.R);
  extern __shared__ double smem[];
  double* M = smem;
  double* red = smem + LDM * QR_CMAX;
  const int tid = threadIdx.x;
  if (c <= 0) return;
  const double* __restrict__ R0 = refp(bufs, S.R0);
  const size_t RR = (size_t)rmax * rmax;
  int have = 0;
  for (int s = 0; s < S.nseg; ++s) {
    const double* Rs = R0 + RR * s;
    for (int e = tid; e < c * c; e += 256) {
      int i = e % c, l = e / c;
      M[have + i + l * LDM] = Rs[i + (size_t)l * rmax];
    }
    __syncthreads();
    int mrows = have + c;
    house_qr_lds(M, mrows, c, red);
    have = min(mrows, c);
    __syncthreads();
  }
  for (int e = tid; e < c * c; e += 256) {
    int i = e % c, l = e / c;
    R[i + (size_t)l * rmax] = (i < have && i <= l) ? M[i + l * LDM] : 0.0;
  }
}

// ------------------------------------------------------------------ small SVD
// One-sided Jacobi (Hestenes) on the columns of an n x n matrix A in LDS
// (ld = SM), accumulating the right rotations in V: A V = U S.  Disjoint
// column pairs of a round-robin ordering are processed by the 4 waves.
constexpr int SM = 96;

__device__ void jacobi_svd_lds(double* A, double* V, int n, int* pairs, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < n * n; e += 256) {
    int i = e % n, j = e / n;
    V[i + j * SM] = (i == j) ? 1.0 : 0.0;
  }
  const int np = (n + 1) & ~1;   // even count (a dummy column n when odd)
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) red[0] = 0.0;
    __syncthreads();
    double offmax = 0.0;
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      // round-robin pairing of 0..np-1 (index np-1 fixed)
      for (int t = wave; t < np / 2; t += 4) {
        int a, b;
        if (t == 0) {
          a = np - 1;
          b = rnd;
        } else {
          a = (rnd + t) % (np - 1);
          b = (rnd - t + (np - 1)) % (np - 1);
        }
        if (a >= n || b >= n) continue;
        int p = min(a, b), q = max(a, b);
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < n; i += 64) {
          double x = A[i + p * SM], y = A[i + q * SM];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        for (int o = 32; o > 0; o >>= 1) {
          al += __shfl_down(al, o);
          be += __shfl_down(be, o);
          ga += __shfl_down(ga, o);
        }
        al = __shfl(al, 0);
        be = __shfl(be, 0);
        ga = __shfl(ga, 0);
        if (ga == 0.0 || al == 0.0 || be == 0.0) continue;
        double rel = fabs(ga) / sqrt(al * be);
        offmax = fmax(offmax, rel);
        if (rel < 1e-15) continue;
        double zeta = (be - al) / (2.0 * ga);
        double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / sqrt(1.0 + tt * tt);
        double sn = cs * tt;
        for (int i = lane; i < n; i += 64) {
          double x = A[i + p * SM], y = A[i + q * SM];
          A[i + p * SM] = cs * x - sn * y;
          A[i + q * SM] = sn * x + cs * y;
          double vx = V[i + p * SM], vy = V[i + q * SM];
          V[i + p * SM] = cs * vx - sn * vy;
          V[i + q * SM] = sn * vx + cs * vy;
        }
      }
      __syncthreads();
    }
    // reduce offmax over waves
    if (lane == 0) {
      // atomic max on a double in LDS via CAS-free approach: store per wave
      red[1 + wave] = offmax;
    }
    __syncthreads();
    double om = fmax(fmax(red[1], red[2]), fmax(red[3], red[4]));
    __syncthreads();
    if (om < 1e-15) break;
  }
  (void)pairs;
}

// sort indices of column norms descending (tid 0), ord[0..n)
__device__ void order_desc(const double* A, int n, double* sv, int* ord) {
  if (threadIdx.x == 0) {
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += A[i + j * SM] * A[i + j * SM];
      sv[j] = sqrt(s);
      ord[j] = j;
    }
    for (int a = 1; a < n; ++a) {   // insertion sort, stable, descending
      int x = ord[a];
      int b = a - 1;
      while (b >= 0 && sv[ord[b]] < sv[x]) {
        ord[b + 1] = ord[b];
        --b;
      }
      ord[b + 1] = x;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_small(Bufs bufs, int* __restrict__ dyn,
                                               const SmallJob* __restrict__ jobs, int j0, int rmax,
                                               double eps_run, double tau_run, int* __restrict__ status) {
  const SmallJob J = jobs[j0 + blockIdx.x];
  const int n = dimv(dyn, J.k);
  extern __shared__ double smem[];
  double* A = smem;                 // SM x SM
  double* V = smem + SM * SM;       // SM x SM
  double* sv = V + SM * SM;         // SM
  double* red = sv + SM;            // 8
  int* ord = (int*)(red + 8);       // SM
  const int tid = threadIdx.x;
  const double eps = J.eps == -1.0 ? eps_run : (J.eps == -2.0 ? tau_run : J.eps);
  if (n <= 0) {
    if (tid == 0) dyn[J.out_rank_slot] = 0;
    return;
  }
  const double* __restrict__ R1 = refp(bufs, J.R1);
  const double* __restrict__ R2 = J.kind != SK_SKETCH_P ? refp(bufs, J.R2) : nullptr;
  double* __restrict__ C1 = refp(bufs, J.C1);
  // ---- form the matrix to decompose
  if (J.kind == SK_RECOMP) {
    // A = R1 R2^T (both upper triangular n x n)
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, j = e / n;
      double s = 0.0;
      for (int l = max(i, j); l < n; ++l) s += R1[i + (size_t)l * rmax] * R2[j + (size_t)l * rmax];
      A[i + j * SM] = s;
    }
  } else if (J.kind == SK_SKETCH_P) {
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, j = e / n;
      A[i + j * SM] = R1[i + (size_t)j * rmax];
    }
  } else {
    // A = R1 R2^{-1}: row i solves g R2 = r1 (R2 upper triangular)
    for (int i = tid; i < n; i += 256) {
      for (int j = 0; j < n; ++j) {
        double s = R1[i + (size_t)j * rmax];
        for (int l = 0; l < j; ++l) s -= A[i + l * SM] * R2[l + (size_t)j * rmax];
        double d = R2[j + (size_t)j * rmax];
        A[i + j * SM] = (d != 0.0) ? s / d : 0.0;
      }
    }
  }
  __syncthreads();
  jacobi_svd_lds(A, V, n, nullptr, red);
  __syncthreads();
  order_desc(A, n, sv, ord);
  const double smax = sv[ord[0]];
  int kk = 0;
  if (smax > 0.0 && isfinite(smax)) {
    while (kk < n && sv[ord[kk]] > eps * smax) ++kk;
  } else if (!isfinite(smax)) {
    if (tid == 0) atomicOr(status, STAT_NONFINITE);
  }
  if (kk > J.cap) {
    if (tid == 0) atomicOr(status, STAT_RANK_OVERFLOW);
    kk = J.cap;
  }
  if (J.kind == SK_SKETCH_F && J.sat.maxv >= 0) {
    int sat = dimv(dyn, J.sat);
    if (kk >= sat && tid == 0) atomicOr(status, STAT_SKETCH_SAT);
  }
  if (J.kind == SK_RECOMP) {
    // A V = X S: X_k = A[:,ord]/s ; Y = V[:, ord]
    // CU = R2^T Y_k (n x kk), CV = R1^T X_k S_k^{-1} = R1^T A[:,ord] / s^2
    double* __restrict__ C2 = refp(bufs, J.C2);
    for (int e = tid; e < n * kk; e += 256) {
      int i = e % n, c = e / n;
      int oc = ord[c];
      double s = sv[oc];
      double cu = 0.0, cv = 0.0;
      for (int l = 0; l <= i; ++l) {
        cu += R2[l + (size_t)i * rmax] * V[l + oc * SM];
        cv += R1[l + (size_t)i * rmax] * A[l + oc * SM];
      }
      C1[i + (size_t)c * rmax] = cu;
      C2[i + (size_t)c * rmax] = cv / (s * s);
    }
  } else if (J.kind == SK_SKETCH_P) {
    // P = W_k S_k^{-1}: columns ord[0..kk)
    for (int e = tid; e < n * kk; e += 256) {
      int i = e % n, c = e / n;
      int oc = ord[c];
      C1[i + (size_t)c * rmax] = V[i + oc * SM] / sv[oc];
    }
  } else {
    // C = R2^{-1} Z_k, Z = V[:, ord]; back substitution per column
    for (int c = tid; c < kk; c += 256) {
      int oc = ord[c];
      for (int i = n - 1; i >= 0; --i) {
        double s = V[i + oc * SM];
        for (int l = i + 1; l < n; ++l) s -= R2[i + (size_t)l * rmax] * C1[l + (size_t)c * rmax];
        double d = R2[i + (size_t)i * rmax];
        C1[i + (size_t)c * rmax] = (d != 0.0) ? s / d : 0.0;
      }
    }
  }
  if (tid == 0) dyn[J.out_rank_slot] = kk;
}

// ------------------------------------------------------------------ leaf
// Dense leaf target: each thread owns an 8 x 8 block of the (<=128 x 128)
// tile in registers; term factors are staged through LDS 16 columns at a
// time.  Diagonal targets are then Cholesky-factorised in LDS.
constexpr int LF = 128, LFK = 16;

__global__ __launch_bounds__(256) void k_leaf(Bufs bufs, const int* __restrict__ dyn,
                                              const LeafJob* __restrict__ jobs,
                                              const LeafTerm* __restrict__ terms, int j0,
                                              double* __restrict__ logdet, int* __restrict__ status) {
  const LeafJob J = jobs[j0 + blockIdx.x];
  extern __shared__ double smem[];
  double* Us = smem;                    // LFK x LF
  double* Vs = smem + LFK * LF;         // LFK x LF
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double* __restrict__ Dp = refp(bufs, J.D);
  const int ldd = J.D.ld, p = J.p, q = J.q;
  double acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      int i = ty * 8 + a, j = tx * 8 + b;
      acc[a][b] = (i < p && j < q) ? Dp[i + (size_t)j * ldd] : 0.0;
    }
  for (int t = J.t0; t < J.t1; ++t) {
    const LeafTerm T = terms[t];
    const int k = dimv(dyn, T.k);
    if (k <= 0) continue;
    const double* __restrict__ U = refp(bufs, T.U);
    const double* __restrict__ V = refp(bufs, T.V);
    const int ldu = T.U.ld, ldv = T.V.ld;
    for (int k0 = 0; k0 < k; k0 += LFK) {
      for (int e = tid; e < LFK * LF; e += 256) {
        int i = e & (LF - 1), kk = e >> 7;
        int gk = k0 + kk;
        // row i of the tile -> row i - i0 of U
        int li = i - T.i0, lj = i - T.j0;
        Us[kk * LF + i] = (li >= 0 && li < T.mi && gk < k) ? U[li + (size_t)gk * ldu] : 0.0;
        Vs[kk * LF + i] = (lj >= 0 && lj < T.nj && gk < k) ? V[lj + (size_t)gk * ldv] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < LFK; ++kk) {
        double a[8], b[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
          a[x] = Us[kk * LF + ty * 8 + x];
          b[x] = Vs[kk * LF + tx * 8 + x];
        }
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
          for (int y = 0; y < 8; ++y) acc[x][y] = fma(-a[x], b[y], acc[x][y]);
      }
      __syncthreads();
    }
  }
  if (!J.diag) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        int i = ty * 8 + a, j = tx * 8 + b;
        if (i < p && j < q) Dp[i + (size_t)j * ldd] = acc[a][b];
      }
    return;
  }
  // potrf in LDS (lower), M col-major LF x LF
  double* M = smem;   // reuse (LF*LF doubles = 128 KiB)
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      int i = ty * 8 + a, j = tx * 8 + b;
      M[i + j * LF] = acc[a][b];
    }
  __shared__ int bad;
  if (tid == 0) bad = -1;
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    double d = M[j + j * LF];
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) bad = j;
      __syncthreads();
      break;
    }
    double ljj = sqrt(d);
    double inv = 1.0 / ljj;
    __syncthreads();
    for (int i = j + 1 + tid; i < p; i += 256) M[i + j * LF] *= inv;
    if (tid == 0) M[j + j * LF] = ljj;
    __syncthreads();
    // trailing update of the lower part: columns c in (j, p), rows i >= c
    int w = p - j - 1;
    for (int e = tid; e < w * w; e += 256) {
      int ii = e % w, cc = e / w;
      int i = j + 1 + ii, c = j + 1 + cc;
      if (i >= c) M[i + c * LF] -= M[i + j * LF] * M[c + j * LF];
    }
    __syncthreads();
  }
  if (bad >= 0) {
    if (tid == 0) {
      atomicOr(status, STAT_NOT_SPD);
      atomicMin(status + 1, (int)(J.row0 + bad));
      logdet[J.leaf] = NAN;
    }
    return;
  }
  for (int e = tid; e < p * p; e += 256) {
    int i = e % p, j = e / p;
    Dp[i + (size_t)j * ldd] = (i >= j) ? M[i + j * LF] : 0.0;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < p; ++j) s += log(M[j + j * LF]);
    logdet[J.leaf] = s;
  }
}

// ------------------------------------------------------------------ trsm
// One wave per job: lower triangle of L packed in LDS, each lane owns one
// right-hand-side column.  layout 0: X col-major (p x nc); layout 1: X^T
// stored (element (i,c) at X[c + i*ld]); layout 2: solve L^T x = b.
__global__ __launch_bounds__(64) void k_trsm(Bufs bufs, const int* __restrict__ dyn,
                                             const TrsmJob* __restrict__ jobs, int j0) {
  const TrsmJob J = jobs[j0 + blockIdx.x];
  const int nc = dimv(dyn, J.ncols);
  const int cw = min(J.cw, nc - J.c0);
  if (cw <= 0) return;
  extern __shared__ double smem[];
  const int p = J.p;
  double* Lp = smem;                       // packed lower: row i at i(i+1)/2
  double* Xs = smem + LF * (LF + 1) / 2;   // p x 64 (col-major, ld LF)
  const double* __restrict__ L = refp(bufs, J.L);
  const int ldl = J.L.ld;
  const int lane = threadIdx.x;
  for (int e = lane; e < p * p; e += 64) {
    int i = e % p, j = e / p;
    if (i >= j) Lp[i * (i + 1) / 2 + j] = L[i + (size_t)j * ldl];
  }
  double* __restrict__ X = refp(bufs, J.X);
  const int ldx = J.X.ld;
  const int c = J.c0 + lane;
  if (lane < cw) {
    for (int i = 0; i < p; ++i)
      Xs[i + lane * LF] = (J.layout == 1) ? X[c + (size_t)i * ldx] : X[i + (size_t)c * ldx];
  }
  __syncthreads();
  if (lane < cw) {
    double* x = Xs + lane * LF;
    if (J.layout != 2) {
      for (int i = 0; i < p; ++i) {
        double s = x[i];
        const double* Li = Lp + i * (i + 1) / 2;
        for (int j = 0; j < i; ++j) s -= Li[j] * x[j];
        x[i] = s / Li[i];
      }
    } else {
      for (int i = p - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j < p; ++j) s -= Lp[j * (j + 1) / 2 + i] * x[j];
        x[i] = s / Lp[i * (i + 1) / 2 + i];
      }
    }
    for (int i = 0; i < p; ++i) {
      if (J.layout == 1)
        X[c + (size_t)i * ldx] = x[i];
      else
        X[i + (size_t)c * ldx] = x[i];
    }
  }
}

// ------------------------------------------------------------------ assembly
__global__ __launch_bounds__(256) void k_dense_fill(double* __restrict__ D, const double2* __restrict__ loc,
                                                    const FillJob* __restrict__ jobs, MaternParams P) {
  const FillJob J = jobs[blockIdx.x];
  double* __restrict__ T = D + J.off;
  const int pq = J.p * J.q;
  for (int e = threadIdx.x; e < pq; e += 256) {
    int i = e % J.p, j = e / J.p;
    double2 a = loc[J.r0 + i], b = loc[J.c0 + j];
    double dx = a.x - b.x, dy = a.y - b.y;
    double h = sqrt(dx * dx + dy * dy);
    double v = matern_eval(h, P);
    if (J.diag && i == j) v += P.nugget;
    T[e] = v;
  }
}

// Block-wide argmax of |v| with ties to the lowest index.
__device__ void argmax_abs(double v, int idx, double* sval, int* sidx, double& out_v, int& out_i) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double a = fabs(v);
  int ix = idx;
  for (int o = 32; o > 0; o >>= 1) {
    double a2 = __shfl_down(a, o);
    int i2 = __shfl_down(ix, o);
    if (a2 > a || (a2 == a && i2 < ix)) {
      a = a2;
      ix = i2;
    }
  }
  if (lane == 0) {
    sval[wave] = a;
    sidx[wave] = ix;
  }
  __syncthreads();
  if (tid == 0) {
    double b = sval[0];
    int bi = sidx[0];
    for (int w = 1; w < 4; ++w)
      if (sval[w] > b || (sval[w] == b && sidx[w] < bi)) {
        b = sval[w];
        bi = sidx[w];
      }
    sval[4] = b;
    sidx[4] = bi;
  }
  __syncthreads();
  out_v = sval[4];
  out_i = sidx[4];
  __syncthreads();
}

__device__ double block_sum(double v, double* s8) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  if (lane == 0) s8[wave] = v;
  __syncthreads();
  double r = (s8[0] + s8[1]) + (s8[2] + s8[3]);
  __syncthreads();
  return r;
}

// Partially pivoted ACA (Bebendorf 2000) on C(rows r0.., cols c0..) with the
// exact incremental Frobenius norm of the approximant; stops when
// ||u_k|| ||v_k|| <= eps_aca ||S_k||_F, at min(p,q) or at the capacity.
__global__ __launch_bounds__(256) void k_aca(double* __restrict__ Ub, double* __restrict__ Vb,
                                             int* __restrict__ dyn, const double2* __restrict__ loc,
                                             const AcaJob* __restrict__ jobs, MaternParams P,
                                             double eps_aca, int kcap, int* __restrict__ status) {
  const AcaJob J = jobs[blockIdx.x];
  double* __restrict__ U = Ub + J.off_u;
  double* __restrict__ V = Vb + J.off_v;
  const int p = J.p, q = J.q;
  const int tid = threadIdx.x;
  __shared__ double rowU[64], colV[64];
  __shared__ double sval[8];
  __shared__ int sidx[8];
  __shared__ int used[128];
  __shared__ double s8[8];
  __shared__ double dots[2][64];
  int nused = 0;
  int i = 0;
  int k = 0;
  double nrm2 = 0.0;
  const int kmax = min(min(p, q), kcap);
  int attempts = 0;
  while (k < kmax && attempts < p + 1) {
    ++attempts;
    // pivot row i: residual r_j = C(i, j) - sum_l U[i,l] V[j,l]
    if (tid < k) rowU[tid] = U[i + (size_t)tid * p];
    if (tid == 0 && nused < 128) used[nused] = i;
    nused = min(nused + 1, 128);
    __syncthreads();
    const double2 xi = loc[J.r0 + i];
    double best = -1.0;
    int bj = 0;
    double* vk = V + (size_t)k * q;
    for (int j = tid; j < q; j += 256) {
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
    }
    double pv;
    int js;
    argmax_abs(best < 0 ? 0.0 : best, best < 0 ? 0x7fffffff : bj, sval, sidx, pv, js);
    if (!(pv > 0.0) || !isfinite(pv)) {
      if (!isfinite(pv) && tid == 0) atomicOr(status, STAT_NONFINITE);
      // zero residual row: take the next row not used yet
      int nxt = -1;
      for (int c = 0; c < p && nxt < 0; ++c) {
        bool u = false;
        for (int x = 0; x < nused; ++x) u |= (used[x] == c);
        if (!u) nxt = c;
      }
      if (nxt < 0 || !isfinite(pv)) break;
      i = nxt;
      continue;
    }
    const double piv = vk[js];
    const double ipiv = 1.0 / piv;
    __syncthreads();
    for (int j = tid; j < q; j += 256) vk[j] *= ipiv;
    if (tid < k) colV[tid] = V[js + (size_t)tid * q];
    __syncthreads();
    // column: u_i = C(i, js) - sum_l V[js,l] U[i,l]
    const double2 yj = loc[J.c0 + js];
    double* uk = U + (size_t)k * p;
    double bu = -1.0;
    int bi = 0;
    for (int r = tid; r < p; r += 256) {
      double2 x = loc[J.r0 + r];
      double dx = x.x - yj.x, dy = x.y - yj.y;
      double u = matern_eval(sqrt(dx * dx + dy * dy), P);
      for (int l = 0; l < k; ++l) u -= colV[l] * U[r + (size_t)l * p];
      uk[r] = u;
      double a = fabs(u);
      if (a > bu) {
        bu = a;
        bi = r;
      }
    }
    __syncthreads();
    // norms: ||u||^2, ||v||^2 and cross terms with the previous columns
    double su = 0.0, sv2 = 0.0;
    for (int r = tid; r < p; r += 256) su += uk[r] * uk[r];
    for (int j = tid; j < q; j += 256) sv2 += vk[j] * vk[j];
    su = block_sum(su, s8);
    sv2 = block_sum(sv2, s8);
    double cross = 0.0;
    for (int l = 0; l < k; ++l) {
      double a = 0.0, b = 0.0;
      for (int r = tid; r < p; r += 256) a += U[r + (size_t)l * p] * uk[r];
      for (int j = tid; j < q; j += 256) b += V[j + (size_t)l * q] * vk[j];
      a = block_sum(a, s8);
      b = block_sum(b, s8);
      cross += a * b;
    }
    const double nuv = su * sv2;
    nrm2 += nuv + 2.0 * cross;
    ++k;
    if (sqrt(nuv) <= eps_aca * sqrt(fmax(nrm2, 0.0))) break;
    // next row: argmax |u| over rows not used yet
    double bv;
    int ni;
    argmax_abs(bu < 0 ? 0.0 : bu, bu < 0 ? 0x7fffffff : bi, sval, sidx, bv, ni);
    bool isused = false;
    for (int x = 0; x < nused; ++x) isused |= (used[x] == ni);
    if (isused || !(bv > 0.0)) {
      int nxt = -1;
      for (int c = 0; c < p && nxt < 0; ++c) {
        bool u = false;
        for (int x = 0; x < nused; ++x) u |= (used[x] == c);
        if (!u) nxt = c;
      }
      if (nxt < 0) break;
      ni = nxt;
    }
    i = ni;
  }
  if (k == kmax && kmax < min(p, q) && tid == 0) atomicOr(status, STAT_RANK_OVERFLOW);
  if (tid == 0) dyn[J.rank_slot] = k;
  (void)dots;
}

// ------------------------------------------------------------------ utilities
__global__ void k_copy_rank(int* __restrict__ dyn, const int2* __restrict__ pairs, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dyn[pairs[i].y] = dyn[pairs[i].x];
}

// out[i] = in[perm[i]] (gather) or out[perm[i]] = in[i] (scatter)
__global__ void k_permute(const double* __restrict__ in, double* __restrict__ out,
                          const int* __restrict__ perm, int64_t n, int scatter) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (scatter)
    out[perm[i]] = in[i];
  else
    out[i] = in[perm[i]];
}

// Fixed-order FP64 reduction: partial sums of x[i]^2 (mode 0) or x[i]
// (mode 1) per block of 1024, written to part[]; the host (or a second
// launch with one block) finishes in block order.
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ x, int64_t n, int mode,
                                                double* __restrict__ part) {
  __shared__ double s8[8];
  int64_t base = (int64_t)blockIdx.x * 1024;
  double s = 0.0;
  for (int r = 0; r < 4; ++r) {
    int64_t i = base + threadIdx.x + 256 * r;
    if (i < n) {
      double v = x[i];
      s += mode == 0 ? v * v : v;
    }
  }
  s = block_sum(s, s8);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_matern_probe(const double* __restrict__ h, double* __restrict__ out, int64_t n,
                               MaternParams P) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = matern_eval(h[i], P);
}


// counter-based standard normals: splitmix64 bits, Box-Muller pairs
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__global__ void k_gaussian(double* __restrict__ out, int64_t n, uint64_t seed) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t pair = i >> 1;
  uint64_t a = splitmix64(seed ^ (2 * (uint64_t)pair));
  uint64_t b = splitmix64(seed ^ (2 * (uint64_t)pair + 1));
  double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);   // (0, 1]
  double u2 = (b >> 11) * (1.0 / 9007199254740992.0);           // [0, 1)
  double r = sqrt(-2.0 * log(u1));
  double ang = 6.283185307179586 * u2;
  out[i] = (i & 1) ? r * sin(ang) : r * cos(ang);
}
__global__ void k_fill_value(double* __restrict__ out, int64_t n, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

constexpr size_t LDS_QR = (size_t(LDM) * QR_CMAX + 8) * 8;
constexpr size_t LDS_SMALL = (size_t(2) * SM * SM + SM + 8) * 8 + SM * 4;
constexpr size_t LDS_LEAF = size_t(LF) * LF * 8;
constexpr size_t LDS_TRSM = (size_t(LF) * (LF + 1) / 2 + size_t(LF) * 64) * 8;

hipError_t setup_kernel_attributes() {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_tsqr_seg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_QR);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_tsqr_red, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_QR);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_small, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_SMALL);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_leaf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_LEAF);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_trsm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_TRSM);
  return e;
}

hipError_t launch_stage(const Stage& s, const LaunchCtx& L, hipStream_t st) {
  const int n = s.end - s.begin;
  switch (s.kind) {
    case ST_GEMM:
      if (n > 0) k_gemm<<<n, 256, 0, st>>>(L.bufs, L.dyn, L.gjobs, L.gprods, L.gtiles, s.begin);
      break;
    case ST_TSQR_SEG:
      if (n > 0) k_tsqr_seg<<<n, 256, LDS_QR, st>>>(L.bufs, L.dyn, L.tsegs, s.begin, L.rmax);
      break;
    case ST_TSQR_RED:
      if (n > 0) k_tsqr_red<<<n, 256, LDS_QR, st>>>(L.bufs, L.dyn, L.treds, s.begin, L.rmax);
      break;
    case ST_SMALL:
      if (n > 0)
        k_small<<<n, 256, LDS_SMALL, st>>>(L.bufs, L.dyn, L.smalls, s.begin, L.rmax, L.eps, L.tau, L.status);
      break;
    case ST_LEAF:
      if (n > 0) k_leaf<<<n, 256, LDS_LEAF, st>>>(L.bufs, L.dyn, L.leafs, L.lterms, s.begin, L.logdet, L.status);
      break;
    case ST_TRSM:
      if (n > 0) k_trsm<<<n, 64, LDS_TRSM, st>>>(L.bufs, L.dyn, L.trsms, s.begin);
      break;
    case ST_COPY_RANK:
      if (L.n_copy > 0) k_copy_rank<<<(L.n_copy + 255) / 256, 256, 0, st>>>(L.dyn, L.copy_pairs, L.n_copy);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill(double* D, const double* loc, const FillJob* jobs, int njobs, const MaternParams& P,
                       hipStream_t st) {
  if (njobs > 0) k_dense_fill<<<njobs, 256, 0, st>>>(D, (const double2*)loc, jobs, P);
  return hipGetLastError();
}

hipError_t launch_aca(double* U, double* V, int* dyn, const double* loc, const AcaJob* jobs, int njobs,
                      const MaternParams& P, double eps_aca, int kcap, int* status, hipStream_t st) {
  if (njobs > 0) k_aca<<<njobs, 256, 0, st>>>(U, V, dyn, (const double2*)loc, jobs, P, eps_aca, kcap, status);
  return hipGetLastError();
}

hipError_t launch_permute(const double* in, double* out, const int* perm, int64_t n, int scatter,
                          hipStream_t st) {
  if (n > 0) k_permute<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(in, out, perm, n, scatter);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* x, int64_t n, int mode, double* part, hipStream_t st, int64_t* nparts) {
  int64_t nb = (n + 1023) / 1024;
  *nparts = nb;
  if (nb > 0) k_reduce<<<(unsigned)nb, 256, 0, st>>>(x, n, mode, part);
  return hipGetLastError();
}

hipError_t launch_probe(const double* h, double* out, int64_t n, const MaternParams& P, hipStream_t st) {
  if (n > 0) k_matern_probe<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(h, out, n, P);
  return hipGetLastError();
}

hipError_t launch_gaussian(double* out, int64_t n, uint64_t seed, hipStream_t st) {
  if (n > 0) k_gaussian<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, n, seed);
  return hipGetLastError();
}

hipError_t launch_fill_value(double* out, int64_t n, double v, hipStream_t st) {
  if (n > 0) k_fill_value<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, n, v);
  return hipGetLastError();
}

}  // namespace hc
