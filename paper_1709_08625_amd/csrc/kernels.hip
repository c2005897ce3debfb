// Batched device kernels of the H-matrix likelihood (gfx950, FP64).
//
//   k_gemm       grouped sum-of-products GEMM over variable-size jobs
//   k_tsqr_seg   Householder R factor of a row segment of a tall matrix
//   k_tsqr_red   R factor of a stack of segment R factors
//   k_small      one-sided Jacobi SVDs of the small R-factor products
//                (recompression and randomised-sketch truncation)
//   k_leaf       dense leaf targets: partial-sum update, blocked potrf
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
// the tile, accumulating all products of the job in registers.  Thread
// (ty, tx) owns rows ty + 16x and columns tx + 16y of the tile; when the
// live part of the tile (ranks are known only at run time) is at most 16 or
// 32 rows/columns wide, only NX x NY of the 4 x 4 sub-tile are computed.
// k is streamed through LDS in chunks of GK with the next chunk's global
// loads in flight in registers while the current one is consumed.
constexpr int GT = 64, GK = 32;
constexpr int GR = GK * GT / 256;   // elements of each operand chunk per thread

// Products of a job, resolved once per batch into LDS: operand base
// pointers, leading dimensions, live dimensions and the intersection with
// the tile.  This replaces the per-product chain of dependent loads
// (descriptor -> dynamic dimensions -> buffer table -> data).
// Values known to be equal in every lane, moved to scalar registers.
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_dbl(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(u & 0xffffffffull));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(u >> 32));
  return reinterpret_cast<T*>((static_cast<unsigned long long>(hi) << 32) | lo);
}

constexpr int PBATCH = 32;
struct ProdMeta {
  const double* A;
  const double* B;
  double alpha;
  int lda, ldb, k;
  int pr0, pr1, pc0, pc1;
  int ta, tb;
  int live;
};

// The product pipeline of a tile, shared by the vector and matrix-core
// bodies: products are taken in batches of PBATCH descriptors; element-wise
// additions (tb == 2) go to on_add(M); every other live product streams its
// k range through LDS in chunks of GK, the next (product, chunk) pair's
// global loads in flight while on_chunk(kl) consumes the current chunk.
//
// With G > 1 groups of 256 threads (a work-group of 256 G threads) the
// groups share the descriptors and work in lockstep on their own LDS chunk
// buffers (As, Bs point to the calling group's): group g takes the pairs and
// the additions whose index in the tile's order is g mod G, so G chunks of
// one tile are in flight at once.  Each group accumulates its own partial
// sum; the caller adds them in group order.
template <class T, int G = 1, class AddF, class ChunkF>
__device__ __forceinline__ void gemm_products(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                              const GemmJob& J, const GemmProd* __restrict__ prods, int m,
                                              int n, int r0, int c0, T (*As)[GT + 1], T (*Bs)[GT + 1],
                                              ProdMeta* pm, AddF on_add, ChunkF on_chunk) {
  const int tid = threadIdx.x & 255;
  const int grp = G > 1 ? uniform_int(int(threadIdx.x >> 8)) : 0;
  // element e of a chunk: A chunk is GT x GK, B chunk GK x GT; the index
  // split follows the operand's storage order so that lanes coalesce.  The
  // loads of the next chunk stay in flight while the current one is used.
  // They are buffer loads over a 2 GiB range from the operand's start
  // (scalar base, 32-bit lane offset): an element outside the product's
  // extent gets the offset 2^31, outside that range, and the hardware
  // returns 0 for it without an access, so a chunk arrives masked and goes
  // to LDS as it is.  Descriptor
  // fields are the same in every lane: scalar registers, so that the
  // operand layout is one uniform branch.
  double ra[GR], rb[GR];
  // element r of a thread: with the operand's leading index contiguous
  // (ta == 0 / tb == 1) the thread keeps index tid % 64 and takes k steps of
  // 4 (k = tid / 64 + 4 r); with k contiguous it keeps k = tid % 32 and takes
  // index steps of 8 (tid / 32 + 8 r).  Either way element r sits at a
  // fixed per-thread byte offset plus r times a uniform stride (the planner
  // keeps every operand below 2^28 elements, so a real offset stays below
  // 2^31 - 8), and a range check is one compare.
  auto fetch_op = [&](const double* base, int lead_major, int ld, int lo, int hi, int g0, int kp, int k0,
                      double* dst) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)0x80000000u, 0x00020000);
    if (lead_major) {
      const int gi = g0 + (tid & (GT - 1));
      const bool iok = unsigned(gi - lo) < unsigned(hi - lo);
      const int kb = k0 + (tid >> 6);
      const unsigned off0 = (unsigned(gi - lo) + unsigned(kb) * unsigned(ld)) * 8u;
      const unsigned step = 32u * unsigned(ld);
#pragma unroll
      for (int r = 0; r < GR; ++r) {
        const bool ok = iok && kb + 4 * r < kp;
        const unsigned off = ok ? off0 + unsigned(r) * step : 0x80000000u;
        dst[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
      }
    } else {
      const int gk = k0 + (tid & (GK - 1));
      const bool kok = gk < kp;
      const int ib = g0 + (tid >> 5) - lo;
      const unsigned off0 = (unsigned(gk) + unsigned(ib) * unsigned(ld)) * 8u;
      const unsigned step = 64u * unsigned(ld);
#pragma unroll
      for (int r = 0; r < GR; ++r) {
        const bool ok = kok && unsigned(ib + 8 * r) < unsigned(hi - lo);
        const unsigned off = ok ? off0 + unsigned(r) * step : 0x80000000u;
        dst[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
      }
    }
  };
  auto fetch = [&](const ProdMeta& M, int k0) {
    const int kp = uniform_int(M.k);
    fetch_op(uniform_ptr(M.A), uniform_int(M.ta) == 0, uniform_int(M.lda), uniform_int(M.pr0), uniform_int(M.pr1),
             r0, kp, k0, ra);
    fetch_op(uniform_ptr(M.B), uniform_int(M.tb) == 1, uniform_int(M.ldb), uniform_int(M.pc0), uniform_int(M.pc1),
             c0, kp, k0, rb);
  };
  const ProdMeta* pmc = pm;
  auto stash = [&](const ProdMeta& M) {
    const int ta = uniform_int(M.ta), tb = uniform_int(M.tb);
    const double alpha = uniform_dbl(M.alpha);
    T* __restrict__ Af = &As[0][0];
    T* __restrict__ Bf = &Bs[0][0];
    // element r of the leading-index-contiguous layout lands at
    // [tid / 64 + 4 r][tid % 64], of the k-contiguous one at
    // [tid % 32][tid / 32 + 8 r]: a per-thread base and an immediate offset
    const int lead0 = (tid >> 6) * (GT + 1) + (tid & (GT - 1));
    const int kmaj0 = (tid & (GK - 1)) * (GT + 1) + (tid >> 5);
    if (alpha != 1.0) {
#pragma unroll
      for (int r = 0; r < GR; ++r) ra[r] *= alpha;
    }
    if (ta == 0) {
#pragma unroll
      for (int r = 0; r < GR; ++r) Af[lead0 + 4 * r * (GT + 1)] = T(ra[r]);
    } else {
#pragma unroll
      for (int r = 0; r < GR; ++r) Af[kmaj0 + 8 * r] = T(ra[r]);
    }
    if (tb == 1) {
#pragma unroll
      for (int r = 0; r < GR; ++r) Bf[lead0 + 4 * r * (GT + 1)] = T(rb[r]);
    } else {
#pragma unroll
      for (int r = 0; r < GR; ++r) Bf[kmaj0 + 8 * r] = T(rb[r]);
    }
  };

  // pairs and additions of the earlier batches, modulo G
  int gpair = 0, gadd = 0;
  for (int base = J.p0; base < J.p1; base += PBATCH) {
    const int cnt = min(PBATCH, J.p1 - base);
    __syncthreads();   // the previous batch is consumed
    if (grp == 0 && tid < cnt) {
      const GemmProd Pd = prods[base + tid];
      ProdMeta M;
      M.k = dimv(dyn, Pd.k);
      const int mi = dimv(dyn, Pd.mi), nj = dimv(dyn, Pd.nj);
      M.pr0 = Pd.i0;
      M.pr1 = min(Pd.i0 + mi, m);
      M.pc0 = Pd.j0;
      M.pc1 = min(Pd.j0 + nj, n);
      M.live = (M.k > 0 && mi > 0 && nj > 0 && M.pr1 > r0 && M.pr0 < r0 + GT && M.pc1 > c0 && M.pc0 < c0 + GT) ? 1 : 0;
      M.A = refp(bufs, Pd.A);
      M.B = refp(bufs, Pd.B);
      M.lda = Pd.A.ld;
      M.ldb = Pd.B.ld;
      M.alpha = Pd.alpha;
      M.ta = Pd.ta;
      M.tb = Pd.tb;
      pm[tid] = M;
    }
    __syncthreads();
    // live products and live element-wise additions of partial sums
    // (tb == 2) of the batch as bit masks, the same in every wave
    bool is_prod = false, is_add = false;
    if ((tid & 63) < cnt) {
      const ProdMeta& M = pmc[tid & 63];
      is_prod = M.live && M.tb != 2;
      is_add = M.live && M.tb == 2;
    }
    const unsigned long long prod_mask = __ballot(is_prod), add_mask = __ballot(is_add);
    for (unsigned long long am = add_mask; am != 0ull; am &= am - 1ull) {
      if (gadd == grp) on_add(pmc[__ffsll((long long)am) - 1]);
      if (G > 1) gadd = gadd + 1 == G ? 0 : gadd + 1;
    }
    // products: (product, k-chunk) pairs in order
    auto next_live = [&](int q) {
      const unsigned long long rest = q < 64 ? prod_mask & (~0ull << q) : 0ull;
      return rest != 0ull ? __ffsll((long long)rest) - 1 : cnt;
    };
    if constexpr (G == 1) {
      int q = next_live(0);
      if (q >= cnt) continue;
      int k0 = 0;
      fetch(pmc[q], 0);
      while (q < cnt) {
        if (k0 > 0 || q > 0) __syncthreads();   // LDS tiles of the previous pair consumed
        stash(pmc[q]);
        __syncthreads();
        int nq = q, nk0 = k0 + GK;
        if (nk0 >= pmc[q].k) {
          nq = next_live(q + 1);
          nk0 = 0;
        }
        if (nq < cnt) fetch(pmc[nq], nk0);
        on_chunk(min(GK, pmc[q].k - k0));
        q = nq;
        k0 = nk0;
      }
    } else {
      // (q, k0) moved d pairs on over the live products of the batch
      auto advance = [&](int& q, int& k0, int d) {
        while (q < cnt) {
          const int left = (uniform_int(pmc[q].k) - k0 + GK - 1) / GK;   // pairs from (q, k0) to the end of q
          if (d < left) {
            k0 += d * GK;
            return;
          }
          d -= left;
          q = next_live(q + 1);
          k0 = 0;
        }
      };
      int total = 0;
      for (unsigned long long pmk = prod_mask; pmk != 0ull; pmk &= pmk - 1ull)
        total += (uniform_int(pmc[__ffsll((long long)pmk) - 1].k) + GK - 1) / GK;
      int q = next_live(0), k0 = 0;
      advance(q, k0, grp >= gpair ? grp - gpair : grp - gpair + G);
      gpair = (gpair + total) % G;
      // rounds of the batch: every group stashes and consumes one pair per
      // round; a group without a pair left takes a chunk of the batch's
      // first live product and consumes none of it (no branches
      // around the pipeline, which keeps its registers as in the plain kernel)
      const int rounds = (total + G - 1) / G;
      if (rounds == 0) continue;
      const int qfirst = next_live(0);
      fetch(pmc[q < cnt ? q : qfirst], q < cnt ? k0 : 0);
      for (int rd = 0; rd < rounds; ++rd) {
        if (rd > 0) __syncthreads();   // LDS tiles of the previous round consumed
        const bool real = q < cnt;
        stash(pmc[real ? q : qfirst]);
        __syncthreads();
        int nq = q, nk0 = k0, kl = 0;
        if (real) {
          kl = min(GK, uniform_int(pmc[q].k) - k0);
          advance(nq, nk0, G);
        }
        fetch(pmc[nq < cnt ? nq : qfirst], nq < cnt ? nk0 : 0);
        on_chunk(kl);
        q = nq;
        k0 = nk0;
      }
    }
  }
}

// Vector body: thread (ty, tx) accumulates rows ty + 16 x and columns
// tx + 16 y of the tile (FP32 in mixed precision).
template <class T, int NX, int NY>
__device__ __forceinline__ void gemm_tile(const Bufs* __restrict__ bufs, const int* __restrict__ dyn, const GemmJob& J,
                                          const GemmProd* __restrict__ prods, int m, int n, int r0,
                                          int c0, T (*As)[GT + 1], T (*Bs)[GT + 1], ProdMeta* pm) {
  const int tid = threadIdx.x;
  const int ty = tid & 15, tx = tid >> 4;   // rows follow the lane index (coalesced C and tb==2 access)
  T acc[NX][NY];
#pragma unroll
  for (int a = 0; a < NX; ++a)
#pragma unroll
    for (int b = 0; b < NY; ++b) acc[a][b] = T(0);
  auto on_add = [&](const ProdMeta& M) {
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int y = 0; y < NY; ++y) {
        int gi = r0 + ty + 16 * x, gj = c0 + tx + 16 * y;
        if (gi >= M.pr0 && gi < M.pr1 && gj >= M.pc0 && gj < M.pc1)
          acc[x][y] += T(M.alpha * gmem(M.A)[(gi - M.pr0) + (size_t)(gj - M.pc0) * M.lda]);
      }
  };
  auto on_chunk = [&](int kl) {
#pragma unroll 8
    for (int kk = 0; kk < kl; ++kk) {
      T av[NX], bv[NY];
#pragma unroll
      for (int z = 0; z < NX; ++z) av[z] = As[kk][ty + 16 * z];
#pragma unroll
      for (int z = 0; z < NY; ++z) bv[z] = Bs[kk][tx + 16 * z];
#pragma unroll
      for (int x = 0; x < NX; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y) acc[x][y] = fma(av[x], bv[y], acc[x][y]);
    }
  };
  gemm_products<T>(bufs, dyn, J, prods, m, n, r0, c0, As, Bs, pm, on_add, on_chunk);
  HC_GLOBAL double* __restrict__ C = gmem(refp(bufs, J.C));
  const int ldc = J.C.ld;
#pragma unroll
  for (int x = 0; x < NX; ++x) {
    int gi = r0 + ty + 16 * x;
    if (gi >= m) continue;
#pragma unroll
    for (int y = 0; y < NY; ++y) {
      int gj = c0 + tx + 16 * y;
      if (gj >= n) continue;
      size_t o = gi + (size_t)gj * ldc;
      C[o] = J.zero ? double(acc[x][y]) : C[o] + double(acc[x][y]);
    }
  }
}

// Matrix-core body (FP64): the live 16 x 16 blocks of the tile are spread
// over the four waves; with fewer than four blocks the waves of a block
// split its k steps and their partial sums are added in wave order at the
// end (deterministic).  Each step is one FP64 16x16x4 matrix instruction
// computing the transposed block, D' = B^T A^T, so that lane L holds the
// element (row L % 16, column 4 r + L / 16) of the block in its register r:
// sixteen consecutive rows of a column, a coalesced store.
//
// With G groups (gemm_products) each group runs this body on its own chunk
// buffers; at the end groups 1 .. G-1 hand their sums to group 0 through
// LDS (xred, 16 x 256 (G - 1) doubles), which adds them in group order and
// writes C.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// The k steps of one chunk for a wave holding NB blocks of one block row
// bi, in block columns bj0, bj0 + STRIDE, ...: step s (s = kpart, kpart +
// NSPLIT, ... < ns) multiplies rows 4 s .. 4 s + 3 of the chunk.  Every
// operand sits at a compile-time offset from two per-lane bases, so the
// loop is fully unrolled with no address arithmetic, and its LDS reads do
// not depend on the step guard (rows past the chunk's k are zero and in
// the buffer), so they can be issued ahead of the matrix instructions.
template <int NB, int STRIDE, int NSPLIT>
__device__ __forceinline__ void mfma_chunk(const double (*As)[GT + 1], const double (*Bs)[GT + 1], dbl4* acc,
                                           int bi, int bj0, int li, int lk, int kpart, int ns) {
  constexpr int NS = GK / 4 / NSPLIT;
  constexpr int ROW = 4 * NSPLIT * (GT + 1);
  const double* __restrict__ pa = &As[4 * kpart + lk][16 * bi + li];
  const double* __restrict__ pb = &Bs[4 * kpart + lk][16 * bj0 + li];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double a = pa[i * ROW];
    double b[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) b[t] = pb[i * ROW + 16 * STRIDE * t];
    if (kpart + i * NSPLIT < ns) {
#pragma unroll
      for (int t = 0; t < NB; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[t], a, acc[t], 0, 0, 0);
    }
  }
}

template <int G = 1>
__device__ __forceinline__ void gemm_tile_mfma(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                               const GemmJob& J, const GemmProd* __restrict__ prods, int m,
                                               int n, int r0, int c0, double (*As)[GT + 1], double (*Bs)[GT + 1],
                                               ProdMeta* pm, double* xred = nullptr) {
  const int tid = threadIdx.x & 255, wave = uniform_int(tid >> 6), lane = tid & 63;
  const int grp = G > 1 ? uniform_int(int(threadIdx.x >> 8)) : 0;
  const int li = lane & 15, lk = lane >> 4;
  const int er = min(GT, m - r0), ec = min(GT, n - c0);
  const int nbr = (er + 15) >> 4, nbc = (ec + 15) >> 4, nblk = nbr * nbc;
  const int nsplit = nblk == 1 ? 4 : (nblk == 2 ? 2 : 1);
  // blocks of a wave: one block row bi and nb block columns bj[t] = bj[0] +
  // stride t (16 x 16 blocks of the tile; a wave without blocks only joins
  // the barriers); a tile of one or two blocks splits their k steps over
  // nsplit waves instead
  int kpart = 0, nb = 0, stride = 1;
  int bi[4] = {0, 0, 0, 0}, bj[4] = {0, 0, 0, 0};
  if (nsplit > 1) {
    const int b = wave / nsplit;
    kpart = wave % nsplit;
    nb = 1;
    bi[0] = b % nbr;
    bj[0] = b / nbr;
  } else if (nbr >= 3) {
    nb = wave < nbr ? nbc : 0;
    bi[0] = wave;
  } else if (nbr == 2) {
    bi[0] = wave & 1;
    bj[0] = wave >> 1;
    nb = (nbc - bj[0] + 1) >> 1;
    stride = 2;
  } else {
    nb = wave < nbc ? 1 : 0;
    bj[0] = wave;
  }
#pragma unroll
  for (int t = 1; t < 4; ++t) {
    bi[t] = bi[0];
    bj[t] = bj[0] + stride * t;
  }
  dbl4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  auto on_add = [&](const ProdMeta& M) {
    if (kpart != 0) return;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < nb) {
        const int gi = r0 + 16 * bi[t] + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gj = c0 + 16 * bj[t] + 4 * r + lk;
          if (gi >= M.pr0 && gi < M.pr1 && gj >= M.pc0 && gj < M.pc1)
            acc[t][r] += M.alpha * gmem(M.A)[(gi - M.pr0) + (size_t)(gj - M.pc0) * M.lda];
        }
      }
    }
  };
  auto on_chunk = [&](int kl) {
    const int ns = (kl + 3) >> 2;
    if (nsplit == 4) {
      mfma_chunk<1, 1, 4>(As, Bs, acc, bi[0], bj[0], li, lk, kpart, ns);
    } else if (nsplit == 2) {
      mfma_chunk<1, 1, 2>(As, Bs, acc, bi[0], bj[0], li, lk, kpart, ns);
    } else if (stride == 2) {
      if (nb == 2)
        mfma_chunk<2, 2, 1>(As, Bs, acc, bi[0], bj[0], li, lk, 0, ns);
      else if (nb == 1)
        mfma_chunk<1, 1, 1>(As, Bs, acc, bi[0], bj[0], li, lk, 0, ns);
    } else {
      switch (nb) {
        case 4: mfma_chunk<4, 1, 1>(As, Bs, acc, bi[0], bj[0], li, lk, 0, ns); break;
        case 3: mfma_chunk<3, 1, 1>(As, Bs, acc, bi[0], bj[0], li, lk, 0, ns); break;
        case 2: mfma_chunk<2, 1, 1>(As, Bs, acc, bi[0], bj[0], li, lk, 0, ns); break;
        case 1: mfma_chunk<1, 1, 1>(As, Bs, acc, bi[0], bj[0], li, lk, 0, ns); break;
        default: break;
      }
    }
  };
  gemm_products<double, G>(bufs, dyn, J, prods, m, n, r0, c0, As, Bs, pm, on_add, on_chunk);
  if (nsplit > 1) {
    // partial sums of the k split: waves with kpart > 0 hand theirs over
    double* red = &As[0][0];
    __syncthreads();
    if (kpart > 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(wave * 4 + r) * 64 + lane] = acc[0][r];
    }
    __syncthreads();
    if (kpart == 0) {
      for (int w = 1; w < nsplit; ++w) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[0][r] += red[((wave + w) * 4 + r) * 64 + lane];
      }
    }
  }
  if constexpr (G > 1) {
    __syncthreads();   // every group's chunk buffers are free
    if (grp > 0 && kpart == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) xred[((grp - 1) * 16 + 4 * t + r) * 256 + tid] = acc[t][r];
        }
    }
    __syncthreads();
    if (grp > 0) return;
    if (kpart == 0) {
      for (int g = 1; g < G; ++g) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[t][r] += xred[((g - 1) * 16 + 4 * t + r) * 256 + tid];
          }
      }
    }
  }
  if (kpart != 0) return;
  HC_GLOBAL double* __restrict__ C = gmem(refp(bufs, J.C));
  const int ldc = J.C.ld;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t < nb) {
      const int gi = r0 + 16 * bi[t] + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gj = c0 + 16 * bj[t] + 4 * r + lk;
        if (gi < m && gj < n) {
          const size_t o = gi + (size_t)gj * ldc;
          C[o] = J.zero ? acc[t][r] : C[o] + acc[t][r];
        }
      }
    }
  }
}

// Two work-groups per CU (up to 256 registers a lane): the chunk loop keeps
// the next chunk's loads and the LDS operands of the coming k steps in
// registers, which costs more than the latency a third or fourth
// work-group would hide.
__global__ __launch_bounds__(256, 2) void k_gemm(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
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
  __shared__ ProdMeta pm[PBATCH];
  const int er = min(GT, m - r0), ec = min(GT, n - c0);
  const int nx = er <= 16 ? 1 : (er <= 32 ? 2 : 4), ny = ec <= 16 ? 1 : (ec <= 32 ? 2 : 4);
  if (J.fp32) {
    // mixed precision: FP32 tiles in the same LDS storage, FP32 accumulation
    float(*Af)[GT + 1] = reinterpret_cast<float(*)[GT + 1]>(&As[0][0]);
    float(*Bf)[GT + 1] = reinterpret_cast<float(*)[GT + 1]>(&Bs[0][0]);
    switch (nx * 8 + ny) {
      case 9: gemm_tile<float, 1, 1>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 10: gemm_tile<float, 1, 2>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 12: gemm_tile<float, 1, 4>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 17: gemm_tile<float, 2, 1>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 18: gemm_tile<float, 2, 2>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 20: gemm_tile<float, 2, 4>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 33: gemm_tile<float, 4, 1>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      case 34: gemm_tile<float, 4, 2>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
      default: gemm_tile<float, 4, 4>(bufs, dyn, J, prods, m, n, r0, c0, Af, Bf, pm); break;
    }
    return;
  }
  gemm_tile_mfma(bufs, dyn, J, prods, m, n, r0, c0, As, Bs, pm);
}

// One tile per work-group of GW groups of 256 threads (FP64 jobs only): the
// groups stream disjoint pairs of the tile in lockstep (gemm_products), so a
// tile with many k chunks takes about 1 / GW of the chunk rounds of k_gemm.
// A CU holds one such work-group; the planner uses this kernel for launches
// whose longest tiles, not their number, set the time.
constexpr int GW = GEMM_GROUPS;
constexpr size_t LDS_GEMM_WIDE = size_t(GW) * 2 * GK * (GT + 1) * 8;
static_assert(size_t(GW - 1) * 16 * 256 * 8 <= LDS_GEMM_WIDE, "group sums fit in the chunk buffers");
__global__ __launch_bounds__(256 * GW) void k_gemm_wide(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                                      const GemmJob* __restrict__ jobs,
                                                      const GemmProd* __restrict__ prods,
                                                      const GemmTile* __restrict__ tiles, int t0) {
  const GemmTile T = tiles[t0 + blockIdx.x];
  const GemmJob J = jobs[T.job];
  const int m = dimv(dyn, J.m), n = dimv(dyn, J.n);
  const int r0 = T.ti * GT, c0 = T.tj * GT;
  if (r0 >= m || c0 >= n) return;
  extern __shared__ double smem[];
  __shared__ ProdMeta pm[PBATCH];
  const int grp = int(threadIdx.x >> 8);
  double(*As)[GT + 1] = reinterpret_cast<double(*)[GT + 1]>(smem + size_t(grp) * 2 * GK * (GT + 1));
  double(*Bs)[GT + 1] = reinterpret_cast<double(*)[GT + 1]>(smem + size_t(grp) * 2 * GK * (GT + 1) + GK * (GT + 1));
  gemm_tile_mfma<GW>(bufs, dyn, J, prods, m, n, r0, c0, As, Bs, pm, smem);
}

// ------------------------------------------------------------------ TSQR
// Householder QR in LDS of an mrows x c matrix (col-major, leading dimension
// ldm chosen at run time so that as many rows as possible are reduced per
// pass).  On exit the leading c x c upper triangle holds R.
constexpr int QR_LDS = 160 * 96;     // doubles of the LDS matrix buffer
constexpr int QR_CMAX = 96;          // max columns

// Cross-lane moves inside a row of 16 lanes (DPP: a plain vector
// instruction, no LDS round trip), applied to both halves of a double.
// Every control used here is a permutation of the 16 lanes of a row, so
// each lane has a source and no fill value is needed.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15 - i within 16

__device__ __forceinline__ double wave_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over the 64 lanes of a wave, the same bits in every lane: DPP moves
// inside each row of 16 lanes, then the four row totals read as scalars.
__device__ __forceinline__ double wave_sum64(double v) {
  v += dpp_move<DPP_MIRROR>(v);
  v += dpp_move<DPP_HALF_MIRROR>(v);
  v += dpp_move<DPP_XOR2>(v);
  v += dpp_move<DPP_XOR1>(v);
  return (wave_bcast(v, 0) + wave_bcast(v, 16)) + (wave_bcast(v, 32) + wave_bcast(v, 48));
}

// Sum over each row of 16 lanes, the same bits in every lane of the row.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_move<DPP_MIRROR>(v);
  v += dpp_move<DPP_HALF_MIRROR>(v);
  v += dpp_move<DPP_XOR2>(v);
  v += dpp_move<DPP_XOR1>(v);
  return v;
}

// Largest value over the 64 lanes of a wave (NaN ignored), in every lane.
__device__ __forceinline__ double wave_max64(double v) {
  v = fmax(v, dpp_move<DPP_MIRROR>(v));
  v = fmax(v, dpp_move<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp_move<DPP_XOR2>(v));
  v = fmax(v, dpp_move<DPP_XOR1>(v));
  return fmax(fmax(wave_bcast(v, 0), wave_bcast(v, 16)), fmax(wave_bcast(v, 32), wave_bcast(v, 48)));
}

// Householder QR of an mrows x c matrix in LDS (col-major, leading dimension
// ldm >= 16 RR >= mrows; rows mrows .. 16 RR - 1 of every column are zero on
// entry and stay zero).  Lane 16 t + q of a wave holds rows q + 16 r of one
// column, so a row of 16 lanes reduces a dot product over the column with
// four DPP moves and a wave treats four columns at once: wave w applies the
// reflector of column j to columns j + 1 + 4 w + 16 g + t.  In registers the
// reflector keeps only the rows below j; row j enters through the element
// a_jl read by every lane (v^T a_l = sum_{i>j} x_i a_il + (x_j - alpha) a_jl)
// and is written by one lane.  One barrier per column: a step reads only
// columns >= j, and column j + 1 is final once the step on column j is.
// With KEEP the reflector tails stay below the diagonal, with the leading
// entry in vtop[j] and the scale in beta[j] (H_j = I - beta[j] v_j v_j^T);
// without it the leading min(c, mrows) rows are cleared below the diagonal,
// leaving R there.
template <int RR, bool KEEP>
__device__ void house_qr_rr(double* M, int ldm, int mrows, int c, double* vtop, double* beta) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane & 15, t = lane >> 4;
  const int jn = min(c, mrows);
  for (int j = 0; j < jn; ++j) {
    const double* cj = M + q + j * ldm;
    double v[RR];
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const double x = cj[16 * r];
      v[r] = (q + 16 * r > j) ? x : 0.0;
      if (r & 1) s1 += v[r] * v[r];
      else s0 += v[r] * v[r];
    }
    const double xj = M[j + j * ldm];
    const int g0 = j + 1 + 4 * wave;
    const int lA = g0 + t, lB = lA + 16;
    const bool two = g0 + 16 < c;   // uniform: a second group of columns
    double* cA = M + min(lA, c - 1) * ldm;
    double* cB = M + min(lB, c - 1) * ldm;
    double yA[RR], yB[RR];
    double dA0 = 0.0, dA1 = 0.0, dB0 = 0.0, dB1 = 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      yA[r] = cA[q + 16 * r];
      if (r & 1) dA1 += v[r] * yA[r];
      else dA0 += v[r] * yA[r];
    }
    const double eA = cA[j];
    double eB = 0.0;
    if (two) {
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        yB[r] = cB[q + 16 * r];
        if (r & 1) dB1 += v[r] * yB[r];
        else dB0 += v[r] * yB[r];
      }
      eB = cB[j];
    }
    const double sq = row_sum16(s0 + s1);
    const double dA = row_sum16(dA0 + dA1);
    const double dB = two ? row_sum16(dB0 + dB1) : 0.0;
    const double nrm = sqrt(sq + xj * xj);
    const double alpha = (xj >= 0.0) ? -nrm : nrm;
    const double vtv = 2.0 * nrm * (nrm + fabs(xj));   // v = x - alpha e_j
    const double tau = (vtv > 0.0) ? 2.0 / vtv : 0.0;
    const double vt = xj - alpha;
    if (tau != 0.0) {
      if (lA < c) {
        const double sd = (dA + vt * eA) * tau;
#pragma unroll
        for (int r = 0; r < RR; ++r) cA[q + 16 * r] = yA[r] - sd * v[r];
        if (q == 0) cA[j] = eA - sd * vt;
      }
      if (two && lB < c) {
        const double sd = (dB + vt * eB) * tau;
#pragma unroll
        for (int r = 0; r < RR; ++r) cB[q + 16 * r] = yB[r] - sd * v[r];
        if (q == 0) cB[j] = eB - sd * vt;
      }
      for (int g = g0 + 32; g < c; g += 16) {
        const int l = g + t;
        double* cl = M + min(l, c - 1) * ldm;
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          yA[r] = cl[q + 16 * r];
          if (r & 1) d1 += v[r] * yA[r];
          else d0 += v[r] * yA[r];
        }
        const double e = cl[j];
        const double sd = (row_sum16(d0 + d1) + vt * e) * tau;
        if (l < c) {
#pragma unroll
          for (int r = 0; r < RR; ++r) cl[q + 16 * r] = yA[r] - sd * v[r];
          if (q == 0) cl[j] = e - sd * vt;
        }
      }
    }
    __syncthreads();
    // column j is final; later steps touch only columns > j
    if (wave == 0) {
      if (KEEP) {
        if (lane == 0) {
          vtop[j] = vt;
          beta[j] = tau;
          M[j + j * ldm] = alpha;
        }
      } else {
        if (lane == 0) M[j + j * ldm] = alpha;
        for (int i = j + 1 + lane; i < jn; i += 64) M[i + j * ldm] = 0.0;
      }
    }
  }
  __syncthreads();
}

// house_qr_rr for rr = ceil(mrows / 16) blocks of rows, 1 <= rr <= RR
template <int RR, bool KEEP>
__device__ __forceinline__ void house_qr_blocks(int rr, double* M, int ldm, int mrows, int c, double* vtop,
                                                double* beta) {
  if constexpr (RR <= 1) {
    house_qr_rr<1, KEEP>(M, ldm, mrows, c, vtop, beta);
  } else {
    if (rr >= RR) house_qr_rr<RR, KEEP>(M, ldm, mrows, c, vtop, beta);
    else house_qr_blocks<RR - 1, KEEP>(rr, M, ldm, mrows, c, vtop, beta);
  }
}

// Zero rows mrows .. 16 ceil(mrows / 16) - 1 of columns 0 .. c-1 (the padding
// the 16-row blocks of house_qr_rr read); the caller synchronises.
__device__ __forceinline__ void qr_zero_pad(double* M, int ldm, int mrows, int c) {
  const int pad = ((mrows + 15) & ~15) - mrows;
  for (int e = threadIdx.x; e < pad * c; e += blockDim.x) M[mrows + e % pad + (e / pad) * ldm] = 0.0;
}

constexpr int QR_RM = 24;              // row registers per lane in the TSQR QR
constexpr int QR_ROWS = 16 * QR_RM;    // rows reduced per pass

// R of the mrows x c matrix in LDS (mrows <= QR_ROWS, ldm a multiple of 16
// and >= mrows): pads the last block of rows with zeros, then factors.
__device__ __forceinline__ void house_qr_lds(double* M, int ldm, int mrows, int c) {
  qr_zero_pad(M, ldm, mrows, c);
  __syncthreads();
  house_qr_blocks<QR_RM, false>((mrows + 15) >> 4, M, ldm, mrows, c, nullptr, nullptr);
}

__device__ __forceinline__ int qr_ldm(int c) { return (QR_LDS / (c > 0 ? c : 1)) & ~15; }

__global__ __launch_bounds__(256) void k_tsqr_seg(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                                  const TsqrSeg* __restrict__ segs, int s0, int rmax) {
  const TsqrSeg S = segs[s0 + blockIdx.x];
  const int c = dimv(dyn, S.cols);
  double* __restrict__ R = refp(bufs, S.R);
  extern __shared__ double smem[];
  double* M = smem;
  const int tid = threadIdx.x;
  if (c <= 0) return;
  const int ldm = qr_ldm(c);
  const int prow = min(ldm, QR_ROWS);
  const double* __restrict__ X = refp(bufs, S.X);
  const int ld = S.X.ld;
  int have = 0;
  for (int base = 0, nr = 0; base < S.rows; base += nr) {
    nr = min(prow - have, S.rows - base);
    for (int b0 = 0; b0 < nr * c; b0 += 2048) {
      double r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int e = b0 + u * 256 + tid;
        int i = e % nr, l = e / nr;
        r[u] = (e < nr * c) ? X[(size_t)(base + i) + (size_t)l * ld] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int e = b0 + u * 256 + tid;
        int i = e % nr, l = e / nr;
        if (e < nr * c) M[have + i + l * ldm] = r[u];
      }
    }
    __syncthreads();
    int mrows = have + nr;
    house_qr_lds(M, ldm, mrows, c);
    have = min(mrows, c);
  }
  for (int e = tid; e < c * c; e += 256) {
    int i = e % c, l = e / c;
    R[i + (size_t)l * rmax] = (i < have && i <= l) ? M[i + l * ldm] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_tsqr_red(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                                  const TsqrRed* __restrict__ reds, int r0i, int rmax) {
  const TsqrRed S = reds[r0i + blockIdx.x];
  const int c = dimv(dyn, S.cols);
  double* __restrict__ R = refp(bufs, S.R);
  extern __shared__ double smem[];
  double* M = smem;
  const int tid = threadIdx.x;
  if (c <= 0) return;
  const int ldm = qr_ldm(c);
  const int prow = min(ldm, QR_ROWS);
  const double* __restrict__ R0 = refp(bufs, S.R0);
  const size_t RR = (size_t)rmax * rmax;
  int have = 0;
  int s = 0;
  while (s < S.nseg) {
    // stack as many segment R factors as fit under the current R
    int mrows = have;
    const int s_start = s;
    while (s < S.nseg && mrows + c <= prow) {
      const double* Rs = R0 + RR * s;
      for (int e = tid; e < c * c; e += 256) {
        int i = e % c, l = e / c;
        M[mrows + i + l * ldm] = Rs[i + (size_t)l * rmax];
      }
      mrows += c;
      ++s;
    }
    if (s == s_start) break;   // cannot happen for c <= 80 (2c <= prow)
    __syncthreads();
    house_qr_lds(M, ldm, mrows, c);
    have = min(mrows, c);
  }
  for (int e = tid; e < c * c; e += 256) {
    int i = e % c, l = e / c;
    R[i + (size_t)l * rmax] = (i < have && i <= l) ? M[i + l * ldm] : 0.0;
  }
}

// ------------------------------------------------------------------ small SVD
// Orders a wave's LDS stores before its later loads from other lanes (a
// wave executes its LDS instructions in order; this keeps the compiler from
// moving them and waits for completion).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One-sided Jacobi (Hestenes) on the columns of an n x n matrix A in LDS
// (ld = SM), accumulating the right rotations in V: A V = U S.  All disjoint
// column pairs of a round-robin round are processed at once, each by a group
// of g lanes (g a power of two, groups aligned inside a wave).  Pairs of
// columns whose squared norms are both below thr2 are skipped: callers set
// thr2 well below their truncation threshold, and such pairs only slow the
// convergence.
constexpr int SM = 80;
// a sweep whose largest squared cosine between paired columns stays below
// this ends the iteration (cosine 1e-3)
constexpr double JACOBI_STOP2 = 1e-6;

__device__ void jacobi_svd_lds(double* A, double* V, int n, double thr2, double* red) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += 256) {
    int i = e % n, j = e / n;
    V[i + j * SM] = (i == j) ? 1.0 : 0.0;
  }
  const int np = (n + 1) & ~1;
  const int npairs = np / 2;
  int g = 64;
  while (g > 1 && npairs * g > 256) g >>= 1;
  const int grp = tid / g, gl = tid % g;
  const double tol = fmax(1e-14, 8.0 * 2.220446049250313e-16 * n);
  const double tol2 = tol * tol;
  constexpr int RU = 8;   // rows per lane kept in registers during a rotation
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off2 = 0.0;   // max over pairs of ga^2 / (al be)
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      if (grp < npairs) {
        int a, b;
        if (grp == 0) {
          a = np - 1;
          b = rnd;
        } else {
          a = (rnd + grp) % (np - 1);
          b = (rnd - grp + (np - 1)) % (np - 1);
        }
        if (a < n && b < n) {
          const int pp = min(a, b), qq = max(a, b);
          double* __restrict__ Ap = A + pp * SM;
          double* __restrict__ Aq = A + qq * SM;
          double xr[RU], yr[RU];
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const int i = gl + g * u;
            xr[u] = i < n ? Ap[i] : 0.0;
            yr[u] = i < n ? Aq[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            al = fma(xr[u], xr[u], al);
            be = fma(yr[u], yr[u], be);
            ga = fma(xr[u], yr[u], ga);
          }
          for (int i = gl + g * RU; i < n; i += g) {
            double x = Ap[i], y = Aq[i];
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
          for (int o = g >> 1; o > 0; o >>= 1) {
            al += __shfl_xor(al, o);
            be += __shfl_xor(be, o);
            ga += __shfl_xor(ga, o);
          }
          if (ga != 0.0 && al != 0.0 && be != 0.0 && (al >= thr2 || be >= thr2)) {
            const double g2 = ga * ga, ab = al * be;
            off2 = fmax(off2, g2 / ab);
            if (g2 >= tol2 * ab) {
              // tangent of the rotation angle: the smaller root of
              // t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 ga), written
              // without the division by ga
              const double d = be - al;
              const double h = sqrt(fma(d, d, 4.0 * g2));
              const double tt = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) / (fabs(d) + h);
              const double cs = 1.0 / sqrt(fma(tt, tt, 1.0));
              const double sn = cs * tt;
#pragma unroll
              for (int u = 0; u < RU; ++u) {
                const int i = gl + g * u;
                if (i < n) {
                  Ap[i] = cs * xr[u] - sn * yr[u];
                  Aq[i] = sn * xr[u] + cs * yr[u];
                }
              }
              for (int i = gl + g * RU; i < n; i += g) {
                double x = Ap[i], y = Aq[i];
                Ap[i] = cs * x - sn * y;
                Aq[i] = sn * x + cs * y;
              }
              double* __restrict__ Vp = V + pp * SM;
              double* __restrict__ Vq = V + qq * SM;
              for (int i = gl; i < n; i += g) {
                double vx = Vp[i], vy = Vq[i];
                Vp[i] = cs * vx - sn * vy;
                Vq[i] = sn * vx + cs * vy;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) off2 = fmax(off2, __shfl_xor(off2, o));
    if ((tid & 63) == 0) red[tid >> 6] = off2;
    __syncthreads();
    double om = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    if (om < JACOBI_STOP2) break;   // see jacobi_wg_rounds
  }
}

// Rotation of a Jacobi pair from al = |x|^2, be = |y|^2, ga = x.y: the
// tangent is the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (be - al) /
// (2 ga), written without the division by ga.  Hardware reciprocal and
// reciprocal square root with one Newton step each: c^2 + s^2 = 1 to a few
// ulp, which is all a rotation needs (the angle itself may be inexact).
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double& cs, double& sn) {
  const double d = be - al;
  const double q = fma(d, d, 4.0 * ga * ga);
  const double h = q * rsq_nr(q);
  const double tt = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) * rcp_nr(fabs(d) + h);
  cs = rsq_nr(fma(tt, tt, 1.0));
  sn = cs * tt;
}

// Sum over an aligned group of G lanes; every lane of the group gets the
// same bits (each level adds a lane's value to its partner's, and the
// partner computes the same two operands in the other order).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 64) v += __shfl_xor(v, 32);
  if constexpr (G >= 32) v += __shfl_xor(v, 16);
  if constexpr (G >= 16) v += dpp_move<DPP_MIRROR>(v);
  if constexpr (G >= 8) v += dpp_move<DPP_HALF_MIRROR>(v);
  if constexpr (G >= 4) v += dpp_move<DPP_XOR2>(v);
  if constexpr (G >= 2) v += dpp_move<DPP_XOR1>(v);
  return v;
}

// Work-group one-sided Jacobi for n <= 64 (all 256 threads; V accumulated,
// V must hold the identity or a start basis): G lanes per column pair
// (pairs * G <= 256, G <= 16 so that a group lies in one row of 16 lanes and
// reduces with DPP), RU >= n / G rows of both columns of A and V per lane
// in registers for the round, one barrier per round.
template <int G, int RU>
__device__ void jacobi_wg_rounds(double* A, double* V, int n, double thr2) {
  const int tid = threadIdx.x;
  const int np = (n + 1) & ~1;
  const int npairs = np / 2;
  const int grp = tid / G, gl = tid % G;
  const double tol = fmax(1e-14, 8.0 * 2.220446049250313e-16 * n);
  const double tol2 = tol * tol;
  const int m1 = np - 1;
  for (int sweep = 0; sweep < 30; ++sweep) {
    int big = 0;
    int a = grp == 0 ? m1 : grp % m1, b = grp == 0 ? 0 : (m1 - grp % m1) % m1;
    for (int rnd = 0; rnd < m1; ++rnd) {
      if (grp < npairs && a < n && b < n) {
        const int pp = min(a, b), qq = max(a, b);
        double* __restrict__ Ap = A + pp * SM;
        double* __restrict__ Aq = A + qq * SM;
        double* __restrict__ Vp = V + pp * SM;
        double* __restrict__ Vq = V + qq * SM;
        // rows n .. G RU - 1 are zero (padded by jacobi_wg) and stay zero
        double xr[RU], yr[RU], vx[RU], vy[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          const int i = gl + G * u;
          xr[u] = Ap[i];
          yr[u] = Aq[i];
          vx[u] = Vp[i];
          vy[u] = Vq[i];
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          al = fma(xr[u], xr[u], al);
          be = fma(yr[u], yr[u], be);
          ga = fma(xr[u], yr[u], ga);
        }
        al = group_sum<G>(al);
        be = group_sum<G>(be);
        ga = group_sum<G>(ga);
        if (ga != 0.0 && al != 0.0 && be != 0.0 && (al >= thr2 || be >= thr2)) {
          const double g2 = ga * ga, ab = al * be;
          if (g2 >= tol2 * ab) {
            if (g2 >= JACOBI_STOP2 * ab) big = 1;
            double cs, sn;
            jacobi_rotation(al, be, ga, cs, sn);
#pragma unroll
            for (int u = 0; u < RU; ++u) {
              const int i = gl + G * u;
              Ap[i] = cs * xr[u] - sn * yr[u];
              Aq[i] = sn * xr[u] + cs * yr[u];
              Vp[i] = cs * vx[u] - sn * vy[u];
              Vq[i] = sn * vx[u] + cs * vy[u];
            }
          }
        }
      }
      if (grp > 0) {
        a = a + 1 == m1 ? 0 : a + 1;
        b = b + 1 == m1 ? 0 : b + 1;
      } else {
        b += 1;
      }
      __syncthreads();
    }
    // converged once no pair of a sweep had a cosine above 1e-3: the
    // convergence is quadratic, so the sweep leaves the columns orthogonal
    // to about 1e-6 and their norms within about 1e-12 of the singular
    // values (relative); the truncation error, the norm of the dropped
    // columns of A V with V orthogonal, is exact whatever cosines remain
    if (!__syncthreads_or(big)) break;
  }
}

// Zero rows n .. rows - 1 of the first n columns of A and V (ld SM).
__device__ __forceinline__ void jacobi_zero_pad(double* A, double* V, int n, int rows) {
  const int pad = rows - n;
  for (int e = threadIdx.x; e < pad * n; e += 256) {
    const int i = n + e % pad, j = e / pad;
    A[i + j * SM] = 0.0;
    V[i + j * SM] = 0.0;
  }
  __syncthreads();
}

// The row span G RU of a round is the smallest multiple of the group width
// that covers n (a lane's rows of a column pair, loaded and stored per
// round, are what a round costs).
__device__ void jacobi_wg(double* A, double* V, int n, double thr2) {
  if (n <= 16) {
    jacobi_zero_pad(A, V, n, 16);
    jacobi_wg_rounds<16, 1>(A, V, n, thr2);
  } else if (n <= 32) {
    jacobi_zero_pad(A, V, n, 32);
    jacobi_wg_rounds<16, 2>(A, V, n, thr2);
  } else if (n <= 40) {
    jacobi_zero_pad(A, V, n, 40);
    jacobi_wg_rounds<8, 5>(A, V, n, thr2);
  } else if (n <= 48) {
    jacobi_zero_pad(A, V, n, 48);
    jacobi_wg_rounds<8, 6>(A, V, n, thr2);
  } else {
    jacobi_zero_pad(A, V, n, 64);
    jacobi_wg_rounds<8, 8>(A, V, n, thr2);
  }
}

// Work-group Jacobi for n <= 64 with V := identity first.
__device__ void jacobi_svd_wg(double* A, double* V, int n, double thr2, double* red) {
  (void)red;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += 256) {
    int i = e % n, j = e / n;
    V[i + j * SM] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_wg(A, V, n, thr2);
  __syncthreads();
}

// Squared Frobenius norm of the n x n matrix A in LDS, returned to every
// thread (uses red[4..7]).
__device__ double fro2_lds(const double* A, int n, double* red) {
  const int tid = threadIdx.x;
  double f = 0.0;
  for (int e = tid; e < n * n; e += 256) {
    double v = A[(e % n) + (e / n) * SM];
    f += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
  __syncthreads();
  if ((tid & 63) == 0) red[4 + (tid >> 6)] = f;
  __syncthreads();
  return red[4] + red[5] + red[6] + red[7];
}

// singular values (column norms of A) and the order by decreasing value,
// ties to the lower index: ord[r] = column of rank r
__device__ void order_desc(const double* A, int n, double* sv, int* ord) {
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += 256) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += A[i + j * SM] * A[i + j * SM];
    sv[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < n; j += 256) {
    int r = 0;
    for (int i = 0; i < n; ++i) r += (sv[i] > sv[j]) || (sv[i] == sv[j] && i < j);
    ord[r] = j;
  }
  __syncthreads();
}

__device__ __forceinline__ int upk(int i, int j) { return j * (j + 1) / 2 + i; }   // i <= j

// bulk copy of the upper triangle of an n x n matrix (ld) into packed LDS,
// loads issued 8 at a time before the stores
__device__ void load_upper(const double* __restrict__ R, int ld, int n, double* Rp) {
  const int tid = threadIdx.x;
  for (int base = 0; base < n * n; base += 2048) {
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int i = e % n, j = e / n;
      r[u] = (e < n * n && i <= j) ? R[i + (size_t)j * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int i = e % n, j = e / n;
      if (e < n * n && i <= j) Rp[upk(i, j)] = r[u];
    }
  }
}

// Rank-revealing orthogonalisation of a sketch: Householder QR with column
// pivoting of the n x n upper-triangular R_Y in LDS (A, ld SM), stopped at
// the first pivot |R'_jj| <= tau |R'_00|.  Returns the kept count k; on exit
// A holds R' in its leading k x k upper triangle and piv[0..k) the chosen
// columns.  Column norms are downdated and recomputed when the downdate
// loses more than half of the digits.
__device__ int qrcp_lds(double* A, int n, double tau, double* cn, double* cn0, int* piv,
                        double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int s_piv, s_stop;
  for (int j = tid; j < n; j += 256) {
    double c = 0.0;
    for (int i = 0; i <= j; ++i) c += A[i + j * SM] * A[i + j * SM];
    cn[j] = c;
    cn0[j] = c;
    piv[j] = j;
  }
  if (tid == 0) s_stop = n;
  __syncthreads();
  int k = n;
  for (int j = 0; j < n; ++j) {
    // pivot: the largest remaining norm, ties to the lowest column
    if (wave == 0) {
      double bv = -1.0;
      int bi = n;
      for (int l = j + lane; l < n; l += 64)
        if (cn[l] > bv) {
          bv = cn[l];
          bi = l;
        }
      for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(bv, o);
        int oi = __shfl_xor(bi, o);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) s_piv = bi;
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j) {
      for (int i = tid; i < n; i += 256) {
        double t = A[i + j * SM];
        A[i + j * SM] = A[i + p * SM];
        A[i + p * SM] = t;
      }
      if (tid == 0) {
        double t = cn[j];
        cn[j] = cn[p];
        cn[p] = t;
        t = cn0[j];
        cn0[j] = cn0[p];
        cn0[p] = t;
        int q = piv[j];
        piv[j] = piv[p];
        piv[p] = q;
      }
    }
    __syncthreads();
    // Householder reflector of column j, rows j..n-1 (exact norm)
    if (wave == 0) {
      double sq = 0.0;
      for (int i = j + lane; i < n; i += 64) sq += A[i + j * SM] * A[i + j * SM];
      for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
      if (lane == 0) {
        const double nrm = sqrt(sq);
        if (j == 0) red[2] = nrm;
        const double r0 = (j == 0) ? nrm : red[2];
        if (!(nrm > tau * r0) || !(nrm > 0.0)) {
          s_stop = j;
        } else {
          const double a = A[j + j * SM];
          const double alpha = (a >= 0.0) ? -nrm : nrm;
          const double vtv = 2.0 * nrm * (nrm + fabs(a));
          red[0] = alpha;
          red[1] = 2.0 / vtv;
          A[j + j * SM] = a - alpha;
        }
      }
    }
    __syncthreads();
    if (s_stop <= j) {
      k = j;
      break;
    }
    const double beta = red[1];
    for (int l = j + 1 + wave; l < n; l += 4) {
      double sdot = 0.0;
      for (int i = j + lane; i < n; i += 64) sdot += A[i + j * SM] * A[i + l * SM];
      for (int o = 32; o > 0; o >>= 1) sdot += __shfl_xor(sdot, o);
      sdot *= beta;
      for (int i = j + lane; i < n; i += 64) A[i + l * SM] -= sdot * A[i + j * SM];
    }
    __syncthreads();
    if (tid == 0) A[j + j * SM] = red[0];
    for (int l = j + 1 + tid; l < n; l += 256) {
      const double r = A[j + l * SM];
      double c = cn[l] - r * r;
      if (!(c > 1e-8 * cn0[l])) {
        c = 0.0;
        for (int i = j + 1; i < n; ++i) c += A[i + l * SM] * A[i + l * SM];
        cn0[l] = c;
      }
      cn[l] = c;
    }
    __syncthreads();
  }
  return k;
}

// Single-wave column-pivoted QR for n <= 64 (lanes = columns).  The matrix
// is kept transposed in LDS (row i at T[i * TLD], lane l owns column l), so
// a lane's accesses are conflict-free and the pivot column is read by every
// lane as a broadcast; steps are ordered by wave-scope fences, not barriers.
// Same contract as qrcp_lds: returns k, with R' in pivot order
// (R'[r][c] = T[r * TLD + piv[c]]) and piv[0..n) a permutation whose first
// k entries are the chosen columns.
constexpr int TLD = 65;

__device__ int qrcp_wave(double* T, int n, double tau, int* piv, int* kout) {
  const int lane = threadIdx.x;   // called by the first wave only
  bool active = lane < n;
  double cn = 0.0;
  if (active)
    for (int i = 0; i < n; ++i) cn = fma(T[i * TLD + lane], T[i * TLD + lane], cn);
  double cn0 = cn;
  double r0 = 0.0;
  int k = n;
  for (int j = 0; j < n; ++j) {
    // pivot: the largest remaining norm, ties to the lowest column (a wave
    // max-reduction, then the lowest lane holding the maximum)
    const double bv = active ? cn : -1.0;
    const double mx = wave_max64(bv);
    const unsigned long long hit = __ballot(active && bv == mx);
    if (hit == 0ull) {   // only NaN norms remain
      k = j;
      break;
    }
    const int p = __ffsll((long long)hit) - 1;
    // exact norm of the pivot column below row j (broadcast reads, four
    // partial sums)
    double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
    int i = j;
    for (; i + 3 < n; i += 4) {
      q0 = fma(T[i * TLD + p], T[i * TLD + p], q0);
      q1 = fma(T[(i + 1) * TLD + p], T[(i + 1) * TLD + p], q1);
      q2 = fma(T[(i + 2) * TLD + p], T[(i + 2) * TLD + p], q2);
      q3 = fma(T[(i + 3) * TLD + p], T[(i + 3) * TLD + p], q3);
    }
    for (; i < n; ++i) q0 = fma(T[i * TLD + p], T[i * TLD + p], q0);
    const double nrm = sqrt((q0 + q1) + (q2 + q3));
    if (j == 0) r0 = nrm;
    if (!(nrm > tau * r0) || !(nrm > 0.0)) {
      k = j;
      break;
    }
    const double a = T[j * TLD + p];
    const double alpha = (a >= 0.0) ? -nrm : nrm;
    const double beta = 2.0 / (2.0 * nrm * (nrm + fabs(a)));
    const double vj = a - alpha;
    if (lane == p) active = false;
    if (active) {
      double w0 = vj * T[j * TLD + lane], w1 = 0.0, w2 = 0.0, w3 = 0.0;
      int i2 = j + 1;
      for (; i2 + 3 < n; i2 += 4) {
        w0 = fma(T[i2 * TLD + p], T[i2 * TLD + lane], w0);
        w1 = fma(T[(i2 + 1) * TLD + p], T[(i2 + 1) * TLD + lane], w1);
        w2 = fma(T[(i2 + 2) * TLD + p], T[(i2 + 2) * TLD + lane], w2);
        w3 = fma(T[(i2 + 3) * TLD + p], T[(i2 + 3) * TLD + lane], w3);
      }
      for (; i2 < n; ++i2) w0 = fma(T[i2 * TLD + p], T[i2 * TLD + lane], w0);
      const double w = ((w0 + w1) + (w2 + w3)) * beta;
      T[j * TLD + lane] -= w * vj;
      for (int i3 = j + 1; i3 < n; ++i3) T[i3 * TLD + lane] -= w * T[i3 * TLD + p];
      const double r = T[j * TLD + lane];
      double c = cn - r * r;
      if (!(c > 1e-8 * cn0)) {
        c = 0.0;
        for (int i3 = j + 1; i3 < n; ++i3) c = fma(T[i3 * TLD + lane], T[i3 * TLD + lane], c);
        cn0 = c;
      }
      cn = c;
    }
    if (lane == p) T[j * TLD + p] = alpha;
    if (lane == 0) piv[j] = p;
    wave_sync_lds();
  }
  // the columns never chosen follow in increasing order, so that piv[0..n)
  // is a permutation (their rows of the result are zero)
  const unsigned long long rest = __ballot(active);
  if (active) piv[k + __popcll(rest & ((1ull << lane) - 1ull))] = lane;
  if (lane == 0) *kout = k;
  wave_sync_lds();
  return k;
}

// Single-wave column-pivoted QR for n <= RU, with the contract of qrcp_wave
// (same pivot rule, stopping rule and output).  A lane keeps its column in
// registers with the row of the current step at index 0: after each step
// the registers shift down by one, so every register index is static.  The
// pivot column goes through xs (RU doubles of LDS) as a broadcast, and each
// row of T is stored as it becomes final.
template <int RU>
__device__ int qrcp_reg(double* T, int n, double tau, int* piv, int* kout, double* xs) {
  const int lane = threadIdx.x;   // called by the first wave only
  bool active = lane < n;
  double col[RU];
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    const double v = T[u * TLD + (active ? lane : 0)];
    col[u] = (active && u < n) ? v : 0.0;
  }
  double cn = 0.0;
#pragma unroll
  for (int u = 0; u < RU; ++u) cn = fma(col[u], col[u], cn);
  double cn0 = cn;
  double r0 = 0.0;
  int k = n;
  for (int j = 0; j < n; ++j) {
    // pivot: the largest remaining norm, ties to the lowest column
    const double bv = active ? cn : -1.0;
    const double mx = wave_max64(bv);
    const unsigned long long hit = __ballot(active && bv == mx);
    if (hit == 0ull) {   // only NaN norms remain
      k = j;
      break;
    }
    const int p = __ffsll((long long)hit) - 1;
    if (lane == p) {
#pragma unroll
      for (int u = 0; u < RU; ++u) xs[u] = col[u];
    }
    wave_sync_lds();
    double x[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) x[u] = xs[u];
    // exact norm of the pivot column from row j on (four partial sums)
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < RU; ++u) q[u & 3] = fma(x[u], x[u], q[u & 3]);
    const double nrm = sqrt((q[0] + q[1]) + (q[2] + q[3]));
    if (j == 0) r0 = nrm;
    if (!(nrm > tau * r0) || !(nrm > 0.0)) {
      k = j;
      break;
    }
    const double a = x[0];
    const double alpha = (a >= 0.0) ? -nrm : nrm;
    const double beta = 2.0 / (2.0 * nrm * (nrm + fabs(a)));
    const double vj = a - alpha;
    if (lane == p) {
      active = false;
      T[j * TLD + p] = alpha;
    }
    if (active) {
      double w[4] = {vj * col[0], 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 1; u < RU; ++u) w[(u - 1) & 3] = fma(x[u], col[u], w[(u - 1) & 3]);
      const double ws = ((w[0] + w[1]) + (w[2] + w[3])) * beta;
      col[0] -= ws * vj;
#pragma unroll
      for (int u = 1; u < RU; ++u) col[u] -= ws * x[u];
      T[j * TLD + lane] = col[0];
      const double r = col[0];
      double c = cn - r * r;
      if (!(c > 1e-8 * cn0)) {
        c = 0.0;
#pragma unroll
        for (int u = 1; u < RU; ++u) c = fma(col[u], col[u], c);
        cn0 = c;
      }
      cn = c;
    }
    if (lane == 0) piv[j] = p;
    // row j + 1 to register 0
#pragma unroll
    for (int u = 0; u + 1 < RU; ++u) col[u] = col[u + 1];
    col[RU - 1] = 0.0;
    wave_sync_lds();   // xs is rewritten by the next step
  }
  // the columns never chosen follow in increasing order, so that piv[0..n)
  // is a permutation (their rows of the result are zero)
  const unsigned long long rest = __ballot(active);
  if (active) piv[k + __popcll(rest & ((1ull << lane) - 1ull))] = lane;
  if (lane == 0) *kout = k;
  wave_sync_lds();
  return k;
}

// Lane-private vectors of RU doubles with compile-time register indices:
// an element at a run-time index is read or written by a select over all of
// them (no dynamic register indexing).
template <int RU>
__device__ __forceinline__ double reg_get(const double (&r)[RU], int j) {
  double x = 0.0;
#pragma unroll
  for (int u = 0; u < RU; ++u) x = (u == j) ? r[u] : x;
  return x;
}
template <int RU>
__device__ __forceinline__ void reg_set(double (&r)[RU], int j, double x) {
#pragma unroll
  for (int u = 0; u < RU; ++u) r[u] = (u == j) ? x : r[u];
}

// Second half of the truncation by the work-group, G lanes per output column
// c < kk (tid / G), lane s holding rows s + G r (r < R; G R = 32 for n <= 32,
// 64 for n <= 64).  Z = Q2 V[:, ord[c]] (reflectors applied last to first,
// each read as a broadcast, each dot product reduced over the G lanes with
// DPP moves), then C1[:, c] = R2^{-1} Z[:, c] by back substitution, each new
// entry passed along the G lanes of its column by a lane permute.
template <int G, int R>
__device__ void sketch_f_out_wg(const double* V, const double* R1, const double* R2, const double* beta,
                                const int* ord, int n, int kk, double* __restrict__ C1, int rmax) {
  constexpr int NR = G * R;
  const int tid = threadIdx.x, c = tid / G, s = tid % G, lane = tid & 63;
  const bool act = c < kk;
  const int oc = act ? ord[c] : 0;
  double z[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int u = s + G * r;
    const double x = V[(u < n ? u : 0) + oc * SM];
    z[r] = (act && u < n) ? x : 0.0;
  }
#pragma unroll
  for (int j = NR - 1; j >= 0; --j) {
    if (j >= n) continue;
    const double bj = beta[j];
    const double v0 = beta[SM + j];
    const int base = j * n - j * (j + 1) / 2 - j - 1;   // packed reflector tail, rows > j
    double cv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = s + G * r;
      const bool tail = u > j && u < n;
      const double t = R1[tail ? base + u : 0];
      cv[r] = (u == j) ? v0 : (tail ? t : 0.0);
    }
    double d = cv[0] * z[0];
#pragma unroll
    for (int r = 1; r < R; ++r) d = fma(cv[r], z[r], d);
    d = group_sum<G>(d) * bj;
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = (bj != 0.0) ? fma(-d, cv[r], z[r]) : z[r];   // bj == 0: H_j = I
  }
#pragma unroll
  for (int i = NR - 1; i >= 0; --i) {
    if (i >= n) continue;
    const double* col = R2 + i * (i + 1) / 2;   // packed upper column i
    const double dg = col[i];
    double x = (dg != 0.0) ? z[i / G] / dg : 0.0;   // right on the lane holding row i
    x = __shfl(x, (lane & ~(G - 1)) | (i % G));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = s + G * r;
      const double cu = col[u < i ? u : 0];
      z[r] = (u == i) ? x : ((u < i) ? fma(-cu, x, z[r]) : z[r]);
    }
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = s + G * r;
      if (u < n) C1[u + (size_t)c * rmax] = z[r];
    }
  }
}

// M = R1 R2^{-1} row by row with G lanes per row i (tid / G), lane s holding
// the entries l = s + G r (r < R; G R >= n): entry j is the row's dot product
// so far with column j of R2 (reduced over the G lanes by DPP), subtracted
// from R1's entry and divided by the diagonal.
template <int G, int R>
__device__ void sketch_f_m_wg(const double* R1, const double* R2, int n, double* A) {
  const int tid = threadIdx.x, i = tid / G, s = tid % G;
  double g[R];
#pragma unroll
  for (int r = 0; r < R; ++r) g[r] = 0.0;
  for (int j = 0; j < n; ++j) {
    const double* col = R2 + j * (j + 1) / 2;   // column j of R2 (rows <= j)
    double p = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int l = s + G * r;
      const double c = col[l < j ? l : 0];
      p = fma(l < j ? g[r] : 0.0, c, p);
    }
    p = group_sum<G>(p);
    const double a = (i < n && i <= j) ? R1[upk(i, j)] : 0.0;
    const double d = col[j];
    const double gj = (d != 0.0) ? (a - p) / d : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (j == s + G * r) g[r] = gj;
  }
  if (i < n) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (s + G * r < n) A[i + (s + G * r) * SM] = g[r];
  }
}

// C1 = Pi R'_k^{-1} for n <= G R by the work-group: G lanes per column
// c < k (tid / G), lane s holding rows s + G r; column c of R'_k^{-1} by
// column-oriented substitution from e_c (R' read as a broadcast), each new
// entry passed along the column's lanes by a lane permute; then row piv[u]
// of C1 for every u < n (zero for u > c).
template <int G, int R>
__device__ void sketch_p_inv_wg(const double* T, const int* piv, int n, int kk, double* __restrict__ C1,
                                int rmax) {
  const int tid = threadIdx.x, c = tid / G, s = tid % G, lane = tid & 63;
  double x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = (s + G * r == c) ? 1.0 : 0.0;
#pragma unroll
  for (int l = G * R - 1; l >= 0; --l) {
    if (l < kk) {
      const int pl = piv[l];
      double xl = x[l / G] / T[l * TLD + pl];   // right on the lane holding row l
      xl = __shfl(xl, (lane & ~(G - 1)) | (l % G));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int u = s + G * r;
        const double t = T[(u < l ? u : 0) * TLD + pl];
        x[r] = (u == l) ? xl : ((u < l) ? fma(-t, xl, x[r]) : x[r]);
      }
    }
  }
  if (c < kk) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = s + G * r;
      if (u < n) C1[piv[u] + (size_t)c * rmax] = (u <= c) ? x[r] : 0.0;
    }
  }
}

// Householder QR of the n x n matrix M in LDS (ld SM) that keeps the
// reflectors: on exit R is in the upper triangle, v_j below the diagonal of
// column j with its leading entry in vtop[j], and H_j = I - beta[j] v_j v_j^T,
// so that M = H_0 H_1 ... H_{n-1} R.
__device__ void house_qr_keep(double* M, int n, double* vtop, double* beta) {
  qr_zero_pad(M, SM, n, n);
  __syncthreads();
  house_qr_blocks<SM / 16, true>((n + 15) >> 4, M, SM, n, n, vtop, beta);
}

// A randomised sketch Y = M Omega of width r yields a near-optimal basis of
// the kept rank k only while at least two of its directions are discarded
// (the expected error of the range finder is bounded by the tail singular
// values once the oversampling is >= 2).  A kept rank of r - 1 or more with
// r below min(p, q) therefore means the sketch may have missed part of M's
// column space at accuracy eps; a sketch of width min(p, q) spans it.
__device__ __forceinline__ bool sketch_saturated(int kept, int r, int full) {
  return r < full && kept + 1 >= r;
}

// Truncation result of a sketched low-rank target (one thread): the kept rank
// is the block's candidate rank hint for the next factorisation's sketch
// width; a saturated sketch proposes its width plus max(8, width / 4) (a
// modest step: the kernels for widths up to 64 are much faster) and raises
// STAT_SKETCH_SAT (and STAT_SAT_CAP when the sketch was already as wide as
// the plan allows).
__device__ __forceinline__ void sketch_report(const SmallJob& J, int* __restrict__ dyn, int kept,
                                              int* __restrict__ status) {
  if (J.sat.maxv < 0) return;
  const int r = dimv(dyn, J.sat);
  const bool sat = sketch_saturated(kept, r, J.full);
  if (J.cand_slot >= 0) dyn[J.cand_slot] = sat ? r + max(8, r / 4) : kept;
  if (sat) {
    atomicOr(status, r >= J.sat.maxv ? (STAT_SKETCH_SAT | STAT_SAT_CAP) : STAT_SKETCH_SAT);
    atomicAdd(status + 2, 1);   // saturated blocks of this factorisation
  }
}

// Small dense problems built from upper-triangular R factors.
//   SK_RECOMP   SVD of A = R1 R2^T = X S Y^T (one-sided Jacobi on A):
//               CU = R2^T Y_k, CV = R1^T X_k S_k^{-1}, k = #{s > eps s_1}
//   SK_SKETCH_P column-pivoted QR of R1 = R_Y (rank-revealing, stopped at
//               tau): C1 = Pi_k R'_k^{-1}, so that Y C1 has orthonormal
//               columns; the kept count is written as the rank
//   SK_SKETCH_F SVD of A = R1 R2^{-1}: C1 = R2^{-1} Y_k, k = #{s > eps s_1}
__global__ __launch_bounds__(256) void k_small(const Bufs* __restrict__ bufs, int* __restrict__ dyn,
                                               const SmallJob* __restrict__ jobs, int j0, int rmax,
                                               double eps_run, double tau_run, int fixed_rank,
                                               int* __restrict__ status) {
  const SmallJob J = jobs[j0 + blockIdx.x];
  const int n = dimv(dyn, J.k);
  extern __shared__ double smem[];
  double* A = smem;                          // SM x SM
  double* V = A + SM * SM;                   // SM x SM
  double* R1 = V + SM * SM;                  // packed upper, SM(SM+1)/2
  double* R2 = R1 + SM * (SM + 1) / 2;       // packed upper
  double* sv = R2 + SM * (SM + 1) / 2;       // SM
  double* red = sv + SM;                     // 8
  double* beta = red + 8;                    // 2 SM: reflector factors, leading entries
  int* ord = (int*)(beta + 2 * SM);          // SM
  const int tid = threadIdx.x;
  const double eps = J.eps == -1.0 ? eps_run : (J.eps == -2.0 ? tau_run : J.eps);
  if (n <= 0) {
    if (tid == 0) dyn[J.out_rank_slot] = 0;
    return;
  }
  double* __restrict__ C1 = refp(bufs, J.C1);
  load_upper(refp(bufs, J.R1), rmax, n, R1);
  if (J.kind != SK_SKETCH_P) load_upper(refp(bufs, J.R2), rmax, n, R2);
  __syncthreads();
  if (J.kind == SK_SKETCH_P && n <= 32) {
    // pivoted QR on R1 transposed into V (row i at V[i * TLD]) by the first
    // wave, then the inverse by the work-group
    __shared__ int s_kr;
    for (int e = tid; e < n * n; e += 256) {
      int i = e / n, l = e % n;
      V[i * TLD + l] = (i <= l) ? R1[upk(i, l)] : 0.0;
    }
    __syncthreads();
    if (tid < 64) qrcp_reg<32>(V, n, eps, ord, &s_kr, sv);
    __syncthreads();
    sketch_p_inv_wg<8, 4>(V, ord, n, s_kr, C1, rmax);
    if (tid == 0) dyn[J.out_rank_slot] = s_kr;
    return;
  }
  if (J.kind == SK_SKETCH_P && n <= 64) {
    // single-wave pivoted QR on R1 transposed into V (row i at V[i * TLD])
    __shared__ int s_k;
    for (int e = tid; e < n * n; e += 256) {
      int i = e / n, l = e % n;
      V[i * TLD + l] = (i <= l) ? R1[upk(i, l)] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      // the register variant (a lane's column in registers) up to 40 rows
      if (n <= 40)
        qrcp_reg<40>(V, n, eps, ord, &s_k, sv);
      else
        qrcp_wave(V, n, eps, ord, &s_k);
    }
    __syncthreads();
    const int kk = s_k;
    // C1 = Pi R'_k^{-1} with four lanes per column
    sketch_p_inv_wg<4, 16>(V, ord, n, kk, C1, rmax);
    if (tid == 0) dyn[J.out_rank_slot] = kk;
    return;
  }
  if (J.kind == SK_SKETCH_P) {
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, j = e / n;
      A[i + j * SM] = (i <= j) ? R1[upk(i, j)] : 0.0;
    }
    __syncthreads();
    // column norms in sv and in R2's (unused) storage; R'^{-1} into V
    const int kk = qrcp_lds(A, n, eps, sv, R2, ord, red);
    double* Xi = V;
    for (int c = tid; c < kk; c += 256) {
      for (int i = c; i >= 0; --i) {
        double acc = (i == c) ? 1.0 : 0.0;
        for (int l = i + 1; l <= c; ++l) acc -= A[i + l * SM] * Xi[l + c * SM];
        Xi[i + c * SM] = acc / A[i + i * SM];
      }
    }
    __syncthreads();
    // C1 = Pi_k X: row ord[i] of C1 is row i of X; rows of dropped columns are 0
    for (int e = tid; e < n * kk; e += 256) {
      int i = e % n, c = e / n;
      double v = (i <= c) ? Xi[i + c * SM] : 0.0;
      if (i >= kk) v = 0.0;
      C1[ord[i] + (size_t)c * rmax] = v;
    }
    if (tid == 0) dyn[J.out_rank_slot] = kk;
    return;
  }
  if (J.kind == SK_SKETCH_F && n <= 64) {
    // The truncation: the work-group forms M = R1 R2^{-1} (eight lanes per
    // row for n <= 32, four for n <= 64), M^T = Q2 R2' (Householder,
    // reflectors kept), one-sided Jacobi on B = R2'^T with V, then
    // Z = Q2 V[:, ord] and C1 = R2^{-1} Z_k (eight or four lanes per column).
    __shared__ int s_kk;
    // (the row span G R of a lane group: the smallest that covers n)
    if (n <= 32)
      sketch_f_m_wg<8, 4>(R1, R2, n, A);
    else if (n <= 40)
      sketch_f_m_wg<4, 10>(R1, R2, n, A);
    else if (n <= 48)
      sketch_f_m_wg<4, 12>(R1, R2, n, A);
    else
      sketch_f_m_wg<4, 16>(R1, R2, n, A);
    // M^T = Q2 R2' by the work-group (reflectors kept), then the reflector
    // tails to R1's packed storage (free now) and B = R2'^T into A
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int i = e % n, j = e / n;
      V[i + j * SM] = A[j + i * SM];
    }
    __syncthreads();
    house_qr_keep(V, n, sv, beta);
    for (int e = tid; e < n * n; e += 256) {
      const int i = e % n, j = e / n;
      if (i > j) R1[j * n - j * (j + 1) / 2 + (i - j - 1)] = V[i + j * SM];
      A[i + j * SM] = (i >= j) ? V[j + i * SM] : 0.0;
    }
    for (int j = tid; j < n; j += 256) beta[SM + j] = sv[j];
    // one-sided Jacobi on B by the whole work-group
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int i = e % n, j = e / n;
      V[i + j * SM] = (i == j) ? 1.0 : 0.0;
    }
    {
      const double f2 = fro2_lds(A, n, red);
      const double dt = 1e-3 * eps;
      jacobi_wg(A, V, n, dt * dt * f2);
    }
    __syncthreads();
    if (tid < 64) {
      const int lane = tid;
      // singular values and their order (ties to the lower index)
      if (lane < n) {
        double q = 0.0;
        for (int i = 0; i < n; ++i) q = fma(A[i + lane * SM], A[i + lane * SM], q);
        sv[lane] = sqrt(q);
      }
      wave_sync_lds();
      if (lane < n) {
        // a NaN sorts last, so that ord is a permutation whatever sv holds
        const double me = sv[lane] == sv[lane] ? sv[lane] : -1.0;
        int r = 0;
        for (int i = 0; i < n; ++i) {
          const double o = sv[i] == sv[i] ? sv[i] : -1.0;
          r += (o > me) || (o == me && i < lane);
        }
        ord[r] = lane;
      }
      wave_sync_lds();
      const double smax = sv[ord[0]];
      int kk = 0;
      if (smax > 0.0 && isfinite(smax)) {
        while (kk < n && sv[ord[kk]] > eps * smax) ++kk;
      } else if (!isfinite(smax) && lane == 0) {
        atomicOr(status, STAT_NONFINITE);
      }
      if (fixed_rank > 0) kk = min(kk, fixed_rank);
      if (kk > J.cap) {
        if (lane == 0) {
          atomicOr(status, STAT_RANK_OVERFLOW);
          if (J.need_slot >= 0) atomicMax(dyn + J.need_slot, kk);
        }
        kk = J.cap;
      }
      if (lane == 0) sketch_report(J, dyn, kk, status);
      if (lane == 0) s_kk = kk;
    }
    __syncthreads();
    if (n <= 32)
      sketch_f_out_wg<8, 4>(V, R1, R2, beta, ord, n, s_kk, C1, rmax);
    else
      sketch_f_out_wg<4, 16>(V, R1, R2, beta, ord, n, s_kk, C1, rmax);
    if (tid == 0) dyn[J.out_rank_slot] = s_kk;
    return;
  }
  // ---- form the matrix to decompose
  if (J.kind == SK_RECOMP) {
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, j = e / n;
      double acc = 0.0;
      for (int l = max(i, j); l < n; ++l) acc += R1[upk(i, l)] * R2[upk(j, l)];
      A[i + j * SM] = acc;
    }
  } else {
    // row i solves g R2 = r1_i (R2 upper triangular)
    for (int i = tid; i < n; i += 256) {
      for (int j = 0; j < n; ++j) {
        double acc = (i <= j) ? R1[upk(i, j)] : 0.0;
        for (int l = 0; l < j; ++l) acc -= A[i + l * SM] * R2[upk(l, j)];
        double d = R2[upk(j, j)];
        A[i + j * SM] = (d != 0.0) ? acc / d : 0.0;
      }
    }
  }
  __syncthreads();
  // SK_SKETCH_F: with M^T = Q2 R2 (reflectors kept in R1's packed storage,
  // which is free now), M = R2^T Q2^T, and one-sided Jacobi on B = R2^T
  // (B V = U S) gives the right singular vectors of M as Q2 V; B converges
  // in about half the sweeps M itself needs.
  double* vtop = sv;                    // reused after the reflectors are saved
  if (J.kind == SK_SKETCH_F) {
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, j = e / n;
      V[i + j * SM] = A[j + i * SM];
    }
    __syncthreads();
    house_qr_keep(V, n, vtop, beta);
    // reflectors (strictly lower part) to packed storage, B = R2^T into A
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, j = e / n;
      if (i > j) R1[j * n - j * (j + 1) / 2 + (i - j - 1)] = V[i + j * SM];
      A[i + j * SM] = (i >= j) ? V[j + i * SM] : 0.0;
    }
    for (int j = tid; j < n; j += 256) beta[SM + j] = vtop[j];
    __syncthreads();
  }
  {
    const double f2 = fro2_lds(A, n, red);
    const double dt = 1e-3 * eps;
    if (n <= 64)
      jacobi_svd_wg(A, V, n, dt * dt * f2, red);
    else
      jacobi_svd_lds(A, V, n, dt * dt * f2, red);
  }
  __syncthreads();
  order_desc(A, n, sv, ord);
  const double smax = sv[ord[0]];
  int kk = 0;
  if (smax > 0.0 && isfinite(smax)) {
    while (kk < n && sv[ord[kk]] > eps * smax) ++kk;
  } else if (!isfinite(smax)) {
    if (tid == 0) atomicOr(status, STAT_NONFINITE);
  }
  if (fixed_rank > 0) kk = min(kk, fixed_rank);
  if (kk > J.cap) {
    if (tid == 0) {
      atomicOr(status, STAT_RANK_OVERFLOW);
      if (J.need_slot >= 0) atomicMax(dyn + J.need_slot, kk);
    }
    kk = J.cap;
  }
  if (J.kind == SK_SKETCH_F && tid == 0) sketch_report(J, dyn, kk, status);
  if (J.kind == SK_RECOMP) {
    // A V = X S: CU = R2^T Y_k, CV = R1^T X_k S_k^{-1} = R1^T A[:,ord] / s^2
    double* __restrict__ C2 = refp(bufs, J.C2);
    for (int e = tid; e < n * kk; e += 256) {
      int i = e % n, c = e / n;
      int oc = ord[c];
      double s = sv[oc];
      double cu = 0.0, cv = 0.0;
      for (int l = 0; l <= i; ++l) {
        cu += R2[upk(l, i)] * V[l + oc * SM];
        cv += R1[upk(l, i)] * A[l + oc * SM];
      }
      C1[i + (size_t)c * rmax] = cu;
      C2[i + (size_t)c * rmax] = cv / (s * s);
    }
  } else {
    // Z_k = Q2 V[:, ord[0..k)] into A (reflectors applied last to first),
    // then C = R2^{-1} Z_k by back substitution, one thread per column, in V
    __syncthreads();
    for (int e = tid; e < n * kk; e += 256) {
      int i = e % n, c = e / n;
      A[i + c * SM] = V[i + ord[c] * SM];
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      const double b = beta[j];
      if (b != 0.0) {
        // v = (vtop_j, v_{j+1..n-1}) on rows j..n-1; column c of Z by one thread
        const double* vj = R1 + j * n - j * (j + 1) / 2;
        const double v0 = beta[SM + j];
        for (int c = tid; c < kk; c += 256) {
          double d = v0 * A[j + c * SM];
          for (int i = j + 1; i < n; ++i) d += vj[i - j - 1] * A[i + c * SM];
          d *= b;
          A[j + c * SM] -= d * v0;
          for (int i = j + 1; i < n; ++i) A[i + c * SM] -= d * vj[i - j - 1];
        }
      }
      __syncthreads();
    }
    for (int c = tid; c < kk; c += 256) {
      for (int i = n - 1; i >= 0; --i) {
        double acc = A[i + c * SM];
        for (int l = i + 1; l < n; ++l) acc -= R2[upk(i, l)] * V[l + c * SM];
        double d = R2[upk(i, i)];
        V[i + c * SM] = (d != 0.0) ? acc / d : 0.0;
      }
    }
    __syncthreads();
    for (int e = tid; e < n * kk; e += 256) {
      int i = e % n, c = e / n;
      C1[i + (size_t)c * rmax] = V[i + c * SM];
    }
  }
  if (tid == 0) dyn[J.out_rank_slot] = kk;
}

// ------------------------------------------------------------------ leaf
// value of v in lane `lane` (uniform) of the wave

// Diagonal leaf factorisation (potrf, lower) of an updated tile of order
// p <= 128.  Each thread owns an 8 x 8 block of the tile in registers (rows
// ty + 16a with ty the lane index mod 16, so that loads coalesce; columns
// tx + 16b).  Blocked right-looking Cholesky: each 16-column panel is copied
// to LDS, factorised there column by column, copied back, and applied to the
// trailing columns from registers.
//
// A pivot counts as zero, and the leaf as not positive definite, when it does
// not exceed 64 p u times the diagonal entry of the updated tile (u = 2^-53):
// the rounding error of a leaf Cholesky is of order p u |a_jj|, so an exactly
// singular leaf (two coincident locations without a nugget: two equal
// columns) gives a pivot of that size and either sign, while a positive
// definite one stays far above it.
constexpr int LF = 128, LPW = 16, LPLD = LPW + 1;
constexpr double PIVOT_REL = 64.0 * 0x1p-53;

__global__ __launch_bounds__(256) void k_leaf(const Bufs* __restrict__ bufs, const LeafJob* __restrict__ jobs,
                                              int j0, double* __restrict__ logdet, int* __restrict__ status) {
  const LeafJob J = jobs[j0 + blockIdx.x];
  extern __shared__ double smem[];
  double* Pn = smem;                  // LF x LPLD panel (row i at Pn[i * LPLD])
  double* dg = smem + LF * LPLD;      // diagonal of the factor
  double* thr = dg + LF;              // zero-pivot threshold per column
  const int tid = threadIdx.x, ty = tid & 15, tx = tid >> 4;
  double* __restrict__ Dp = refp(bufs, J.D);
  const int ldd = J.D.ld, p = J.p;
  for (int i = tid; i < p; i += 256) thr[i] = PIVOT_REL * p * fabs(Dp[i + (size_t)i * ldd]);
  double acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      int i = ty + 16 * a, j = tx + 16 * b;
      acc[a][b] = (i < p && j < p) ? Dp[i + (size_t)j * ldd] : 0.0;
    }
  __shared__ int s_bad;
  if (tid == 0) s_bad = -1;
  int bad = -1;
  // register arrays are only indexed by compile-time constants (predicated
  // copies), so that nothing is demoted to indexed register access
#pragma unroll 1
  for (int bb = 0; bb < LF / LPW; ++bb) {
    const int jb = bb * LPW;
    if (jb >= p || bad >= 0) break;
    const int w = min(LPW, p - jb);
    // panel columns jb..jb+w-1 (owned by the threads' column group bb) to LDS;
    // rows above the panel are zero
#pragma unroll
    for (int b = 0; b < LF / LPW; ++b) {
      if (b == bb) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          int i = ty + 16 * a;
          Pn[i * LPLD + tx] = (i >= jb && i < p) ? acc[a][b] : 0.0;
        }
      }
    }
    __syncthreads();
    // the first wave factorises the panel in registers: lane l holds rows
    // jb + l and jb + 64 + l; the pivot row jb + c is lane c, and the entries
    // of column c needed by every lane are read with readlane
    if (tid < 64) {
      const int lane = tid;
      const int ra = jb + lane, rb = jb + 64 + lane;
      double x0[LPW], x1[LPW];
#pragma unroll
      for (int c = 0; c < LPW; ++c) {
        x0[c] = ra < p ? Pn[ra * LPLD + c] : 0.0;
        x1[c] = rb < p ? Pn[rb * LPLD + c] : 0.0;
      }
      int wbad = -1;
#pragma unroll
      for (int c = 0; c < LPW; ++c) {
        if (c < w && wbad < 0) {
          const double d = wave_bcast(x0[c], c);
          if (!(d > thr[jb + c]) || !isfinite(d)) {
            wbad = jb + c;
          } else {
            const double ljj = sqrt(d), inv = 1.0 / ljj;
            if (lane == c)
              x0[c] = ljj;
            else if (lane > c)
              x0[c] *= inv;
            x1[c] *= inv;
            if (lane == 0) dg[jb + c] = ljj;
#pragma unroll
            for (int c2 = c + 1; c2 < LPW; ++c2) {
              if (c2 < w) {
                const double l = wave_bcast(x0[c], c2);
                if (lane >= c2) x0[c2] = fma(-x0[c], l, x0[c2]);
                x1[c2] = fma(-x1[c], l, x1[c2]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < LPW; ++c) {
        if (ra < p) Pn[ra * LPLD + c] = x0[c];
        if (rb < p) Pn[rb * LPLD + c] = x1[c];
      }
      if (lane == 0) s_bad = wbad;
    }
    __syncthreads();
    bad = s_bad;
    if (bad >= 0) break;
    // factorised panel back to the owners; trailing update of later columns
#pragma unroll
    for (int b = 0; b < LF / LPW; ++b) {
      if (b == bb) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          int r = ty + 16 * a;
          acc[a][b] = (r >= jb + tx && r < p) ? Pn[r * LPLD + tx] : 0.0;
        }
      }
    }
#pragma unroll 2
    for (int c = 0; c < w; ++c) {
      double av[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) av[a] = Pn[(ty + 16 * a) * LPLD + c];
#pragma unroll
      for (int b = 1; b < LF / LPW; ++b) {
        if (b > bb && b * 16 < p) {
          const double lj = Pn[(tx + 16 * b) * LPLD + c];
#pragma unroll
          for (int a = 0; a < 8; ++a) acc[a][b] = fma(-av[a], lj, acc[a][b]);
        }
      }
    }
    __syncthreads();   // the panel buffer is rewritten by the next panel
  }
  if (bad >= 0) {
    if (tid == 0) {
      atomicOr(status, STAT_NOT_SPD);
      atomicMin(status + 1, (int)(J.row0 + bad));
      logdet[J.leaf] = NAN;
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      int i = ty + 16 * a, j = tx + 16 * b;
      if (i < p && j < p) Dp[i + (size_t)j * ldd] = (i >= j) ? acc[a][b] : 0.0;
    }
  // log of the diagonal in parallel, summed in index order by one thread
  for (int j = tid; j < p; j += 256) Pn[j] = log(dg[j]);
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < p; ++j) s += Pn[j];
    logdet[J.leaf] = s;
  }
}

// ------------------------------------------------------------------ trsm
// One work-group per job: the lower triangle of L packed in LDS, the (up to
// 64) right-hand-side columns row-major in LDS (conflict-free per lane).
// Blocked substitution: a 16-row diagonal block is solved with one lane per
// column, then the rows below (above, for L^T) are updated by all threads.
// layout 0: X col-major (p x nc); layout 1: X^T stored (element (i,c) at
// X[c + i*ld]); layout 2: solve L^T x = b.
constexpr int TB = 16;
__global__ __launch_bounds__(256) void k_trsm(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                              const TrsmJob* __restrict__ jobs, int j0) {
  const TrsmJob J = jobs[j0 + blockIdx.x];
  const int nc = dimv(dyn, J.ncols);
  const int cw = min(J.cw, nc - J.c0);
  if (cw <= 0) return;
  extern __shared__ double smem[];
  const int p = J.p;
  double* Lp = smem;                       // packed lower: row i at i(i+1)/2
  double* Xs = smem + LF * (LF + 1) / 2;   // p x 64 row-major
  const double* __restrict__ L = refp(bufs, J.L);
  const int ldl = J.L.ld;
  const int tid = threadIdx.x;
  // loads are issued 8 at a time before their LDS stores (latency hiding)
  for (int base = 0; base < p * p; base += 2048) {
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int i = e % p, j = e / p;
      r[u] = (e < p * p && i >= j) ? L[i + (size_t)j * ldl] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int i = e % p, j = e / p;
      if (e < p * p && i >= j) Lp[i * (i + 1) / 2 + j] = r[u];
    }
  }
  double* __restrict__ X = refp(bufs, J.X);
  const int ldx = J.X.ld;
  for (int base = 0; base < p * 64; base += 2048) {
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int c, i;
      if (J.layout == 1) {
        c = e & 63;
        i = e >> 6;
      } else {
        i = e % p;
        c = e / p;
      }
      if (J.layout == 3)
        r[u] = (e < p * 64 && c < cw && i == J.c0 + c) ? 1.0 : 0.0;   // columns of the identity
      else
        r[u] = (e < p * 64 && c < cw) ? (J.layout == 1 ? X[(J.c0 + c) + (size_t)i * ldx] : X[i + (size_t)(J.c0 + c) * ldx])
                                      : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int c, i;
      if (J.layout == 1) {
        c = e & 63;
        i = e >> 6;
      } else {
        i = e % p;
        c = e / p;
      }
      if (e < p * 64 && c < cw) Xs[i * 64 + c] = r[u];
    }
  }
  __shared__ double rdiag[LF];
  __syncthreads();
  for (int i = tid; i < p; i += 256) rdiag[i] = 1.0 / Lp[i * (i + 1) / 2 + i];
  __syncthreads();
  if (J.layout != 2) {
    for (int b0 = 0; b0 < p; b0 += TB) {
      const int b1 = min(b0 + TB, p);
      if (tid < cw) {
        // the block's 16 unknowns of this column stay in registers
        double xr[TB];
#pragma unroll
        for (int u = 0; u < TB; ++u) xr[u] = (b0 + u < b1) ? Xs[(b0 + u) * 64 + tid] : 0.0;
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          if (b0 + u < b1) {
            const double* Li = Lp + (b0 + u) * (b0 + u + 1) / 2 + b0;
            double s0 = xr[u], s1 = 0.0;
#pragma unroll
            for (int v = 0; v < u; ++v) {
              if (v & 1)
                s1 = fma(-Li[v], xr[v], s1);
              else
                s0 = fma(-Li[v], xr[v], s0);
            }
            xr[u] = (s0 + s1) * rdiag[b0 + u];
          }
        }
#pragma unroll
        for (int u = 0; u < TB; ++u)
          if (b0 + u < b1) Xs[(b0 + u) * 64 + tid] = xr[u];
      }
      __syncthreads();
      // rows below the block: thread owns column c = tid & 63 and rows
      // b1 + (tid >> 6) + 4u; four independent accumulations per pass
      {
        const int c = tid & 63;
        if (c < cw) {
          for (int i0 = b1 + (tid >> 6); i0 < p; i0 += 16) {
            double acc4[4] = {0.0, 0.0, 0.0, 0.0};
            int ro[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              int i = i0 + 4 * u;
              ro[u] = i < p ? i * (i + 1) / 2 : 0;
            }
            for (int j = b0; j < b1; ++j) {
              double xj = Xs[j * 64 + c];
#pragma unroll
              for (int u = 0; u < 4; ++u) acc4[u] += Lp[ro[u] + j] * xj;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              int i = i0 + 4 * u;
              if (i < p) Xs[i * 64 + c] -= acc4[u];
            }
          }
        }
      }
      __syncthreads();
    }
  } else {
    for (int b1 = p; b1 > 0; b1 -= TB) {
      const int b0 = max(b1 - TB, 0);
      if (tid < cw) {
        for (int i = b1 - 1; i >= b0; --i) {
          double s = Xs[i * 64 + tid];
          for (int j = i + 1; j < b1; ++j) s -= Lp[j * (j + 1) / 2 + i] * Xs[j * 64 + tid];
          Xs[i * 64 + tid] = s / Lp[i * (i + 1) / 2 + i];
        }
      }
      __syncthreads();
      for (int e = tid; e < b0 * 64; e += 256) {
        int c = e & 63, i = e >> 6;
        if (c < cw) {
          double s = 0.0;
          for (int j = b0; j < b1; ++j) s += Lp[j * (j + 1) / 2 + i] * Xs[j * 64 + c];
          Xs[i * 64 + c] -= s;
        }
      }
      __syncthreads();
    }
  }
  if (J.layout == 1) {
    for (int e = tid; e < p * 64; e += 256) {
      int c = e & 63, i = e >> 6;
      if (c < cw) X[(J.c0 + c) + (size_t)i * ldx] = Xs[e];
    }
  } else {
    for (int e = tid; e < p * 64; e += 256) {
      int i = e % p, c = e / p;
      if (c < cw) X[i + (size_t)(J.c0 + c) * ldx] = Xs[i * 64 + c];
    }
  }
}

// X <- L X with L the stored inverse of a diagonal leaf factor (lower
// triangular, p <= 128) and X a panel of up to 64 columns (layout 0: col-major;
// layout 1: X^T stored).  No dependency chain: thread (tr, tc) accumulates
// rows tr + 16a (a < 8) of columns 4 tc .. 4 tc + 3 over k = 0 .. i.
__global__ __launch_bounds__(256) void k_trmm(const Bufs* __restrict__ bufs, const int* __restrict__ dyn,
                                              const TrsmJob* __restrict__ jobs, int j0) {
  const TrsmJob J = jobs[j0 + blockIdx.x];
  const int nc = dimv(dyn, J.ncols);
  const int cw = min(J.cw, nc - J.c0);
  if (cw <= 0) return;
  extern __shared__ double smem[];
  const int p = J.p;
  double* Lp = smem;                       // packed lower: row i at i(i+1)/2
  double* Xs = smem + LF * (LF + 1) / 2;   // p x 64 row-major
  const double* __restrict__ L = refp(bufs, J.L);
  const int ldl = J.L.ld;
  const int tid = threadIdx.x;
  for (int base = 0; base < p * p; base += 2048) {
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int i = e % p, j = e / p;
      r[u] = (e < p * p && i >= j) ? L[i + (size_t)j * ldl] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int i = e % p, j = e / p;
      if (e < p * p && i >= j) Lp[i * (i + 1) / 2 + j] = r[u];
    }
  }
  double* __restrict__ X = refp(bufs, J.X);
  const int ldx = J.X.ld;
  for (int base = 0; base < p * 64; base += 2048) {
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int c = (J.layout == 1) ? (e & 63) : (e / p), i = (J.layout == 1) ? (e >> 6) : (e % p);
      r[u] = (e < p * 64 && c < cw) ? (J.layout == 1 ? X[(J.c0 + c) + (size_t)i * ldx] : X[i + (size_t)(J.c0 + c) * ldx])
                                    : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256 + tid;
      int c = (J.layout == 1) ? (e & 63) : (e / p), i = (J.layout == 1) ? (e >> 6) : (e % p);
      if (e < p * 64) Xs[i * 64 + c] = (c < cw) ? r[u] : 0.0;
    }
  }
  __syncthreads();
  const int tr = tid & 15, tc = tid >> 4;
  double acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  if (4 * tc < cw) {
    for (int k = 0; k < p; ++k) {
      double xb[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) xb[b] = Xs[k * 64 + 4 * tc + b];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int i = tr + 16 * a;
        if (i >= k && i < p) {
          const double l = Lp[i * (i + 1) / 2 + k];
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(l, xb[b], acc[a][b]);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int i = tr + 16 * a;
    if (i >= p) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = 4 * tc + b;
      if (c >= cw) continue;
      if (J.layout == 1)
        X[(J.c0 + c) + (size_t)i * ldx] = acc[a][b];
      else
        X[i + (size_t)(J.c0 + c) * ldx] = acc[a][b];
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
                                             double eps_aca, int kcap, int cap_ok, int* __restrict__ status) {
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
  const int kmax = min(min(p, q), min(kcap, J.cap));
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
  if (k == kmax && kmax < min(p, q) && !cap_ok && tid == 0) {
    atomicOr(status, STAT_RANK_OVERFLOW);
    if (J.need_slot >= 0) atomicMax(dyn + J.need_slot, kmax + 1);
  }
  if (tid == 0) dyn[J.rank_slot] = k;
  (void)dots;
}

// ------------------------------------------------------------------ utilities
// After the assembly, per low-rank block (x: rank slot, y: sketch-width slot,
// z: rank-hint slot, w: candidate-hint slot): the sketch width of the sweep
// is the larger of the assembled rank and the hint, plus the oversampling.
__global__ void k_copy_rank(int* __restrict__ dyn, const int4* __restrict__ slots, int n, int oversample) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int4 s = slots[i];
    dyn[s.y] = max(dyn[s.x], dyn[s.z]) + oversample;
  }
}

// After a factorisation whose sketches saturated: the candidate hints it
// wrote become the rank hints.
__global__ void k_adopt_hints(int* __restrict__ dyn, const int4* __restrict__ slots, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dyn[slots[i].z] = dyn[slots[i].w];
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
// Partial sums of 1024 entries per work-group: mode 0 sum x_i^2, mode 1
// sum x_i, mode 2 sum x_i y_i (fixed order: deterministic).
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ x, const double* __restrict__ y,
                                                int64_t n, int mode, double* __restrict__ part) {
  __shared__ double s8[8];
  int64_t base = (int64_t)blockIdx.x * 1024;
  double s = 0.0;
  for (int r = 0; r < 4; ++r) {
    int64_t i = base + threadIdx.x + 256 * r;
    if (i < n) {
      double v = x[i];
      s += mode == 0 ? v * v : (mode == 1 ? v : v * y[i]);
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


// y = C x with the exact entries of Eq. (3) evaluated on the fly (plus the
// nugget on the diagonal): one row per thread, the columns streamed through
// LDS in tiles of 256 locations, summed in increasing column order.
__global__ __launch_bounds__(256) void k_exact_matvec(const double2* __restrict__ loc, const double* __restrict__ x,
                                                      double* __restrict__ y, int64_t n, MaternParams P) {
  __shared__ double2 sl[256];
  __shared__ double sx[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double2 me = i < n ? loc[i] : make_double2(0.0, 0.0);
  double acc = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    sl[threadIdx.x] = j < n ? loc[j] : make_double2(0.0, 0.0);
    sx[threadIdx.x] = j < n ? x[j] : 0.0;
    __syncthreads();
    const int m = (int)min<int64_t>(256, n - j0);
    for (int t = 0; t < m; ++t) {
      const double dx = me.x - sl[t].x, dy = me.y - sl[t].y;
      acc = fma(matern_eval(sqrt(dx * dx + dy * dy), P), sx[t], acc);
    }
    __syncthreads();
  }
  if (i < n) y[i] = fma(P.nugget, x[i], acc);
}

hipError_t launch_exact_matvec(const double* loc, const double* x, double* y, int64_t n, const MaternParams& P,
                               hipStream_t st) {
  if (n > 0) k_exact_matvec<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const double2*)loc, x, y, n, P);
  return hipGetLastError();
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

constexpr size_t LDS_QR = (size_t(QR_LDS) + 8) * 8;
constexpr size_t LDS_SMALL = (size_t(2) * SM * SM + size_t(SM) * (SM + 1) + SM + 8 + 2 * SM) * 8 + SM * 4;
constexpr size_t LDS_LEAF = size_t(LF * LPLD + 2 * LF) * 8;
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
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_trmm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_TRSM);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_gemm_wide, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_GEMM_WIDE);
  return e;
}

hipError_t launch_stage(const Stage& s, const LaunchCtx& L, hipStream_t st) {
  const int n = s.end - s.begin;
  switch (s.kind) {
    case ST_GEMM:
      if (n > 0) k_gemm<<<n, 256, 0, st>>>(L.dbufs, L.dyn, L.gjobs, L.gprods, L.gtiles, s.begin);
      break;
    case ST_GEMM_WIDE:
      if (n > 0)
        k_gemm_wide<<<n, 256 * GW, LDS_GEMM_WIDE, st>>>(L.dbufs, L.dyn, L.gjobs, L.gprods, L.gtiles, s.begin);
      break;
    case ST_TSQR_SEG:
      if (n > 0) k_tsqr_seg<<<n, 256, LDS_QR, st>>>(L.dbufs, L.dyn, L.tsegs, s.begin, L.rmax);
      break;
    case ST_TSQR_RED:
      if (n > 0) k_tsqr_red<<<n, 256, LDS_QR, st>>>(L.dbufs, L.dyn, L.treds, s.begin, L.rmax);
      break;
    case ST_SMALL:
      if (n > 0)
        k_small<<<n, 256, LDS_SMALL, st>>>(L.dbufs, L.dyn, L.smalls, s.begin, L.rmax, L.eps, L.tau, L.fixed_rank,
                                           L.status);
      break;
    case ST_LEAF:
      if (n > 0) k_leaf<<<n, 256, LDS_LEAF, st>>>(L.dbufs, L.leafs, s.begin, L.logdet, L.status);
      break;
    case ST_TRSM:
      if (n > 0) k_trsm<<<n, 256, LDS_TRSM, st>>>(L.dbufs, L.dyn, L.trsms, s.begin);
      break;
    case ST_TRMM:
      if (n > 0) k_trmm<<<n, 256, LDS_TRSM, st>>>(L.dbufs, L.dyn, L.trsms, s.begin);
      break;
    case ST_COPY_RANK:
      if (L.n_copy > 0)
        k_copy_rank<<<(L.n_copy + 255) / 256, 256, 0, st>>>(L.dyn, L.copy_pairs, L.n_copy, L.oversample);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adopt_hints(const LaunchCtx& L, hipStream_t st) {
  if (L.n_copy > 0) k_adopt_hints<<<(L.n_copy + 255) / 256, 256, 0, st>>>(L.dyn, L.copy_pairs, L.n_copy);
  return hipGetLastError();
}

hipError_t launch_fill(double* D, const double* loc, const FillJob* jobs, int njobs, const MaternParams& P,
                       hipStream_t st) {
  if (njobs > 0) k_dense_fill<<<njobs, 256, 0, st>>>(D, (const double2*)loc, jobs, P);
  return hipGetLastError();
}

hipError_t launch_aca(double* U, double* V, int* dyn, const double* loc, const AcaJob* jobs, int njobs,
                      const MaternParams& P, double eps_aca, int kcap, int cap_ok, int* status, hipStream_t st) {
  if (njobs > 0)
    k_aca<<<njobs, 256, 0, st>>>(U, V, dyn, (const double2*)loc, jobs, P, eps_aca, kcap, cap_ok, status);
  return hipGetLastError();
}

hipError_t launch_permute(const double* in, double* out, const int* perm, int64_t n, int scatter,
                          hipStream_t st) {
  if (n > 0) k_permute<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(in, out, perm, n, scatter);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* x, const double* y, int64_t n, int mode, double* part, hipStream_t st,
                         int64_t* nparts) {
  int64_t nb = (n + 1023) / 1024;
  *nparts = nb;
  if (nb > 0) k_reduce<<<(unsigned)nb, 256, 0, st>>>(x, y, n, mode, part);
  return hipGetLastError();
}

// y = a x + b y
__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], b * y[i]);
}

hipError_t launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t st) {
  if (n > 0) k_axpby<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(y, x, a, b, n);
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
