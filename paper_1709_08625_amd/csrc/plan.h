// Host-side plan of the H-matrix assembly and H-Cholesky sweep, plus the POD
// job descriptors the GPU kernels execute.  Everything here is a function of
// the two trees only (never of theta), so one plan serves every likelihood
// evaluation on the same locations; ranks are data dependent and are read by
// the kernels from a device array of "dynamic dimensions".
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

namespace hc {

// ---------------------------------------------------------------- buffers
// Every matrix operand is addressed relative to one of these device buffers,
// so plans do not depend on allocation addresses.
enum BufId : int32_t {
  B_DENSE = 0,   // dense leaves (col-major, one tile per dense block)
  B_U = 1,       // low-rank U factors, p x cap col-major per block (cap: the block's rank room)
  B_V = 2,       // low-rank V factors, q x cap col-major per block
  B_SCR = 3,     // per-step scratch (reset every step)
  B_OMEGA = 4,   // fixed Gaussian test matrix (Nmax x rcap col-major)
  B_RHS = 5,     // right-hand side solved inside the sweep (cluster order)
  B_PERS = 6,    // persistent scratch (assembly, R factors, coefficients)
  B_LINV = 7,    // inverses of the diagonal leaf factors (p x p col-major per leaf)
  B_COUNT = 8
};

struct Ref {
  int32_t buf;
  int32_t ld;
  int64_t off;  // element offset
};

// A dimension: static value (slot < 0) or min(dyn[slot] + add, maxv).
struct Dim {
  int32_t slot;
  int32_t add;
  int32_t maxv;
};
inline Dim dim_static(int v) { return Dim{-1, 0, v}; }
inline Dim dim_dyn(int slot, int maxv, int add = 0) { return Dim{slot, add, maxv}; }

// ---------------------------------------------------------------- GEMM jobs
// C[i0+i, j0+j] (+)= alpha * sum_kk op(A)[i,kk] * op(B)[kk,j]
// op(A) is m x k: ta=0 -> A[i + kk*lda], ta=1 -> A[kk + i*lda]
// op(B) is k x n: tb=0 -> B[kk + j*ldb], tb=1 -> B[j + kk*ldb]
struct GemmProd {
  Ref A;
  Ref B;
  Dim k;
  Dim mi;      // rows of C touched by this product (from i0)
  Dim nj;      // cols of C touched by this product (from j0)
  int32_t i0, j0;
  int32_t ta, tb;
  double alpha;
};

struct GemmJob {
  Ref C;
  Dim m, n;          // extent of C written by this job
  int32_t zero;      // 1: C := sum (C is overwritten on its m x n extent)
  int32_t p0, p1;    // products [p0, p1)
  int32_t fp32;      // 1: products accumulated in FP32 (mixed precision)
};

// Tile of a GEMM launch (capacity-based grid, dynamic tiles exit early).
struct GemmTile {
  int32_t job;
  int32_t ti, tj;
  int32_t pad;
};

// ---------------------------------------------------------------- TSQR jobs
// R factor of a tall matrix X (rows x cols, cols <= RMAX): the local stage
// computes one R per segment of consecutive rows; the reduce stage combines
// the segment Rs of one matrix.  R is stored upper-triangular in an
// RMAX x RMAX col-major slot (ld = RMAX) and is zero-padded beyond cols.
struct TsqrSeg {
  Ref X;          // start of this segment (row offset already applied)
  int32_t rows;   // rows in this segment
  Dim cols;
  Ref R;          // output R of this segment
};
struct TsqrRed {
  Ref R0;         // first segment R (ld RMAX), nseg consecutive slots
  int32_t nseg;
  Dim cols;
  Ref R;          // output
};

// ---------------------------------------------------------------- small jobs
enum SmallKind : int32_t {
  SK_RECOMP = 0,   // SVD(RU RV^T) -> CU = RV^T Y_k, CV = RU^T X_k S_k^-1; rank
  SK_SKETCH_P = 1, // SVD(RY) -> P = W_y S_y^-1 (kept dirs), kept count
  SK_SKETCH_F = 2, // Z_k from SVD(RB RQ^-1) -> C = RQ^-1 Z_k; rank
};
struct SmallJob {
  int32_t kind;
  int32_t out_rank_slot;   // dyn slot receiving the new rank / kept count
  Dim k;                   // input width (cols of the R factors)
  Ref R1, R2;              // input R factors (ld RMAX)
  Ref C1, C2;              // outputs (ld RMAX)
  int32_t cap;             // maximal allowed output rank
  Dim sat;                 // sketch width (saturation test); static -1 = none
  int32_t full;            // min(p, q) of the block: a sketch this wide spans
                           // the whole column space and cannot saturate
  int32_t cand_slot;       // dyn slot of the block's candidate rank hint (-1: none)
  double eps;              // < 0: taken from the launch (-1 eps, -2 tau)
  int32_t need_slot = -1;  // dyn slot receiving the untruncated count when it exceeds cap (-1: none)
  int32_t pad = 0;
};

// ---------------------------------------------------------------- leaf jobs
// Diagonal leaf (p <= LEAF_MAX), already updated: factorised in place
// (potrf, lower) and sum log L_ii is stored to logdet[leaf].
struct LeafJob {
  Ref D;
  int32_t p;
  int32_t leaf;     // leaf index for logdet / error reporting
  int64_t row0;     // global cluster-order index of the first row (errors)
};

// ---------------------------------------------------------------- trsm jobs
// X <- L^{-1} X for a panel of right-hand sides, L lower triangular p x p.
// Layout 3 forms the inverse: columns [c0, c0+cw) of X <- L^{-1} (X p x p
// col-major, the identity is generated in place of a load).  The same job
// record drives the multiplication stage ST_TRMM, X <- L X with L the stored
// inverse (layouts 0 and 1 only).
// layout 0: X is p x ncols col-major (ld); layout 1: X^T is stored, i.e.
// element (i, c) of X is at X[c + i*ld] (dense target solved from the right).
struct TrsmJob {
  Ref L;
  int32_t p;
  int32_t layout;
  Ref X;
  Dim ncols;
  int32_t c0;       // first column of this job's chunk
  int32_t cw;       // chunk width
};

// ---------------------------------------------------------------- stages
// ST_FORK: the second lane (stream) waits for the work issued so far on the
// first; ST_JOIN: the first lane waits for the work issued on the second.
// ST_GEMM_WIDE: the same tiles as ST_GEMM, run by the grouped kernel
// (GEMM_GROUPS groups of 256 threads per tile) for launches bound by their
// longest tile.
constexpr int GEMM_GROUPS = 2;   // groups of 256 threads of the grouped GEMM kernel
enum StageKind : int32_t { ST_GEMM = 0, ST_TSQR_SEG, ST_TSQR_RED, ST_SMALL, ST_LEAF, ST_TRSM, ST_COPY_RANK,
                           ST_FORK, ST_JOIN, ST_TRMM, ST_GEMM_WIDE };
struct Stage {
  int32_t kind;
  int32_t begin, end;   // item range in the kind's array (tiles for GEMM)
  int32_t lane = 0;     // 0: the context's stream, 1: its second stream
  int32_t alt = 0;      // GEMM: 1 when the other GEMM kernel may run it too
};

// ---------------------------------------------------------------- tree data
struct BlockInfo {
  int32_t level, a, c, kind;   // kind 1 = LR, 0 = dense
  int64_t r0, r1, c0, c1;      // row/col ranges (cluster order)
  int64_t off_d;               // dense offset (elements) in B_DENSE
  int64_t off_u, off_v;        // LR offsets in B_U / B_V
  int32_t rank_slot;           // dyn slot of the current rank (LR)
  int32_t rank0_slot;          // dyn slot of the ACA rank, then of the sketch width (LR)
  int32_t hint_slot;           // dyn slot of the rank hint of the sweep's sketch width (LR)
  int32_t cand_slot;           // dyn slot of the rank the last factorisation kept (LR)
  int32_t cap;                 // columns of the block's U and V arenas (LR): its rank capacity
  int32_t need_slot;           // dyn slot of the largest rank a truncation or the ACA asked beyond cap (LR)
};

struct Plan {
  // structure
  int64_t n = 0;
  bool mixed = false;   // low-rank GEMM work in FP32 (dense leaves, potrf, solves FP64)
  // rcap: widest randomised sketch (rank + oversampling), rmax = max(rcap, kcap)
  int D = 0, leaf = 0, kcap = 64, rcap = 80, rmax = 80;
  std::vector<std::vector<int64_t>> lo;   // lo[l][i] node start (size 2^l + 1 incl. end)
  std::vector<BlockInfo> blocks;
  std::unordered_map<uint64_t, int32_t> status;   // (l,a,c) -> block id, or -1 = subdivided
  std::vector<int32_t> diag_block;                // leaf j -> block id of (j, j)
  int64_t dense_elems = 0, u_elems = 0, v_elems = 0, linv_elems = 0;
  std::vector<int64_t> linv_off;                  // leaf j -> offset of its inverse in B_LINV
  int32_t n_dyn = 0;                               // dynamic dimension slots

  // executable job arrays (all steps share them; stages index into them)
  std::vector<GemmJob> gjobs;
  std::vector<GemmProd> gprods;
  std::vector<GemmTile> gtiles;
  std::vector<TsqrSeg> tsegs;
  std::vector<TsqrRed> treds;
  std::vector<SmallJob> smalls;
  std::vector<LeafJob> leafs;
  std::vector<TrsmJob> trsms;

  // schedules
  std::vector<Stage> recomp_stages;              // assembly recompression
  std::vector<std::vector<Stage>> steps;          // factorisation sweep (with the fused RHS column)
  int64_t scr_elems = 0;                          // per-step scratch size
  int64_t pers_elems = 0;                         // persistent scratch size
  int64_t omega_rows = 0;

  // forward/backward solve schedules on B_RHS (single vector)
  std::vector<std::vector<Stage>> fsolve_steps;
  std::vector<std::vector<Stage>> bsolve_steps;
  // H-matvec C~ x (assembled matrix), x in B_RHS col 0, y in col 1
  std::vector<Stage> matvec_stages;
  // y = L~ x and y = L~^T x (x in B_RHS col 0, y col 1)
  std::vector<Stage> lmul_stages;
  std::vector<Stage> ltmul_stages;

  int64_t rhs_ld = 0;   // leading dimension of B_RHS (= n), 2 columns

  // statistics
  int64_t n_lr = 0, n_dense = 0, lr_rows = 0;
  int64_t n_launch_fact = 0;
};

inline uint64_t key3(int l, int64_t a, int64_t c) {
  return (uint64_t(l) << 58) | (uint64_t(a) << 29) | uint64_t(c);
}

// Build the plan from the tree structure.  blocks_lac: n_blocks x 4
// (level, row node, col node, kind) in breadth-first order.
// Returns an empty string on success, else an error message.
// The sketch width of a low-rank target is the larger of its assembly rank
// and its rank hint, plus an oversampling chosen at run time (see
// ST_COPY_RANK), at most the block's room + OVERSAMPLE_MAX (rcap = kcap +
// OVERSAMPLE_MAX for a block at the full room).  A factorisation
// writes every target's kept rank (doubled sketch width where the sketch
// saturated) as its candidate hint; the candidates become the hints only
// after a factorisation that saturated, so that the widths, and with them
// the results, change only when a sketch was too narrow.
constexpr int OVERSAMPLE_MAX = 16;
// caps: per block (n_blocks entries, read for low-rank blocks) the columns of
// its U and V arenas, each in [1, kcap]; nullptr gives every block kcap.
std::string build_plan(Plan& P, int64_t n, int D, int leaf, const int64_t* blocks_lac,
                       int64_t n_blocks, int kcap, bool mixed, const int32_t* caps = nullptr);

int64_t node_lo(const Plan& P, int l, int64_t i);
int64_t node_hi(const Plan& P, int l, int64_t i);

}  // namespace hc
