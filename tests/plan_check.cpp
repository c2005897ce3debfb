// Host-side bounds check of a factorisation plan (test infrastructure).
//
// Reads a block tree (n, depth, leaf, count, then count x (level, row node,
// col node, kind) as little-endian int64) from the file argv[1], builds the
// plan with max_rank 64 and the per-block rooms named by argv[2] ("64", any
// other number for every block, or "rand" for seeded rooms in [1, 64]), and
// checks that every operand a kernel may touch lies inside its buffer at the
// largest values its dynamic dimensions can take: GEMM outputs and both
// operands of every product (and each product inside its job's extent), TSQR
// inputs and R slots, the small jobs' R and coefficient slots, the diagonal
// leaves, the triangular solves' factors and panels, and every low-rank
// block's U and V.  Prints one summary line (with the plan's dynamic-slot
// and stage counts, which must not depend on the rooms: a context that grows
// its rooms keeps its rank hints by slot number); exit status 2 on a
// violation.
// Compiled with -DSHRINK=b it under-sizes buffer b by one element, so that a
// test can see the check fail.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "plan.h"

using namespace hc;

namespace {

int64_t g_size[B_COUNT];
long g_bad = 0;

void check(const char* what, const Ref& r, int64_t last, long idx) {
  if (r.buf < 0 || r.buf >= B_COUNT) {
    if (g_bad++ < 10) std::printf("%s %ld: buffer id %d\n", what, idx, r.buf);
    return;
  }
  if (r.off < 0 || r.off + last >= g_size[r.buf])
    if (g_bad++ < 10)
      std::printf("%s %ld: buffer %d offset %lld last %lld size %lld\n", what, idx, r.buf, (long long)r.off,
                  (long long)last, (long long)g_size[r.buf]);
}

// last element of an m x k operand stored col-major (t = 0) or transposed
int64_t last_of(int rows, int cols, int ld, int t) {
  return t ? (cols - 1) + int64_t(rows - 1) * ld : (rows - 1) + int64_t(cols - 1) * ld;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 3) return 1;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 1;
  int64_t hdr[4];
  if (std::fread(hdr, 8, 4, f) != 4) return 1;
  const int64_t n = hdr[0], depth = hdr[1], leaf = hdr[2], nb = hdr[3];
  std::vector<int64_t> blk(size_t(4 * nb));
  if (std::fread(blk.data(), 8, blk.size(), f) != blk.size()) return 1;
  std::fclose(f);
  const std::string mode = argv[2];
  std::vector<int32_t> rooms(size_t(nb), 64);
  std::mt19937 gen(7);
  for (auto& c : rooms) c = mode == "rand" ? 1 + int(gen() % 64) : std::atoi(mode.c_str());
  Plan P;
  const std::string e = build_plan(P, n, int(depth), int(leaf), blk.data(), nb, 64, false, rooms.data());
  if (!e.empty()) {
    std::printf("plan error: %s\n", e.c_str());
    return 1;
  }
  g_size[B_DENSE] = P.dense_elems;
  g_size[B_U] = P.u_elems;
  g_size[B_V] = P.v_elems;
  g_size[B_SCR] = P.scr_elems;
  g_size[B_OMEGA] = P.omega_rows * P.rcap;
  g_size[B_RHS] = 2 * P.rhs_ld;
  g_size[B_PERS] = P.pers_elems;
  g_size[B_LINV] = P.linv_elems;
#ifdef SHRINK
  g_size[SHRINK] -= 1;
#endif
  const int RM = P.rmax;
  const int64_t slot = int64_t(RM) * RM - 1;
  for (size_t j = 0; j < P.gjobs.size(); ++j) {
    const GemmJob& J = P.gjobs[j];
    const int m = J.m.maxv, nn = J.n.maxv;
    if (m > 0 && nn > 0) check("gemm C", J.C, last_of(m, nn, J.C.ld, 0), long(j));
    for (int p = J.p0; p < J.p1; ++p) {
      const GemmProd& Q = P.gprods[size_t(p)];
      const int mi = Q.mi.maxv, nj = Q.nj.maxv, k = Q.k.maxv;
      if (mi <= 0 || nj <= 0 || k <= 0) continue;
      if (Q.i0 < 0 || Q.j0 < 0 || Q.i0 + mi > m || Q.j0 + nj > nn)
        if (g_bad++ < 10) std::printf("product %d outside job %zu\n", p, j);
      check("gemm A", Q.A, last_of(mi, k, Q.A.ld, Q.ta), p);
      check("gemm B", Q.B, last_of(k, nj, Q.B.ld, Q.tb), p);
    }
  }
  for (size_t i = 0; i < P.tsegs.size(); ++i) {
    const TsqrSeg& S = P.tsegs[i];
    if (S.cols.maxv > RM && g_bad++ < 10) std::printf("tsqr segment %zu: %d columns\n", i, S.cols.maxv);
    check("tsqr X", S.X, last_of(S.rows, S.cols.maxv, S.X.ld, 0), long(i));
    check("tsqr R", S.R, slot, long(i));
  }
  for (size_t i = 0; i < P.treds.size(); ++i) {
    check("tsqr R0", P.treds[i].R0, int64_t(P.treds[i].nseg) * RM * RM - 1, long(i));
    check("tsqr Rout", P.treds[i].R, slot, long(i));
  }
  for (size_t i = 0; i < P.smalls.size(); ++i) {
    const SmallJob& J = P.smalls[i];
    if (J.k.maxv > RM && g_bad++ < 10) std::printf("small job %zu: width %d\n", i, J.k.maxv);
    check("small R1", J.R1, slot, long(i));
    if (J.kind != SK_SKETCH_P) check("small R2", J.R2, slot, long(i));
    check("small C1", J.C1, slot, long(i));
    if (J.kind == SK_RECOMP) check("small C2", J.C2, slot, long(i));
  }
  for (size_t i = 0; i < P.leafs.size(); ++i)
    check("leaf", P.leafs[i].D, last_of(P.leafs[i].p, P.leafs[i].p, P.leafs[i].D.ld, 0), long(i));
  for (size_t i = 0; i < P.trsms.size(); ++i) {
    const TrsmJob& T = P.trsms[i];
    check("trsm L", T.L, last_of(T.p, T.p, T.L.ld, 0), long(i));
    const int nc = T.ncols.maxv;
    if (nc > 0) check("trsm X", T.X, last_of(T.p, nc, T.X.ld, T.layout == 1 ? 1 : 0), long(i));
  }
  for (const auto& B : P.blocks) {
    if (B.kind != 1) continue;
    check("U", Ref{B_U, int32_t(B.r1 - B.r0), B.off_u}, (B.r1 - B.r0) * B.cap - 1, 0);
    check("V", Ref{B_V, int32_t(B.c1 - B.c0), B.off_v}, (B.c1 - B.c0) * B.cap - 1, 0);
  }
  size_t stages = P.recomp_stages.size();
  for (const auto& st : P.steps) stages += st.size();
  std::printf("n=%lld rooms %s: %zu GEMM jobs, %zu products, %zu TSQR segments, %zu small jobs; U+V %lld elements; "
              "dynamic slots %d, stages %zu; violations %ld\n",
              (long long)n, mode.c_str(), P.gjobs.size(), P.gprods.size(), P.tsegs.size(), P.smalls.size(),
              (long long)(P.u_elems + P.v_elems), P.n_dyn, stages, g_bad);
  return g_bad ? 2 : 0;
}
