// Planner: turns the cluster tree and block cluster tree into job lists.
//
// The factorisation is a left-looking H-Cholesky over the leaf clusters
// c_0 .. c_{m-1} of a perfect binary cluster tree (Eq. (2) of Sec. 1; H-matrix
// factorisation with the fixed accuracy eps of Sec. 2.2).  For a factor block
// T = (rho, pi) the Cholesky identity gives
//     L(rho,pi) = ( C(rho,pi) - L(rho, <pi) L(pi, <pi)^T ) L(pi,pi)^{-T},
// where "<pi" are the columns before pi.  Those columns are the left
// siblings K of the ancestors of pi that are right sons, so the update is a
// sum of products L(rho,K) L(pi,K)^T; each product is expanded recursively on
// the block tree until one side is a single low-rank or dense leaf, which
// keeps every term of low rank.  The update is applied when the sweep reaches
// the first leaf of pi; low-rank targets are then recompressed to accuracy
// eps by a randomised range finder with exact QR-based truncation, and their
// V factor is solved against L(pi,pi) one leaf row at a time as the sweep
// passes through pi (forward substitution interleaved with the
// factorisation, with the sibling blocks of the cluster tree applied as
// H-matrix-vector products).
#include "plan.h"

#include <algorithm>
#include <cassert>
#include <cstdio>
#include <functional>
#include <map>
#include <tuple>

namespace hc {

static const int TM = 64, TN = 64;   // GEMM tile (must match the kernel)
static const int TSQR_SEG = 384;     // rows per TSQR segment work-group
static const int TSQR_FAN = 16;      // R factors per TSQR reduction work-group
static const int LEAF_MAX = 128;

int64_t node_lo(const Plan& P, int l, int64_t i) { return P.lo[l][i]; }
int64_t node_hi(const Plan& P, int l, int64_t i) { return P.lo[l][i + 1]; }

namespace {

struct Src {
  Ref ref;
  Dim cols;
};

struct Term {
  int64_t r0, r1;   // absolute rows (inside the target's rows)
  int64_t p0, p1;   // absolute rows of the V side (inside the target's cols)
  Src U, V;
};

class Builder {
 public:
  Plan& P;
  // per-step scratch bump allocator
  int64_t scr_top = 0;
  int32_t cur_lane = 0;   // lane of the stages emitted next
  int32_t dyn_base = 0, dyn_top = 0, dyn_max = 0;
  // current stage buffers (one step at a time)
  struct GemmStage {
    std::vector<int32_t> jobs;
  };

  explicit Builder(Plan& p) : P(p) {}

  int64_t scr_alloc(int64_t elems) {
    int64_t o = scr_top;
    scr_top += (elems + 31) / 32 * 32;
    if (scr_top > P.scr_elems) P.scr_elems = scr_top;
    return o;
  }
  int32_t dyn_alloc() {
    int32_t s = dyn_top++;
    if (dyn_top > dyn_max) dyn_max = dyn_top;
    return s;
  }

  // Cached rank x rank cores V_A[K]^T V_B[K] of pairs of low-rank blocks of
  // the factor.  Once the sweep has passed the last leaf of K both panels are
  // final, so every later target that needs the product of the same two
  // blocks over the same K reuses one core in the persistent scratch.  A core
  // is needed only by targets whose column lies in the row cluster of B, so
  // its slot is recycled after the last leaf of that cluster.
  struct CoreKey {
    int32_t a, b;
    int64_t k0, k1;
    bool operator<(const CoreKey& o) const {
      return std::tie(a, b, k0, k1) < std::tie(o.a, o.b, o.k0, o.k1);
    }
  };
  std::map<CoreKey, int64_t> core_slot;
  std::vector<int64_t> core_free;
  std::vector<std::vector<std::pair<CoreKey, int64_t>>> core_release;   // by step
  int64_t core_base = 0, core_top = 0, cur_step = 0;

  void core_reset(int64_t steps) {
    core_slot.clear();
    core_free.clear();
    core_release.assign(steps + 1, {});
    core_top = core_base;
  }
  void core_step(int64_t j) {
    cur_step = j;
    for (auto& e : core_release[j]) {
      core_slot.erase(e.first);
      core_free.push_back(e.second);
    }
    core_release[j].clear();
  }
  // returns the slot offset; *fresh tells the caller to compute it
  int64_t core_get(int32_t a, int32_t b, int64_t k0, int64_t k1, bool* fresh) {
    CoreKey key{a, b, k0, k1};
    auto it = core_slot.find(key);
    if (it != core_slot.end()) {
      *fresh = false;
      return it->second;
    }
    *fresh = true;
    int64_t o;
    if (!core_free.empty()) {
      o = core_free.back();
      core_free.pop_back();
    } else {
      o = core_top;
      core_top += int64_t(P.kcap) * P.kcap;
      if (core_top > P.pers_elems) P.pers_elems = core_top;
    }
    core_slot[key] = o;
    const BlockInfo& B = P.blocks[b];
    int64_t last = ((int64_t(B.a) + 1) << (P.D - B.level)) - 1;   // last leaf of rows(B)
    core_release[std::max<int64_t>(last + 1, cur_step + 1)].push_back({key, o});
    return o;
  }

  // ---------------------------------------------------------------- GEMM
  bool fp32_for(const Ref& C) const { return P.mixed && C.buf != B_DENSE && C.buf != B_RHS; }
  // fp32 < 0: from the output buffer (partial sums take their job's choice)
  int32_t gemm_job(Ref C, Dim m, Dim n, int zero, int fp32 = -1) {
    GemmJob j{};
    j.C = C;
    j.m = m;
    j.n = n;
    j.zero = zero;
    j.p0 = j.p1 = 0;
    // mixed precision: every GEMM except those producing dense leaves or the
    // right-hand side of the fused solve accumulates in FP32
    j.fp32 = fp32 >= 0 ? fp32 : (fp32_for(C) ? 1 : 0);
    P.gjobs.push_back(j);
    pending_prods.emplace_back();
    return int32_t(P.gjobs.size() - 1);
  }
  // products are collected per job, then laid out contiguously at flush
  std::vector<std::vector<GemmProd>> pending_prods;
  int32_t job_base = 0;

  void add_prod(int32_t job, Ref A, int ta, Ref B, int tb, Dim k, int i0, int j0, Dim mi,
                Dim nj, double alpha) {
    GemmProd p{};
    p.A = A;
    p.B = B;
    p.ta = ta;
    p.tb = tb;
    p.k = k;
    p.i0 = i0;
    p.j0 = j0;
    p.mi = mi;
    p.nj = nj;
    p.alpha = alpha;
    pending_prods[job - job_base].push_back(p);
  }

  // close the GEMM jobs created since the last flush into one stage
  void flush_gemm(std::vector<Stage>& out) {
    int32_t nj = int32_t(P.gjobs.size()) - job_base;
    if (nj <= 0) return;
    int32_t t0 = int32_t(P.gtiles.size());
    // estimated k chunks per tile, accumulated over the tiles each product spans
    std::vector<int> tcost;
    // the grouped kernel adds a tile's chunks in another order: launches with
    // a solve job keep the plain kernel, so that the sweep's fused solve and
    // the stand-alone forward solve do the same arithmetic; FP32 jobs need
    // the vector body of the plain kernel
    bool wide_ok = true;
    for (int32_t j = 0; j < nj; ++j) {
      GemmJob& g = P.gjobs[job_base + j];
      g.p0 = int32_t(P.gprods.size());
      const int mt = (g.m.maxv + TM - 1) / TM, nt = (g.n.maxv + TN - 1) / TN;
      const size_t tb = tcost.size();
      tcost.resize(tb + size_t(mt) * nt, 0);
      if (g.C.buf == B_RHS) wide_ok = false;
      for (auto& p : pending_prods[j]) {
        P.gprods.push_back(p);
        if (p.A.buf == B_RHS || p.B.buf == B_RHS) {
          g.fp32 = 0;   // the solve stays FP64
          wide_ok = false;
        }
        const int c = p.tb == 2 ? 1 : chunks(est_k(p.k));
        const int a0 = std::max(0, p.i0 / TM), a1 = std::min(mt, (p.i0 + p.mi.maxv + TM - 1) / TM);
        const int b0 = std::max(0, p.j0 / TN), b1 = std::min(nt, (p.j0 + p.nj.maxv + TN - 1) / TN);
        for (int a = a0; a < a1; ++a)
          for (int b = b0; b < b1; ++b) tcost[tb + size_t(a) * nt + b] += c;
      }
      if (g.fp32) wide_ok = false;
      g.p1 = int32_t(P.gprods.size());
      for (int a = 0; a < mt; ++a)
        for (int b = 0; b < nt; ++b) P.gtiles.push_back(GemmTile{job_base + j, a, b, 0});
    }
    pending_prods.clear();
    job_base = int32_t(P.gjobs.size());
    int32_t t1 = int32_t(P.gtiles.size());
    if (t1 > t0) {
      // heaviest tiles first: work-groups start in tile order, so a launch
      // with more tiles than resident work-groups is scheduled longest first
      std::vector<std::pair<int, int32_t>> cost;
      cost.reserve(size_t(t1 - t0));
      for (int32_t t = t0; t < t1; ++t) cost.emplace_back(-tcost[size_t(t - t0)], t);
      std::stable_sort(cost.begin(), cost.end(),
                       [](const std::pair<int, int32_t>& x, const std::pair<int, int32_t>& y) { return x.first < y.first; });
      std::vector<GemmTile> sorted;
      sorted.reserve(cost.size());
      for (auto& ct : cost) sorted.push_back(P.gtiles[ct.second]);
      std::copy(sorted.begin(), sorted.end(), P.gtiles.begin() + t0);
      // chunk times of the launch, heaviest first: the plain kernel runs 4
      // tiles per CU, each through its chunks one by one; the grouped one
      // runs 1 tile per CU, GEMM_GROUPS chunks of it at a time
      int64_t plain_tot = 0, wide_tot = 0;
      int cmax = 0;
      for (auto& ct : cost) {
        const int c = -ct.first;
        cmax = std::max(cmax, c);
        plain_tot += c;
        wide_tot += (c + GEMM_GROUPS - 1) / GEMM_GROUPS;
      }
      const int64_t plain = std::max<int64_t>(cmax, (plain_tot + 1023) / 1024);
      const int64_t wide = std::max<int64_t>((cmax + GEMM_GROUPS - 1) / GEMM_GROUPS, (wide_tot + 255) / 256);
      out.push_back(Stage{wide_ok && wide < plain ? ST_GEMM_WIDE : ST_GEMM, t0, t1, cur_lane, wide_ok ? 1 : 0});
    }
  }

  // ---------------------------------------------------------------- TSQR
  struct TsqrReq {
    Ref X;
    int64_t rows;
    Dim cols;
    Ref R;   // final R (ld rmax)
  };
  std::vector<TsqrReq> tsqr_pending;
  void tsqr(Ref X, int64_t rows, Dim cols, Ref R) { tsqr_pending.push_back(TsqrReq{X, rows, cols, R}); }
  // Segment R factors are combined by a tree of reductions of at most
  // TSQR_FAN factors each; every tree level is one launch.
  void flush_tsqr(std::vector<Stage>& out) {
    if (tsqr_pending.empty()) return;
    int32_t s0 = int32_t(P.tsegs.size());
    const int64_t RR = int64_t(P.rmax) * P.rmax;
    std::vector<std::vector<TsqrRed>> levels;
    for (auto& q : tsqr_pending) {
      int64_t nseg = (q.rows + TSQR_SEG - 1) / TSQR_SEG;
      if (nseg <= 1) {
        P.tsegs.push_back(TsqrSeg{q.X, int32_t(q.rows), q.cols, q.R});
        continue;
      }
      int64_t base = scr_alloc(nseg * RR);
      for (int64_t s = 0; s < nseg; ++s) {
        Ref X = q.X;
        X.off += s * TSQR_SEG;
        int32_t rows = int32_t(std::min<int64_t>(TSQR_SEG, q.rows - s * TSQR_SEG));
        P.tsegs.push_back(TsqrSeg{X, rows, q.cols, Ref{B_SCR, P.rmax, base + s * RR}});
      }
      int64_t cnt = nseg;
      size_t lv = 0;
      while (cnt > TSQR_FAN) {
        int64_t ng = (cnt + TSQR_FAN - 1) / TSQR_FAN;
        int64_t nb = scr_alloc(ng * RR);
        if (levels.size() <= lv) levels.resize(lv + 1);
        for (int64_t g = 0; g < ng; ++g)
          levels[lv].push_back(TsqrRed{Ref{B_SCR, P.rmax, base + g * TSQR_FAN * RR},
                                       int32_t(std::min<int64_t>(TSQR_FAN, cnt - g * TSQR_FAN)), q.cols,
                                       Ref{B_SCR, P.rmax, nb + g * RR}});
        base = nb;
        cnt = ng;
        ++lv;
      }
      if (levels.size() <= lv) levels.resize(lv + 1);
      levels[lv].push_back(TsqrRed{Ref{B_SCR, P.rmax, base}, int32_t(cnt), q.cols, q.R});
    }
    tsqr_pending.clear();
    int32_t s1 = int32_t(P.tsegs.size());
    if (s1 > s0) out.push_back(Stage{ST_TSQR_SEG, s0, s1});
    for (auto& L : levels) {
      if (L.empty()) continue;
      int32_t r0 = int32_t(P.treds.size());
      for (auto& r : L) P.treds.push_back(r);
      out.push_back(Stage{ST_TSQR_RED, r0, int32_t(P.treds.size())});
    }
  }

  void flush_small(std::vector<Stage>& out, int32_t s0) {
    int32_t s1 = int32_t(P.smalls.size());
    if (s1 > s0) out.push_back(Stage{ST_SMALL, s0, s1});
  }

  // ---------------------------------------------------------------- tree helpers
  int64_t lo(int l, int64_t i) const { return P.lo[l][i]; }
  int64_t hi(int l, int64_t i) const { return P.lo[l][i + 1]; }
  int32_t status(int l, int64_t a, int64_t c) const {
    auto it = P.status.find(key3(l, a, c));
    return it == P.status.end() ? -2 : it->second;
  }
  // region rows node (l,a) x cols node (lk,k): returns block id if covered by
  // a single leaf, -1 if subdivided
  int32_t region(int l, int64_t a, int lk, int64_t k) const {
    int64_t aa = a >> (l - lk);
    int32_t s = status(lk, aa, k);
    if (s != -2) return s;
    int ll = lk;
    int64_t x = aa, y = k;
    while (ll > 0) {
      --ll;
      x >>= 1;
      y >>= 1;
      int32_t t = status(ll, x, y);
      if (t != -2) {
        assert(t >= 0);
        return t;
      }
    }
    fprintf(stderr, "hcov plan: region lookup failed\n");
    abort();
  }

  Dim rank_dim(int32_t b) const { return dim_dyn(P.blocks[b].rank_slot, P.blocks[b].cap); }

  // U of block b restricted to absolute rows [r0, r1)
  Src lr_u(int32_t b, int64_t r0) const {
    const BlockInfo& B = P.blocks[b];
    return Src{Ref{B_U, int32_t(B.r1 - B.r0), B.off_u + (r0 - B.r0)}, rank_dim(b)};
  }
  Src lr_v(int32_t b, int64_t c0) const {
    const BlockInfo& B = P.blocks[b];
    return Src{Ref{B_V, int32_t(B.c1 - B.c0), B.off_v + (c0 - B.c0)}, rank_dim(b)};
  }
  // dense block b restricted to rows starting r0, cols starting c0, width w
  Src dn(int32_t b, int64_t r0, int64_t c0, int w) const {
    const BlockInfo& B = P.blocks[b];
    int32_t ld = int32_t(B.r1 - B.r0);
    return Src{Ref{B_DENSE, ld, B.off_d + (r0 - B.r0) + (c0 - B.c0) * ld}, dim_static(w)};
  }

  // W = L(P, K) X with P = (l,p), K = (lk,k); X has |K| rows (absolute
  // column index c maps to X row c - K.lo).  Emits inner products into the
  // current "A" stage and the accumulation job into the current "B" stage.
  // Returns the scratch W (|P| x X.cols).
  std::vector<int32_t>* stageA_jobs = nullptr;   // (unused, jobs are global)
  struct Pending {
    int32_t jobA_base;
  };

  // Two-phase GEMM emission: phase A jobs go to list A, phase B to list B.
  struct Deferred {
    Ref C;
    Dim m, n;
    int zero;
    std::vector<GemmProd> prods;
  };
  std::vector<Deferred> listA, listB;

  int32_t defer(std::vector<Deferred>& L, Ref C, Dim m, Dim n, int zero) {
    L.push_back(Deferred{C, m, n, zero, {}});
    return int32_t(L.size() - 1);
  }
  static void dprod(Deferred& d, Ref A, int ta, Ref B, int tb, Dim k, int i0, int j0, Dim mi,
                    Dim nj, double alpha) {
    GemmProd p{};
    p.A = A;
    p.B = B;
    p.ta = ta;
    p.tb = tb;
    p.k = k;
    p.i0 = i0;
    p.j0 = j0;
    p.mi = mi;
    p.nj = nj;
    p.alpha = alpha;
    d.prods.push_back(p);
  }
  // Emit deferred jobs as one GEMM stage.  A work-group streams the k
  // chunks of every product of its job that meets its tile, so a job whose
  // busiest tile would stream more than TILE_BUDGET chunks is split: long
  // static-k products are cut into k ranges, and the pieces are packed
  // first-fit into groups whose per-tile cost fits the budget.  Each group
  // writes a partial sum to scratch and a second stage adds the partials
  // into the real output in a fixed order (deterministic, no atomics).
  static constexpr int GKP = 32;            // k chunk of the GEMM kernel
  static constexpr int TILE_BUDGET = 16;    // k chunks per tile and launch
  static constexpr int64_t PART_CAP = int64_t(1) << 23;   // scratch elements per split job
  static int est_k(const Dim& k) { return k.slot < 0 ? k.maxv : std::min(k.maxv, 32); }
  static int chunks(int k) { return (k + GKP - 1) / GKP; }
  void emit(std::vector<Deferred>& L, std::vector<Stage>& out) {
    std::vector<Deferred> finals;
    for (auto& d : L) {
      const int mcap = d.m.maxv, ncap = d.n.maxv;
      const int tr = (mcap + 63) / 64, tc = (ncap + 63) / 64;
      // tile range of a product (capacity-based)
      auto span = [&](const GemmProd& p, int& a0, int& a1, int& b0, int& b1) {
        a0 = p.i0 / 64;
        a1 = std::min(tr, (p.i0 + p.mi.maxv + 63) / 64);
        b0 = p.j0 / 64;
        b1 = std::min(tc, (p.j0 + p.nj.maxv + 63) / 64);
      };
      // busiest tile of the unsplit job
      std::vector<int> cost(size_t(tr) * tc, 0);
      int worst = 0;
      for (auto& p : d.prods) {
        int a0, a1, b0, b1;
        span(p, a0, a1, b0, b1);
        int c = p.tb == 2 ? 1 : chunks(est_k(p.k));
        for (int x = a0; x < a1; ++x)
          for (int y = b0; y < b1; ++y) worst = std::max(worst, cost[size_t(x) * tc + y] += c);
      }
      std::vector<std::vector<GemmProd>> groups;
      if (worst > TILE_BUDGET && int64_t(mcap) * ncap * 2 <= PART_CAP) {
        // pieces: long static-k products cut into k ranges of the budget
        std::vector<GemmProd> pieces;
        const int kcut = TILE_BUDGET * GKP;
        for (auto& p : d.prods) {
          if (p.k.slot >= 0 || p.tb == 2 || p.k.maxv <= kcut) {
            pieces.push_back(p);
            continue;
          }
          for (int k0 = 0; k0 < p.k.maxv; k0 += kcut) {
            GemmProd q = p;
            q.k = dim_static(std::min(kcut, p.k.maxv - k0));
            q.A.off += (p.ta == 0) ? int64_t(k0) * p.A.ld : int64_t(k0);
            q.B.off += (p.tb == 0) ? int64_t(k0) : int64_t(k0) * p.B.ld;
            pieces.push_back(q);
          }
        }
        std::vector<std::vector<int>> gcost;
        const int64_t gmax = std::max<int64_t>(2, PART_CAP / (int64_t(mcap) * ncap));
        for (auto& q : pieces) {
          int a0, a1, b0, b1;
          span(q, a0, a1, b0, b1);
          int c = q.tb == 2 ? 1 : chunks(est_k(q.k));
          size_t g = 0;
          for (; g < groups.size(); ++g) {
            bool fits = true;
            for (int x = a0; x < a1 && fits; ++x)
              for (int y = b0; y < b1 && fits; ++y) fits = gcost[g][size_t(x) * tc + y] + c <= TILE_BUDGET;
            if (fits) break;
          }
          if (g == groups.size()) {
            if (int64_t(groups.size()) >= gmax) {
              g = groups.size() - 1;   // scratch cap: overload the last group
            } else {
              groups.emplace_back();
              gcost.emplace_back(size_t(tr) * tc, 0);
            }
          }
          groups[g].push_back(q);
          for (int x = a0; x < a1; ++x)
            for (int y = b0; y < b1; ++y) gcost[g][size_t(x) * tc + y] += c;
        }
      }
      if (groups.size() <= 1) {
        int32_t j = gemm_job(d.C, d.m, d.n, d.zero);
        for (auto& p : d.prods) add_prod(j, p.A, p.ta, p.B, p.tb, p.k, p.i0, p.j0, p.mi, p.nj, p.alpha);
        continue;
      }
      Deferred fin{d.C, d.m, d.n, d.zero, {}};
      for (auto& g : groups) {
        int64_t pb = scr_alloc(int64_t(mcap) * ncap);
        int32_t j = gemm_job(Ref{B_SCR, mcap, pb}, d.m, d.n, 1, fp32_for(d.C) ? 1 : 0);
        for (auto& p : g) add_prod(j, p.A, p.ta, p.B, p.tb, p.k, p.i0, p.j0, p.mi, p.nj, p.alpha);
        dprod(fin, Ref{B_SCR, mcap, pb}, 0, Ref{B_SCR, mcap, pb}, 2, dim_static(1), 0, 0, d.m, d.n, 1.0);
      }
      finals.push_back(fin);
    }
    L.clear();
    flush_gemm(out);
    if (!finals.empty()) {
      for (auto& d : finals) {
        int32_t j = gemm_job(d.C, d.m, d.n, d.zero);
        for (auto& p : d.prods) add_prod(j, p.A, p.ta, p.B, p.tb, p.k, p.i0, p.j0, p.mi, p.nj, p.alpha);
      }
      flush_gemm(out);
    }
  }

  // add to deferred job `d` (in list B) the contributions of region
  // rows (l,p) x cols (lk,k) times X; W rows are offset by wrow0 = P.lo
  void hmv_pieces(int l, int64_t p, int lk, int64_t k, const Src& X, int64_t xcol0,
                  std::vector<Deferred>& LA, std::vector<Deferred>& LB, int32_t dB, double alpha,
                  int64_t wrow0, bool transpose) {
    int64_t P0 = lo(l, p), P1 = hi(l, p);
    std::function<void(int, int64_t, int64_t)> rec = [&](int lv, int64_t r, int64_t c) {
      int32_t s = status(lv, r, c);
      if (s == -2) {
        fprintf(stderr, "hcov plan: hmv lookup failed\n");
        abort();
      }
      if (s >= 0) {
        piece(s, std::max(lo(lv, r), P0), std::min(hi(lv, r), P1), lo(lv, c), hi(lv, c), X,
              xcol0, LA, LB, dB, alpha, wrow0, transpose);
        return;
      }
      std::vector<int64_t> rc;
      if (lv < l)
        rc.push_back(p >> (l - lv - 1));
      else {
        rc.push_back(2 * r);
        rc.push_back(2 * r + 1);
      }
      for (int64_t rr : rc)
        for (int64_t cc : {2 * c, 2 * c + 1}) rec(lv + 1, rr, cc);
    };
    int32_t st = region(l, p, lk, k);
    if (st >= 0) {
      piece(st, P0, P1, lo(lk, k), hi(lk, k), X, xcol0, LA, LB, dB, alpha, wrow0, transpose);
      return;
    }
    rec(lk, p >> (l - lk), k);
  }

  // one leaf block b restricted to rows [r0,r1) x cols [c0,c1):
  //   W[r0-wrow0 ..] += alpha * Lb[r, c] X[c - xcol0]
  // transpose: W[c - wrow0] += alpha * Lb[r, c]^T X[r - xcol0]
  void piece(int32_t b, int64_t r0, int64_t r1, int64_t c0, int64_t c1, const Src& X,
             int64_t xcol0, std::vector<Deferred>& LA, std::vector<Deferred>& LB, int32_t dB,
             double alpha, int64_t wrow0, bool transpose) {
    const BlockInfo& B = P.blocks[b];
    int nr = int(r1 - r0), nc = int(c1 - c0);
    if (nr <= 0 || nc <= 0) return;
    if (!transpose) {
      if (B.kind == 1 && xblk >= 0) {
        // X is the final V panel of block xblk: T^T = V_xblk[c]^T V_b[c] is a cached core
        bool fresh = false;
        int64_t c = core_get(xblk, b, c0, c1, &fresh);
        if (fresh) {
          int32_t dA = defer(LA, Ref{B_PERS, P.kcap, c}, X.cols, rank_dim(b), 1);
          Ref Xr = X.ref;
          Xr.off += (c0 - xcol0);
          dprod(LA[dA], Xr, 1, lr_v(b, c0).ref, 0, dim_static(nc), 0, 0, X.cols, rank_dim(b), 1.0);
        }
        dprod(LB[dB], lr_u(b, r0).ref, 0, Ref{B_PERS, P.kcap, c}, 1, rank_dim(b), int(r0 - wrow0),
              0, dim_static(nr), X.cols, alpha);
      } else if (B.kind == 1) {
        // T = V_b[c]^T X[c]  (rank x X.cols)
        Src V = lr_v(b, c0);
        int64_t t = scr_alloc(int64_t(P.kcap) * X.cols.maxv);
        int32_t dA = defer(LA, Ref{B_SCR, P.kcap, t}, rank_dim(b), X.cols, 1);
        Ref Xr = X.ref;
        Xr.off += (c0 - xcol0);
        dprod(LA[dA], V.ref, 1, Xr, 0, dim_static(nc), 0, 0, rank_dim(b), X.cols, 1.0);
        Src U = lr_u(b, r0);
        dprod(LB[dB], U.ref, 0, Ref{B_SCR, P.kcap, t}, 0, rank_dim(b), int(r0 - wrow0), 0,
              dim_static(nr), X.cols, alpha);
      } else {
        Src Dm = dn(b, r0, c0, nc);
        Ref Xr = X.ref;
        Xr.off += (c0 - xcol0);
        dprod(LB[dB], Dm.ref, 0, Xr, 0, dim_static(nc), int(r0 - wrow0), 0, dim_static(nr),
              X.cols, alpha);
      }
    } else {
      if (B.kind == 1) {
        Src U = lr_u(b, r0);
        int64_t t = scr_alloc(int64_t(P.kcap) * X.cols.maxv);
        int32_t dA = defer(LA, Ref{B_SCR, P.kcap, t}, rank_dim(b), X.cols, 1);
        Ref Xr = X.ref;
        Xr.off += (r0 - xcol0);
        dprod(LA[dA], U.ref, 1, Xr, 0, dim_static(nr), 0, 0, rank_dim(b), X.cols, 1.0);
        Src V = lr_v(b, c0);
        dprod(LB[dB], V.ref, 0, Ref{B_SCR, P.kcap, t}, 0, rank_dim(b), int(c0 - wrow0), 0,
              dim_static(nc), X.cols, alpha);
      } else {
        Src Dm = dn(b, r0, c0, nc);
        Ref Xr = X.ref;
        Xr.off += (r0 - xcol0);
        dprod(LB[dB], Dm.ref, 1, Xr, 0, dim_static(nr), int(c0 - wrow0), 0, dim_static(nc),
              X.cols, alpha);
      }
    }
  }

  // block whose final V panel is the right-hand side of the current H-matvec
  // (enables the core cache in piece()), or -1
  int32_t xblk = -1;

  // H-matvec producing a fresh scratch W = L(P,K) X
  Src hmatvec(int l, int64_t p, int lk, int64_t k, const Src& X, int64_t xcol0) {
    int64_t P0 = lo(l, p), P1 = hi(l, p);
    int64_t w = scr_alloc((P1 - P0) * int64_t(X.cols.maxv));
    int32_t dB = defer(listB, Ref{B_SCR, int32_t(P1 - P0), w}, dim_static(int(P1 - P0)), X.cols, 1);
    hmv_pieces(l, p, lk, k, X, xcol0, listA, listB, dB, 1.0, P0, false);
    return Src{Ref{B_SCR, int32_t(P1 - P0), w}, X.cols};
  }

  // terms of L(R,K) L(P,K)^T with R = (l,a), P = (l,p), K = (lk,k)
  void pair_terms(int l, int64_t a, int64_t p, int lk, int64_t k, std::vector<Term>& out) {
    int64_t R0 = lo(l, a), R1 = hi(l, a), Q0 = lo(l, p), Q1 = hi(l, p), K0 = lo(lk, k),
            K1 = hi(lk, k);
    int32_t sR = region(l, a, lk, k);
    int32_t sP = region(l, p, lk, k);
    int kR = sR >= 0 ? P.blocks[sR].kind : -1;
    int kP = sP >= 0 ? P.blocks[sP].kind : -1;
    if (kR == 1) {
      Src Ua = lr_u(sR, R0);
      Src Va = lr_v(sR, K0);
      if (kP == 1) {
        // U_t = Ua[R] (Va[K]^T Vb[K]),  V_t = Ub[P]
        Src Vb = lr_v(sP, K0);
        bool fresh = false;
        int64_t c = core_get(sR, sP, K0, K1, &fresh);
        if (fresh) {
          int32_t dA = defer(listA, Ref{B_PERS, P.kcap, c}, rank_dim(sR), rank_dim(sP), 1);
          dprod(listA[dA], Va.ref, 1, Vb.ref, 0, dim_static(int(K1 - K0)), 0, 0, rank_dim(sR),
                rank_dim(sP), 1.0);
        }
        int64_t u = scr_alloc((R1 - R0) * int64_t(P.blocks[sP].cap));
        int32_t dB = defer(listB, Ref{B_SCR, int32_t(R1 - R0), u}, dim_static(int(R1 - R0)),
                           rank_dim(sP), 1);
        dprod(listB[dB], Ua.ref, 0, Ref{B_PERS, P.kcap, c}, 0, rank_dim(sR), 0, 0,
              dim_static(int(R1 - R0)), rank_dim(sP), 1.0);
        out.push_back(Term{R0, R1, Q0, Q1, Src{Ref{B_SCR, int32_t(R1 - R0), u}, rank_dim(sP)},
                           lr_u(sP, Q0)});
      } else {
        xblk = sR;
        Src W = hmatvec(l, p, lk, k, Va, K0);
        xblk = -1;
        out.push_back(Term{R0, R1, Q0, Q1, Ua, W});
      }
      return;
    }
    if (kP == 1) {
      Src Vb = lr_v(sP, K0);
      xblk = sP;
      Src W = hmatvec(l, a, lk, k, Vb, K0);
      xblk = -1;
      out.push_back(Term{R0, R1, Q0, Q1, W, lr_u(sP, Q0)});
      return;
    }
    if (kR == 0 && kP == 0) {
      int w = int(K1 - K0);
      out.push_back(Term{R0, R1, Q0, Q1, dn(sR, R0, K0, w), dn(sP, Q0, K0, w)});
      return;
    }
    if (kR >= 0 || kP >= 0) {
      fprintf(stderr, "hcov plan: dense/subdivided mix\n");
      abort();
    }
    if (lk < l) {
      pair_terms(l, a, p, lk + 1, 2 * k, out);
      pair_terms(l, a, p, lk + 1, 2 * k + 1, out);
    } else {
      for (int64_t ai : {2 * a, 2 * a + 1})
        for (int64_t pj : {2 * p, 2 * p + 1})
          for (int64_t kc : {2 * k, 2 * k + 1}) pair_terms(l + 1, ai, pj, l + 1, kc, out);
    }
  }

  std::vector<Term> update_terms(int l, int64_t a, int64_t b) {
    std::vector<Term> out;
    int lp = l;
    int64_t node = b;
    while (lp >= 1) {
      if (node & 1) pair_terms(l, a, b, lp, node - 1, out);
      node >>= 1;
      --lp;
    }
    return out;
  }

  // ---------------------------------------------------------------- the sweep
  // jobs X <- L_jj^{-1} X in 64-column chunks: by substitution with L_jj
  // (inverse = false) or by multiplication with the stored inverse
  void add_trsm(int64_t j, Ref X, int layout, Dim nc, bool inverse = false) {
    const BlockInfo& Dg = P.blocks[P.diag_block[j]];
    const int pj = int(Dg.r1 - Dg.r0);
    Ref Lr = inverse ? Ref{B_LINV, pj, P.linv_off[j]} : Ref{B_DENSE, pj, Dg.off_d};
    for (int c0 = 0; c0 < nc.maxv; c0 += 64)
      P.trsms.push_back(TrsmJob{Lr, pj, layout, X, nc, c0, std::min(64, nc.maxv - c0)});
  }
  template <class T>
  static std::vector<int32_t> lrs_ids(const std::vector<T>& lrs) {
    std::vector<int32_t> v;
    for (auto& t : lrs) v.push_back(t.b);
    return v;
  }
  std::vector<std::vector<int32_t>> active;   // LR blocks whose column cluster contains leaf j
  // Once the dense targets of step j are updated, a second lane (stream)
  // factorises the diagonal leaf and applies L_jj^{-1} to the dense targets,
  // the panels of the low-rank blocks that started before j and the fused
  // right-hand side, while the first lane recompresses the new low-rank
  // targets: the two sets of work touch disjoint data.
  void fork_leaf(int64_t j, const std::vector<std::pair<int32_t, std::vector<Term>>>& dns,
                 const std::vector<int32_t>& fresh, bool fuse_rhs, std::vector<Stage>& st,
                 std::vector<Deferred>& dense_upd) {
    st.push_back(Stage{ST_FORK, 0, 0});
    // the dense targets (the diagonal leaf among them) are updated on the
    // second lane, ahead of the leaf factorisation
    cur_lane = 1;
    emit(dense_upd, st);
    cur_lane = 0;
    const BlockInfo& B = P.blocks[P.diag_block[j]];
    LeafJob J{};
    J.D = Ref{B_DENSE, int32_t(B.r1 - B.r0), B.off_d};
    J.p = int32_t(B.r1 - B.r0);
    J.leaf = int32_t(j);
    J.row0 = B.r0;
    int32_t l0 = int32_t(P.leafs.size());
    P.leafs.push_back(J);
    st.push_back(Stage{ST_LEAF, l0, l0 + 1, 1});
    // L_jj^{-1} into B_LINV (substitution on the identity), then the
    // second lane's right-hand sides by multiplication with it
    int32_t t0 = int32_t(P.trsms.size());
    add_trsm(j, Ref{B_LINV, J.p, P.linv_off[j]}, 3, dim_static(J.p));
    st.push_back(Stage{ST_TRSM, t0, int32_t(P.trsms.size()), 1});
    const int64_t cj0 = lo(P.D, j);
    t0 = int32_t(P.trsms.size());
    for (auto& dt : dns) {
      const BlockInfo& T = P.blocks[dt.first];
      if (T.a == T.c) continue;
      add_trsm(j, Ref{B_DENSE, int32_t(T.r1 - T.r0), T.off_d}, 1, dim_static(int(T.r1 - T.r0)), true);
    }
    for (int32_t b : active[j]) {
      if (std::find(fresh.begin(), fresh.end(), b) != fresh.end()) continue;
      const BlockInfo& T = P.blocks[b];
      add_trsm(j, Ref{B_V, int32_t(T.c1 - T.c0), T.off_v + (cj0 - T.c0)}, 0, rank_dim(b), true);
    }
    if (fuse_rhs) add_trsm(j, Ref{B_RHS, int32_t(P.rhs_ld), cj0}, 0, dim_static(1), true);
    int32_t t1 = int32_t(P.trsms.size());
    if (t1 > t0) st.push_back(Stage{ST_TRMM, t0, t1, 1});
  }

  void build_steps(bool fuse_rhs, std::vector<std::vector<Stage>>& steps);
  void build_recompress();
  void build_solves();
  void build_matvec();
};

void Builder::build_steps(bool fuse_rhs, std::vector<std::vector<Stage>>& steps) {
  const int D = P.D;
  const int64_t m = int64_t(1) << D;
  std::vector<std::vector<int32_t>> by_start(m);
  for (int32_t b = 0; b < int32_t(P.blocks.size()); ++b) {
    const BlockInfo& B = P.blocks[b];
    by_start[int64_t(B.c) << (D - B.level)].push_back(b);
  }
  // LR blocks whose column cluster contains leaf j are "active" at j
  active.assign(m, {});
  std::unordered_map<uint64_t, std::vector<int32_t>> by_col;
  for (int32_t b = 0; b < int32_t(P.blocks.size()); ++b) {
    const BlockInfo& B = P.blocks[b];
    if (B.kind != 1) continue;
    int64_t f = int64_t(B.c) << (D - B.level), e = int64_t(B.c + 1) << (D - B.level);
    for (int64_t x = f; x < e; ++x) active[x].push_back(b);
    by_col[key3(B.level, B.c, 0)].push_back(b);
  }
  steps.assign(m, {});
  core_reset(m);
  const int RM = P.rmax;
  const int64_t RR = int64_t(RM) * RM;
  for (int64_t j = 0; j < m; ++j) {
    std::vector<Stage>& st = steps[j];
    core_step(j);
    scr_top = 0;
    dyn_top = dyn_base;
    const int64_t cj0 = lo(D, j), cj1 = hi(D, j);
    const int pj = int(cj1 - cj0);

    // ---- update terms of every target starting at j
    struct LrT {
      int32_t b;
      std::vector<Term> terms;
    };
    std::vector<LrT> lrs;
    std::vector<std::pair<int32_t, std::vector<Term>>> dns;
    for (int32_t b : by_start[j]) {
      const BlockInfo& B = P.blocks[b];
      auto terms = update_terms(B.level, B.a, B.c);
      if (B.kind == 1)
        lrs.push_back(LrT{b, std::move(terms)});
      else
        dns.emplace_back(b, std::move(terms));
    }
    emit(listA, st);   // inner products and cores
    emit(listB, st);   // W accumulation and U*core

    // ---- dense targets: D -= sum of the update terms, as GEMM jobs on the
    // target tile (split into partial sums by emit() when long); they run on
    // the second lane (fork_leaf) while this lane forms the sketches
    std::vector<Deferred> listD;
    for (auto& dt : dns) {
      if (dt.second.empty()) continue;
      const BlockInfo& B = P.blocks[dt.first];
      const int p = int(B.r1 - B.r0), q = int(B.c1 - B.c0);
      int32_t d = defer(listD, Ref{B_DENSE, p, B.off_d}, dim_static(p), dim_static(q), 0);
      for (auto& T : dt.second)
        dprod(listD[d], T.U.ref, 0, T.V.ref, 1, T.U.cols, int(T.r0 - B.r0), int(T.p0 - B.c0),
              dim_static(int(T.r1 - T.r0)), dim_static(int(T.p1 - T.p0)), -1.0);
    }
    if (lrs.empty()) fork_leaf(j, dns, lrs_ids(lrs), fuse_rhs, st, listD);

    // ---- randomised recompression of low-rank targets
    if (!lrs.empty()) {
      struct SK {
        int32_t b;
        int64_t p, q;
        Dim r;          // sketch width
        Dim rk;         // kept directions of Y
        int64_t y, qm, bp, ry, rq, rb, pm, c2, bpp;
        std::vector<int64_t> p1, z1;
      };
      std::vector<SK> sk(lrs.size());
      for (size_t t = 0; t < lrs.size(); ++t) {
        const BlockInfo& B = P.blocks[lrs[t].b];
        SK& s = sk[t];
        s.b = lrs[t].b;
        s.p = B.r1 - B.r0;
        s.q = B.c1 - B.c0;
        // the widest sketch a block can use: its capacity plus the oversampling
        // bound (a wider kept rank overflows the capacity anyway)
        int rmaxT = int(std::min<int64_t>({s.p, s.q, int64_t(B.cap) + OVERSAMPLE_MAX}));
        // after the assembly the rank0 slot holds rank + oversampling
        s.r = Dim{B.rank0_slot, 0, rmaxT};
        s.rk = dim_dyn(dyn_alloc(), rmaxT);
        s.y = scr_alloc(s.p * rmaxT);
        s.qm = scr_alloc(s.p * rmaxT);
        s.bp = scr_alloc(s.q * rmaxT);
        s.ry = scr_alloc(RR);
        s.rq = scr_alloc(RR);
        s.rb = scr_alloc(RR);
        s.pm = scr_alloc(RR);
        s.c2 = scr_alloc(RR);
        // P1 = V^T Omega for A and each term
        Dim kA = rank_dim(s.b);
        int64_t pa = scr_alloc(int64_t(B.cap) * rmaxT);
        s.p1.push_back(pa);
        int32_t d = defer(listA, Ref{B_SCR, B.cap, pa}, kA, s.r, 1);
        dprod(listA[d], Ref{B_V, int32_t(s.q), B.off_v}, 1, Ref{B_OMEGA, int32_t(P.omega_rows), 0},
              0, dim_static(int(s.q)), 0, 0, kA, s.r, 1.0);
        for (auto& T : lrs[t].terms) {
          int kc = T.V.cols.maxv;
          int64_t o = scr_alloc(int64_t(kc) * rmaxT);
          s.p1.push_back(o);
          int32_t dd = defer(listA, Ref{B_SCR, kc, o}, T.V.cols, s.r, 1);
          dprod(listA[dd], T.V.ref, 1,
                Ref{B_OMEGA, int32_t(P.omega_rows), T.p0 - B.c0}, 0,
                dim_static(int(T.p1 - T.p0)), 0, 0, T.V.cols, s.r, 1.0);
        }
      }
      fork_leaf(j, dns, lrs_ids(lrs), fuse_rhs, st, listD);
      emit(listA, st);
      // Y = U_A P1_A - sum U_t P1_t
      for (size_t t = 0; t < lrs.size(); ++t) {
        const BlockInfo& B = P.blocks[sk[t].b];
        SK& s = sk[t];
        int32_t d = defer(listB, Ref{B_SCR, int32_t(s.p), s.y}, dim_static(int(s.p)), s.r, 1);
        dprod(listB[d], Ref{B_U, int32_t(s.p), B.off_u}, 0, Ref{B_SCR, B.cap, s.p1[0]}, 0,
              rank_dim(s.b), 0, 0, dim_static(int(s.p)), s.r, 1.0);
        for (size_t i = 0; i < lrs[t].terms.size(); ++i) {
          auto& T = lrs[t].terms[i];
          dprod(listB[d], T.U.ref, 0, Ref{B_SCR, T.V.cols.maxv, s.p1[i + 1]}, 0, T.U.cols,
                int(T.r0 - B.r0), 0, dim_static(int(T.r1 - T.r0)), s.r, -1.0);
        }
      }
      emit(listB, st);
      // R_Y
      for (auto& s : sk) tsqr(Ref{B_SCR, int32_t(s.p), s.y}, s.p, s.r, Ref{B_SCR, RM, s.ry});
      flush_tsqr(st);
      // P from SVD(R_Y)
      int32_t sm0 = int32_t(P.smalls.size());
      for (auto& s : sk) {
        SmallJob J{};
        J.kind = SK_SKETCH_P;
        J.out_rank_slot = s.rk.slot;
        J.k = s.r;
        J.R1 = Ref{B_SCR, RM, s.ry};
        J.C1 = Ref{B_SCR, RM, s.pm};
        J.cap = s.rk.maxv;
        J.sat = dim_static(-1);
        J.full = 0;
        J.cand_slot = -1;
        J.eps = -2.0;           // tau from the context at run time
        P.smalls.push_back(J);
      }
      flush_small(st, sm0);
      // Q = Y P
      for (auto& s : sk) {
        int32_t d = defer(listA, Ref{B_SCR, int32_t(s.p), s.qm}, dim_static(int(s.p)), s.rk, 1);
        dprod(listA[d], Ref{B_SCR, int32_t(s.p), s.y}, 0, Ref{B_SCR, RM, s.pm}, 0, s.r, 0, 0,
              dim_static(int(s.p)), s.rk, 1.0);
      }
      emit(listA, st);
      // Z1 = U^T Q for A and terms
      for (size_t t = 0; t < lrs.size(); ++t) {
        const BlockInfo& B = P.blocks[sk[t].b];
        SK& s = sk[t];
        int rmaxT = s.r.maxv;
        int64_t za = scr_alloc(int64_t(B.cap) * rmaxT);
        s.z1.push_back(za);
        int32_t d = defer(listA, Ref{B_SCR, B.cap, za}, rank_dim(s.b), s.rk, 1);
        dprod(listA[d], Ref{B_U, int32_t(s.p), B.off_u}, 1, Ref{B_SCR, int32_t(s.p), s.qm}, 0,
              dim_static(int(s.p)), 0, 0, rank_dim(s.b), s.rk, 1.0);
        for (auto& T : lrs[t].terms) {
          int kc = T.U.cols.maxv;
          int64_t o = scr_alloc(int64_t(kc) * rmaxT);
          s.z1.push_back(o);
          int32_t dd = defer(listA, Ref{B_SCR, kc, o}, T.U.cols, s.rk, 1);
          dprod(listA[dd], T.U.ref, 1, Ref{B_SCR, int32_t(s.p), s.qm + (T.r0 - B.r0)}, 0,
                dim_static(int(T.r1 - T.r0)), 0, 0, T.U.cols, s.rk, 1.0);
        }
      }
      emit(listA, st);
      // B' = V_A Z1_A - sum V_t Z1_t
      for (size_t t = 0; t < lrs.size(); ++t) {
        const BlockInfo& B = P.blocks[sk[t].b];
        SK& s = sk[t];
        int32_t d = defer(listB, Ref{B_SCR, int32_t(s.q), s.bp}, dim_static(int(s.q)), s.rk, 1);
        dprod(listB[d], Ref{B_V, int32_t(s.q), B.off_v}, 0, Ref{B_SCR, B.cap, s.z1[0]}, 0,
              rank_dim(s.b), 0, 0, dim_static(int(s.q)), s.rk, 1.0);
        for (size_t i = 0; i < lrs[t].terms.size(); ++i) {
          auto& T = lrs[t].terms[i];
          dprod(listB[d], T.V.ref, 0, Ref{B_SCR, T.U.cols.maxv, s.z1[i + 1]}, 0, T.V.cols,
                int(T.p0 - B.c0), 0, dim_static(int(T.p1 - T.p0)), s.rk, -1.0);
        }
      }
      emit(listB, st);
      // second lane, once B' exists: B''_t = L_jj^{-1} B'_t on the leaf-j rows
      // (the first rows of every target that starts at j), while this lane
      // computes R_Q, R_B' and the truncation
      st.push_back(Stage{ST_FORK, 0, 0});
      {
        const BlockInfo& Dg = P.blocks[P.diag_block[j]];
        const int pd = int(Dg.r1 - Dg.r0);
        for (auto& s2 : sk) {
          s2.bpp = scr_alloc(int64_t(pd) * s2.r.maxv);
          int32_t d = defer(listA, Ref{B_SCR, pd, s2.bpp}, dim_static(pd), s2.rk, 1);
          dprod(listA[d], Ref{B_LINV, pd, P.linv_off[j]}, 0, Ref{B_SCR, int32_t(s2.q), s2.bp}, 0,
                dim_static(pd), 0, 0, dim_static(pd), s2.rk, 1.0);
        }
        cur_lane = 1;
        emit(listA, st);
        cur_lane = 0;
      }
      // R_Q and R_B'
      for (auto& s : sk) {
        tsqr(Ref{B_SCR, int32_t(s.p), s.qm}, s.p, s.rk, Ref{B_SCR, RM, s.rq});
        tsqr(Ref{B_SCR, int32_t(s.q), s.bp}, s.q, s.rk, Ref{B_SCR, RM, s.rb});
      }
      flush_tsqr(st);
      // C2 = R_Q^{-1} Z_k, new rank
      sm0 = int32_t(P.smalls.size());
      for (auto& s : sk) {
        SmallJob J{};
        J.kind = SK_SKETCH_F;
        J.out_rank_slot = P.blocks[s.b].rank_slot;
        J.k = s.rk;
        J.R1 = Ref{B_SCR, RM, s.rb};
        J.R2 = Ref{B_SCR, RM, s.rq};
        J.C1 = Ref{B_SCR, RM, s.c2};
        J.cap = P.blocks[s.b].cap;
        J.need_slot = P.blocks[s.b].need_slot;
        J.sat = s.r;            // saturation if the kept rank nearly fills r
        J.full = int32_t(std::min(s.p, s.q));
        J.cand_slot = P.blocks[s.b].cand_slot;
        J.eps = -1.0;           // filled at run time from the context eps
        P.smalls.push_back(J);
      }
      flush_small(st, sm0);
      // U := Q C2, V := B' C2 with the leaf-j rows of V from B'' (already
      // multiplied by L_jj^{-1}: the second lane joins first)
      st.push_back(Stage{ST_JOIN, 0, 0});
      const int pdj = int(cj1 - cj0);
      for (auto& s : sk) {
        const BlockInfo& B = P.blocks[s.b];
        int32_t d = defer(listA, Ref{B_U, int32_t(s.p), B.off_u}, dim_static(int(s.p)),
                          rank_dim(s.b), 1);
        dprod(listA[d], Ref{B_SCR, int32_t(s.p), s.qm}, 0, Ref{B_SCR, RM, s.c2}, 0, s.rk, 0, 0,
              dim_static(int(s.p)), rank_dim(s.b), 1.0);
        int32_t d2 = defer(listA, Ref{B_V, int32_t(s.q), B.off_v}, dim_static(int(s.q)),
                           rank_dim(s.b), 1);
        dprod(listA[d2], Ref{B_SCR, pdj, s.bpp}, 0, Ref{B_SCR, RM, s.c2}, 0, s.rk, 0, 0,
              dim_static(pdj), rank_dim(s.b), 1.0);
        if (s.q > pdj)
          dprod(listA[d2], Ref{B_SCR, int32_t(s.q), s.bp + pdj}, 0, Ref{B_SCR, RM, s.c2}, 0, s.rk,
                pdj, 0, dim_static(int(s.q) - pdj), rank_dim(s.b), 1.0);
      }
      emit(listA, st);
    }

    // ---- without low-rank targets the second lane joins here
    if (lrs.empty()) st.push_back(Stage{ST_JOIN, 0, 0});

    // ---- sibling update: the ancestor t1 whose last leaf is c_j, a left son
    {
      int lv = D;
      int64_t node = j;
      while (lv >= 1 && (node & 1) == 1) {
        node >>= 1;
        --lv;
      }
      if (lv >= 1) {
        const int64_t t1 = node, t2 = node + 1;
        const int64_t T1a = lo(lv, t1), T2a = lo(lv, t2), T2b = hi(lv, t2);
        auto rhs = [&](Ref Xbase, int64_t xrow0, Dim cols) {
          // X rows are indexed from absolute row xrow0
          Src Xs{Xbase, cols};
          Ref Out = Xbase;
          Out.off += (T2a - xrow0);
          int32_t dB = defer(listB, Out, dim_static(int(T2b - T2a)), cols, 0);
          hmv_pieces(lv, t2, lv, t1, Xs, xrow0, listA, listB, dB, -1.0, T2a, false);
        };
        // targets whose column cluster is the parent of t1 or an ancestor of it
        for (int lvl = lv - 1; lvl >= 0; --lvl) {
          auto it = by_col.find(key3(lvl, t1 >> (lv - lvl), 0));
          if (it == by_col.end()) continue;
          for (int32_t b : it->second) {
            const BlockInfo& B = P.blocks[b];
            xblk = b;
            rhs(Ref{B_V, int32_t(B.c1 - B.c0), B.off_v}, B.c0, rank_dim(b));
            xblk = -1;
          }
        }
        if (fuse_rhs) rhs(Ref{B_RHS, int32_t(P.rhs_ld), 0}, 0, dim_static(1));
        emit(listA, st);
        emit(listB, st);
      }
    }
  }
  if (dyn_max > P.n_dyn) P.n_dyn = dyn_max;
}

// Assembly recompression of every low-rank block (ACA output in U, V with
// rank0 columns): R_U, R_V by TSQR, SVD(R_U R_V^T), U := U C_U, V := V C_V.
// Done in chunks so the R slots fit in the persistent scratch.
void Builder::build_recompress() {
  const int RM = P.rmax;
  const int64_t RR = int64_t(RM) * RM;
  std::vector<int32_t> lrb;
  for (int32_t b = 0; b < int32_t(P.blocks.size()); ++b)
    if (P.blocks[b].kind == 1) lrb.push_back(b);
  const size_t CH = 2048;
  int64_t pers_max = 0;
  for (size_t c0 = 0; c0 < lrb.size(); c0 += CH) {
    size_t c1 = std::min(lrb.size(), c0 + CH);
    scr_top = 0;
    // the R slots live in the persistent scratch; segment Rs in the step scratch
    int64_t pers = 0;
    std::vector<int64_t> ru(c1 - c0), rv(c1 - c0), cu(c1 - c0), cv(c1 - c0);
    for (size_t i = c0; i < c1; ++i) {
      ru[i - c0] = pers;
      pers += RR;
      rv[i - c0] = pers;
      pers += RR;
      cu[i - c0] = pers;
      pers += RR;
      cv[i - c0] = pers;
      pers += RR;
    }
    pers_max = std::max(pers_max, pers);
    for (size_t i = c0; i < c1; ++i) {
      const BlockInfo& B = P.blocks[lrb[i]];
      Dim k0 = dim_dyn(B.rank0_slot, B.cap);
      tsqr(Ref{B_U, int32_t(B.r1 - B.r0), B.off_u}, B.r1 - B.r0, k0, Ref{B_PERS, RM, ru[i - c0]});
      tsqr(Ref{B_V, int32_t(B.c1 - B.c0), B.off_v}, B.c1 - B.c0, k0, Ref{B_PERS, RM, rv[i - c0]});
    }
    flush_tsqr(P.recomp_stages);
    int32_t sm0 = int32_t(P.smalls.size());
    for (size_t i = c0; i < c1; ++i) {
      const BlockInfo& B = P.blocks[lrb[i]];
      SmallJob J{};
      J.kind = SK_RECOMP;
      J.out_rank_slot = B.rank_slot;
      J.k = dim_dyn(B.rank0_slot, B.cap);
      J.R1 = Ref{B_PERS, RM, ru[i - c0]};
      J.R2 = Ref{B_PERS, RM, rv[i - c0]};
      J.C1 = Ref{B_PERS, RM, cu[i - c0]};
      J.C2 = Ref{B_PERS, RM, cv[i - c0]};
      J.cap = B.cap;
      J.sat = dim_static(-1);
      J.full = 0;
      J.cand_slot = -1;
      J.eps = -1.0;
      P.smalls.push_back(J);
    }
    flush_small(P.recomp_stages, sm0);
    for (size_t i = c0; i < c1; ++i) {
      const BlockInfo& B = P.blocks[lrb[i]];
      Dim k0 = dim_dyn(B.rank0_slot, B.cap);
      int32_t d = defer(listA, Ref{B_U, int32_t(B.r1 - B.r0), B.off_u},
                        dim_static(int(B.r1 - B.r0)), rank_dim(lrb[i]), 1);
      dprod(listA[d], Ref{B_U, int32_t(B.r1 - B.r0), B.off_u}, 0, Ref{B_PERS, RM, cu[i - c0]}, 0,
            k0, 0, 0, dim_static(int(B.r1 - B.r0)), rank_dim(lrb[i]), 1.0);
      int32_t d2 = defer(listA, Ref{B_V, int32_t(B.c1 - B.c0), B.off_v},
                         dim_static(int(B.c1 - B.c0)), rank_dim(lrb[i]), 1);
      dprod(listA[d2], Ref{B_V, int32_t(B.c1 - B.c0), B.off_v}, 0, Ref{B_PERS, RM, cv[i - c0]}, 0,
            k0, 0, 0, dim_static(int(B.c1 - B.c0)), rank_dim(lrb[i]), 1.0);
    }
    emit(listA, P.recomp_stages);
  }
  P.recomp_stages.push_back(Stage{ST_COPY_RANK, 0, 0});
  P.pers_elems = std::max(P.pers_elems, pers_max);
}

// Forward (L v = z) and backward (L^T x = v) substitution on B_RHS col 0.
void Builder::build_solves() {
  const int D = P.D;
  const int64_t m = int64_t(1) << D;
  P.fsolve_steps.assign(m, {});
  P.bsolve_steps.assign(m, {});
  Ref X{B_RHS, int32_t(P.rhs_ld), 0};
  for (int64_t j = 0; j < m; ++j) {
    auto& st = P.fsolve_steps[j];
    scr_top = 0;
    int64_t c0 = lo(D, j);
    int pj = int(hi(D, j) - c0);
    // the same arithmetic as the solve fused into the factorisation sweep:
    // multiplication by the stored inverse of L_jj
    int32_t t0 = int32_t(P.trsms.size());
    P.trsms.push_back(TrsmJob{Ref{B_LINV, pj, P.linv_off[j]}, pj, 0, Ref{B_RHS, int32_t(P.rhs_ld), c0},
                              dim_static(1), 0, 1});
    st.push_back(Stage{ST_TRMM, t0, t0 + 1});
    int lv = D;
    int64_t node = j;
    while (lv >= 1 && (node & 1) == 1) {
      node >>= 1;
      --lv;
    }
    if (lv >= 1) {
      int64_t t1 = node, t2 = node + 1;
      int64_t T2a = lo(lv, t2), T2b = hi(lv, t2);
      Ref Out = X;
      Out.off += T2a;
      int32_t dB = defer(listB, Out, dim_static(int(T2b - T2a)), dim_static(1), 0);
      hmv_pieces(lv, t2, lv, t1, Src{X, dim_static(1)}, 0, listA, listB, dB, -1.0, T2a, false);
      emit(listA, st);
      emit(listB, st);
    }
  }
  // backward: j descending; x_j = L_jj^{-T} v_j; then for the ancestor t2
  // whose first leaf is c_j and which is a right son: v[t1] -= L(t2,t1)^T x[t2]
  for (int64_t jj = m - 1; jj >= 0; --jj) {
    auto& st = P.bsolve_steps[m - 1 - jj];
    scr_top = 0;
    int64_t c0 = lo(D, jj);
    int pj = int(hi(D, jj) - c0);
    int32_t t0 = int32_t(P.trsms.size());
    P.trsms.push_back(TrsmJob{Ref{B_DENSE, pj, P.blocks[P.diag_block[jj]].off_d}, pj, 2,
                              Ref{B_RHS, int32_t(P.rhs_ld), c0}, dim_static(1), 0, 1});
    st.push_back(Stage{ST_TRSM, t0, t0 + 1});
    int lv = D;
    int64_t node = jj;
    while (lv >= 1 && (node & 1) == 0) {
      node >>= 1;
      --lv;
    }
    if (lv >= 1) {
      int64_t t2 = node, t1 = node - 1;
      int64_t T1a = lo(lv, t1), T1b = hi(lv, t1);
      Ref Out = X;
      Out.off += T1a;
      int32_t dB = defer(listB, Out, dim_static(int(T1b - T1a)), dim_static(1), 0);
      hmv_pieces(lv, t2, lv, t1, Src{X, dim_static(1)}, 0, listA, listB, dB, -1.0, T1a, true);
      emit(listA, st);
      emit(listB, st);
    }
  }
}

// y = C~ x on the assembled matrix (x = B_RHS col 0, y = col 1), y = L~ x
// and y = L~^T x on the factor.  Output rows are split by leaf cluster so
// every job owns its rows.
void Builder::build_matvec() {
  const int D = P.D;
  const int64_t m = int64_t(1) << D;
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<Stage>& out = pass == 0 ? P.matvec_stages : (pass == 1 ? P.lmul_stages : P.ltmul_stages);
    scr_top = 0;
    Ref X{B_RHS, int32_t(P.rhs_ld), 0};
    std::vector<int32_t> jobB(m);
    for (int64_t j = 0; j < m; ++j) {
      Ref Y{B_RHS, int32_t(P.rhs_ld), P.rhs_ld + lo(D, j)};
      jobB[j] = defer(listB, Y, dim_static(int(hi(D, j) - lo(D, j))), dim_static(1), 1);
    }
    for (int32_t b = 0; b < int32_t(P.blocks.size()); ++b) {
      const BlockInfo& B = P.blocks[b];
      // leaf rows covered by the block rows / cols
      auto leaf_of = [&](int64_t r) {
        // leaf containing absolute row r (leaves are contiguous, sizes differ by <= 1)
        int64_t lo_ = 0, hi_ = m - 1;
        while (lo_ < hi_) {
          int64_t mid = (lo_ + hi_ + 1) / 2;
          if (lo(D, mid) <= r) lo_ = mid; else hi_ = mid - 1;
        }
        return lo_;
      };
      bool diag = (B.a == B.c);
      for (int side = 0; side < 2; ++side) {
        if (pass == 2 && side == 0) continue;   // L^T x: the transposed lower part only
        if (side == 1 && diag && pass != 2) break;   // diagonal tiles hold both triangles (C) / lower (L)
        if (side == 1 && pass == 1) break;   // L x uses the lower part only
        // side 0: y[rows] += M x[cols]; side 1: y[cols] += M^T x[rows]
        int64_t o0 = side == 0 ? B.r0 : B.c0, o1 = side == 0 ? B.r1 : B.c1;
        int64_t i0 = side == 0 ? B.c0 : B.r0, i1 = side == 0 ? B.c1 : B.r1;
        int64_t tmp = -1;
        if (B.kind == 1) {
          tmp = scr_alloc(P.kcap);
          int32_t dA = defer(listA, Ref{B_SCR, P.kcap, tmp}, rank_dim(b), dim_static(1), 1);
          Ref inner = side == 0 ? Ref{B_V, int32_t(B.c1 - B.c0), B.off_v}
                                : Ref{B_U, int32_t(B.r1 - B.r0), B.off_u};
          Ref xs = X;
          xs.off += i0;
          dprod(listA[dA], inner, 1, xs, 0, dim_static(int(i1 - i0)), 0, 0, rank_dim(b),
                dim_static(1), 1.0);
        }
        for (int64_t L = leaf_of(o0); L < m && lo(D, L) < o1; ++L) {
          int64_t a = std::max(o0, lo(D, L)), e = std::min(o1, hi(D, L));
          Deferred& dj = listB[jobB[L]];
          if (B.kind == 1) {
            Ref outer = side == 0 ? Ref{B_U, int32_t(B.r1 - B.r0), B.off_u + (a - B.r0)}
                                  : Ref{B_V, int32_t(B.c1 - B.c0), B.off_v + (a - B.c0)};
            dprod(dj, outer, 0, Ref{B_SCR, P.kcap, tmp}, 0, rank_dim(b), int(a - lo(D, L)), 0,
                  dim_static(int(e - a)), dim_static(1), 1.0);
          } else {
            int32_t ld = int32_t(B.r1 - B.r0);
            Ref xs = X;
            xs.off += i0;
            if (side == 0)
              dprod(dj, Ref{B_DENSE, ld, B.off_d + (a - B.r0)}, 0, xs, 0,
                    dim_static(int(i1 - i0)), int(a - lo(D, L)), 0, dim_static(int(e - a)),
                    dim_static(1), 1.0);
            else
              dprod(dj, Ref{B_DENSE, ld, B.off_d + (a - B.c0) * ld}, 1, xs, 0,
                    dim_static(int(i1 - i0)), int(a - lo(D, L)), 0, dim_static(int(e - a)),
                    dim_static(1), 1.0);
          }
        }
      }
    }
    emit(listA, out);
    emit(listB, out);
  }
}

}  // namespace

std::string build_plan(Plan& P, int64_t n, int D, int leaf, const int64_t* blk, int64_t nb,
                       int kcap, bool mixed, const int32_t* caps) {
  P = Plan();
  P.mixed = mixed;
  P.n = n;
  P.D = D;
  P.leaf = leaf;
  P.kcap = kcap;
  P.rcap = kcap + OVERSAMPLE_MAX;
  P.rmax = std::max(P.rcap, kcap);
  if (kcap > 64 || kcap < 1) return "rank capacity must be in [1, 64]";
  if (P.rmax > 80) return "rank capacity plus oversampling must not exceed 80";
  // node ranges: left son takes ceil(s/2)
  P.lo.resize(D + 1);
  P.lo[0] = {0, n};
  for (int l = 1; l <= D; ++l) {
    auto& prev = P.lo[l - 1];
    auto& cur = P.lo[l];
    int64_t cnt = int64_t(1) << (l - 1);
    cur.resize(2 * cnt + 1);
    for (int64_t i = 0; i < cnt; ++i) {
      int64_t a = prev[i], b = prev[i + 1];
      cur[2 * i] = a;
      cur[2 * i + 1] = a + (b - a + 1) / 2;
    }
    cur[2 * cnt] = n;
  }
  int64_t m = int64_t(1) << D;
  for (int64_t i = 0; i < m; ++i)
    if (P.lo[D][i + 1] - P.lo[D][i] > LEAF_MAX) return "leaf larger than 128";
  P.blocks.resize(nb);
  P.diag_block.assign(m, -1);
  int32_t dyn = 0;
  for (int64_t b = 0; b < nb; ++b) {
    BlockInfo& B = P.blocks[b];
    B.level = int32_t(blk[4 * b]);
    B.a = int32_t(blk[4 * b + 1]);
    B.c = int32_t(blk[4 * b + 2]);
    B.kind = int32_t(blk[4 * b + 3]);
    B.r0 = P.lo[B.level][B.a];
    B.r1 = P.lo[B.level][B.a + 1];
    B.c0 = P.lo[B.level][B.c];
    B.c1 = P.lo[B.level][B.c + 1];
    int64_t p = B.r1 - B.r0, q = B.c1 - B.c0;
    if (B.kind == 1) {
      B.cap = caps ? caps[b] : kcap;
      if (B.cap < 1 || B.cap > kcap) return "block rank capacity outside [1, kcap]";
      B.off_u = P.u_elems;
      P.u_elems += p * B.cap;
      B.off_v = P.v_elems;
      P.v_elems += q * B.cap;
      B.off_d = -1;
      B.rank_slot = dyn++;
      B.rank0_slot = dyn++;
      B.hint_slot = dyn++;
      B.cand_slot = dyn++;
      B.need_slot = dyn++;
      P.n_lr++;
      P.lr_rows += p + q;
    } else {
      B.off_d = P.dense_elems;
      P.dense_elems += p * q;
      B.off_u = B.off_v = -1;
      B.rank_slot = B.rank0_slot = B.hint_slot = B.cand_slot = B.need_slot = -1;
      B.cap = 0;
      P.n_dense++;
      if (B.level != D) return "dense block above the leaf level";
      if (B.a == B.c) P.diag_block[B.a] = int32_t(b);
    }
    P.status[key3(B.level, B.a, B.c)] = int32_t(b);
    int l = B.level;
    int64_t x = B.a, y = B.c;
    while (l > 0) {
      --l;
      x >>= 1;
      y >>= 1;
      uint64_t k = key3(l, x, y);
      if (P.status.count(k)) break;
      P.status[k] = -1;
    }
  }
  for (int64_t i = 0; i < m; ++i)
    if (P.diag_block[i] < 0) return "missing diagonal leaf";
  P.linv_off.resize(m);
  for (int64_t i = 0; i < m; ++i) {
    const int64_t pj = P.lo[D][i + 1] - P.lo[D][i];
    P.linv_off[i] = P.linv_elems;
    P.linv_elems += pj * pj;
  }
  P.rhs_ld = n;
  P.omega_rows = std::max<int64_t>(n, 1);
  Builder Bd(P);
  Bd.dyn_base = dyn;
  Bd.dyn_top = dyn;
  Bd.dyn_max = dyn;
  P.n_dyn = dyn;
  Bd.build_recompress();
  Bd.core_base = P.pers_elems;   // cores live above the assembly R slots
  // one sweep serves both uses: without an observation vector the fused
  // right-hand side is a zero column (a few flops per step)
  Bd.build_steps(true, P.steps);
  Bd.build_solves();
  Bd.build_matvec();
  if (Bd.dyn_max > P.n_dyn) P.n_dyn = Bd.dyn_max;
  // the GEMM kernel addresses an element of a product operand by a byte
  // offset below 2^31 from the operand's start, 2^31 being its masked one
  for (const GemmProd& g : P.gprods) {
    if (g.tb == 2) continue;
    const int64_t kk = g.k.maxv, mi = g.mi.maxv, nj = g.nj.maxv;
    const int64_t a = g.ta == 0 ? mi + kk * g.A.ld : kk + mi * g.A.ld;
    const int64_t b = g.tb == 0 ? kk + nj * g.B.ld : nj + kk * g.B.ld;
    if (std::max(a, b) >= (int64_t(1) << 28)) return "a GEMM operand spans 2^28 elements or more";
  }
  int64_t launches = 0;
  for (auto& s : P.steps)
    for (auto& x : s) launches += (x.kind != ST_FORK && x.kind != ST_JOIN) ? 1 : 0;
  P.n_launch_fact = launches;
  return "";
}

}  // namespace hc
