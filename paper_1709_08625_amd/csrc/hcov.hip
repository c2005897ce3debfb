// C ABI of the hcov library: context, assembly, H-Cholesky sweep, solves.
// Declarations and citations are in include/hcov.h.
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hcov.h"
#include "common.h"
#include "launch.h"
#include "plan.h"
#include "tree.h"

using namespace hc;

struct hcov_ctx {
  int64_t n = 0;
  int leaf = 0, D = 0;
  double eta = 2.0, eps = 1e-8;
  hcov_opts opts{};
  hipStream_t stream = nullptr;
  hcov_theta theta{};
  MaternParams mp{};
  Plan plan;
  std::vector<int64_t> perm;
  std::vector<double> bbox;
  std::vector<int64_t> blocks_lac;
  // device memory
  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;
  size_t n_base_allocs = 0;   // allocations that do not depend on the plan (locations, permutation)
  int64_t bytes = 0;
  // per-block rank capacities (opts.initial_rank_cap; empty: max_rank everywhere)
  bool sizing = false;
  std::vector<int32_t> caps;
  int64_t n_replans = 0;
  bool plan_ok = false;       // plan-dependent buffers exist (false after a failed rebuild)
  double* d_loc = nullptr;     // double2[n], cluster order
  int* d_perm = nullptr;       // int32[n]
  double* d_buf[B_COUNT] = {};
  int* d_dyn = nullptr;
  int* d_status = nullptr;
  double* d_logdet = nullptr;  // per leaf
  double* d_part = nullptr;    // reduction partials
  double* d_tmp = nullptr;     // n doubles
  FillJob* d_fill = nullptr;
  AcaJob* d_aca = nullptr;
  int n_fill = 0, n_aca = 0;
  // large blocks: multi-work-group ACA
  AcaJob* d_acab = nullptr;
  int n_acab = 0, n_brow = 0, n_bcol = 0;
  AcaBigChunk *d_brow = nullptr, *d_bcol = nullptr;
  int *d_brow_first = nullptr, *d_brow_count = nullptr, *d_bcol_first = nullptr, *d_bcol_count = nullptr;
  AcaBigState* d_bstate = nullptr;
  double *d_bpart = nullptr, *d_bacc = nullptr;
  int* d_bactive = nullptr;
  LaunchCtx L{};
  // a copy of the assembled C~ (opts.keep_matrix): its dense and low-rank
  // arenas and dynamic dimensions, and the launch context that addresses them
  bool keep = false, kept_valid = false;
  double* d_keep[3] = {};      // dense, U, V
  int* d_dyn_keep = nullptr;
  LaunchCtx Lc{};
  double* d_vec = nullptr;     // 6 n doubles: vectors of the iterations (PCG, power method)
  int pcg_iters = 0;
  double pcg_relres = 0.0;
  // kernel profiling (HIP events around every launch of one stage kind)
  int prof_kind = -1;
  // second lane of the factorisation sweep (see ST_FORK / ST_JOIN)
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // the sweep captured as a graph (index 1: with the fused right-hand side),
  // replayed on gstream between two events of the caller's stream
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<hipGraphExec_t> gexec;      // segments of whole steps, replayed in order
  bool graph_failed = false;
  int64_t n_replays = 0;
  int64_t n_retries = 0;       // factorisations redone with wider sketches
  int sat_last = 0;            // saturated sketches of the last factorisation
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
  std::vector<Stage> prof_stages;
  std::vector<double> prof_times;   // per-launch ms of the last profiling session
  std::vector<std::pair<int, int>> prof_where;   // (sweep step, stage) of each profiled launch, step -1 outside
  int prof_step = -1;                            // sweep step being launched
  bool tuned = false;                            // the GEMM kernel choice was timed (opts.autotune)
  int64_t n_switched = 0;                        // GEMM launches the tuning moved to the other kernel
  // state
  bool assembled = false, factored = false;
  double ms_tree = 0, ms_asm = 0, ms_fact = 0, ms_solve = 0;
  std::string err;
};

namespace {

const char* kErr[] = {"ok", "invalid argument", "matrix not positive definite", "out of memory",
                      "call out of order", "device error", "rank capacity exceeded", "not completed yet"};

int fail(hcov_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, x)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, HCOV_EDEVICE, std::string("HIP: ") + hipGetErrorString(e_) + " in " #x); \
  } while (0)

void* dev_alloc(hcov_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (c->opts.alloc) {
    p = c->opts.alloc(bytes, c->opts.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    c->allocs.push_back(p);
    c->alloc_bytes.push_back(bytes);
    c->bytes += int64_t(bytes);
  }
  return p;
}

template <class T>
T* upload(hcov_ctx* c, const std::vector<T>& v) {
  T* d = (T*)dev_alloc(c, v.size() * sizeof(T));
  if (!d) return nullptr;
  if (!v.empty() && hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return nullptr;
  return d;
}

// Temme's Gamma_1, Gamma_2 (Temme 1975): Gamma_1(mu) = (1/Gamma(1-mu) -
// 1/Gamma(1+mu)) / (2 mu), Gamma_2(mu) = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2.
// For |mu| < 1e-3 the Taylor series of 1/Gamma(1+z) (Abramowitz & Stegun
// 6.1.34) avoids the cancellation; otherwise long double tgamma suffices.
void temme_gammas(double mu, double& g1, double& g2) {
  if (std::fabs(mu) < 1e-3) {
    const double eg = 0.57721566490153286061;    // a1 (Euler's constant)
    const double a2 = -0.6558780715202538;
    const double a3 = -0.0420026350340952;
    const double a4 = 0.1665386113822915;
    const double a5 = -0.0421977345555443;
    double m2 = mu * mu;
    g1 = -(eg + a3 * m2 + a5 * m2 * m2);
    g2 = 1.0 + a2 * m2 + a4 * m2 * m2;
  } else {
    long double m = mu;
    long double ip = 1.0L / std::tgamma(1.0L - m), im = 1.0L / std::tgamma(1.0L + m);
    g1 = double((ip - im) / (2.0L * m));
    g2 = double((ip + im) / 2.0L);
  }
}

MaternParams make_params(const hcov_theta& t) {
  MaternParams P{};
  P.sigma2 = t.sigma2;
  P.inv_ell = 1.0 / t.ell;
  P.nu = t.nu;
  P.nugget = t.nugget;
  if (t.nu == 0.5)
    P.kind = 1;
  else if (t.nu == 1.5)
    P.kind = 2;
  else if (t.nu == 2.5)
    P.kind = 3;
  else
    P.kind = 0;
  long double nu = t.nu;
  P.norm = double((long double)t.sigma2 * std::pow(2.0L, 1.0L - nu) / std::tgamma(nu));
  int N = int(std::floor(t.nu + 0.5));
  double mu = t.nu - N;
  P.N = N;
  P.mu = mu;
  temme_gammas(mu, P.g1, P.g2);
  P.gp = 1.0 / (P.g2 - mu * P.g1);
  P.gm = 1.0 / (P.g2 + mu * P.g1);
  if (std::fabs(mu) < 1e-8) {
    double x = M_PI * mu;
    P.mupi = 1.0 + x * x / 6.0;
  } else {
    P.mupi = double((long double)M_PI * mu / std::sin((long double)M_PI * mu));
  }
  return P;
}

bool theta_ok(const hcov_theta& t) {
  return std::isfinite(t.sigma2) && std::isfinite(t.ell) && std::isfinite(t.nu) && std::isfinite(t.nugget) &&
         t.sigma2 > 0 && t.ell > 0 && t.nu > 0 && t.nu <= 20.0 && t.nugget >= 0;
}

int tree_depth(int64_t n, int leaf) {
  int D = 0;
  while ((n + (int64_t(1) << D) - 1) / (int64_t(1) << D) > leaf) ++D;
  return D;
}

int run_stages(hcov_ctx* c, const std::vector<Stage>& st, const LaunchCtx* Lx = nullptr) {
  const LaunchCtx& LC = Lx ? *Lx : c->L;
  for (const Stage& s : st) {
    if (s.kind == ST_FORK) {
      HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
      HIPCHK(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
      continue;
    }
    if (s.kind == ST_JOIN) {
      HIPCHK(c, hipEventRecord(c->ev_join, c->stream2));
      HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
      continue;
    }
    hipStream_t sm = s.lane ? c->stream2 : c->stream;
    if (s.kind == c->prof_kind || (s.kind == ST_GEMM_WIDE && c->prof_kind == ST_GEMM)) {
      hipEvent_t a, b;
      HIPCHK(c, hipEventCreate(&a));
      HIPCHK(c, hipEventCreate(&b));
      HIPCHK(c, hipEventRecord(a, sm));
      HIPCHK(c, launch_stage(s, LC, sm));
      HIPCHK(c, hipEventRecord(b, sm));
      c->prof_ev.emplace_back(a, b);
      c->prof_stages.push_back(s);
      c->prof_where.emplace_back(c->prof_step, int(&s - st.data()));
    } else {
      HIPCHK(c, launch_stage(s, LC, sm));
    }
  }
  return HCOV_OK;
}

inline int dyn_value(const std::vector<int>& dyn, const Dim& d) {
  if (d.slot < 0) return d.maxv;
  int v = dyn[d.slot] + d.add;
  return v < d.maxv ? v : d.maxv;
}

// Algorithmic work of one stage with the current dynamic dimensions: FP64
// flops and the bytes its operands must move at least once (each product
// reads its A and B operands; each job writes its output and, when it
// accumulates, reads it too; elements of 8 bytes, 4 for FP32 jobs).
void stage_work(const Plan& P, const std::vector<int>& dyn, const Stage& s, double* flops, double* bytes) {
  double f = 0.0, b = 0.0;
  if (s.kind == ST_GEMM || s.kind == ST_GEMM_WIDE) {
    // the tiles of a launch are sorted by cost, so one job's tiles need not
    // be adjacent: count every job of the launch once
    std::vector<int> jobs;
    jobs.reserve(size_t(s.end - s.begin));
    for (int t = s.begin; t < s.end; ++t) jobs.push_back(P.gtiles[t].job);
    std::sort(jobs.begin(), jobs.end());
    jobs.erase(std::unique(jobs.begin(), jobs.end()), jobs.end());
    for (int j : jobs) {
      const GemmJob& J = P.gjobs[j];
      int m = dyn_value(dyn, J.m), n = dyn_value(dyn, J.n);
      if (m <= 0 || n <= 0) continue;
      const double el = J.fp32 ? 4.0 : 8.0;
      b += 8.0 * double(m) * double(n) * (J.zero ? 1.0 : 2.0);
      for (int q = J.p0; q < J.p1; ++q) {
        const GemmProd& G = P.gprods[q];
        int k = dyn_value(dyn, G.k);
        int mi = std::min(dyn_value(dyn, G.mi), m - G.i0), nj = std::min(dyn_value(dyn, G.nj), n - G.j0);
        if (mi > 0 && nj > 0 && k > 0) {
          if (G.tb == 2) {   // partial-sum addition: one operand of mi x nj
            f += double(mi) * double(nj);
            b += el * double(mi) * double(nj);
          } else {
            f += 2.0 * k * double(mi) * double(nj);
            b += el * double(k) * (double(mi) + double(nj));
          }
        }
      }
    }
  } else if (s.kind == ST_LEAF) {
    for (int t = s.begin; t < s.end; ++t) {
      const double p = P.leafs[t].p;
      f += p * p * p / 3.0;
      b += 16.0 * p * p;
    }
  } else if (s.kind == ST_TRSM || s.kind == ST_TRMM) {
    for (int t = s.begin; t < s.end; ++t) {
      const TrsmJob& J = P.trsms[t];
      int nc = dyn_value(dyn, J.ncols);
      int cw = std::min(J.cw, nc - J.c0);
      if (cw > 0) {
        f += double(J.p) * J.p * cw;
        b += 8.0 * double(J.p) * (J.p + 2.0 * cw);
      }
    }
  }
  *flops = f;
  *bytes = b;
}

// Internal (positive) result of a factorisation whose sketches saturated
// below the widest width: the saturated blocks' rank hints were doubled, and
// the caller re-assembles and factorises again with the wider sketches.
constexpr int SAT_RETRY = 1;
constexpr double MIXED_EPS_FLOOR = 1e-6;
constexpr int MAX_SKETCH_RETRIES = 4;
// Internal (positive) result of an assembly or factorisation in which a
// block asked for more rank than its arena holds, below max_rank: the
// capacities were grown and the plan must be rebuilt before a repeat.
constexpr int GROW_REPLAN = 2;
constexpr int MAX_REPLANS = 8;

int setup_plan(hcov_ctx* c);
int replan(hcov_ctx* c);

// Raises the capacity of every low-rank block whose ACA or truncation asked
// for more than it holds (dyn need slots): to at least twice the old
// capacity and 3/2 of the request, rounded up to 8, at most max_rank.  The
// same rebuild gives blocks whose kept rank fills 3/4 of their room or more
// room for 3/2 of it, so that the next parameters rarely force another.
// Returns the number of overflowing blocks grown (0: none could grow, no
// rebuild is due), or an error.
int grow_caps(hcov_ctx* c) {
  const Plan& P = c->plan;
  std::vector<int> dyn(P.n_dyn + 1);
  HIPCHK(c, hipMemcpyAsync(dyn.data(), c->d_dyn, dyn.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int kcap = P.kcap;
  int grown = 0;
  auto up8 = [](int x) { return (x + 7) / 8 * 8; };
  std::vector<int32_t> next(c->caps);
  for (size_t b = 0; b < P.blocks.size(); ++b) {
    const BlockInfo& B = P.blocks[b];
    if (B.kind != 1 || B.cap >= kcap) continue;
    const int need = dyn[B.need_slot], kept = dyn[B.rank_slot];
    int want = B.cap;
    if (need > B.cap) {
      want = std::max(2 * B.cap, up8(need + need / 2));
      ++grown;
    } else if (4 * kept >= 3 * B.cap) {
      want = up8(kept + kept / 2);
    }
    next[b] = int32_t(std::min(kcap, std::max(B.cap, want)));
  }
  if (grown) c->caps.swap(next);
  return grown;
}

int check_status(hcov_ctx* c, bool spd_matters) {
  int st[3];
  HIPCHK(c, hipMemcpyAsync(st, c->d_status, 12, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (spd_matters) c->sat_last = st[2];
  if (c->sizing && (st[0] & STAT_RANK_OVERFLOW)) {
    const int g = grow_caps(c);
    if (g < 0) return g;
    if (g > 0) {
      c->factored = false;
      // widened sketch hints of this factorisation carry over to the rebuilt plan
      if (spd_matters && (st[0] & STAT_SKETCH_SAT) && !(st[0] & STAT_SAT_CAP))
        HIPCHK(c, launch_adopt_hints(c->L, c->stream));
      return GROW_REPLAN;
    }
  }
  if (spd_matters && (st[0] & STAT_SKETCH_SAT)) {
    // a saturated sketch may also have spoiled a later pivot: the retry (or
    // the error) comes first
    c->factored = false;
    if (st[0] & STAT_SAT_CAP)
      return fail(c, HCOV_ERANK, "a low-rank block's randomised sketch saturated at the widest width (its room + 16)");
    // the saturated blocks' doubled widths (and every other block's kept rank)
    // become the hints of the next factorisation, retried here or later
    HIPCHK(c, launch_adopt_hints(c->L, c->stream));
    if (c->opts.on_saturation == HCOV_SAT_RETRY) return SAT_RETRY;
    return fail(c, HCOV_ERANK, "a low-rank block's randomised sketch saturated (on_saturation = HCOV_SAT_ERROR)");
  }
  if (spd_matters && (st[0] & STAT_NOT_SPD)) {
    c->factored = false;
    return fail(c, HCOV_ENOTSPD, "non-positive pivot at cluster-order row " + std::to_string(st[1]));
  }
  if (st[0] & STAT_NONFINITE) return fail(c, HCOV_ENOTSPD, "non-finite matrix entry");
  if (st[0] & STAT_RANK_OVERFLOW) return fail(c, HCOV_ERANK, "a low-rank block exceeded max_rank");
  return HCOV_OK;
}

int reset_status(hcov_ctx* c) {
  static const int init[3] = {0, 0x7fffffff, 0};
  HIPCHK(c, hipMemcpyAsync(c->d_status, init, 12, hipMemcpyHostToDevice, c->stream));
  return HCOV_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int assemble(hcov_ctx* c) {
  if (!c->plan_ok) return fail(c, HCOV_ESTATE, "the plan rebuild of a capacity growth failed; context unusable");
  double t0 = now_ms();
  c->mp = make_params(c->theta);
  int r = reset_status(c);
  if (r) return r;
  HIPCHK(c, launch_fill(c->d_buf[B_DENSE], c->d_loc, c->d_fill, c->n_fill, c->mp, c->stream));
  const int cap_ok = c->opts.fixed_rank > 0 ? 1 : 0;
  HIPCHK(c, launch_aca(c->d_buf[B_U], c->d_buf[B_V], c->d_dyn, c->d_loc, c->d_aca, c->n_aca, c->mp,
                       c->eps * c->opts.aca_eps_factor, c->plan.kcap, cap_ok, c->d_status, c->stream));
  HIPCHK(c, run_aca_big(c->d_buf[B_U], c->d_buf[B_V], c->d_dyn, c->d_loc, c->d_acab, c->n_acab, c->d_brow,
                        c->n_brow, c->d_bcol, c->n_bcol, c->d_brow_first, c->d_brow_count, c->d_bcol_first,
                        c->d_bcol_count, c->d_bstate, c->d_bpart, c->d_bacc, c->d_bactive, c->mp,
                        c->eps * c->opts.aca_eps_factor, c->plan.kcap, cap_ok, c->d_status, c->stream));
  r = run_stages(c, c->plan.recomp_stages);
  if (r) return r;
  r = check_status(c, false);
  if (r) {
    c->ms_asm = now_ms() - t0;
    return r;
  }
  c->kept_valid = false;
  if (c->keep) {
    // C~ for products after the factorisation (H-matvec, PCG, error norms)
    const Plan& P = c->plan;
    HIPCHK(c, hipMemcpyAsync(c->d_keep[0], c->d_buf[B_DENSE], P.dense_elems * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_keep[1], c->d_buf[B_U], P.u_elems * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_keep[2], c->d_buf[B_V], P.v_elems * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_dyn_keep, c->d_dyn, (P.n_dyn + 1) * 4, hipMemcpyDeviceToDevice, c->stream));
    c->kept_valid = true;
  }
  c->ms_asm = now_ms() - t0;
  c->assembled = true;
  c->factored = false;
  return HCOV_OK;
}

// fixed-order sum of part[0..np) on the host after a device partial reduction
int reduce_dev(hcov_ctx* c, const double* x, int64_t n, int mode, double* out, const double* y = nullptr) {
  int64_t np = 0;
  HIPCHK(c, launch_reduce(x, y, n, mode, c->d_part, c->stream, &np));
  std::vector<double> h(np);
  if (np) HIPCHK(c, hipMemcpyAsync(h.data(), c->d_part, np * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // pairwise in fixed order
  while (h.size() > 1) {
    std::vector<double> g((h.size() + 1) / 2);
    for (size_t i = 0; i < g.size(); ++i) g[i] = h[2 * i] + (2 * i + 1 < h.size() ? h[2 * i + 1] : 0.0);
    h.swap(g);
  }
  *out = h.empty() ? 0.0 : h[0];
  return HCOV_OK;
}

// Captures the launches of the sweep (both lanes, joined by the fork/join
// events) on gstream into graphs of whole steps, each of at most
// GRAPH_STAGES stages (a graph is one long dependency chain; bounded
// segments keep the runtime's per-graph work bounded).  Kernel arguments are
// fixed for the life of the context (sizes that change with theta live in
// device memory), so the segments serve every later factorisation.  Any
// failure leaves the context on per-stage launches.
constexpr size_t GRAPH_STAGES = 1500;

void capture_sweep(hcov_ctx* c, const std::vector<std::vector<Stage>>& steps) {
  hipStream_t user = c->stream;
  c->stream = c->gstream;
  bool ok = true;
  size_t j = 0;
  while (ok && j < steps.size()) {
    if (hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      ok = false;
      break;
    }
    size_t staged = 0;
    while (j < steps.size() && (staged == 0 || staged + steps[j].size() <= GRAPH_STAGES)) {
      if (run_stages(c, steps[j]) != HCOV_OK) ok = false;
      staged += steps[j].size();
      ++j;
      if (!ok) break;
    }
    hipGraph_t g = nullptr;
    const bool ended = hipStreamEndCapture(c->gstream, &g) == hipSuccess;
    hipGraphExec_t ge = nullptr;
    ok = ok && ended && g && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (ok) c->gexec.push_back(ge);
  }
  c->stream = user;
  if (!ok) {
    for (auto ge : c->gexec)
      if (ge) (void)hipGraphExecDestroy(ge);
    c->gexec.clear();
    c->graph_failed = true;
    c->err.clear();
    (void)hipGetLastError();
  }
}

int factor(hcov_ctx* c, const double* z_dev_cluster, bool fuse) {
  if (!c->plan_ok) return fail(c, HCOV_ESTATE, "the plan rebuild of a capacity growth failed; context unusable");
  if (!c->assembled) return fail(c, HCOV_ESTATE, "matrix not assembled");
  double t0 = now_ms();
  int r = reset_status(c);
  if (r) return r;
  (void)z_dev_cluster;   // with fuse, the right-hand side is already in B_RHS
  // without an observation vector the sweep's right-hand-side column is zero
  if (!fuse) HIPCHK(c, launch_fill_value(c->d_buf[B_RHS], c->n, 0.0, c->stream));
  const auto& steps = c->plan.steps;
  if (c->gstream && c->prof_kind < 0 && !c->graph_failed && c->gexec.empty()) capture_sweep(c, steps);
  if (c->gstream && c->prof_kind < 0 && !c->gexec.empty()) {
    HIPCHK(c, hipEventRecord(c->ev_in, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->gstream, c->ev_in, 0));
    for (auto ge : c->gexec) HIPCHK(c, hipGraphLaunch(ge, c->gstream));
    c->n_replays += 1;
    HIPCHK(c, hipEventRecord(c->ev_out, c->gstream));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_out, 0));
  } else {
    for (size_t j = 0; j < steps.size(); ++j) {
      c->prof_step = int(j);
      r = run_stages(c, steps[j]);
      c->prof_step = -1;
      if (r) return r;
    }
  }
  c->assembled = false;   // C~ is overwritten by the factor
  r = check_status(c, true);
  c->ms_fact = now_ms() - t0;
  if (r) return r;
  c->factored = true;
  return HCOV_OK;
}

int to_cluster(hcov_ctx* c, const double* z, int where, double* dst);

// Assembly (if needed) and factorisation; with `z` the forward solve of z is
// fused into the sweep.  A saturated sketch re-assembles C~ and factorises
// again with the saturated blocks' sketches widened (at most
// MAX_SKETCH_RETRIES times).
int factorise_once(hcov_ctx* c, const double* z, int where);

// Launches of one stage kind (ST_GEMM: both GEMM kernels) are bracketed by
// events from here on.
int profile_begin(hcov_ctx* c, int kind) {
  c->prof_kind = kind;
  c->prof_ev.clear();
  c->prof_stages.clear();
  c->prof_where.clear();
  return HCOV_OK;
}

// Waits for the profiled launches and turns their events into prof_times
// (ms, launch order; prof_where says where each was launched); summed ms,
// algorithmic flops and bytes to the optional outputs.
int profile_collect(hcov_ctx* c, double* ms_out, double* fl_out, double* by_out) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream2));
  std::vector<int> dyn(c->plan.n_dyn + 1);
  HIPCHK(c, hipMemcpyAsync(dyn.data(), c->d_dyn, dyn.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ms = 0.0, fl = 0.0, by = 0.0;
  c->prof_times.clear();
  int rc = HCOV_OK;
  for (size_t i = 0; i < c->prof_ev.size(); ++i) {
    float t = 0.f;
    if (rc == HCOV_OK && hipEventElapsedTime(&t, c->prof_ev[i].first, c->prof_ev[i].second) != hipSuccess)
      rc = fail(c, HCOV_EDEVICE, "event timing failed");
    ms += t;
    c->prof_times.push_back(t);
    double f1 = 0.0, b1 = 0.0;
    stage_work(c->plan, dyn, c->prof_stages[i], &f1, &b1);
    fl += f1;
    by += b1;
    (void)hipEventDestroy(c->prof_ev[i].first);
    (void)hipEventDestroy(c->prof_ev[i].second);
  }
  c->prof_ev.clear();
  c->prof_stages.clear();
  if (ms_out) *ms_out = ms;
  if (fl_out) *fl_out = fl;
  if (by_out) *by_out = by;
  return rc;
}

// opts.autotune: the two GEMM kernels are timed on every sweep launch that
// both may run (two factorisations with events around the GEMM launches,
// the second with those launches switched to the other kernel), and each
// launch keeps the faster one.  Saturation retries inside the timed
// factorisations only add samples (the minimum per launch counts).
int autotune_once(hcov_ctx* c, const double* z, int where) {
  const int64_t rp0 = c->n_replans;
  auto& steps = c->plan.steps;
  auto is_gemm = [](const Stage& s) { return s.kind == ST_GEMM || s.kind == ST_GEMM_WIDE; };
  std::vector<std::vector<double>> best[2];
  for (int pass = 0; pass < 2; ++pass) {
    best[pass].assign(steps.size(), {});
    for (size_t j = 0; j < steps.size(); ++j) best[pass][j].assign(steps[j].size(), 1e300);
    if (pass == 1)
      for (auto& st : steps)
        for (auto& s : st)
          if (is_gemm(s) && s.alt) s.kind = s.kind == ST_GEMM ? ST_GEMM_WIDE : ST_GEMM;
    int r = profile_begin(c, ST_GEMM);
    if (r) return r;
    r = factorise_once(c, z, where);
    int r2 = profile_collect(c, nullptr, nullptr, nullptr);
    c->prof_kind = -1;
    if (r) return r;
    if (r2) return r2;
    // a capacity growth rebuilt the plan (its stages are the planner's
    // again): the caller starts the tuning over
    if (c->n_replans != rp0) return HCOV_OK;
    for (size_t i = 0; i < c->prof_where.size(); ++i) {
      const auto& w = c->prof_where[i];
      if (w.first < 0) continue;
      double& b = best[pass][size_t(w.first)][size_t(w.second)];
      b = std::min(b, c->prof_times[i]);
    }
  }
  // the stages are in their pass-1 (switched) state: switch back where the
  // planner's choice was not slower
  int64_t moved = 0;
  for (size_t j = 0; j < steps.size(); ++j)
    for (size_t i = 0; i < steps[j].size(); ++i) {
      Stage& s = steps[j][i];
      if (!is_gemm(s) || !s.alt) continue;
      if (best[0][j][i] <= best[1][j][i])
        s.kind = s.kind == ST_GEMM ? ST_GEMM_WIDE : ST_GEMM;
      else
        ++moved;
    }
  c->n_switched = moved;
  c->tuned = true;
  return HCOV_OK;
}

int autotune(hcov_ctx* c, const double* z, int where) {
  for (int round = 0; round <= MAX_REPLANS && !c->tuned; ++round) {
    const int r = autotune_once(c, z, where);
    if (r) return r;
  }
  return HCOV_OK;
}

int factorise(hcov_ctx* c, const double* z, int where) {
  if (c->opts.autotune && !c->tuned) {
    int r = autotune(c, z, where);
    if (r) return r;
  }
  return factorise_once(c, z, where);
}

int factorise_once(hcov_ctx* c, const double* z, int where) {
  int attempt = 0, grows = 0;
  auto grow = [&]() -> int {
    if (++grows > MAX_REPLANS)
      return fail(c, HCOV_ERANK, "block rank capacities still growing after " + std::to_string(MAX_REPLANS) +
                                     " plan rebuilds");
    return replan(c);
  };
  for (;;) {
    int r;
    if (!c->assembled) {
      r = assemble(c);
      if (r == GROW_REPLAN) {
        r = grow();
        if (r) return r;
        continue;
      }
      if (r) return r;
    }
    if (z) {
      r = to_cluster(c, z, where, c->d_buf[B_RHS]);
      if (r) return r;
    }
    r = factor(c, nullptr, z != nullptr);
    if (r == GROW_REPLAN) {
      r = grow();
      if (r) return r;
      continue;
    }
    if (r != SAT_RETRY) return r;
    if (attempt >= MAX_SKETCH_RETRIES)
      return fail(c, HCOV_ERANK, "sketches still saturated after " + std::to_string(MAX_SKETCH_RETRIES) +
                                     " retries with doubled widths");
    ++attempt;
    c->n_retries += 1;
  }
}

int to_cluster(hcov_ctx* c, const double* z, int where, double* dst) {
  if (where == HCOV_HOST) {
    HIPCHK(c, hipMemcpyAsync(c->d_tmp, z, c->n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_permute(c->d_tmp, dst, c->d_perm, c->n, 0, c->stream));
  } else {
    HIPCHK(c, launch_permute(z, dst, c->d_perm, c->n, 0, c->stream));
  }
  return HCOV_OK;
}

int from_cluster(hcov_ctx* c, const double* src, double* x, int where) {
  if (where == HCOV_HOST) {
    HIPCHK(c, launch_permute(src, c->d_tmp, c->d_perm, c->n, 1, c->stream));
    HIPCHK(c, hipMemcpyAsync(x, c->d_tmp, c->n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, launch_permute(src, x, c->d_perm, c->n, 1, c->stream));
  }
  return HCOV_OK;
}

int logdet_sum(hcov_ctx* c, double* out) {
  int64_t m = int64_t(1) << c->D;
  double s = 0;
  int r = reduce_dev(c, c->d_logdet, m, 1, &s);
  if (r) return r;
  *out = 2.0 * s;
  return HCOV_OK;
}

// Plan, device buffers, job arrays and launch contexts of the current block
// capacities (c->caps; empty: every block at max_rank).  Everything
// allocated here comes after the first n_base_allocs allocations of the
// context, so that release_plan can give it back before a rebuild.
int setup_plan(hcov_ctx* c) {
  const int64_t n = c->n;
  const hcov_opts& o = c->opts;
  // plan
  int64_t nb = int64_t(c->blocks_lac.size() / 4);
  std::string e = build_plan(c->plan, n, c->D, c->leaf, c->blocks_lac.data(), nb, o.max_rank,
                             o.precision == HCOV_MIXED, c->caps.empty() ? nullptr : c->caps.data());
  if (!e.empty()) {
    c->err = e;
    return HCOV_EINVAL;
  }
  Plan& P = c->plan;
  // memory estimate check
  size_t need = size_t(P.dense_elems + P.u_elems + P.v_elems + P.scr_elems + P.pers_elems + P.omega_rows * P.rcap +
                       2 * P.rhs_ld + P.linv_elems) * 8;
  if (c->keep) need += size_t(P.dense_elems + P.u_elems + P.v_elems + 6 * n) * 8;
  if (o.mem_cap_bytes && need > o.mem_cap_bytes) {
    c->err = "estimate " + std::to_string(need) + " bytes exceeds the memory cap";
    return HCOV_ENOMEM;
  }
  c->d_buf[B_DENSE] = (double*)dev_alloc(c, P.dense_elems * 8);
  c->d_buf[B_U] = (double*)dev_alloc(c, P.u_elems * 8);
  c->d_buf[B_V] = (double*)dev_alloc(c, P.v_elems * 8);
  c->d_buf[B_SCR] = (double*)dev_alloc(c, P.scr_elems * 8);
  c->d_buf[B_OMEGA] = (double*)dev_alloc(c, P.omega_rows * P.rcap * 8);
  c->d_buf[B_RHS] = (double*)dev_alloc(c, 2 * P.rhs_ld * 8);
  c->d_buf[B_PERS] = (double*)dev_alloc(c, P.pers_elems * 8);
  c->d_buf[B_LINV] = (double*)dev_alloc(c, P.linv_elems * 8);
  c->d_dyn = (int*)dev_alloc(c, (P.n_dyn + 1) * 4);
  c->d_status = (int*)dev_alloc(c, 16);
  int64_t m = int64_t(1) << c->D;
  c->d_logdet = (double*)dev_alloc(c, m * 8);
  c->d_part = (double*)dev_alloc(c, ((n + 1023) / 1024 + m / 1024 + 8) * 8);
  c->d_tmp = (double*)dev_alloc(c, n * 8);
  for (int b = 0; b < B_COUNT; ++b)
    if (!c->d_buf[b]) return HCOV_ENOMEM;
  if (c->keep) {
    c->d_keep[0] = (double*)dev_alloc(c, P.dense_elems * 8);
    c->d_keep[1] = (double*)dev_alloc(c, P.u_elems * 8);
    c->d_keep[2] = (double*)dev_alloc(c, P.v_elems * 8);
    c->d_dyn_keep = (int*)dev_alloc(c, (P.n_dyn + 1) * 4);
    c->d_vec = (double*)dev_alloc(c, 6 * n * 8);
    if (!c->d_keep[0] || !c->d_keep[1] || !c->d_keep[2] || !c->d_dyn_keep || !c->d_vec) return HCOV_ENOMEM;
  }
  if (!c->d_dyn || !c->d_status || !c->d_logdet || !c->d_part || !c->d_tmp) return HCOV_ENOMEM;
  if (hipMemsetAsync(c->d_dyn, 0, (P.n_dyn + 1) * 4, c->stream) != hipSuccess) return HCOV_EDEVICE;
  // fixed Gaussian test matrix of the randomised range finder
  if (launch_gaussian(c->d_buf[B_OMEGA], P.omega_rows * P.rcap, o.seed ? o.seed : 0x5eed5eedULL, c->stream) !=
      hipSuccess)
    return HCOV_EDEVICE;
  // job arrays
  std::vector<FillJob> fj;
  std::vector<AcaJob> aj;
  std::vector<int4> cp;
  for (auto& B : P.blocks) {
    if (B.kind == 0) {
      fj.push_back(FillJob{B.off_d, B.r0, B.c0, int32_t(B.r1 - B.r0), int32_t(B.c1 - B.c0), B.a == B.c ? 1 : 0, 0});
    } else {
      aj.push_back(AcaJob{B.off_u, B.off_v, B.r0, B.c0, int32_t(B.r1 - B.r0), int32_t(B.c1 - B.c0), B.rank0_slot,
                          B.cap, B.need_slot, 0});
      cp.push_back(make_int4(B.rank_slot, B.rank0_slot, B.hint_slot, B.cand_slot));
    }
  }
  // blocks with more than ACA_BIG_SPLIT rows + columns: multi-work-group ACA
  const int ACA_BIG_SPLIT = 2048;
  std::vector<AcaJob> big, small;
  for (auto& a : aj) (int64_t(a.p) + a.q > ACA_BIG_SPLIT ? big : small).push_back(a);
  std::stable_sort(small.begin(), small.end(), [](const AcaJob& a, const AcaJob& b) {
    return int64_t(a.p) + a.q > int64_t(b.p) + b.q;
  });
  aj = small;
  {
    std::vector<AcaBigChunk> rows, cols;
    std::vector<int> rf, rcn, cf, ccn;
    for (int b = 0; b < int(big.size()); ++b) {
      rf.push_back(int(rows.size()));
      for (int c0 = 0; c0 < big[b].q; c0 += ACA_BIG_CHUNK) rows.push_back(AcaBigChunk{b, c0});
      rcn.push_back(int(rows.size()) - rf.back());
      cf.push_back(int(cols.size()));
      for (int c0 = 0; c0 < big[b].p; c0 += ACA_BIG_CHUNK) cols.push_back(AcaBigChunk{b, c0});
      ccn.push_back(int(cols.size()) - cf.back());
    }
    c->n_acab = int(big.size());
    c->n_brow = int(rows.size());
    c->n_bcol = int(cols.size());
    if (c->n_acab > 0) {
      c->d_acab = upload(c, big);
      c->d_brow = upload(c, rows);
      c->d_bcol = upload(c, cols);
      c->d_brow_first = upload(c, rf);
      c->d_brow_count = upload(c, rcn);
      c->d_bcol_first = upload(c, cf);
      c->d_bcol_count = upload(c, ccn);
      c->d_bstate = (AcaBigState*)dev_alloc(c, size_t(c->n_acab) * ACA_BIG_STATE_BYTES);
      c->d_bpart = (double*)dev_alloc(c, size_t(std::max(c->n_brow, c->n_bcol)) * ACA_BIG_PREC * 8);
      c->d_bacc = (double*)dev_alloc(c, size_t(c->n_acab) * ACA_BIG_PREC * 8);
      c->d_bactive = (int*)dev_alloc(c, 16);
      if (!c->d_acab || !c->d_brow || !c->d_bcol || !c->d_brow_first || !c->d_brow_count || !c->d_bcol_first ||
          !c->d_bcol_count || !c->d_bstate || !c->d_bpart || !c->d_bacc || !c->d_bactive)
        return HCOV_ENOMEM;
    }
  }
  c->n_fill = int(fj.size());
  c->n_aca = int(aj.size());
  c->d_fill = upload(c, fj);
  c->d_aca = upload(c, aj);
  c->L = LaunchCtx{};
  LaunchCtx& L = c->L;
  for (int b = 0; b < B_COUNT; ++b) L.bufs.p[b] = c->d_buf[b];
  std::vector<Bufs> btab(1, L.bufs);
  L.dbufs = upload(c, btab);
  L.dyn = c->d_dyn;
  L.gjobs = upload(c, P.gjobs);
  L.gprods = upload(c, P.gprods);
  L.gtiles = upload(c, P.gtiles);
  L.tsegs = upload(c, P.tsegs);
  L.treds = upload(c, P.treds);
  L.smalls = upload(c, P.smalls);
  L.leafs = upload(c, P.leafs);
  L.trsms = upload(c, P.trsms);
  L.copy_pairs = upload(c, cp);
  L.n_copy = int(cp.size());
  L.rmax = P.rmax;
  L.oversample = o.oversample;
  L.fixed_rank = o.fixed_rank;
  // FP32 accumulation leaves noise of order 1e-7 relative in the low-rank
  // products: in mixed precision the truncations keep singular values above
  // max(eps, 1e-6) of the largest, so that noise is not kept as rank
  L.eps = o.precision == HCOV_MIXED ? std::max(c->eps, MIXED_EPS_FLOOR) : c->eps;
  L.tau = std::min(1e-10, 1e-2 * c->eps);
  L.logdet = c->d_logdet;
  L.status = c->d_status;
  if (!L.dbufs || !L.gjobs || !L.gprods || !L.gtiles || !L.tsegs || !L.treds || !L.smalls || !L.leafs ||
      !L.trsms || !L.copy_pairs || !c->d_fill || !c->d_aca)
    return HCOV_ENOMEM;
  if (c->keep) {
    // the launch context of the kept C~: its own arenas and dimensions
    c->Lc = L;
    c->Lc.bufs.p[B_DENSE] = c->d_keep[0];
    c->Lc.bufs.p[B_U] = c->d_keep[1];
    c->Lc.bufs.p[B_V] = c->d_keep[2];
    std::vector<Bufs> kt(1, c->Lc.bufs);
    c->Lc.dbufs = upload(c, kt);
    c->Lc.dyn = c->d_dyn_keep;
    if (!c->Lc.dbufs) return HCOV_ENOMEM;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return HCOV_EDEVICE;
  c->plan_ok = true;
  return HCOV_OK;
}

// Gives back everything setup_plan allocated (after the streams drained)
// and drops the captured sweep and any pending profiling events.
int release_plan(hcov_ctx* c) {
  if (c->stream2) HIPCHK(c, hipStreamSynchronize(c->stream2));
  if (c->gstream) HIPCHK(c, hipStreamSynchronize(c->gstream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->plan_ok = false;
  for (auto g : c->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  c->gexec.clear();
  for (auto& ev : c->prof_ev) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  c->prof_ev.clear();
  c->prof_stages.clear();
  c->prof_where.clear();
  for (size_t i = c->allocs.size(); i-- > c->n_base_allocs;) {
    if (c->opts.free)
      c->opts.free(c->allocs[i], c->opts.alloc_user);
    else
      (void)hipFree(c->allocs[i]);
    c->bytes -= int64_t(c->alloc_bytes[i]);
  }
  c->allocs.resize(c->n_base_allocs);
  c->alloc_bytes.resize(c->n_base_allocs);
  for (auto& b : c->d_buf) b = nullptr;
  c->d_dyn = c->d_status = nullptr;
  c->d_logdet = c->d_part = c->d_tmp = nullptr;
  c->d_fill = nullptr;
  c->d_aca = c->d_acab = nullptr;
  c->n_fill = c->n_aca = c->n_acab = c->n_brow = c->n_bcol = 0;
  c->d_brow = c->d_bcol = nullptr;
  c->d_brow_first = c->d_brow_count = c->d_bcol_first = c->d_bcol_count = nullptr;
  c->d_bstate = nullptr;
  c->d_bpart = c->d_bacc = nullptr;
  c->d_bactive = nullptr;
  for (auto& k : c->d_keep) k = nullptr;
  c->d_dyn_keep = nullptr;
  c->d_vec = nullptr;
  c->L = LaunchCtx{};
  c->Lc = LaunchCtx{};
  c->kept_valid = false;
  return HCOV_OK;
}

// Rebuilds the plan at the grown capacities.  The dynamic slots keep their
// numbering (it depends on the trees only), so the rank hints carry over;
// the need slots start again from zero.  C~ must be assembled again.
int replan(hcov_ctx* c) {
  const int32_t n_dyn = c->plan.n_dyn;
  std::vector<int> dyn(size_t(n_dyn) + 1);
  HIPCHK(c, hipMemcpyAsync(dyn.data(), c->d_dyn, dyn.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int r = release_plan(c);
  if (r) return r;
  r = setup_plan(c);
  if (r) {
    c->plan_ok = false;
    return r;
  }
  if (c->plan.n_dyn != n_dyn) {
    c->plan_ok = false;
    return fail(c, HCOV_EDEVICE, "plan rebuild changed the dynamic slots");
  }
  for (const auto& B : c->plan.blocks)
    if (B.kind == 1) dyn[B.need_slot] = 0;
  HIPCHK(c, hipMemcpyAsync(c->d_dyn, dyn.data(), dyn.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->assembled = c->factored = false;
  c->tuned = false;   // the rebuilt stages carry the planner's kernel choice
  c->n_switched = 0;
  c->n_replans += 1;
  return HCOV_OK;
}

// Assembly, repeated after each capacity growth it triggers.
int assemble_grown(hcov_ctx* c) {
  for (int g = 0;; ++g) {
    int r = assemble(c);
    if (r != GROW_REPLAN) return r;
    if (g >= MAX_REPLANS)
      return fail(c, HCOV_ERANK, "block rank capacities still growing after " + std::to_string(MAX_REPLANS) +
                                     " plan rebuilds");
    r = replan(c);
    if (r) return r;
  }
}

}  // namespace

extern "C" {

void hcov_opts_default(hcov_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = HCOV_FP64;
  o->max_rank = 64;
  o->aca_eps_factor = 0.1;
  o->fuse_solve = 1;
  o->use_graphs = 1;
  o->oversample = 10;
  o->on_saturation = HCOV_SAT_RETRY;
  o->keep_matrix = 0;
  o->quad_mode = HCOV_QUAD_DIRECT;
  o->pcg_tol = 1e-6;
  o->pcg_max_iter = 150;
  o->fixed_rank = 0;
  o->adm_rule = HCOV_ADM_MIN;
}

const char* hcov_strerror(int code) {
  if (code > 0 || code < -7) return "unknown error";
  return kErr[-code];
}

const char* hcov_last_error(const hcov_ctx* c) { return c ? c->err.c_str() : ""; }

int hcov_build(const double* locs, int64_t n, hcov_theta theta, double eps, int leaf, double eta,
               const hcov_opts* opts, void* hip_stream, hcov_ctx** out) {
  if (!out) return HCOV_EINVAL;
  *out = nullptr;
  if (!locs || n < 1 || n > (int64_t(1) << 30) || leaf < 2 || leaf > 128 || !(eta > 0) || !std::isfinite(eta) ||
      !(eps > 0 && eps < 1) || !theta_ok(theta))
    return HCOV_EINVAL;
  hcov_opts o;
  hcov_opts_default(&o);
  if (opts) o = *opts;
  if (o.max_rank < 1 || o.max_rank > 64 || !(o.aca_eps_factor > 0) || o.aca_eps_factor > 1) return HCOV_EINVAL;
  if (o.precision != HCOV_FP64 && o.precision != HCOV_MIXED) return HCOV_EINVAL;
  if (o.oversample < 2 || o.oversample > 64) return HCOV_EINVAL;
  if (o.on_saturation != HCOV_SAT_RETRY && o.on_saturation != HCOV_SAT_ERROR) return HCOV_EINVAL;
  if (o.quad_mode != HCOV_QUAD_DIRECT && o.quad_mode != HCOV_QUAD_PCG) return HCOV_EINVAL;
  if (!(o.pcg_tol > 0 && o.pcg_tol < 1) || o.pcg_max_iter < 1) return HCOV_EINVAL;
  if (o.fixed_rank < 0 || o.fixed_rank > o.max_rank) return HCOV_EINVAL;
  if (o.adm_rule != HCOV_ADM_MIN && o.adm_rule != HCOV_ADM_MAX && o.adm_rule != HCOV_ADM_WEAK) return HCOV_EINVAL;
  if (o.autotune != 0 && o.autotune != 1) return HCOV_EINVAL;
  if (o.initial_rank_cap < 0 || o.initial_rank_cap > o.max_rank) return HCOV_EINVAL;
  std::vector<double> h(2 * n);
  for (int64_t i = 0; i < 2 * n; ++i) {
    if (!std::isfinite(locs[i])) return HCOV_EINVAL;
    h[i] = locs[i] + 0.0;   // -0.0 -> +0.0
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return HCOV_EDEVICE;
  hcov_ctx* c = new hcov_ctx();
  c->n = n;
  c->leaf = leaf;
  c->eta = eta;
  c->eps = eps;
  c->opts = o;
  c->keep = o.keep_matrix != 0 || o.quad_mode == HCOV_QUAD_PCG;
  c->stream = (hipStream_t)hip_stream;
  if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      (o.use_graphs && (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess))) {
    if (c->stream2) (void)hipStreamDestroy(c->stream2);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    delete c;
    return HCOV_EDEVICE;
  }
  c->theta = theta;
  c->D = tree_depth(n, leaf);
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] { attr_err = setup_kernel_attributes(); });
  if (attr_err != hipSuccess) {
    hcov_destroy(c);
    return HCOV_EDEVICE;
  }
  auto bail = [&](int code) {
    hcov_destroy(c);
    return code;
  };
  double t0 = now_ms();
  // node ranges from the sizes alone (left son takes ceil(s/2))
  std::vector<std::vector<int64_t>> lo(c->D + 1);
  lo[0] = {0, n};
  for (int l = 1; l <= c->D; ++l) {
    int64_t cnt = int64_t(1) << (l - 1);
    lo[l].resize(2 * cnt + 1);
    for (int64_t i = 0; i < cnt; ++i) {
      int64_t a = lo[l - 1][i], b = lo[l - 1][i + 1];
      lo[l][2 * i] = a;
      lo[l][2 * i + 1] = a + (b - a + 1) / 2;
    }
    lo[l][2 * cnt] = n;
  }
  // temporaries of the tree build are stream ordered (no device-wide sync)
  double* d_orig = nullptr;
  if (hipMallocAsync(&d_orig, n * 16, c->stream) != hipSuccess) return bail(HCOV_ENOMEM);
  if (hipMemcpyAsync(d_orig, h.data(), n * 16, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipFreeAsync(d_orig, c->stream);
    return bail(HCOV_EDEVICE);
  }
  TreeOut T;
  std::string e = build_trees(d_orig, n, leaf, c->D, eta, o.adm_rule, lo, c->stream, T);
  if (!e.empty()) {
    (void)hipFreeAsync(d_orig, c->stream);
    c->err = e;
    return bail(HCOV_EDEVICE);
  }
  c->perm = T.perm;
  c->bbox = T.bbox;
  c->blocks_lac = T.blocks;
  c->ms_tree = now_ms() - t0;
  // cluster-order locations and permutation (library owned)
  c->d_perm = (int*)dev_alloc(c, n * 4);
  c->d_loc = (double*)dev_alloc(c, n * 16);
  if (!c->d_perm || !c->d_loc) {
    (void)hipFreeAsync(d_orig, c->stream);
    (void)hipFreeAsync(T.d_perm, c->stream);
    return bail(HCOV_ENOMEM);
  }
  hipMemcpyAsync(c->d_perm, T.d_perm, n * 4, hipMemcpyDeviceToDevice, c->stream);
  {
    std::vector<double> lc(2 * n);
    for (int64_t i = 0; i < n; ++i) {
      lc[2 * i] = h[2 * T.perm[i]];
      lc[2 * i + 1] = h[2 * T.perm[i] + 1];
    }
    hipMemcpyAsync(c->d_loc, lc.data(), n * 16, hipMemcpyHostToDevice, c->stream);
    (void)hipFreeAsync(d_orig, c->stream);
    (void)hipFreeAsync(T.d_perm, c->stream);
    hipStreamSynchronize(c->stream);
  }
  c->n_base_allocs = c->allocs.size();
  c->sizing = o.initial_rank_cap > 0 && o.fixed_rank == 0;
  if (c->sizing) {
    const int64_t nb = int64_t(c->blocks_lac.size() / 4);
    c->caps.assign(size_t(nb), int32_t(std::min(o.initial_rank_cap, o.max_rank)));
  }
  {
    const int rs = setup_plan(c);
    if (rs) return bail(rs);
  }
  int r = assemble_grown(c);
  if (r != HCOV_OK && r != HCOV_ERANK) {
    std::string keep = c->err;
    hcov_destroy(c);
    (void)keep;
    return r;
  }
  *out = c;
  return r;
}

int hcov_set_theta(hcov_ctx* c, hcov_theta theta) {
  if (!c) return HCOV_EINVAL;
  if (!theta_ok(theta)) return fail(c, HCOV_EINVAL, "theta out of domain");
  c->theta = theta;
  c->assembled = c->factored = false;
  return assemble_grown(c);
}

int hcov_cholesky(hcov_ctx* c) {
  if (!c) return HCOV_EINVAL;
  if (c->factored) return HCOV_OK;
  return factorise(c, nullptr, HCOV_HOST);
}

int hcov_logdet(hcov_ctx* c, double* out) {
  if (!c || !out) return HCOV_EINVAL;
  if (!c->factored) return fail(c, HCOV_ESTATE, "logdet requires hcov_cholesky");
  return logdet_sum(c, out);
}

static int fwd_sweep(hcov_ctx* c) {
  for (const auto& st : c->plan.fsolve_steps) {
    int r = run_stages(c, st);
    if (r) return r;
  }
  return HCOV_OK;
}

int hcov_forward(hcov_ctx* c, const double* z, double* v, double* quad, int where) {
  if (!c || !z) return HCOV_EINVAL;
  if (!c->factored) return fail(c, HCOV_ESTATE, "forward solve requires hcov_cholesky");
  double t0 = now_ms();
  int r = to_cluster(c, z, where, c->d_buf[B_RHS]);
  if (r) return r;
  r = fwd_sweep(c);
  if (r) return r;
  if (quad) {
    r = reduce_dev(c, c->d_buf[B_RHS], c->n, 0, quad);
    if (r) return r;
  }
  if (v) {
    if (where == HCOV_HOST) {
      HIPCHK(c, hipMemcpyAsync(v, c->d_buf[B_RHS], c->n * 8, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
      HIPCHK(c, hipMemcpyAsync(v, c->d_buf[B_RHS], c->n * 8, hipMemcpyDeviceToDevice, c->stream));
    }
  }
  c->ms_solve = now_ms() - t0;
  return HCOV_OK;
}

int hcov_solve(hcov_ctx* c, const double* z, double* x, int where) {
  if (!c || !z || !x) return HCOV_EINVAL;
  if (!c->factored) return fail(c, HCOV_ESTATE, "solve requires hcov_cholesky");
  int r = to_cluster(c, z, where, c->d_buf[B_RHS]);
  if (r) return r;
  r = fwd_sweep(c);
  if (r) return r;
  for (const auto& st : c->plan.bsolve_steps) {
    r = run_stages(c, st);
    if (r) return r;
  }
  return from_cluster(c, c->d_buf[B_RHS], x, where);
}

int hcov_sample(hcov_ctx* c, const double* xi, double* y, int where) {
  if (!c || !xi || !y) return HCOV_EINVAL;
  if (!c->factored) return fail(c, HCOV_ESTATE, "sample requires hcov_cholesky");
  if (where == HCOV_HOST)
    HIPCHK(c, hipMemcpyAsync(c->d_buf[B_RHS], xi, c->n * 8, hipMemcpyHostToDevice, c->stream));
  else
    HIPCHK(c, hipMemcpyAsync(c->d_buf[B_RHS], xi, c->n * 8, hipMemcpyDeviceToDevice, c->stream));
  int r = run_stages(c, c->plan.lmul_stages);
  if (r) return r;
  return from_cluster(c, c->d_buf[B_RHS] + c->plan.rhs_ld, y, where);
}

int hcov_matvec(hcov_ctx* c, const double* x, double* y, int where) {
  if (!c || !x || !y) return HCOV_EINVAL;
  if (!c->assembled && !c->kept_valid)
    return fail(c, HCOV_ESTATE, "matvec needs the assembled matrix (or opts.keep_matrix after a factorisation)");
  int r = to_cluster(c, x, where, c->d_buf[B_RHS]);
  if (r) return r;
  r = run_stages(c, c->plan.matvec_stages, c->assembled ? nullptr : &c->Lc);
  if (r) return r;
  return from_cluster(c, c->d_buf[B_RHS] + c->plan.rhs_ld, y, where);
}

// ---------------------------------------------------------------- products on
// device vectors in cluster order (n doubles each), through the B_RHS columns

static int d2d(hcov_ctx* c, double* dst, const double* src) {
  HIPCHK(c, hipMemcpyAsync(dst, src, c->n * 8, hipMemcpyDeviceToDevice, c->stream));
  return HCOV_OK;
}

// y = C~ x: the assembled matrix, or its kept copy after a factorisation
static int apply_C(hcov_ctx* c, const double* x, double* y) {
  if (!c->assembled && !c->kept_valid) return fail(c, HCOV_ESTATE, "C~ is neither assembled nor kept");
  int r = d2d(c, c->d_buf[B_RHS], x);
  if (!r) r = run_stages(c, c->plan.matvec_stages, c->assembled ? nullptr : &c->Lc);
  if (!r) r = d2d(c, y, c->d_buf[B_RHS] + c->plan.rhs_ld);
  return r;
}

// y = (L~ L~^T)^{-1} x by the forward and backward H-triangular solves
static int apply_Minv(hcov_ctx* c, const double* x, double* y) {
  int r = d2d(c, c->d_buf[B_RHS], x);
  if (!r) r = fwd_sweep(c);
  for (size_t i = 0; !r && i < c->plan.bsolve_steps.size(); ++i) r = run_stages(c, c->plan.bsolve_steps[i]);
  if (!r) r = d2d(c, y, c->d_buf[B_RHS]);
  return r;
}

// y = L~ L~^T x
static int apply_M(hcov_ctx* c, const double* x, double* y) {
  double* col0 = c->d_buf[B_RHS];
  double* col1 = col0 + c->plan.rhs_ld;
  int r = d2d(c, col0, x);
  if (!r) r = run_stages(c, c->plan.ltmul_stages);
  if (!r) r = d2d(c, col0, col1);
  if (!r) r = run_stages(c, c->plan.lmul_stages);
  if (!r) r = d2d(c, y, col1);
  return r;
}

static int dot(hcov_ctx* c, const double* x, const double* y, double* out) {
  return reduce_dev(c, x, c->n, 2, out, y);
}

static int axpby(hcov_ctx* c, double* y, const double* x, double a, double b) {
  HIPCHK(c, launch_axpby(y, x, a, b, c->n, c->stream));
  return HCOV_OK;
}

// q = b^T C~^{-1} b by conjugate gradients on the kept C~ with the H-Cholesky
// factor as preconditioner (the listing of Appendix B evaluates the quadratic
// form by CG with the factor, 150 iterations, tolerance 1e-6), started from
// the preconditioner's solution.  b: device, cluster order.
static int pcg_quad(hcov_ctx* c, const double* b, double* quad) {
  const int64_t n = c->n;
  double* x = c->d_vec;
  double* rr = x + n;
  double* z = rr + n;
  double* p = z + n;
  double* w = p + n;
  double bb = 0.0, rn2 = 0.0, rz = 0.0, rz_old = 1.0, pw = 0.0;
  int r = apply_Minv(c, b, x);
  if (!r) r = apply_C(c, x, w);
  if (!r) r = d2d(c, rr, b);
  if (!r) r = axpby(c, rr, w, -1.0, 1.0);
  if (!r) r = dot(c, b, b, &bb);
  if (r) return r;
  int it = 0;
  for (;; ++it) {
    r = dot(c, rr, rr, &rn2);
    if (r) return r;
    if (!(rn2 > c->opts.pcg_tol * c->opts.pcg_tol * bb) || it >= c->opts.pcg_max_iter) break;
    r = apply_Minv(c, rr, z);
    if (!r) r = dot(c, rr, z, &rz);
    if (!r) r = it == 0 ? d2d(c, p, z) : axpby(c, p, z, 1.0, rz / rz_old);
    if (!r) r = apply_C(c, p, w);
    if (!r) r = dot(c, p, w, &pw);
    if (r) return r;
    if (!(pw > 0.0) || !std::isfinite(pw)) return fail(c, HCOV_ENOTSPD, "CG: C~ is not positive definite");
    const double alpha = rz / pw;
    r = axpby(c, x, p, alpha, 1.0);
    if (!r) r = axpby(c, rr, w, -alpha, 1.0);
    if (r) return r;
    rz_old = rz;
  }
  c->pcg_iters = it;
  c->pcg_relres = bb > 0 ? std::sqrt(rn2 / bb) : 0.0;
  return dot(c, b, x, quad);
}

int hcov_loglik(hcov_ctx* c, const double* z, int where, double* out_ll, double* out_logdet, double* out_quad) {
  if (!c || !z || !out_ll) return HCOV_EINVAL;
  int r;
  double quad = 0, ld = 0;
  if (c->opts.quad_mode == HCOV_QUAD_PCG) {
    if (!c->factored) {
      r = factorise(c, nullptr, where);
      if (r) return r;
    }
    double* b = c->d_vec + 5 * c->n;
    r = to_cluster(c, z, where, b);
    if (!r) r = pcg_quad(c, b, &quad);
    if (r) return r;
  } else if (!c->factored) {
    if (c->opts.fuse_solve) {
      r = factorise(c, z, where);
      if (r) return r;
      r = reduce_dev(c, c->d_buf[B_RHS], c->n, 0, &quad);
      if (r) return r;
    } else {
      r = factorise(c, nullptr, where);
      if (r) return r;
      r = hcov_forward(c, z, nullptr, &quad, where);
      if (r) return r;
    }
  } else {
    r = hcov_forward(c, z, nullptr, &quad, where);
    if (r) return r;
  }
  r = logdet_sum(c, &ld);
  if (r) return r;
  double n = double(c->n);
  *out_ll = -0.5 * n * std::log(2.0 * M_PI) - 0.5 * ld - 0.5 * quad;
  if (out_logdet) *out_logdet = ld;
  if (out_quad) *out_quad = quad;
  return HCOV_OK;
}

int hcov_factor_matvec(hcov_ctx* c, const double* x, double* y, int where) {
  if (!c || !x || !y) return HCOV_EINVAL;
  if (!c->factored) return fail(c, HCOV_ESTATE, "L~ L~^T x requires hcov_cholesky");
  if (!c->keep) return fail(c, HCOV_ESTATE, "L~ L~^T x needs opts.keep_matrix (vector workspace)");
  double* b = c->d_vec + 5 * c->n;
  int r = to_cluster(c, x, where, b);
  if (!r) r = apply_M(c, b, c->d_vec);
  if (!r) r = from_cluster(c, c->d_vec, y, where);
  return r;
}

int hcov_error_norms(hcov_ctx* c, int iters, uint64_t seed, double* norm_c, double* err_fact, double* err_inv) {
  if (!c || iters < 1) return HCOV_EINVAL;
  if (!c->factored || !c->kept_valid)
    return fail(c, HCOV_ESTATE, "error norms need a factorised context with opts.keep_matrix");
  const int64_t n = c->n;
  double* v = c->d_vec;
  double* w = v + n;
  double* u = w + n;
  double* t = u + n;
  int r = HCOV_OK;
  // one power iteration: v <- op(v) / ||op(v)||, returns ||op(v)|| for unit v
  auto power = [&](int which, uint64_t sd, double* est) -> int {
    HIPCHK(c, launch_gaussian(v, n, sd, c->stream));
    double nv = 0.0;
    int rc = dot(c, v, v, &nv);
    if (rc) return rc;
    rc = axpby(c, v, v, 0.0, 1.0 / std::sqrt(nv));
    double lam = 0.0;
    for (int k = 0; !rc && k < iters; ++k) {
      if (which == 0) {                      // C~ v
        rc = apply_C(c, v, w);
      } else if (which == 1) {               // (C~ - L~L~^T) v
        rc = apply_C(c, v, w);
        if (!rc) rc = apply_M(c, v, u);
        if (!rc) rc = axpby(c, w, u, -1.0, 1.0);
      } else {                               // A^T A v, A = I - (L~L~^T)^{-1} C~
        rc = apply_C(c, v, t);
        if (!rc) rc = apply_Minv(c, t, u);
        if (!rc) rc = axpby(c, u, v, 1.0, -1.0);   // u = A v
        if (!rc) rc = dot(c, u, u, &lam);          // ||A v||^2
        if (!rc) rc = apply_Minv(c, u, t);
        if (!rc) rc = apply_C(c, t, w);
        if (!rc) rc = axpby(c, w, u, 1.0, -1.0);   // w = A^T u
      }
      double nw = 0.0;
      if (!rc) rc = dot(c, w, w, &nw);
      if (rc) break;
      if (which != 2) lam = nw;
      if (!(nw > 0.0)) break;
      rc = axpby(c, v, w, 1.0 / std::sqrt(nw), 0.0);
    }
    *est = std::sqrt(lam);
    return rc;
  };
  double e0 = 0, e1 = 0, e2 = 0;
  r = power(0, seed, &e0);
  if (!r) r = power(1, seed + 1, &e1);
  if (!r) r = power(2, seed + 2, &e2);
  if (r) return r;
  if (norm_c) *norm_c = e0;
  if (err_fact) *err_fact = e1;
  if (err_inv) *err_inv = e2;
  return HCOV_OK;
}

int hcov_exact_matvec(hcov_ctx* c, const double* x, double* y, int where) {
  if (!c || !x || !y) return HCOV_EINVAL;
  int r = to_cluster(c, x, where, c->d_buf[B_RHS]);
  if (r) return r;
  HIPCHK(c, launch_exact_matvec(c->d_loc, c->d_buf[B_RHS], c->d_buf[B_RHS] + c->plan.rhs_ld, c->n, c->mp,
                                c->stream));
  return from_cluster(c, c->d_buf[B_RHS] + c->plan.rhs_ld, y, where);
}

int hcov_exact_norms(hcov_ctx* c, int iters, uint64_t seed, double* err_c, double* err_cinv) {
  if (!c || iters < 1) return HCOV_EINVAL;
  if (!c->factored || !c->kept_valid)
    return fail(c, HCOV_ESTATE, "exact error norms need a factorised context with opts.keep_matrix");
  const int64_t n = c->n;
  double* v = c->d_vec;
  double* w = v + n;
  double* u = w + n;
  double* t = u + n;
  auto exact = [&](const double* a, double* b) -> int {
    HIPCHK(c, launch_exact_matvec(c->d_loc, a, b, n, c->mp, c->stream));
    return HCOV_OK;
  };
  auto power = [&](int which, uint64_t sd, double* est) -> int {
    HIPCHK(c, launch_gaussian(v, n, sd, c->stream));
    double nv = 0.0, lam = 0.0;
    int rc = dot(c, v, v, &nv);
    if (!rc) rc = axpby(c, v, v, 0.0, 1.0 / std::sqrt(nv));
    for (int k = 0; !rc && k < iters; ++k) {
      if (which == 0) {                      // (C - C~) v
        rc = exact(v, w);
        if (!rc) rc = apply_C(c, v, u);
        if (!rc) rc = axpby(c, w, u, -1.0, 1.0);
      } else {                               // B^T B v, B = C (L~L~^T)^{-1} - I
        rc = apply_Minv(c, v, t);
        if (!rc) rc = exact(t, u);
        if (!rc) rc = axpby(c, u, v, -1.0, 1.0);   // u = B v
        if (!rc) rc = dot(c, u, u, &lam);
        if (!rc) rc = exact(u, t);
        if (!rc) rc = apply_Minv(c, t, w);
        if (!rc) rc = axpby(c, w, u, -1.0, 1.0);   // w = B^T u
      }
      double nw = 0.0;
      if (!rc) rc = dot(c, w, w, &nw);
      if (rc) break;
      if (which == 0) lam = nw;
      if (!(nw > 0.0)) break;
      rc = axpby(c, v, w, 1.0 / std::sqrt(nw), 0.0);
    }
    *est = std::sqrt(lam);
    return rc;
  };
  double e0 = 0, e1 = 0;
  int r = power(0, seed, &e0);
  if (!r) r = power(1, seed + 1, &e1);
  if (r) return r;
  if (err_c) *err_c = e0;
  if (err_cinv) *err_cinv = e1;
  return HCOV_OK;
}

int hcov_stats(const hcov_ctx* c, hcov_stats_t* s) {
  if (!c || !s) return HCOV_EINVAL;
  std::memset(s, 0, sizeof(*s));
  const Plan& P = c->plan;
  s->n = c->n;
  s->leaf = c->leaf;
  s->depth = c->D;
  s->n_dense_blocks = P.n_dense;
  s->n_lr_blocks = P.n_lr;
  s->dense_entries = P.dense_elems;
  s->lr_rows = P.lr_rows;
  s->bytes_device = c->bytes;
  s->ms_tree = c->ms_tree;
  s->ms_assemble = c->ms_asm;
  s->ms_factor = c->ms_fact;
  s->ms_solve = c->ms_solve;
  s->n_steps = int64_t(1) << c->D;
  s->n_launches_factor = P.n_launch_fact;
  s->n_graph_replays = c->n_replays;
  s->n_sketch_retries = c->n_retries;
  s->sketch_saturated = c->sat_last;
  s->pcg_iters = c->pcg_iters;
  s->pcg_relres = c->pcg_relres;
  s->n_autotune_switched = c->n_switched;
  s->n_gemm_grouped = 0;
  for (const auto& st : P.steps)
    for (const auto& x : st) s->n_gemm_grouped += x.kind == ST_GEMM_WIDE ? 1 : 0;
  // ranks
  std::vector<int> dyn(P.n_dyn + 1);
  if (hipMemcpyAsync(dyn.data(), c->d_dyn, dyn.size() * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return HCOV_EDEVICE;
  int64_t sum = 0, rows = 0, mx = 0;
  double fb = double(P.dense_elems);
  for (auto& B : P.blocks) {
    if (B.kind != 1) continue;
    int k = dyn[B.rank_slot];
    mx = std::max<int64_t>(mx, k);
    sum += k;
    rows += (B.r1 - B.r0) + (B.c1 - B.c0);
    fb += double(k) * double((B.r1 - B.r0) + (B.c1 - B.c0));
  }
  s->max_rank_seen = int(mx);
  {
    // planned GEMM work of one factorisation at these ranks
    double fl = 0.0, by = 0.0;
    for (const auto& st : P.steps)
      for (const auto& x : st)
        if (x.kind == ST_GEMM || x.kind == ST_GEMM_WIDE) {
          double f1 = 0.0, b1 = 0.0;
          stage_work(P, dyn, x, &f1, &b1);
          fl += f1;
          by += b1;
        }
    s->gemm_flops_factor = fl;
    s->gemm_bytes_factor = by;
  }
  s->n_replans = c->n_replans;
  s->bytes_lowrank = (P.u_elems + P.v_elems) * 8;
  {
    // sketch width of every low-rank block in the last factorisation
    double w = 0.0;
    for (auto& B : P.blocks)
      if (B.kind == 1)
        w += double(std::min<int64_t>({int64_t(dyn[B.rank0_slot]), B.r1 - B.r0, B.c1 - B.c0, int64_t(P.rcap)}));
    s->mean_sketch_width = P.n_lr ? w / double(P.n_lr) : 0.0;
  }
  s->mean_rank = P.n_lr ? double(sum) / double(P.n_lr) : 0.0;
  s->bytes_factor = int64_t(fb * 8.0);
  (void)rows;
  return HCOV_OK;
}

int hcov_estimate_bytes(const double* locs, int64_t n, double eps, int leaf, double eta, const hcov_opts* opts,
                        size_t* out) {
  (void)eps;
  if (!locs || !out || n < 1 || leaf < 2 || leaf > 128 || !(eta > 0)) return HCOV_EINVAL;
  hcov_opts o;
  hcov_opts_default(&o);
  if (opts) o = *opts;
  // upper bound from sizes alone: dense leaves near the diagonal scale with n,
  // low-rank storage with n log n.  The exact figure needs the trees and the
  // plan (built on the device and the host at hcov_build); the serving
  // admission runs at submission, before either exists, so it takes this
  // conservative bound (documented in the header).
  int D = tree_depth(n, leaf);
  double L = double(leaf);
  double dense = 16.0 * double(n) * L;                   // ~C_sp leaves per row
  double lr = 12.0 * double(n) * double(D + 1) * 2.0 * o.max_rank;
  double scratch = 8.0 * double(n) * 96.0;
  *out = size_t((dense + lr + scratch + double(n) * (74 + 4)) * 8.0);
  return HCOV_OK;
}

int hcov_perm(const hcov_ctx* c, int64_t* perm) {
  if (!c || !perm) return HCOV_EINVAL;
  std::memcpy(perm, c->perm.data(), c->n * 8);
  return HCOV_OK;
}

int hcov_tree_sizes(const hcov_ctx* c, int* depth, int64_t* nb) {
  if (!c || !depth || !nb) return HCOV_EINVAL;
  *depth = c->D;
  *nb = int64_t(c->blocks_lac.size() / 4);
  return HCOV_OK;
}

int hcov_tree_dump(const hcov_ctx* c, double* bbox, int64_t* blocks) {
  if (!c) return HCOV_EINVAL;
  if (bbox) std::memcpy(bbox, c->bbox.data(), c->bbox.size() * 8);
  if (blocks) std::memcpy(blocks, c->blocks_lac.data(), c->blocks_lac.size() * 8);
  return HCOV_OK;
}

void hcov_destroy(hcov_ctx* c) {
  if (!c) return;
  if (c->stream2) (void)hipStreamSynchronize(c->stream2);
  if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  for (auto g : c->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->stream2) (void)hipStreamDestroy(c->stream2);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  for (void* p : c->allocs) {
    if (c->opts.free)
      c->opts.free(p, c->opts.alloc_user);
    else
      hipFree(p);
  }
  delete c;
}

int hcov_profile_begin(hcov_ctx* c, int stage_kind) {
  if (!c || stage_kind < 0 || stage_kind > ST_TRMM || stage_kind == ST_COPY_RANK || stage_kind == ST_FORK ||
      stage_kind == ST_JOIN)
    return HCOV_EINVAL;
  return profile_begin(c, stage_kind);
}

int hcov_profile_end(hcov_ctx* c, int64_t* launches, double* total_ms, double* flops, double* bytes) {
  if (!c) return HCOV_EINVAL;
  const int64_t nl = int64_t(c->prof_ev.size());
  const int rc = profile_collect(c, total_ms, flops, bytes);
  if (launches) *launches = nl;
  c->prof_kind = -1;
  return rc;
}

int hcov_profile_times(const hcov_ctx* c, double* times_ms, int64_t max_n, int64_t* n_out) {
  if (!c) return HCOV_EINVAL;
  const int64_t n = int64_t(c->prof_times.size());
  if (n_out) *n_out = n;
  if (times_ms)
    for (int64_t i = 0; i < std::min(n, max_n); ++i) times_ms[i] = c->prof_times[size_t(i)];
  return HCOV_OK;
}

// Matérn of Eq. (3) on the device for given distances (test access to the
// device K_nu): h, out are host arrays of n doubles.
int hcov_matern_eval(hcov_theta theta, const double* h, double* out, int64_t n) {
  if (!h || !out || n < 0 || !theta_ok(theta)) return HCOV_EINVAL;
  if (n == 0) return HCOV_OK;
  MaternParams P = make_params(theta);
  double *dh = nullptr, *dout = nullptr;
  if (hipMalloc(&dh, n * 8) != hipSuccess) return HCOV_ENOMEM;
  if (hipMalloc(&dout, n * 8) != hipSuccess) {
    hipFree(dh);
    return HCOV_ENOMEM;
  }
  int rc = HCOV_OK;
  if (hipMemcpy(dh, h, n * 8, hipMemcpyHostToDevice) != hipSuccess || launch_probe(dh, dout, n, P, nullptr) != hipSuccess ||
      hipMemcpy(out, dout, n * 8, hipMemcpyDeviceToHost) != hipSuccess)
    rc = HCOV_EDEVICE;
  hipFree(dh);
  hipFree(dout);
  return rc;
}

}  // extern "C"
// ------------------------------------------------------------ no-allocation variant
// hcov_matern_eval without any allocation: the device staging of distances
// and results lives in a fixed array of this library (each GPU holds its own
// copy), whose device address is looked up once per device.
namespace {
constexpr int64_t NOALLOC_MAX = HCOV_NOALLOC_MAX_N;
__device__ __align__(256) double scratch[2 * NOALLOC_MAX];   // [0, MAX): h, [MAX, 2 MAX): out
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu[MAX_DEVICES];
double* scratch_ptr[MAX_DEVICES] = {};
}  // namespace

extern "C" int hcov_matern_eval_noalloc(hcov_theta theta, const double* h, double* out, int64_t n) {
  if (!h || !out || n < 0 || !theta_ok(theta) || n > NOALLOC_MAX) return HCOV_EINVAL;
  if (n == 0) return HCOV_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return HCOV_EDEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu[dev]);
  if (!scratch_ptr[dev]) {
    // the host-side name `scratch` is not a device address: resolve it once
    // per device, with that device current
    double* p = nullptr;
    if (hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HCOV_EDEVICE;
    scratch_ptr[dev] = p;
  }
  double* dh = scratch_ptr[dev];
  double* dout = dh + NOALLOC_MAX;
  const MaternParams P = make_params(theta);
  if (hipMemcpyAsync(dh, h, size_t(n) * 8, hipMemcpyHostToDevice, nullptr) != hipSuccess ||
      launch_probe(dh, dout, n, P, nullptr) != hipSuccess ||
      hipMemcpyAsync(out, dout, size_t(n) * 8, hipMemcpyDeviceToHost, nullptr) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess)
    return HCOV_EDEVICE;
  return HCOV_OK;
}
