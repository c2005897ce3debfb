// Cluster tree and block cluster tree on the GPU (Sec. 2.2, Appendix A).
//
// Cluster tree: recursive bisection into two equal-sized subsets by an
// axis-parallel cut across the longer side of the cluster's bounding box.
// Level-synchronous: at each level every node's points are ordered by
// (coordinate on the node's split axis, original index) with one device-wide
// radix sort (the library's own, below) of the 64-bit key (node << 32 | rank
// on that axis), where the rank of a point on an axis is its position in the
// global order (coordinate, index); the first ceil(s/2) points of a node form
// its left son.  Leaves are finally ordered by original index.  Bounding boxes are
// exact min/max reductions, so the result is bit-identical to the CPU
// reference.
//
// Block cluster tree: breadth-first expansion from (root, root) keeping the
// lower triangle; a pair is a low-rank leaf when the standard admissibility
// condition min(diam^2) <= eta^2 dist^2 holds with dist^2 > 0 (evaluated with
// single IEEE operations, no contraction), a dense leaf at the leaf level,
// otherwise it is replaced by its son pairs.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tree.h"

#pragma clang fp contract(off)

namespace hc {

#define TCHK(x)                                                              \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) return std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x; \
  } while (0)

__device__ __forceinline__ unsigned long long ord_key(double v) {
  unsigned long long u = __double_as_longlong(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_val(unsigned long long k) {
  unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(u);
}

__global__ void k_axis_keys(const double2* __restrict__ loc, int64_t n, int axis,
                            unsigned long long* __restrict__ key, int* __restrict__ val) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = axis == 0 ? loc[i].x : loc[i].y;
  key[i] = ord_key(v);
  val[i] = (int)i;
}

__global__ void k_scatter_rank(const int* __restrict__ order, int64_t n, int* __restrict__ rank) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  rank[order[i]] = (int)i;
}

// node containing position p at a level (lo has cnt+1 entries)
__device__ __forceinline__ int node_of(const int64_t* __restrict__ lo, int cnt, int64_t p) {
  int a = 0, b = cnt - 1;
  while (a < b) {
    int m = (a + b + 1) >> 1;
    if (lo[m] <= p)
      a = m;
    else
      b = m - 1;
  }
  return a;
}

__global__ void k_bbox_init(unsigned long long* __restrict__ bb, int cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  bb[4 * i + 0] = ~0ull;   // xmin
  bb[4 * i + 1] = 0ull;    // xmax
  bb[4 * i + 2] = ~0ull;   // ymin
  bb[4 * i + 3] = 0ull;    // ymax
}

__global__ void k_bbox(const double2* __restrict__ loc, const int* __restrict__ perm, int64_t n,
                       const int64_t* __restrict__ lo, int cnt, unsigned long long* __restrict__ bb) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool act = p < n;
  int node = act ? node_of(lo, cnt, p) : -1;
  unsigned long long kx = 0, ky = 0;
  if (act) {
    double2 v = loc[perm[p]];
    kx = ord_key(v.x);
    ky = ord_key(v.y);
  }
  unsigned long long xmn = act ? kx : ~0ull, xmx = act ? kx : 0ull;
  unsigned long long ymn = act ? ky : ~0ull, ymx = act ? ky : 0ull;
  // whole wave in one node: reduce in the wave first
  int n0 = __shfl(node, 0);
  bool same = __all(node == n0 || node < 0);
  if (same) {
    for (int o = 32; o > 0; o >>= 1) {
      unsigned long long a = __shfl_down(xmn, o), b = __shfl_down(xmx, o);
      unsigned long long c = __shfl_down(ymn, o), d = __shfl_down(ymx, o);
      xmn = a < xmn ? a : xmn;
      xmx = b > xmx ? b : xmx;
      ymn = c < ymn ? c : ymn;
      ymx = d > ymx ? d : ymx;
    }
    if ((threadIdx.x & 63) == 0 && n0 >= 0) {
      atomicMin(&bb[4 * n0 + 0], xmn);
      atomicMax(&bb[4 * n0 + 1], xmx);
      atomicMin(&bb[4 * n0 + 2], ymn);
      atomicMax(&bb[4 * n0 + 3], ymx);
    }
  } else if (act) {
    atomicMin(&bb[4 * node + 0], xmn);
    atomicMax(&bb[4 * node + 1], xmx);
    atomicMin(&bb[4 * node + 2], ymn);
    atomicMax(&bb[4 * node + 3], ymx);
  }
}

__global__ void k_bbox_decode(const unsigned long long* __restrict__ bb, int cnt, double* __restrict__ out,
                              signed char* __restrict__ axis) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  double x0 = ord_val(bb[4 * i]), x1 = ord_val(bb[4 * i + 1]);
  double y0 = ord_val(bb[4 * i + 2]), y1 = ord_val(bb[4 * i + 3]);
  out[4 * i] = x0;
  out[4 * i + 1] = x1;
  out[4 * i + 2] = y0;
  out[4 * i + 3] = y1;
  double ex = x1 - x0, ey = y1 - y0;
  axis[i] = (ex >= ey) ? 0 : 1;
}

__global__ void k_level_keys(const int* __restrict__ perm, int64_t n, const int64_t* __restrict__ lo,
                             int cnt, const signed char* __restrict__ axis, const int* __restrict__ rx,
                             const int* __restrict__ ry, unsigned long long* __restrict__ key, int final_sort) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  int node = node_of(lo, cnt, p);
  int pt = perm[p];
  unsigned int r;
  if (final_sort)
    r = (unsigned int)pt;
  else
    r = (unsigned int)(axis[node] == 0 ? rx[pt] : ry[pt]);
  key[p] = ((unsigned long long)node << 32) | r;
}

// ---------------------------------------------------------------- block tree
// Admissibility of two clusters of one level by their bounding boxes
// (Appendix A): rule 0 the standard Adm_eta, min(diam) <= eta dist
// (Eq. (stand_cond)); rule 1 its max form, max(diam) <= eta dist; rule 2 the
// weak admissibility Adm_W (Eq. (wead_adm)): any two different clusters.
// Squared forms, single IEEE operations (no contraction), so that the host
// reference gets the same bits.
__device__ __forceinline__ bool admissible(const double* bt, const double* bs, double eta2, int rule) {
  if (rule == 2) return true;
  double dx = fmax(fmax(0.0, bs[0] - bt[1]), bt[0] - bs[1]);
  double dy = fmax(fmax(0.0, bs[2] - bt[3]), bt[2] - bs[3]);
  double dist2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
  if (!(dist2 > 0.0)) return false;
  double ext = bt[1] - bt[0], eyt = bt[3] - bt[2];
  double dt = __dadd_rn(__dmul_rn(ext, ext), __dmul_rn(eyt, eyt));
  double exs = bs[1] - bs[0], eys = bs[3] - bs[2];
  double ds = __dadd_rn(__dmul_rn(exs, exs), __dmul_rn(eys, eys));
  return (rule == 1 ? fmax(dt, ds) : fmin(dt, ds)) <= __dmul_rn(eta2, dist2);
}

// classify: out_kind: 0 dense leaf, 1 LR leaf, 2 subdivided; nch: children count
__global__ void k_classify(const int2* __restrict__ fr, int cnt, const double* __restrict__ bbl,
                           double eta2, int rule, int is_leaf_level, int* __restrict__ isleaf, int* __restrict__ nch,
                           int* __restrict__ kind) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  int t = fr[i].x, s = fr[i].y;
  int k;
  if (t != s && admissible(bbl + 4 * t, bbl + 4 * s, eta2, rule))
    k = 1;
  else if (is_leaf_level)
    k = 0;
  else
    k = 2;
  kind[i] = k;
  isleaf[i] = k != 2;
  nch[i] = k != 2 ? 0 : (t == s ? 3 : 4);
}

__global__ void k_expand(const int2* __restrict__ fr, int cnt, const int* __restrict__ kind,
                         const int* __restrict__ lpos, const int* __restrict__ cpos, int level,
                         int4* __restrict__ leaves, int leaf_base, int2* __restrict__ next) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  int t = fr[i].x, s = fr[i].y, k = kind[i];
  if (k != 2) {
    leaves[leaf_base + lpos[i]] = make_int4(level, t, s, k);
    return;
  }
  int o = cpos[i];
  if (t == s) {
    next[o] = make_int2(2 * t, 2 * t);
    next[o + 1] = make_int2(2 * t + 1, 2 * t);
    next[o + 2] = make_int2(2 * t + 1, 2 * t + 1);
  } else {
    next[o] = make_int2(2 * t, 2 * s);
    next[o + 1] = make_int2(2 * t, 2 * s + 1);
    next[o + 2] = make_int2(2 * t + 1, 2 * s);
    next[o + 3] = make_int2(2 * t + 1, 2 * s + 1);
  }
}

static int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of unsigned 32-bit counts: each work-group scans 1024
// entries (4 a thread, the thread totals scanned by shuffles inside a wave
// and through LDS across the four waves) and writes its total; the totals
// are scanned the same way (recursively) and added back.
constexpr int SC_THREADS = 256, SC_ITEMS = 4, SC_TILE = SC_THREADS * SC_ITEMS;

__global__ __launch_bounds__(SC_THREADS) void k_scan_tile(const unsigned* __restrict__ in, unsigned* __restrict__ out,
                                                          int64_t n, unsigned* __restrict__ totals) {
  __shared__ unsigned wsum[SC_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = int64_t(blockIdx.x) * SC_TILE + int64_t(tid) * SC_ITEMS;
  unsigned v[SC_ITEMS], t = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    t += v[i];
  }
  // inclusive scan of the thread totals inside the wave
  unsigned x = t;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  unsigned before = x - t;
  for (int w = 0; w < wave; ++w) before += wsum[w];
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    if (base + i < n) out[base + i] = before;
    before += v[i];
  }
  if (totals && tid == SC_THREADS - 1) totals[blockIdx.x] = before;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_add(unsigned* __restrict__ out, int64_t n,
                                                         const unsigned* __restrict__ offs) {
  const int64_t i = int64_t(blockIdx.x) * SC_TILE + threadIdx.x;
  const unsigned a = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SC_ITEMS; ++k)
    if (i + k * SC_THREADS < n) out[i + k * SC_THREADS] += a;
}

// Scratch (unsigned entries) that exclusive_sum needs for n entries.
static int64_t scan_scratch(int64_t n) {
  const int64_t nb = nblk(n, SC_TILE);
  return nb > 1 ? 2 * nb + scan_scratch(nb) : 1;
}

// out[i] = in[0] + ... + in[i-1] for i < n (in and out may not alias);
// scratch holds scan_scratch(n) entries.
static std::string exclusive_sum(const unsigned* in, unsigned* out, int64_t n, unsigned* scratch, hipStream_t st) {
  if (n <= 0) return "";
  const int nb = nblk(n, SC_TILE);
  if (nb == 1) {
    k_scan_tile<<<1, SC_THREADS, 0, st>>>(in, out, n, nullptr);
    TCHK(hipGetLastError());
    return "";
  }
  unsigned* totals = scratch;
  k_scan_tile<<<nb, SC_THREADS, 0, st>>>(in, out, n, totals);
  TCHK(hipGetLastError());
  // the totals are scanned in place through the rest of the scratch
  unsigned* sums = scratch + nb;
  std::string e = exclusive_sum(totals, sums, nb, sums + nb, st);
  if (!e.empty()) return e;
  k_scan_add<<<nb, SC_THREADS, 0, st>>>(out, n, sums);
  TCHK(hipGetLastError());
  return "";
}

// ------------------------------------------------------------------ sort
// Stable least-significant-digit radix sort of (64-bit key, 32-bit value)
// pairs on the bits [0, endbit) of the key, 8 bits a pass.  A pass counts
// the digits of each tile of 2048 keys (digit-major table: digit d of tile
// b at d * tiles + b), scans the table, and scatters: inside a tile the
// keys go in index order, a key's position among the earlier keys of its
// digit coming from the wave (ballots of the digit's bits: the lanes with
// the same digit, and the rank among them), the earlier waves of the same
// round (per-wave digit counts in LDS) and the earlier rounds (a running
// count per digit).
constexpr int RS_THREADS = 256, RS_ITEMS = 8, RS_TILE = RS_THREADS * RS_ITEMS, RS_BINS = 256;

__global__ __launch_bounds__(RS_THREADS) void k_rs_count(const unsigned long long* __restrict__ keys, int64_t n,
                                                         int shift, int tiles, unsigned* __restrict__ table) {
  __shared__ unsigned cnt[RS_BINS];
  const int tid = threadIdx.x;
  cnt[tid] = 0u;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * RS_TILE;
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t idx = base + i * RS_THREADS + tid;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 0xff], 1u);
  }
  __syncthreads();
  table[int64_t(tid) * tiles + blockIdx.x] = cnt[tid];
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const unsigned long long* __restrict__ kin,
                                                           const int* __restrict__ vin, int64_t n, int shift,
                                                           int tiles, const unsigned* __restrict__ offs,
                                                           unsigned long long* __restrict__ kout,
                                                           int* __restrict__ vout) {
  __shared__ unsigned run[RS_BINS];
  __shared__ unsigned wcnt[RS_THREADS / 64][RS_BINS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  run[tid] = offs[int64_t(tid) * tiles + blockIdx.x];
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t base = int64_t(blockIdx.x) * RS_TILE;
  for (int it = 0; it < RS_ITEMS; ++it) {
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    const int64_t idx = base + it * RS_THREADS + tid;
    const bool valid = idx < n;
    const unsigned long long key = valid ? kin[idx] : 0ull;
    const int d = int((key >> shift) & 0xff);
    // lanes of this wave holding a valid key with the same digit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    const unsigned rank = unsigned(__popcll(peers & below));
    if (valid && rank == 0u) wcnt[wave][d] = unsigned(__popcll(peers));
    __syncthreads();
    if (valid) {
      unsigned pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
    unsigned add = 0u;
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) add += wcnt[w][tid];
    run[tid] += add;
  }
}

// Scratch (unsigned entries) that radix_sort needs for n pairs.
static int64_t sort_scratch(int64_t n) {
  const int64_t t = int64_t(RS_BINS) * nblk(n, RS_TILE);
  return 2 * t + scan_scratch(t);
}

// Sorts (kin, vin) by the key bits [0, endbit) into (kout, vout); kin and
// vin are overwritten (ping-pong buffers).
static std::string radix_sort(unsigned long long* kin, int* vin, unsigned long long* kout, int* vout, int64_t n,
                              int endbit, unsigned* scratch, hipStream_t st) {
  if (n <= 0) return "";
  const int tiles = nblk(n, RS_TILE);
  const int64_t t = int64_t(RS_BINS) * tiles;
  unsigned* table = scratch;
  unsigned* offs = scratch + t;
  unsigned* sscr = scratch + 2 * t;
  const int passes = (endbit + 7) / 8;
  unsigned long long *ka = kin, *kb = kout;
  int *va = vin, *vb = vout;
  for (int p = 0; p < passes; ++p) {
    k_rs_count<<<tiles, RS_THREADS, 0, st>>>(ka, n, 8 * p, tiles, table);
    TCHK(hipGetLastError());
    std::string e = exclusive_sum(table, offs, t, sscr, st);
    if (!e.empty()) return e;
    k_rs_scatter<<<tiles, RS_THREADS, 0, st>>>(ka, va, n, 8 * p, tiles, offs, kb, vb);
    TCHK(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  // after an odd number of passes the result is in (kout, vout) already
  if (ka != kout) {
    TCHK(hipMemcpyAsync(kout, ka, n * 8, hipMemcpyDeviceToDevice, st));
    TCHK(hipMemcpyAsync(vout, va, n * 4, hipMemcpyDeviceToDevice, st));
  }
  return "";
}

std::string build_trees(const double* d_loc, int64_t n, int leaf_max, int D, double eta, int rule,
                        const std::vector<std::vector<int64_t>>& lo, hipStream_t st, TreeOut& out) {
  (void)leaf_max;
  const double2* loc = (const double2*)d_loc;
  // global ranks along x and y
  unsigned long long *kin = nullptr, *kout = nullptr;
  int *vin = nullptr, *vout = nullptr, *rx = nullptr, *ry = nullptr, *perm = nullptr;
  TCHK(hipMallocAsync(&kin, n * 8, st));
  TCHK(hipMallocAsync(&kout, n * 8, st));
  TCHK(hipMallocAsync(&vin, n * 4, st));
  TCHK(hipMallocAsync(&vout, n * 4, st));
  TCHK(hipMallocAsync(&rx, n * 4, st));
  TCHK(hipMallocAsync(&ry, n * 4, st));
  TCHK(hipMallocAsync(&perm, n * 4, st));
  unsigned* tmp = nullptr;
  TCHK(hipMallocAsync(&tmp, sort_scratch(n) * 4, st));
  for (int ax = 0; ax < 2; ++ax) {
    k_axis_keys<<<nblk(n, 256), 256, 0, st>>>(loc, n, ax, kin, vin);
    TCHK(hipGetLastError());
    {
      std::string e = radix_sort(kin, vin, kout, vout, n, 64, tmp, st);
      if (!e.empty()) return e;
    }
    k_scatter_rank<<<nblk(n, 256), 256, 0, st>>>(vout, n, ax == 0 ? rx : ry);
    TCHK(hipGetLastError());
  }
  // identity permutation
  {
    std::vector<int> id(n);
    for (int64_t i = 0; i < n; ++i) id[i] = (int)i;
    TCHK(hipMemcpyAsync(perm, id.data(), n * 4, hipMemcpyHostToDevice, st));
    TCHK(hipStreamSynchronize(st));
  }
  int64_t total_nodes = (int64_t(2) << D) - 1;
  double* bbox_all = nullptr;
  TCHK(hipMallocAsync(&bbox_all, total_nodes * 4 * 8, st));
  unsigned long long* bbk = nullptr;
  signed char* axis = nullptr;
  int64_t* dlo = nullptr;
  TCHK(hipMallocAsync(&bbk, ((int64_t)1 << D) * 4 * 8, st));
  TCHK(hipMallocAsync(&axis, ((int64_t)1 << D), st));
  TCHK(hipMallocAsync(&dlo, (((int64_t)1 << D) + 1) * 8, st));
  for (int l = 0; l <= D; ++l) {
    int cnt = 1 << l;
    TCHK(hipMemcpyAsync(dlo, lo[l].data(), (cnt + 1) * 8, hipMemcpyHostToDevice, st));
    k_bbox_init<<<nblk(cnt, 256), 256, 0, st>>>(bbk, cnt);
    k_bbox<<<nblk(n, 256), 256, 0, st>>>(loc, perm, n, dlo, cnt, bbk);
    k_bbox_decode<<<nblk(cnt, 256), 256, 0, st>>>(bbk, cnt, bbox_all + ((int64_t)cnt - 1) * 4, axis);
    TCHK(hipGetLastError());
    // sort points inside each node: by axis rank (levels < D), by index at D
    k_level_keys<<<nblk(n, 256), 256, 0, st>>>(perm, n, dlo, cnt, axis, rx, ry, kin, l == D ? 1 : 0);
    TCHK(hipGetLastError());
    TCHK(hipMemcpyAsync(vin, perm, n * 4, hipMemcpyDeviceToDevice, st));
    int endbit = 32 + (l == 0 ? 1 : l + 1);
    {
      std::string e = radix_sort(kin, vin, kout, perm, n, endbit, tmp, st);
      if (!e.empty()) return e;
    }
    TCHK(hipStreamSynchronize(st));
    // lo for the next level is only used by the next iteration
  }
  // download perm and bboxes
  out.perm.resize(n);
  {
    std::vector<int> ph(n);
    TCHK(hipMemcpyAsync(ph.data(), perm, n * 4, hipMemcpyDeviceToHost, st));
    TCHK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) out.perm[i] = ph[i];
  }
  out.bbox.resize(total_nodes * 4);
  TCHK(hipMemcpyAsync(out.bbox.data(), bbox_all, total_nodes * 4 * 8, hipMemcpyDeviceToHost, st));
  TCHK(hipStreamSynchronize(st));
  out.d_perm = perm;

  // ---------------- block tree
  const double eta2 = eta * eta;
  int2* fr = nullptr;
  int2* nx = nullptr;
  int *isl = nullptr, *nch = nullptr, *knd = nullptr, *lpos = nullptr, *cpos = nullptr;
  int4* leaves = nullptr;
  int64_t fr_cap = 0, wk_cap = 0, leaf_cap = 1 << 16;
  // work arrays sized for a frontier of c pairs (contents not preserved)
  auto ensure_work = [&](int64_t c) -> std::string {
    if (c <= wk_cap) return "";
    int64_t nc = std::max<int64_t>(1024, wk_cap);
    while (nc < c) nc *= 2;
    if (nx) TCHK(hipFreeAsync(nx, st));
    if (isl) TCHK(hipFreeAsync(isl, st));
    if (nch) TCHK(hipFreeAsync(nch, st));
    if (knd) TCHK(hipFreeAsync(knd, st));
    if (lpos) TCHK(hipFreeAsync(lpos, st));
    if (cpos) TCHK(hipFreeAsync(cpos, st));
    wk_cap = nc;
    TCHK(hipMallocAsync(&nx, (wk_cap * 4) * 8, st));
    TCHK(hipMallocAsync(&isl, (wk_cap + 1) * 4, st));
    TCHK(hipMallocAsync(&nch, (wk_cap + 1) * 4, st));
    TCHK(hipMallocAsync(&knd, (wk_cap + 1) * 4, st));
    TCHK(hipMallocAsync(&lpos, (wk_cap + 1) * 4, st));
    TCHK(hipMallocAsync(&cpos, (wk_cap + 1) * 4, st));
    return "";
  };
  // frontier array (contents not preserved: it is rewritten from nx)
  auto ensure_fr = [&](int64_t c) -> std::string {
    if (c <= fr_cap) return "";
    int64_t nc = std::max<int64_t>(1024, fr_cap);
    while (nc < c) nc *= 2;
    if (fr) TCHK(hipFreeAsync(fr, st));
    fr_cap = nc;
    TCHK(hipMallocAsync(&fr, fr_cap * 8, st));
    return "";
  };
  {
    std::string g = ensure_fr(1);
    if (!g.empty()) return g;
  }
  TCHK(hipMallocAsync(&leaves, leaf_cap * 16, st));
  {
    int2 root = make_int2(0, 0);
    TCHK(hipMemcpyAsync(fr, &root, 8, hipMemcpyHostToDevice, st));
  }
  int64_t cnt = 1, nleaves = 0;
  unsigned* stmp = nullptr;
  int64_t stmpb = 0;
  for (int l = 0; l <= D && cnt > 0; ++l) {
    std::string g = ensure_work(cnt + 1);
    if (!g.empty()) return g;
    k_classify<<<nblk(cnt, 256), 256, 0, st>>>(fr, (int)cnt, bbox_all + ((int64_t(1) << l) - 1) * 4,
                                                eta2, rule, l == D, isl, nch, knd);
    TCHK(hipGetLastError());
    const int64_t need2 = scan_scratch(cnt + 1);
    if (need2 > stmpb) {
      if (stmp) TCHK(hipFreeAsync(stmp, st));
      stmpb = need2 * 2;
      TCHK(hipMallocAsync(&stmp, stmpb * 4, st));
    }
    TCHK(hipMemsetAsync(isl + cnt, 0, 4, st));
    TCHK(hipMemsetAsync(nch + cnt, 0, 4, st));
    {
      std::string e = exclusive_sum((const unsigned*)isl, (unsigned*)lpos, cnt + 1, stmp, st);
      if (e.empty()) e = exclusive_sum((const unsigned*)nch, (unsigned*)cpos, cnt + 1, stmp, st);
      if (!e.empty()) return e;
    }
    int tot[2];
    TCHK(hipMemcpyAsync(&tot[0], lpos + cnt, 4, hipMemcpyDeviceToHost, st));
    TCHK(hipMemcpyAsync(&tot[1], cpos + cnt, 4, hipMemcpyDeviceToHost, st));
    TCHK(hipStreamSynchronize(st));
    if (nleaves + tot[0] > leaf_cap) {
      int64_t nc = leaf_cap;
      while (nc < nleaves + tot[0]) nc *= 2;
      int4* l2 = nullptr;
      TCHK(hipMallocAsync(&l2, nc * 16, st));
      TCHK(hipMemcpyAsync(l2, leaves, nleaves * 16, hipMemcpyDeviceToDevice, st));
      TCHK(hipStreamSynchronize(st));
      TCHK(hipFreeAsync(leaves, st));
      leaves = l2;
      leaf_cap = nc;
    }
    if (tot[1] > wk_cap * 4) return "block tree frontier overflow";
    k_expand<<<nblk(cnt, 256), 256, 0, st>>>(fr, (int)cnt, knd, lpos, cpos, l, leaves, (int)nleaves, nx);
    TCHK(hipGetLastError());
    TCHK(hipStreamSynchronize(st));
    nleaves += tot[0];
    cnt = tot[1];
    if (cnt > 0) {
      std::string g2 = ensure_fr(cnt);
      if (!g2.empty()) return g2;
      TCHK(hipMemcpyAsync(fr, nx, cnt * 8, hipMemcpyDeviceToDevice, st));
      TCHK(hipStreamSynchronize(st));
    }
  }
  std::vector<int4> lh(nleaves);
  TCHK(hipMemcpyAsync(lh.data(), leaves, nleaves * 16, hipMemcpyDeviceToHost, st));
  TCHK(hipStreamSynchronize(st));
  out.blocks.resize(nleaves * 4);
  for (int64_t i = 0; i < nleaves; ++i) {
    out.blocks[4 * i] = lh[i].x;
    out.blocks[4 * i + 1] = lh[i].y;
    out.blocks[4 * i + 2] = lh[i].z;
    out.blocks[4 * i + 3] = lh[i].w;
  }
  hipFreeAsync(fr, st);
  hipFreeAsync(nx, st);
  hipFreeAsync(isl, st);
  hipFreeAsync(nch, st);
  hipFreeAsync(knd, st);
  hipFreeAsync(lpos, st);
  hipFreeAsync(cpos, st);
  hipFreeAsync(leaves, st);
  if (stmp) hipFreeAsync(stmp, st);
  hipFreeAsync(kin, st);
  hipFreeAsync(kout, st);
  hipFreeAsync(vin, st);
  hipFreeAsync(vout, st);
  hipFreeAsync(rx, st);
  hipFreeAsync(ry, st);
  hipFreeAsync(tmp, st);
  hipFreeAsync(bbox_all, st);
  hipFreeAsync(bbk, st);
  hipFreeAsync(axis, st);
  hipFreeAsync(dlo, st);
  return "";
}

}  // namespace hc
