// Cluster tree and block cluster tree on the GPU (Sec. 2.2, Appendix A).
//
// Cluster tree: recursive bisection into two equal-sized subsets by an
// axis-parallel cut across the longer side of the cluster's bounding box.
// Level-synchronous: at each level every node's points are ordered by
// (coordinate on the node's split axis, original index) with one device-wide
// radix sort of the 64-bit key (node << 32 | rank on that axis), where the
// rank of a point on an axis is its position in the global order
// (coordinate, index); the first ceil(s/2) points of a node form its left
// son.  Leaves are finally ordered by original index.  Bounding boxes are
// exact min/max reductions, so the result is bit-identical to the CPU
// reference.
//
// Block cluster tree: breadth-first expansion from (root, root) keeping the
// lower triangle; a pair is a low-rank leaf when the standard admissibility
// condition min(diam^2) <= eta^2 dist^2 holds with dist^2 > 0 (evaluated with
// single IEEE operations, no contraction), a dense leaf at the leaf level,
// otherwise it is replaced by its son pairs.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

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
  void* tmp = nullptr;
  size_t tmpb = 0, need = 0;
  TCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, (int)n, 0, 64, st));
  tmpb = need;
  TCHK(hipMallocAsync(&tmp, tmpb + 256, st));
  for (int ax = 0; ax < 2; ++ax) {
    k_axis_keys<<<nblk(n, 256), 256, 0, st>>>(loc, n, ax, kin, vin);
    TCHK(hipGetLastError());
    size_t tb = tmpb;
    TCHK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, vin, vout, (int)n, 0, 64, st));
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
    size_t tb = tmpb;
    int endbit = 32 + (l == 0 ? 1 : l + 1);
    TCHK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, vin, perm, (int)n, 0, endbit, st));
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
  void* stmp = nullptr;
  size_t stmpb = 0;
  for (int l = 0; l <= D && cnt > 0; ++l) {
    std::string g = ensure_work(cnt + 1);
    if (!g.empty()) return g;
    k_classify<<<nblk(cnt, 256), 256, 0, st>>>(fr, (int)cnt, bbox_all + ((int64_t(1) << l) - 1) * 4,
                                                eta2, rule, l == D, isl, nch, knd);
    TCHK(hipGetLastError());
    size_t need2 = 0;
    TCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, need2, isl, lpos, (int)cnt + 1, st));
    if (need2 > stmpb) {
      if (stmp) TCHK(hipFreeAsync(stmp, st));
      stmpb = need2 * 2;
      TCHK(hipMallocAsync(&stmp, stmpb, st));
    }
    TCHK(hipMemsetAsync(isl + cnt, 0, 4, st));
    TCHK(hipMemsetAsync(nch + cnt, 0, 4, st));
    size_t tb = stmpb;
    TCHK(hipcub::DeviceScan::ExclusiveSum(stmp, tb, isl, lpos, (int)cnt + 1, st));
    tb = stmpb;
    TCHK(hipcub::DeviceScan::ExclusiveSum(stmp, tb, nch, cpos, (int)cnt + 1, st));
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
