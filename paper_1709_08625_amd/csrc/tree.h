// GPU construction of the cluster tree and the block cluster tree.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace hc {

struct TreeOut {
  std::vector<int64_t> perm;     // cluster position -> original index
  std::vector<double> bbox;      // (2^(D+1)-1) x 4, level order
  std::vector<int64_t> blocks;   // n_blocks x 4 (level, row, col, kind)
  int* d_perm = nullptr;         // device copy of perm (int32), owned by caller
};

// d_loc: device double2[n] in original order.  lo: node starts per level
// (from the sizes alone).  rule: 0 standard (min), 1 max form, 2 weak
// admissibility.  Returns "" on success.
std::string build_trees(const double* d_loc, int64_t n, int leaf_max, int D, double eta, int rule,
                        const std::vector<std::vector<int64_t>>& lo, hipStream_t st, TreeOut& out);

}  // namespace hc
