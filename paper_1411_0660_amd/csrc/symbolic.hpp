// symbolic.hpp -- fill-reducing ordering and assembly tree of dense fronts for
// the sparse LU of H - sigma (host side, computed once per chain length L).
#pragma once

#include <cstdint>
#include <vector>

namespace mbl {

// Symmetric sparsity pattern in CSR (diagonal may be present; it is ignored by
// the ordering).
struct Pattern {
    int64_t n = 0;
    std::vector<int32_t> rowptr, col;
};

// One dense front of the multifrontal factorisation: the pivots are the
// contiguous new indices [first, first + p), the contribution rows are the
// sorted new indices contrib[cptr .. cptr + c).  The front matrix is m x m with
// m = p + c, local order = pivots then contribution rows.
struct Front {
    int32_t first = 0, p = 0, c = 0;
    int32_t parent = -1;
    int32_t level = 0;              // 0 for leaves, 1 + max(children) otherwise
    int64_t cptr = 0;               // offset into FrontTree::contrib
    std::vector<int32_t> children;  // in creation order
    int32_t m() const { return p + c; }
};

struct FrontTree {
    int64_t n = 0;
    std::vector<int32_t> perm;      // new -> old index
    std::vector<int32_t> iperm;     // old -> new index
    std::vector<Front> fronts;      // post-order: children before parents
    std::vector<int32_t> contrib;   // concatenated contribution-row lists
    int32_t n_levels = 0;
    // statistics
    int64_t nnz_factor = 0, front_entries = 0, max_m = 0, max_p = 0;
    double flops = 0.0;
    double seconds = 0.0;
};

struct NdOptions {
    int leaf_size = 96;       // subgraphs at most this large become one front
    double imbalance = 0.05;  // allowed deviation from an even split
    int fm_passes = 6;
    int init_tries = 8;
    uint64_t seed = 0x5eed;
};

// Nested dissection with multilevel vertex separators, then the front
// structure (pivots, contribution rows, tree levels, statistics).
FrontTree build_front_tree(const Pattern &A, const NdOptions &opt);

// Local index of every contribution row of child `ch` inside its parent front.
void child_relative_map(const FrontTree &t, int ch, std::vector<int32_t> &map);

}  // namespace mbl
