// Host check of the nested-dissection front tree (no GPU): builds the S^z
// sector pattern of the periodic chain of length L (the sparsity of H in
// Eq. (1): the diagonal plus one entry per antiparallel neighbour pair), runs
// the product's symbolic analysis on it, and prints the pattern, the ordering
// and the fronts as JSON for tests/test_symbolic_host.py.
#include "symbolic.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace mbl;

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const int L = atoi(argv[1]);
    const int nup = (L + 1) / 2;
    std::vector<uint32_t> basis;
    for (uint32_t w = 0; w < (1u << L); w++)
        if (__builtin_popcount(w) == nup) basis.push_back(w);
    Pattern A;
    A.n = (int64_t)basis.size();
    A.rowptr.push_back(0);
    for (size_t i = 0; i < basis.size(); i++) {
        const uint32_t w = basis[i];
        std::vector<int32_t> cols{(int32_t)i};
        for (int s = 0; s < L; s++) {
            const int t = (s + 1) % L;
            if (((w >> s) & 1) != ((w >> t) & 1)) {
                const uint32_t v = w ^ (1u << s) ^ (1u << t);
                cols.push_back((int32_t)(std::lower_bound(basis.begin(), basis.end(), v) - basis.begin()));
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        for (int32_t c : cols) A.col.push_back(c);
        A.rowptr.push_back((int32_t)A.col.size());
    }
    NdOptions opt;
    if (argc > 2) opt.leaf_size = atoi(argv[2]);
    const FrontTree t = build_front_tree(A, opt);
    printf("{\"n\": %lld, \"nnz_factor\": %lld, \"front_entries\": %lld, \"flops\": %.17g, \"n_levels\": %d,\n",
           (long long)t.n, (long long)t.nnz_factor, (long long)t.front_entries, t.flops, t.n_levels);
    printf("\"rowptr\": [");
    for (size_t i = 0; i < A.rowptr.size(); i++) printf("%s%d", i ? "," : "", A.rowptr[i]);
    printf("],\n\"col\": [");
    for (size_t i = 0; i < A.col.size(); i++) printf("%s%d", i ? "," : "", A.col[i]);
    printf("],\n\"perm\": [");
    for (size_t i = 0; i < t.perm.size(); i++) printf("%s%d", i ? "," : "", t.perm[i]);
    printf("],\n\"fronts\": [");
    for (size_t f = 0; f < t.fronts.size(); f++) {
        const Front &fr = t.fronts[f];
        printf("%s\n{\"first\": %d, \"p\": %d, \"c\": %d, \"parent\": %d, \"level\": %d, \"children\": [",
               f ? "," : "", fr.first, fr.p, fr.c, fr.parent, fr.level);
        for (size_t k = 0; k < fr.children.size(); k++) printf("%s%d", k ? "," : "", fr.children[k]);
        printf("], \"contrib\": [");
        for (int32_t k = 0; k < fr.c; k++) printf("%s%d", k ? "," : "", t.contrib[fr.cptr + k]);
        printf("]}");
    }
    printf("]}\n");
    return 0;
}
