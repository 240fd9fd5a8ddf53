// Host test of the TSQR tree indexing (paper_2604_05319_amd/csrc/tsqr_tree.h):
// for every chunk count, the nodes that the merge kernels address (every level
// of ceil-halving up to the root) lie inside the tree_nodes(n) slots the host
// allocates per problem, and no two nodes share a slot.
#include <cstdio>
#include <vector>

#include "../../paper_2604_05319_amd/csrc/tsqr_tree.h"

int main() {
    int failures = 0;
    for (int n = 1; n <= 4096; ++n) {
        const int total = hn::tree_nodes(n);
        std::vector<int> used(total, 0);
        int cnt = n, L = 0;
        for (;;) {
            const int off = hn::tree_levoff(n, L);
            for (int i = 0; i < cnt; ++i) {
                const int slot = off + i;
                if (slot < 0 || slot >= total) {
                    std::printf("FAIL n=%d level %d node %d -> slot %d of %d\n", n, L, i, slot, total);
                    ++failures;
                } else if (used[slot]++) {
                    std::printf("FAIL n=%d slot %d used twice\n", n, slot);
                    ++failures;
                }
            }
            if (cnt == 1) break;
            cnt = (cnt + 1) / 2;
            ++L;
        }
        if (L != hn::tree_depth(n)) {
            std::printf("FAIL n=%d depth %d vs %d\n", n, L, hn::tree_depth(n));
            ++failures;
        }
        if (failures > 20) break;
    }
    if (failures) return 1;
    std::printf("tree host test ok\n");
    return 0;
}
