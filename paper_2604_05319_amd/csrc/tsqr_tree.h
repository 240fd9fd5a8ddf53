// Index arithmetic of the TSQR reduction tree of a merge: chunk R factors are
// combined pairwise, level by level (cnt[0] = chunks, cnt[L+1] = ceil(cnt[L]/2)),
// until one root remains; node (L, i) is stored at tree_levoff(n, L) + i.
// Plain functions for the host (scratch sizing, tests) and the device.
#pragma once

#if defined(__HIPCC__)
#define HN_TREE_HD __host__ __device__
#else
#define HN_TREE_HD
#endif

namespace hn {

// first node of level L of the tree over n chunks
HN_TREE_HD constexpr int tree_levoff(int n, int L) {
    int off = 0, cnt = n;
    for (int i = 0; i < L; ++i) {
        off += cnt;
        cnt = (cnt + 1) / 2;
    }
    return off;
}

// nodes of the tree over n chunks (more than 2n - 1 when n is not a power of two)
HN_TREE_HD constexpr int tree_nodes(int n) {
    int total = n, cnt = n;
    while (cnt > 1) {
        cnt = (cnt + 1) / 2;
        total += cnt;
    }
    return total;
}

// number of levels above the chunks
HN_TREE_HD constexpr int tree_depth(int n) {
    int d = 0;
    for (int cnt = n; cnt > 1; cnt = (cnt + 1) / 2) ++d;
    return d;
}

}  // namespace hn
