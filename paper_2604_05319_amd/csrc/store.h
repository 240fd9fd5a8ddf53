// Row append kernels: argument struct and launchers.
#pragma once

#include "common.h"

namespace hn {

struct AppendArgs {
    const cd* row;  // (n+1) x npair
    int n, npair, nt, k;
    int ls, lw;     // leaf of row n: first row/column and width
    int slot;       // tail slot of row n (n - first unmerged row)
    cd* leaf;       // leaf triangle base (pair 0)
    cd* tail;       // tail base
    cd* band;       // retarded band or nullptr
    // batched objects (grid dimension y): element strides from one object to the next
    long long kRow, kLeaf, kTail, kBand;
};

hipError_t launch_append_hodlr(const AppendArgs& a, int nk, hipStream_t st);
// both components' rows n in one launch (grid dimension z = component)
hipError_t launch_append_hodlr2(const AppendArgs& a0, const AppendArgs& a1, int nk, hipStream_t st);
hipError_t launch_append_dense(cd* dst, const cd* row, int n, int npair, long long trin,
                               hipStream_t st);

}  // namespace hn
