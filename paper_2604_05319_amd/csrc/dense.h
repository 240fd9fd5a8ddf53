// Dense baseline kernels: argument struct and launcher.
#pragma once

#include "common.h"

namespace hn {

struct DenseArgs {
    int n, nt, norb;
    double h;
    Weights W;
    const cd* sigR;
    const cd* sigL;
    const cd* L[2];      // packed lower triangles, pair-major: L[q*trin + t1(t1+1)/2 + t2]
    long long trin;      // nt(nt+1)/2
    cd* colR;            // [row band][m][npair] partial column sums (retarded)
    cd* colL;            // [row band][m][npair] partial column sums (lesser)
    cd* rowL;            // [64-column chunk][j][npair] partial row dots (lesser output)
    cd* outR;
    cd* outL;
};

int dense_band_count(int nt);    // 128-row bands (column-sum partials)
int dense_chunk_count(int nt);   // 64-column chunks (row-dot partials)
hipError_t dense_init();
hipError_t launch_dense_history(const DenseArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);

}  // namespace hn
