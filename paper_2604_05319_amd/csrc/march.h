// Rows of G^R in the paper's orientation: argument struct and launcher.
#pragma once

#include "common.h"

namespace hn {

// Each row n of G^R solves its own Volterra problem along the relative time: the right
// form of the retarded equation, marched from the diagonal leftwards over the compressed
// Sigma^R history held by a handle (stored as its retarded component, merges finished).
// One workgroup per row; rows nlo..nhi in one launch.
struct MarchArgs {
    int nt, norb, npair, RC, k, nlvl, ring;
    int n0;              // first unmerged row of the stored Sigma (tail rows n0..last)
    int ls;              // dense tail columns [0, ls)
    int nlo, nhi;        // rows of this launch (nlo >= k)
    double h;
    Weights W;
    StepWeights S;
    // Sigma^R storage of the handle (retarded component)
    const cd* U;
    const cd* V;
    const double* Sv;
    const int* rank;
    const int* cur;
    long long bU, bV, bS, bRank;
    const long long* Uoff;
    const long long* Voff;
    const long long* Loff;
    const int* blk;      // 5 per block: level, r0, r1, c0, c1
    const int* leafs;    // 2 per leaf: s0, s1
    const int* rowLeaf;  // leaf index of each row
    const int* cover;    // [l * nt + m]: block with m in its column range (>= 0) or ~block
    const cd* leaf;
    const cd* tail;
    const cd* band;      // band[(m (k+1) + i) npair + q] = Sigma^R(m+i, m)
    const cd* eps;       // eps(t_j), [nt][npair]
    cd* rows;            // row n at rows + (n - nlo) * rowStride: G^R(t_n, t_m), m = 0..n
    long long rowStride;
    cd* proj;            // per row and level: the current block's projections [NORB][npair][32]
    cd* minv;            // [m][a][b]: M_m^{-1}, M_m = i a_0/h - eps(t_m) - h omega_0 Sigma(m, m)
};

// M_m^{-1} for the columns m = 0..mcount-1 (the same for every row), then the rows
// nlo..nhi, longest first; a.proj holds nhi - nlo + 1 rows of projections.
hipError_t launch_march_minv(const MarchArgs& a, int mcount, hipStream_t st);
hipError_t launch_row_march(const MarchArgs& a, hipStream_t st);

}  // namespace hn
