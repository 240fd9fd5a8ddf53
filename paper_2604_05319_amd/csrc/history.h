// History-integral kernels over HODLR storage: argument structs and launchers.
#pragma once

#include "common.h"

namespace hn {

// A projection task: rows [chunk*kch, +kch) of U (which = 0) or V (which = 1)
// (kch: HistArgs::kch, the handle's chunk rows)
// of block b, orbital pair q, component comp.  Active once row `act` is merged
// (U: the chunk's first row; V: the block's first row).  At norb 4, and with
// matrix-core projections (HistArgs::mfproj) at norb 16, q is the shared orbital
// index beta of the norb pairs the task takes.
struct FactTask {
    int comp, b, q, which, chunk, act;
};

struct HistArgs {
    int n;          // current step
    int n0[2];      // first row not yet merged, per component
    int last[2];    // last appended row, per component
    int ls[2];      // tail rows (n0..last) hold columns [0, ls) for rows >= nsplit and
    int lslo[2];    // [0, lslo) for rows < nsplit (the panel whose merge is still in flight)
    int nsplit[2];
    int ring;       // tail row r sits in slot r % ring
    int nt, norb, npair, RC, nlvl, nb, P;
    int nk;         // objects in the batch (grid dimension y)
    int wantR, wantL;
    int adj;        // adjoint of I^R: sigL holds Ibar(n, m) rows, outL receives dI/dSigma^R (see launch_history)
    double h;
    Weights W;
    const cd* sigR;   // Sigma^R(n, j), j = 0..n
    const cd* sigL;   // Sigma^<(s, n), s = 0..n
    cd* sigRT;        // norb 16: scratch for Sigma^R(n, j) with its orbital indices swapped
    long long kInT;   // its object stride
    int kch;          // factor rows per projection chunk (task and partial slot)
    int f32;          // factors stored as complex float (cf) instead of complex double
    int mfproj;       // norb = 16 with cf factors and RC <= 16: projections on the matrix
                      // cores, one task per (block, factor, chunk, orbital index beta)
    int mfcomb;       // with mfproj and every leaf starting at a multiple of 16: the
                      // expansions of the combine on the matrix cores, 16-column tiles
    const void* U[2]; // factor storage, element type cd or cf
    const void* V[2];
    const double* S[2];
    const int* rank[2];
    // double-buffered factors: block b of component c is read from buffer cur[c][b];
    // buffer 1 of U / V / S / rank lies bU / bV / bS / bRank elements after buffer 0
    const int* cur[2];
    long long bU, bV, bS, bRank;
    const cd* leaf[2];
    const cd* tail[2];
    const cd* band;   // retarded band: band[(m*(k+1) + i)*npair + q] = G^R(m+i, m)
    const int* blk;   // 5 per block: level, r0, r1, c0, c1
    const int* leafs; // 2 per leaf: s0, s1
    const int* cover; // [l*nt + m]
    const long long* Uoff;
    const long long* Voff;
    const long long* Loff;
    const FactTask* ft[2];
    const long long* partoff;  // per (comp, b, q, which): first chunk-partial slot
    int nf[2];       // active projection tasks per component
    int nfpad;       // nf[0] + nf[1] rounded up to a multiple of 8 (of 32 at norb 4)
    int nleaf;       // active leaves
    int nleaftask;   // leaf tasks in the grid (after the XCD-grouping remap)
    int ntailchunk[2];
    int ntailtask;
    cd* part;        // [partial slot][a][RC]  S_r * projection of one chunk
    cd* proj;        // [comp][b][q][which][a][RC]  S_r * projection (sum of the chunks)
    cd* leafR;       // [pair group][m][a][c]   leaf pieces, one slot per pair group
    cd* leafLR;
    cd* leafLL;
    cd* tailcol[2];  // [m][a][c]       column sums over the tail rows
    cd* tailpart[2]; // [chunk][slot][a][c]  row dots of the tail rows, per column chunk
    cd* tailrow[2];  // [slot][a][c]         row dots of the tail rows (sum over the chunks)
    cd* outR;
    cd* outL;
    // factor-gradient mode (fgrad = 1, with wantR = wantL = adj = 1 and no dense
    // pieces): the step's projections x_n U and Ibar_n V feed fgrad_kernel, which adds
    // the step's contributions to dL/d(U, S, V) of the retarded factors (FP64 copies
    // Ud, Vd) into dU, dV (laid out like one buffer of U, V) and dS ([b][pair][RC])
    int fgrad;
    const cd* Ud;
    const cd* Vd;
    cd* dU;
    cd* dV;
    double* dS;
    // batched objects (grid dimension y): element strides from one object's
    // data to the next; the geometry and the task lists are shared
    long long kIn, kOut;   // Sigma rows, output rows
    long long kU, kV, kS, kRank, kLeaf, kTail, kBand;
    long long kProj, kPart, kLeafOut, kLeafOutLL, kTailcol, kTailpart, kTailrow;
};

// Adjoint mode (adj = 1, wantR = 0, wantL = 1): the comp-0 row-dot path of the
// second lesser term is driven by x(m) = Ibar(n, m) instead of the folded
// Sigma^< slice, which gives y(j) = sum_{m<=j} Ibar(n,m) G^R(j,m)^dagger; the
// combine scales it by the end weight of j and adds the start / short-interval
// corrections, so outL(j) = h sum_{m<=j} w^{(n-m)}_{j-m} Ibar(n,m) G^R(j,m)^dagger.
// The lesser component is not touched.
//
// ev: nullptr, or four events recorded before hist_tasks, after it, after
// proj_reduce and after hist_combine (per-kernel timing on the launch stream)
hipError_t launch_history(const HistArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);
hipError_t history_init();

}  // namespace hn
