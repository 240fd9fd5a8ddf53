// Incremental TSVD merge: argument structs and launcher.
#pragma once

#include "common.h"

namespace hn {

constexpr int kW = 32;                  // max width r + panel of a merge (SVD size)
constexpr int kMergeCH = 128;           // rows of Z per chunk workgroup
constexpr int kMaxMergeBlk = 24;        // blocks merged by one panel (<= nlvl)
constexpr int kNodeQ = 2 * kW * kW + kW;  // reflectors (2W x W) + tau (W) of a tree node
constexpr int kChunkQ = kMergeCH * kW + kW;  // reflectors (CH x W) + tau (W) of a chunk

struct MergeBlk {
    int b;          // block index in the factor arrays (rank/S are [b][pair])
    int c0;         // first column of the block
    int ncols;      // |C_b|
    int ldU;        // row capacity of U (|R_b|)
    int kb;         // rows already merged
    int nchunks;    // ceil(ncols / kMergeCH)
    int task_off;   // first chunk task of this block (pair-major inside)
    int utask_off;  // first U task of this block (inside the U segment)
    int nutask;     // U tasks per pair
    int nnodes;     // tree nodes per pair (2 * nchunks)
    long long node_base;  // first node of pair 0 of this block in the scratch
    long long chunk_base; // first chunk slot of pair 0 of this block in chunkQ
    long long Uoff, Voff; // element offsets of the block in U / V (pair 0, rank 0)
    int rd;               // factor buffer holding the block's current TSVD (read); the
                          // update goes to buffer rd ^ flip
};

struct MergeArgs {
    int pp;        // rows in this panel
    int npair;     // norb^2
    int RC;        // rank capacity per block and pair
    double tol;    // eps_SVD (absolute)
    int nblk;
    MergeBlk blk[kMaxMergeBlk];
    int ntask_v;   // chunk tasks (merge_up grid; first part of merge_down grid)
    int ntask_u;   // U-row tasks (second part of merge_down grid)
    cd* U;         // FP64 factors (the merge works on these), buffer 0
    cd* V;
    cf* U32;       // complex-float mirrors of U and V read by the history kernels, or nullptr
    cf* V32;
    double* S;
    int* rank;
    // panel row i, pair q, absolute column s at src[slot*src_row + q*src_pair + s]
    // with slot = (src_first + i) % src_ring
    const cd* src;
    long long src_row, src_pair;
    int src_first, src_ring;
    // scratch
    cd* nodeR;     // [node][W*W]
    cd* nodeQ;     // [node][kNodeQ]
    cd* chunkQ;    // [chunk slot][kChunkQ]: chunk QR of merge_up, reused by merge_down
    int* nodecnt;  // [node]
    cd* UK;        // [problem][W*W]
    cd* VR;        // [problem][W*W]
    double* Sold;  // [problem][W]
    int* rold;     // [problem]
    int* err;      // device error flags (bit 0: rank cap reached)
    // double buffering: buffer 1 of U / V (and mirrors) / S / rank lies bU / bV / bS /
    // bRank elements after buffer 0; flip = 1 writes the update into the other buffer,
    // flip = 0 updates in place
    int flip;
    long long bU, bV, bS, bRank;
    // batched objects (grid dimension y): element strides from one object to the next
    long long kU, kV, kS, kRank, kSrc, kNodeR, kNodeQ, kNodeCnt, kProbW2, kProbW, kProb, kChunkQ;
};

hipError_t launch_merge(const MergeArgs& a, int nk, hipStream_t st);
// cur[b] ^= 1 for the n blocks listed (n <= kMaxMergeBlk): the merged blocks'
// updated TSVDs become current
hipError_t launch_flip(int* cur, const int* blocks, int n, hipStream_t st);
hipError_t merge_init();

}  // namespace hn
