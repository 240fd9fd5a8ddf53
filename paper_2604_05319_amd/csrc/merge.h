// Incremental TSVD merge: argument structs and launcher.
#pragma once

#include "common.h"
#include "tsqr_tree.h"

namespace hn {

// Width w = r + panel of a merge (the size of its small SVD) is at most the
// merge width W, one of two compiled widths: 32 (128-row chunks) or 48
// (96-row chunks, for rank capacities above 32 - panel).
constexpr int kWSmall = 32;
constexpr int kWLarge = 48;
constexpr int kW = kWLarge;             // widest merge
constexpr int kMaxMergeBlk = 24;        // blocks merged by one panel (<= nlvl)

__host__ __device__ constexpr int merge_ch(int W) { return W <= kWSmall ? 128 : 96; }   // rows of Z per chunk
__host__ __device__ constexpr int node_q(int W) { return 2 * W * W + W; }            // explicit Q (2W x W), W spare
__host__ __device__ constexpr int chunk_q(int W) { return merge_ch(W) * W + W; }      // explicit Q (CH x W), W spare
inline int merge_width(int rank_cap, int panel) { return rank_cap + panel <= kWSmall ? kWSmall : kWLarge; }

struct MergeBlk {
    int b;          // block index in the factor arrays (rank/S are [b][pair])
    int c0;         // first column of the block
    int ncols;      // |C_b|
    int ldU;        // row capacity of U (|R_b|)
    int kb;         // rows already merged
    int nchunks;    // ceil(ncols / CH)
    int task_off;   // first chunk task of this block (pair-major inside)
    int utask_off;  // first U task of this block (inside the U segment)
    int nutask;     // U tasks per pair
    int nnodes;     // tree nodes per pair (at least tree_nodes(nchunks))
    long long node_base;  // first node of pair 0 of this block in the scratch
    long long chunk_base; // first chunk slot of pair 0 of this block in chunkQ
    long long Uoff, Voff; // element offsets of the block in U / V (pair 0, rank 0)
    int rd;               // factor buffer holding the block's current TSVD (read); the
                          // update goes to buffer rd ^ flip
};

struct MergeArgs {
    int W;         // merge width (kWSmall or kWLarge): selects the kernel instance
    int pp;        // rows in this panel
    int npair;     // norb^2
    int RC;        // rank capacity per block and pair of the updated factors
    int RCr;       // rank capacity of the factors read (equal to RC except for a
                   // final merge into buffers of another capacity)
    double tol;    // eps_SVD (absolute) of this merge
    int nblk;
    MergeBlk blk[kMaxMergeBlk];
    int ntask_v;   // chunk tasks (merge_up grid; first part of merge_down grid)
    int ntask_u;   // U-row tasks (second part of merge_down grid)
    // factors: the current TSVD is read from Ur/Vr/Sr/rankr and the update written to
    // U/V/S/rank (the same arrays in the HODLR store)
    const cd* Ur;
    const cd* Vr;
    const double* Sr;
    const int* rankr;
    cd* U;
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
    cd* nodeQ;     // [node][node_q(W)]: explicit Q of each tree node's QR
    cd* chunkQ;    // [chunk slot][chunk_q(W)]: explicit Q of merge_up's chunk QR, used by merge_down
    int* nodecnt;  // [node]
    cd* UK;        // [problem][W*W]
    cd* VR;        // [problem][W*W]
    double* Sold;  // [problem][W]
    int* rold;     // [problem]
    int* err;      // device error flags (bit 0: rank cap reached, bit 1: non-finite data)
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
// p[i] = v for i < n (clears flags and counters without a memset node)
hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t st);
hipError_t merge_init();

}  // namespace hn
