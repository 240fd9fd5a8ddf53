// Incremental truncated-SVD update of HODLR blocks (section "Hierarchical
// decomposition": finished rows are folded into the block's TSVD as they
// arrive; singular values below eps_SVD are dropped).
//
// A block B (rows so far) ~ U S V^dagger receives a panel A_p of Pp new rows.
// With Z = [V S, A_p^dagger] (cols x w, w = r + Pp) and Z = Q R (QR),
//     [B; A_p] = blkdiag(U, I) Z^dagger = blkdiag(U, I) R^dagger Q^dagger,
// so an SVD R^dagger = U_K Sigma V_R^dagger gives the updated factors
//     U' = blkdiag(U, I) U_K,   S' = Sigma,   V' = Q V_R,
// truncated to the singular values >= eps.  The paper updates one row at a
// time; here a panel of rows is merged at once.
//
// Device design (one problem = one block x one orbital pair):
//   merge_up:   the columns of the block are cut into chunks of kCH rows of Z;
//               each workgroup builds its chunk of Z in LDS, factors it with
//               Householder reflections and keeps the explicit thin Q.  The R
//               factors are combined pairwise up a binary tree (each node's
//               explicit Q kept too); the last workgroup to arrive at a node does
//               the combine (no waiting), and the one arriving at the root
//               runs a one-sided Jacobi SVD of R^dagger and truncates.
//   merge_down: each chunk workgroup pulls V_R down the tree to its chunk (at
//               every level the node's Q rows of its side times the current
//               factor), multiplies by its chunk's Q and writes its rows of V';
//               further workgroups rewrite the rows of U'.
#include "merge.h"
#include "trunc.h"

namespace hn {

namespace {

constexpr int NT = 256;

__device__ inline double warp_sum(double v, int width) {
    for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

// block-wide sum of one double (all threads get the result)
__device__ double block_sum(double v, double* red) {
    v = warp_sum(v, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// Householder QR of an nrows x ncols column-major LDS matrix A (lda = nrows),
// nrows >= ncols.  On exit R is in the upper triangle, the reflector vectors
// (v_j = 1 implicit) below it, and tau[j] holds the scalars: A = H_0..H_{n-1} R
// with H_j = I - tau_j v_j v_j^dagger.
//
// One barrier per column: the thread group that updates column j+1 also sums
// its squared entries below the diagonal (the next reflector's norm), and the
// scaling of reflector j into v_j (with the diagonal beta_j) is written during
// step j+1, when no thread reads column j any more.  Threads: groups of
// TPC = NT / W per trailing column, group g updates column j + 1 + g.
template <int W>
__device__ void reflector(cd alpha, double sig2, cd& beta_out, cd& t, cd& scale) {
    double beta = alpha.x;
    t = mk(0.0, 0.0);
    scale = mk(0.0, 0.0);
    const double nrm0 = sqrt(norm2(alpha) + sig2);
    // no reflection for an exactly zero column, or one so small (or not finite)
    // that 1/(alpha - beta) would overflow: tau = 0, H_j = I
    if (!(sig2 == 0.0 && alpha.y == 0.0) && nrm0 > 1e-150 && nrm0 < 1e150) {
        beta = alpha.x >= 0.0 ? -nrm0 : nrm0;
        t = mk((beta - alpha.x) / beta, -alpha.y / beta);
        const cd d = alpha - mk(beta, 0.0);  // 1/(alpha - beta)
        const double dn = norm2(d);
        scale = mk(d.x / dn, -d.y / dn);
    }
    beta_out = mk(beta, 0.0);
}

// threads per column of a W-wide factorization: a power of two, at most NT / W
__host__ __device__ constexpr int cols_tpc(int W) { return NT / W >= 8 ? 8 : (NT / W >= 4 ? 4 : 2); }

template <int W>
__device__ __attribute__((noinline)) void hh_qr(cd* A, int nrows, int ncols, cd* tau,
                                                double* red) {
    constexpr int TPC = cols_tpc(W);  // threads per trailing column
    const int tid = threadIdx.x;
    const int g = tid / TPC, l = tid % TPC;
    // norm of column 0 below the diagonal
    {
        double part = 0.0;
        for (int i = 1 + tid; i < nrows; i += NT) part += norm2(A[i]);
        const double s0 = block_sum(part, red);
        __syncthreads();
        if (tid == 0) red[8] = s0;
        __syncthreads();
    }
    cd pbeta = mk(0.0, 0.0), pt = mk(0.0, 0.0), pscale = mk(0.0, 0.0);   // reflector j - 1
    for (int j = 0; j < ncols; ++j) {
        cd* aj = A + (size_t)j * nrows;
        const double sig2 = red[8 + (j & 1)];
        const cd alpha = aj[j];
        cd beta, t, scale;
        reflector<W>(alpha, sig2, beta, t, scale);
        // finish reflector j - 1 (nobody reads column j - 1 in this step)
        if (j > 0) {
            cd* ap = A + (size_t)(j - 1) * nrows;
            for (int i = j + tid; i < nrows; i += NT) ap[i] = ap[i] * pscale;
            if (tid == 0) {
                ap[j - 1] = pbeta;
                tau[j - 1] = pt;
            }
        }
        // apply H_j^dagger to the trailing columns: a_c -= conj(tau) v (v^dagger a_c),
        // v_j = 1 and v_i = scale * a_ij below the diagonal
        const int c = j + 1 + g;
        cd dot = mk(0.0, 0.0);
        if (c < ncols) {
            const cd* ac = A + (size_t)c * nrows;
            cd d2 = mk(0.0, 0.0);
            for (int i = j + 1 + l; i < nrows; i += TPC) fmac_(d2, aj[i], ac[i]);
            dot = conj(scale) * d2;
            if (l == 0) dot = dot + ac[j];
        }
        dot.x = warp_sum(dot.x, TPC);
        dot.y = warp_sum(dot.y, TPC);
        double nrm_next = 0.0;
        if (c < ncols) {
            cd* ac = A + (size_t)c * nrows;
            const cd f = conj(t) * dot;
            if (l == 0) ac[j] = ac[j] - f;
            const cd fs = scale * f;
            for (int i = j + 1 + l; i < nrows; i += TPC) {
                const cd v = ac[i] - aj[i] * fs;
                ac[i] = v;
                if (i > j + 1) nrm_next += norm2(v);
            }
        }
        nrm_next = warp_sum(nrm_next, TPC);   // every lane takes part in the shuffles
        if (g == 0 && l == 0) red[8 + ((j + 1) & 1)] = nrm_next;   // column j + 1's group
        pbeta = beta;
        pt = t;
        pscale = scale;
        __syncthreads();
    }
    if (ncols > 0) {
        const int j = ncols;
        cd* ap = A + (size_t)(j - 1) * nrows;
        for (int i = j + tid; i < nrows; i += NT) ap[i] = ap[i] * pscale;
        if (tid == 0) {
            ap[j - 1] = pbeta;
            tau[j - 1] = pt;
        }
    }
    __syncthreads();
}

// Explicit thin Q of hh_qr's factorization in place of the reflectors: A (nrows x
// ncols, column-major) <- H_0 H_1 .. H_{ncols-1} [I; 0].  Formed from the last
// reflector backwards: column j of the result is H_j e_j = e_j - tau_j v_j (rows
// above j zero), and H_j is applied to the columns right of j, which hold the
// columns formed so far.  One barrier per column: reflector j is copied to
// vbuf[(j & 1) * nrows ..] a step ahead, so that column j can be overwritten while
// the groups of the columns right of it still read v_j.  R (the upper triangle) is
// overwritten; the caller stores it first.
template <int W>
__device__ __attribute__((noinline)) void hh_form_q(cd* A, int nrows, int ncols, const cd* tau, cd* vbuf) {
    constexpr int TPC = cols_tpc(W);
    const int tid = threadIdx.x;
    const int g = tid / TPC, l = tid % TPC;
    if (ncols <= 0) return;
    {
        const int j = ncols - 1;
        cd* vb = vbuf + (size_t)(j & 1) * nrows;
        for (int i = j + 1 + tid; i < nrows; i += NT) vb[i] = A[(size_t)j * nrows + i];
    }
    __syncthreads();
    for (int j = ncols - 1; j >= 0; --j) {
        const cd* v = vbuf + (size_t)(j & 1) * nrows;   // v_j below row j (v_j = 1 at row j)
        const cd t = tau[j];
        if (j > 0) {   // reflector j - 1 for the next step (its column is not touched here)
            cd* vn = vbuf + (size_t)((j - 1) & 1) * nrows;
            for (int i = j + tid; i < nrows; i += NT) vn[i] = A[(size_t)(j - 1) * nrows + i];
        }
        // columns c > j: a_c -= tau_j v_j (v_j^dagger a_c) over rows j..nrows-1
        const int c = j + 1 + g;
        cd dot = mk(0.0, 0.0);
        if (c < ncols) {
            const cd* ac = A + (size_t)c * nrows;
            for (int i = j + l; i < nrows; i += TPC) fmac_(dot, i == j ? mk(1.0, 0.0) : v[i], ac[i]);
        }
        dot.x = warp_sum(dot.x, TPC);   // every lane takes part in the shuffles
        dot.y = warp_sum(dot.y, TPC);
        if (c < ncols) {
            cd* ac = A + (size_t)c * nrows;
            const cd f = t * dot;
            for (int i = j + l; i < nrows; i += TPC) ac[i] = ac[i] - (i == j ? mk(1.0, 0.0) : v[i]) * f;
        }
        // column j: e_j - tau_j v_j
        cd* aj = A + (size_t)j * nrows;
        for (int i = tid; i < nrows; i += NT)
            aj[i] = i > j ? -(t * v[i]) : (i == j ? mk(1.0 - t.x, -t.y) : mk(0.0, 0.0));
        __syncthreads();
    }
}

// one-sided (Hestenes) Jacobi on the columns of M (n x n, column-major, n even,
// ld = n), accumulating the rotations in J (starts as identity).
// A pair (p, q) is rotated while its coupling |m_p^dagger m_q| exceeds both
// 1e-15 |m_p| |m_q| (relative orthogonality) and 1e-30 |M|_F^2 (round-off of the
// whole matrix): columns at round-off level, which exact-low-rank panels produce,
// would otherwise keep the sweeps going without changing any singular value
// above 1e-15 |M|_F.
__device__ __attribute__((noinline)) void jacobi_svd(cd* M, cd* J, int n, int* flag, double* red) {
    const int tid = threadIdx.x;
    const int npairs = n / 2;
    int tpp = NT / npairs;
    if (tpp > 64) tpp = 64;
    // round down to a power of two
    int p2 = 1;
    while (p2 * 2 <= tpp) p2 *= 2;
    tpp = p2;
    for (int i = tid; i < n * n; i += NT) J[i] = mk((i % (n + 1)) == 0 ? 1.0 : 0.0, 0.0);
    double f2 = 0.0;
    for (int i = tid; i < n * n; i += NT) f2 += norm2(M[i]);
    const double floor2 = 1e-30 * block_sum(f2, red);   // |M|_F^2 is invariant under the rotations
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < n - 1; ++round) {
            const int pi = tid / tpp, l = tid % tpp;
            int p = -1, q = -1;
            if (pi < npairs) {
                // circle method: position 0 fixed, positions 1..n-1 rotate
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (n - 1)) + 1; };
                p = player(pi);
                q = player(n - 1 - pi);
            }
            double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
            if (pi < npairs) {
                const cd* mp = M + (size_t)p * n;
                const cd* mq = M + (size_t)q * n;
                for (int i = l; i < n; i += tpp) {
                    cd x = mp[i], y = mq[i];
                    al += norm2(x);
                    be += norm2(y);
                    gr += x.x * y.x + x.y * y.y;  // conj(x) y
                    gi += x.x * y.y - x.y * y.x;
                }
            }
            al = warp_sum(al, tpp);
            be = warp_sum(be, tpp);
            gr = warp_sum(gr, tpp);
            gi = warp_sum(gi, tpp);
            if (pi < npairs) {
                double ag = sqrt(gr * gr + gi * gi);
                if (ag > 1e-15 * sqrt(al * be) && ag > floor2 && ag > 1e-300) {
                    double zeta = (be - al) / (2.0 * ag);
                    double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                    cd e = mk(gr / ag, gi / ag);  // e^{i theta}
                    cd se = s * e, sec = s * conj(e);
                    cd* mp = M + (size_t)p * n;
                    cd* mq = M + (size_t)q * n;
                    cd* jp = J + (size_t)p * n;
                    cd* jq = J + (size_t)q * n;
                    for (int i = l; i < n; i += tpp) {
                        cd x = mp[i], y = mq[i];
                        mp[i] = c * x - sec * y;
                        mq[i] = se * x + c * y;
                        cd u = jp[i], v = jq[i];
                        jp[i] = c * u - sec * v;
                        jq[i] = se * u + c * v;
                    }
                    if (l == 0) *flag = 1;
                }
            }
            __syncthreads();
        }
        if (*flag == 0) break;
        __syncthreads();
    }
    __syncthreads();
}

// per-object data of object blockIdx.y of a batch (the kernel arguments
// hold object 0 and the strides)
#define OBJ ((long long)blockIdx.y)
__device__ inline cf* m_U32(const MergeArgs& a) { return a.U32 ? a.U32 + OBJ * a.kU : nullptr; }
__device__ inline cf* m_V32(const MergeArgs& a) { return a.V32 ? a.V32 + OBJ * a.kV : nullptr; }
__device__ inline const cd* m_src(const MergeArgs& a) { return a.src + OBJ * a.kSrc; }
__device__ inline cd* m_nodeR(const MergeArgs& a) { return a.nodeR + OBJ * a.kNodeR; }
__device__ inline cd* m_nodeQ(const MergeArgs& a) { return a.nodeQ + OBJ * a.kNodeQ; }
__device__ inline int* m_nodecnt(const MergeArgs& a) { return a.nodecnt + OBJ * a.kNodeCnt; }
__device__ inline cd* m_chunkQ(const MergeArgs& a) { return a.chunkQ + OBJ * a.kChunkQ; }
__device__ inline cd* m_UK(const MergeArgs& a) { return a.UK + OBJ * a.kProbW2; }
__device__ inline cd* m_VR(const MergeArgs& a) { return a.VR + OBJ * a.kProbW2; }
__device__ inline double* m_Sold(const MergeArgs& a) { return a.Sold + OBJ * a.kProbW; }
__device__ inline int* m_rold(const MergeArgs& a) { return a.rold + OBJ * a.kProb; }

// the block's current (read) and updated (write) factor buffers
__device__ inline const cd* rd_U(const MergeArgs& a, const MergeBlk& B) { return a.Ur + OBJ * a.kU + B.rd * a.bU; }
__device__ inline const cd* rd_V(const MergeArgs& a, const MergeBlk& B) { return a.Vr + OBJ * a.kV + B.rd * a.bV; }
__device__ inline const double* rd_S(const MergeArgs& a, const MergeBlk& B) { return a.Sr + OBJ * a.kS + B.rd * a.bS; }
__device__ inline const int* rd_rank(const MergeArgs& a, const MergeBlk& B) {
    return a.rankr + OBJ * a.kRank + B.rd * a.bRank;
}
__device__ inline long long wr_buf(const MergeArgs& a, const MergeBlk& B) { return B.rd ^ a.flip; }
__device__ inline cd* wr_U(const MergeArgs& a, const MergeBlk& B) { return a.U + OBJ * a.kU + wr_buf(a, B) * a.bU; }
__device__ inline cd* wr_V(const MergeArgs& a, const MergeBlk& B) { return a.V + OBJ * a.kV + wr_buf(a, B) * a.bV; }
__device__ inline double* wr_S(const MergeArgs& a, const MergeBlk& B) { return a.S + OBJ * a.kS + wr_buf(a, B) * a.bS; }
__device__ inline int* wr_rank(const MergeArgs& a, const MergeBlk& B) {
    return a.rank + OBJ * a.kRank + wr_buf(a, B) * a.bRank;
}
__device__ inline cf* wr_U32(const MergeArgs& a, const MergeBlk& B) {
    return a.U32 ? m_U32(a) + wr_buf(a, B) * a.bU : nullptr;
}
__device__ inline cf* wr_V32(const MergeArgs& a, const MergeBlk& B) {
    return a.V32 ? m_V32(a) + wr_buf(a, B) * a.bV : nullptr;
}

// ranks come from device memory; every index derived from them is kept
// inside the capacity the host allocated, whatever the memory holds
__device__ inline int clamp_rank(int r, int cap) { return r < 0 ? 0 : (r > cap ? cap : r); }

struct Ctx {
    int slot, q, chunk;
    const MergeBlk* B;
};

__device__ inline Ctx decode_task(const MergeArgs& a, int task) {
    Ctx c{};
    int s = 0;
    while (s + 1 < a.nblk && task >= a.blk[s + 1].task_off) ++s;
    c.slot = s;
    c.B = &a.blk[s];
    int local = task - a.blk[s].task_off;
    c.q = local / c.B->nchunks;
    c.chunk = local % c.B->nchunks;
    return c;
}

__device__ inline size_t prob_index(const MergeArgs& a, const Ctx& c) {
    return (size_t)c.slot * a.npair + c.q;
}


// Build the chunk of Z = [V S, A_p^dagger] into LDS (column-major, CH rows,
// zero padded) and factor it.
template <int W>
__device__ void chunk_qr(const MergeArgs& a, const Ctx& c, int r_old, const double* s_old,
                         cd* A, cd* tau, double* red) {
    constexpr int CH = merge_ch(W);
    const MergeBlk& B = *c.B;
    const int w = r_old + a.pp;
    const int row0 = c.chunk * CH;
    const int nr = min(CH, B.ncols - row0);
    const cd* V = rd_V(a, B) + B.Voff + (size_t)c.q * a.RCr * B.ncols;
    for (int idx = threadIdx.x; idx < CH * w; idx += NT) {
        int col = idx / CH, i = idx % CH;
        cd z = mk(0.0, 0.0);
        if (i < nr) {
            int s = row0 + i;  // column of the block (relative)
            if (col < r_old) {
                z = s_old[col] * V[(size_t)col * B.ncols + s];
            } else {
                int pr = col - r_old;
                const size_t slot = (size_t)((a.src_first + pr) % a.src_ring);
                z = conj(m_src(a)[slot * a.src_row + (size_t)c.q * a.src_pair + B.c0 + s]);
            }
        }
        A[idx] = z;
    }
    __syncthreads();
    hh_qr<W>(A, CH, w, tau, red);
}

template <int W>
__global__ void __launch_bounds__(NT) merge_up_kernel(MergeArgs a) {
    constexpr int CH = merge_ch(W), NQ = node_q(W), CQ = chunk_q(W);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int XR = CH > 2 * W ? CH : 2 * W;
    cd* A = reinterpret_cast<cd*>(smem_raw);               // CH x W (also 2W x W, and M, J)
    cd* tau = A + (size_t)XR * W;                          // W
    double* red = reinterpret_cast<double*>(tau + W);      // 16
    cd* vbuf = reinterpret_cast<cd*>(red + 16);            // 2 XR: reflectors while Q is formed
    __shared__ int sflag;
    __shared__ double s_old[W];
    __shared__ double ssig[W];
    __shared__ int sperm[W];
    __shared__ int sbad;

    Ctx c = decode_task(a, blockIdx.x);
    const MergeBlk& B = *c.B;
    const size_t pidx = prob_index(a, c);
    const size_t fq = (size_t)B.b * a.npair + c.q;
    const int r_old = clamp_rank(rd_rank(a, B)[fq], min(a.RCr, W - a.pp));
    const int w = r_old + a.pp;
    for (int i = threadIdx.x; i < W; i += NT) s_old[i] = i < r_old ? rd_S(a, B)[fq * a.RCr + i] : 0.0;
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();

    chunk_qr<W>(a, c, r_old, s_old, A, tau, red);

    const long long nbase = B.node_base + (long long)c.q * B.nnodes;
    cd* nodeR = m_nodeR(a) + (size_t)nbase * W * W;
    cd* nodeQ = m_nodeQ(a) + (size_t)nbase * NQ;
    int* nodecnt = m_nodecnt(a) + nbase;
    {
        cd* dst = nodeR + (size_t)c.chunk * W * W;
        for (int e = threadIdx.x; e < W * W; e += NT) {
            int col = e / W, i = e % W;
            dst[e] = (col < w && i <= col) ? A[(size_t)col * CH + i] : mk(0.0, 0.0);
        }
    }
    __syncthreads();   // R is read before the explicit Q overwrites it
    hh_form_q<W>(A, CH, w, tau, vbuf);
    {   // keep the chunk's explicit Q (CH x w) for merge_down
        cd* cq = m_chunkQ(a) + (size_t)(B.chunk_base + (long long)c.q * B.nchunks + c.chunk) * CQ;
        for (int e = threadIdx.x; e < CH * w; e += NT) cq[e] = A[e];
    }
    __threadfence();
    __syncthreads();

    int idx = c.chunk, L = 0, cnt = B.nchunks;
    while (cnt > 1) {
        const int parent = idx >> 1;
        const int offL = tree_levoff(B.nchunks, L), offP = tree_levoff(B.nchunks, L + 1);
        if ((idx ^ 1) < cnt) {
            if (threadIdx.x == 0) sflag = atomicAdd(&nodecnt[offP + parent], 1);
            __syncthreads();
            if (sflag == 0) return;  // first to arrive: the sibling finishes this node
            __threadfence();
            if (threadIdx.x == 0) nodecnt[offP + parent] = 0;
            const cd* rl = nodeR + (size_t)(offL + 2 * parent) * W * W;
            const cd* rr = nodeR + (size_t)(offL + 2 * parent + 1) * W * W;
            const int nr2 = 2 * w;
            for (int e = threadIdx.x; e < nr2 * w; e += NT) {
                int col = e / nr2, i = e % nr2;
                A[e] = (i < w) ? rl[(size_t)col * W + i] : rr[(size_t)col * W + (i - w)];
            }
            __syncthreads();
            hh_qr<W>(A, nr2, w, tau, red);
            cd* dst = nodeR + (size_t)(offP + parent) * W * W;
            for (int e = threadIdx.x; e < W * W; e += NT) {
                int col = e / W, i = e % W;
                dst[e] = (col < w && i <= col) ? A[(size_t)col * nr2 + i] : mk(0.0, 0.0);
            }
            __syncthreads();   // R is read before the explicit Q overwrites it
            hh_form_q<W>(A, nr2, w, tau, vbuf);
            cd* qd = nodeQ + (size_t)(offP + parent) * NQ;   // explicit Q (2w x w)
            for (int e = threadIdx.x; e < nr2 * w; e += NT) qd[e] = A[e];
            __threadfence();
            __syncthreads();
        } else {
            const cd* src = nodeR + (size_t)(offL + idx) * W * W;
            cd* dst = nodeR + (size_t)(offP + parent) * W * W;
            for (int e = threadIdx.x; e < W * W; e += NT) dst[e] = src[e];
            __threadfence();
            __syncthreads();
        }
        idx = parent;
        cnt = (cnt + 1) / 2;
        ++L;
    }

    // root: one-sided Jacobi SVD of R^dagger, truncation, commit rank and S
    const cd* R = nodeR + (size_t)tree_levoff(B.nchunks, L) * W * W;
    const int ne = (w + 1) & ~1;
    cd* M = A;
    cd* J = A + (size_t)ne * ne;
    for (int e = threadIdx.x; e < ne * ne; e += NT) {
        int col = e / ne, i = e % ne;  // M[i][col] = conj(R[col][i])
        M[e] = (i < w && col < w) ? conj(R[(size_t)i * W + col]) : mk(0.0, 0.0);
    }
    __syncthreads();
    jacobi_svd(M, J, ne, &sflag, red);
    for (int i = threadIdx.x; i < ne; i += NT) {
        double s = 0.0;
        for (int r = 0; r < ne; ++r) s += norm2(M[(size_t)i * ne + r]);
        bool bad = false;
        ssig[i] = trunc_key(sqrt(s), &bad);
        if (bad) sbad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && sbad) atomicOr(a.err, 2);
    // descending order; all keys are finite, so this is a permutation of 0..ne-1
    for (int i = threadIdx.x; i < ne; i += NT) sperm[trunc_position(ssig, ne, i)] = i;
    __syncthreads();
    bool over = false;
    const int rnew = trunc_rank(ssig, sperm, ne, a.tol, a.RC, &over);
    if (threadIdx.x == 0) {
        if (over) atomicOr(a.err, 1);
        m_rold(a)[pidx] = r_old;
        wr_rank(a, B)[fq] = rnew;
    }
    for (int i = threadIdx.x; i < W; i += NT) m_Sold(a)[pidx * W + i] = s_old[i];
    for (int i = threadIdx.x; i < a.RC; i += NT) wr_S(a, B)[fq * a.RC + i] = i < rnew ? ssig[sperm[i]] : 0.0;
    cd* UK = m_UK(a) + pidx * W * W;
    cd* VR = m_VR(a) + pidx * W * W;
    for (int e = threadIdx.x; e < w * rnew; e += NT) {
        int col = e / w, i = e % w;
        int src = min(max(sperm[col], 0), ne - 1);
        double inv = 1.0 / ssig[src];
        UK[(size_t)col * W + i] = inv * M[(size_t)src * ne + i];
        VR[(size_t)col * W + i] = J[(size_t)src * ne + i];
    }
}

template <int W>
__global__ void __launch_bounds__(NT) merge_down_kernel(MergeArgs a) {
    constexpr int CH = merge_ch(W), NQ = node_q(W), CQ = chunk_q(W);
    constexpr int YPT = (W * W + NT - 1) / NT;   // entries of T per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // V_R pulled down the tree: at each level the half of the node's explicit Q that
    // belongs to this chunk's side times T, then the chunk's explicit Q times T gives
    // the chunk's rows of V' (plain products, the Q factors read from global memory)
    cd* T = reinterpret_cast<cd*>(smem_raw);   // W x W (column-major, ld W)

    if ((int)blockIdx.x < a.ntask_v) {
        Ctx c = decode_task(a, blockIdx.x);
        const MergeBlk& B = *c.B;
        const size_t pidx = prob_index(a, c);
        const size_t fq = (size_t)B.b * a.npair + c.q;
        const int r_old = clamp_rank(m_rold(a)[pidx], min(a.RCr, W - a.pp));
        const int rnew = clamp_rank(wr_rank(a, B)[fq], a.RC);
        const int w = r_old + a.pp;
        // the chunk's explicit Q from merge_up (CH x w, column-major)
        const cd* cq = m_chunkQ(a) + (size_t)(B.chunk_base + (long long)c.q * B.nchunks + c.chunk) * CQ;
        const cd* VR = m_VR(a) + pidx * W * W;
        for (int e = threadIdx.x; e < W * W; e += NT) {
            int col = e / W, i = e % W;
            T[e] = (col < rnew && i < w) ? VR[(size_t)col * W + i] : mk(0.0, 0.0);
        }
        __syncthreads();
        const long long nbase = B.node_base + (long long)c.q * B.nnodes;
        const cd* nodeQ = m_nodeQ(a) + (size_t)nbase * NQ;
        int depth = 0;
        for (int cnt = B.nchunks; cnt > 1; cnt = (cnt + 1) / 2) ++depth;
        for (int L = depth; L >= 1; --L) {
            int cntBelow = B.nchunks;
            for (int i = 0; i < L - 1; ++i) cntBelow = (cntBelow + 1) / 2;
            const int node = c.chunk >> L;
            const int child = c.chunk >> (L - 1);
            if (2 * node + 1 >= cntBelow) continue;  // single child: Q = identity
            const int slot = child & 1;
            const int nr2 = 2 * w;
            // T <- Q_node[slot w .. slot w + w - 1, 0 .. w - 1] T
            const cd* Qn = nodeQ + (size_t)(tree_levoff(B.nchunks, L) + node) * NQ + slot * w;
            cd y[YPT];
#pragma unroll
            for (int u = 0; u < YPT; ++u) {
                const int e = threadIdx.x + u * NT;
                y[u] = mk(0.0, 0.0);
                if (e < w * rnew) {
                    const int col = e / w, i = e % w;
                    cd acc = mk(0.0, 0.0);
                    for (int kk = 0; kk < w; ++kk) fma_(acc, Qn[(size_t)kk * nr2 + i], T[(size_t)col * W + kk]);
                    y[u] = acc;
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < YPT; ++u) {
                const int e = threadIdx.x + u * NT;
                if (e < w * rnew) T[(size_t)(e / w) * W + e % w] = y[u];
            }
            __syncthreads();
        }
        // the chunk's rows of V' = Q_chunk T
        const int row0 = c.chunk * CH;
        const int nr = min(CH, B.ncols - row0);
        const size_t vo = B.Voff + (size_t)c.q * a.RC * B.ncols;
        cd* V = wr_V(a, B) + vo;
        cf* V32 = a.V32 ? wr_V32(a, B) + vo : nullptr;
        for (int e = threadIdx.x; e < nr * rnew; e += NT) {
            int col = e / nr, i = e % nr;
            cd x = mk(0.0, 0.0);
            for (int kk = 0; kk < w; ++kk) fma_(x, cq[(size_t)kk * CH + i], T[(size_t)col * W + kk]);
            V[(size_t)col * B.ncols + row0 + i] = x;
            if (V32) V32[(size_t)col * B.ncols + row0 + i] = from_cd<cf>(x);
        }
        return;
    }
    // U rows: old rows U' = U U_K[0:r_old, :], new rows U' = U_K[r_old + i, :]
    const int t = blockIdx.x - a.ntask_v;
    int s = 0;
    while (s + 1 < a.nblk && t >= a.blk[s + 1].utask_off) ++s;
    const MergeBlk& B = a.blk[s];
    const int local = t - B.utask_off;
    const int q = local / B.nutask, ut = local % B.nutask;
    const size_t pidx = (size_t)s * a.npair + q;
    const size_t fq = (size_t)B.b * a.npair + q;
    const int r_old = clamp_rank(m_rold(a)[pidx], min(a.RCr, W - a.pp));
    const int rnew = clamp_rank(wr_rank(a, B)[fq], a.RC);
    const cd* UK = m_UK(a) + pidx * W * W;
    const cd* Uold = rd_U(a, B) + B.Uoff + (size_t)q * a.RCr * B.ldU;
    const size_t uo = B.Uoff + (size_t)q * a.RC * B.ldU;
    cd* U = wr_U(a, B) + uo;
    cf* U32 = a.U32 ? wr_U32(a, B) + uo : nullptr;
    const int row = ut * NT + threadIdx.x;
    const int nrows = B.kb + a.pp;
    if (row >= nrows) return;
    if (row < B.kb) {
        cd u[W];
#pragma unroll
        for (int r = 0; r < W; ++r) u[r] = (r < r_old) ? Uold[(size_t)r * B.ldU + row] : mk(0.0, 0.0);
        for (int col = 0; col < rnew; ++col) {
            cd acc = mk(0.0, 0.0);
#pragma unroll
            for (int r = 0; r < W; ++r)
                if (r < r_old) fma_(acc, u[r], UK[(size_t)col * W + r]);
            U[(size_t)col * B.ldU + row] = acc;
            if (U32) U32[(size_t)col * B.ldU + row] = from_cd<cf>(acc);
        }
    } else {
        const int pr = r_old + (row - B.kb);
        for (int col = 0; col < rnew; ++col) {
            const cd x = UK[(size_t)col * W + pr];
            U[(size_t)col * B.ldU + row] = x;
            if (U32) U32[(size_t)col * B.ldU + row] = from_cd<cf>(x);
        }
    }
}

template <int W>
size_t merge_up_smem() {
    constexpr int CH = merge_ch(W), XR = CH > 2 * W ? CH : 2 * W;
    return (size_t)XR * W * sizeof(cd) + (size_t)W * sizeof(cd) + 16 * sizeof(double) + (size_t)2 * XR * sizeof(cd);
}
template <int W>
size_t merge_down_smem(int RC) {
    (void)RC;
    return (size_t)W * W * sizeof(cd);
}

template <int W>
hipError_t launch_merge_w(const MergeArgs& a, int nk, hipStream_t st) {
    merge_up_kernel<W><<<dim3(a.ntask_v, nk), NT, merge_up_smem<W>(), st>>>(a);
    merge_down_kernel<W><<<dim3(a.ntask_v + a.ntask_u, nk), NT, merge_down_smem<W>(a.RC), st>>>(a);
    return hipGetLastError();
}

struct FlipList {
    int n;
    int b[kMaxMergeBlk];
};

__global__ void flip_kernel(int* cur, FlipList f) {
    const int i = threadIdx.x;
    if (i < f.n) cur[f.b[i]] ^= 1;
}

__global__ void fill_int_kernel(int* p, long long n, int v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_merge(const MergeArgs& a, int nk, hipStream_t st) {
    if (a.ntask_v == 0) return hipSuccess;
    if (a.RC < 1 || a.RC > a.W || a.pp < 1 || a.pp >= a.W) return hipErrorInvalidValue;
    for (int i = 0; i < a.nblk; ++i)   // every tree node of a problem has its own slot
        if (a.blk[i].nnodes < tree_nodes(a.blk[i].nchunks)) return hipErrorInvalidValue;
    if (a.W == kWSmall) return launch_merge_w<kWSmall>(a, nk, st);
    if (a.W == kWLarge) return launch_merge_w<kWLarge>(a, nk, st);
    return hipErrorInvalidValue;
}

hipError_t launch_flip(int* cur, const int* blocks, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n > kMaxMergeBlk) return hipErrorInvalidValue;
    FlipList f{};
    f.n = n;
    for (int i = 0; i < n; ++i) f.b[i] = blocks[i];
    flip_kernel<<<1, 64, 0, st>>>(cur, f);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    fill_int_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t merge_init() {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f, size_t bytes) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    };
    set((const void*)merge_up_kernel<kWSmall>, merge_up_smem<kWSmall>());
    set((const void*)merge_down_kernel<kWSmall>, merge_down_smem<kWSmall>(kWSmall));
    set((const void*)merge_up_kernel<kWLarge>, merge_up_smem<kWLarge>());
    set((const void*)merge_down_kernel<kWLarge>, merge_down_smem<kWLarge>(kWLarge));
    return e;
}

}  // namespace hn
