// History integrals at step n over HODLR storage.
//
// For every m <= n (right-hand sides of the retarded and lesser Kadanoff-Baym
// equations, Gregory weights from the appendix on integration):
//   I^R(n,m) = h sum_{j=m..n} w^{(n-m)}_{j-m} Sigma^R(n,j) G^R(j,m)
//   I^<(n,m) = h sum_{s<=n} w^{(n)}_s Sigma^R(n,s) G^<(s,m)
//            + h sum_{s<=m} w^{(m)}_s Sigma^<(n,s) G^A(s,m)
// The weights differ from one only within k+1 points of an interval end, so
// the weights that depend on n alone are folded into the Sigma rows:
//   x (j) = (1 + (omega_{n-j} - 1)[n-j <= k]) Sigma^R(n,j)       (retarded)
//   x1(s) = w^{(n)}_s Sigma^R(n,s)                               (lesser, 1st term)
//   x2(s) = (1 + (omega_s - 1)[s <= k]) Sigma^<(n,s)             (lesser, 2nd term)
// and the rest (start weights of I^R, end weights of the second lesser term,
// and intervals shorter than k) becomes a band correction on the dense band
// G^R(m+i, m), i <= k.  The folded row then multiplies the stored lower
// triangles piece by piece:
//   dense leaves     column sums and row dots of each leaf triangle
//   dense tail rows  rows appended since the last compression panel
//   HODLR blocks     per orbital pair, project the row onto one factor
//                    (x U or x V, scaled by S), then expand with the other.
// Kernel 1 (hist_tasks) does the projections, leaves and tail rows as a flat
// list of workgroup tasks; kernel 2 (hist_combine) expands, adds the pieces
// and the band corrections for each output column m.
#include "history.h"

#include <type_traits>

namespace hn {

namespace {

constexpr int NT = 256;

__device__ inline double wsum64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// task id -> (group, member) so that the members of a group land on one XCD
// (workgroups are dealt round-robin over the 8 XCDs) and share its L2
__device__ inline bool xcd_group(int id, int ngroups, int nmem, int& g, int& mem) {
    const int blk = id / (8 * nmem), rem = id % (8 * nmem);
    mem = rem / 8;
    g = blk * 8 + rem % 8;
    return g < ngroups;
}

// acc[idx] += v with a run-time idx, without dynamic register indexing
template <int N>
__device__ inline void add_at(cd (&acc)[N], int idx, cd v) {
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i == idx) acc[i] = acc[i] + v;
}

// per-object data of object blockIdx.y of a batch (the kernel arguments
// hold object 0 and the strides)
#define OBJ ((long long)blockIdx.y)
__device__ inline const cd* p_sigR(const HistArgs& A) { return A.sigR ? A.sigR + OBJ * A.kIn : nullptr; }
__device__ inline const cd* p_sigL(const HistArgs& A) { return A.sigL ? A.sigL + OBJ * A.kIn : nullptr; }
// Sigma^R(n, j) with the orbital indices swapped ([j][b][a], norb 16 only)
__device__ inline const cd* p_sigRT(const HistArgs& A) { return A.sigRT + OBJ * A.kInT; }
__device__ inline cd* p_outR(const HistArgs& A) { return A.outR ? A.outR + OBJ * A.kOut : nullptr; }
__device__ inline cd* p_outL(const HistArgs& A) { return A.outL ? A.outL + OBJ * A.kOut : nullptr; }
// factor buffer holding block b's current TSVD
__device__ inline long long buf_of(const HistArgs& A, int c, int b) { return A.cur[c][b] & 1; }
template <class FT>
__device__ inline const FT* p_U(const HistArgs& A, int c, int b) {
    return static_cast<const FT*>(A.U[c]) + OBJ * A.kU + buf_of(A, c, b) * A.bU;
}
template <class FT>
__device__ inline const FT* p_V(const HistArgs& A, int c, int b) {
    return static_cast<const FT*>(A.V[c]) + OBJ * A.kV + buf_of(A, c, b) * A.bV;
}
__device__ inline const double* p_S(const HistArgs& A, int c, int b) {
    return A.S[c] + OBJ * A.kS + buf_of(A, c, b) * A.bS;
}
__device__ inline const int* p_rank(const HistArgs& A, int c, int b) {
    return A.rank[c] + OBJ * A.kRank + buf_of(A, c, b) * A.bRank;
}
__device__ inline const cd* p_leaf(const HistArgs& A, int c) { return A.leaf[c] + OBJ * A.kLeaf; }
__device__ inline const cd* p_tail(const HistArgs& A, int c) { return A.tail[c] + OBJ * A.kTail; }
__device__ inline cd* p_tailcol(const HistArgs& A, int c) { return A.tailcol[c] + OBJ * A.kTailcol; }
__device__ inline cd* p_tailpart(const HistArgs& A, int c) { return A.tailpart[c] + OBJ * A.kTailpart; }
__device__ inline cd* p_tailrow(const HistArgs& A, int c) { return A.tailrow[c] + OBJ * A.kTailrow; }
__device__ inline const cd* p_band(const HistArgs& A) { return A.band + OBJ * A.kBand; }
__device__ inline cd* p_proj(const HistArgs& A) { return A.proj + OBJ * A.kProj; }
__device__ inline cd* p_part(const HistArgs& A) { return A.part + OBJ * A.kPart; }
__device__ inline cd* p_leafR(const HistArgs& A) { return A.leafR + OBJ * A.kLeafOut; }
__device__ inline cd* p_leafLR(const HistArgs& A) { return A.leafLR + OBJ * A.kLeafOut; }
__device__ inline cd* p_leafLL(const HistArgs& A) { return A.leafLL + OBJ * A.kLeafOutLL; }

// ranks come from device memory: clamp them to the allocated capacity
__device__ inline int rank_of(const HistArgs& A, int comp, int b, int q) {
    const int r = p_rank(A, comp, b)[(size_t)b * A.npair + q];
    return r < 0 ? 0 : (r > A.RC ? A.RC : r);
}

__device__ inline size_t proj_slot(const HistArgs& A, int comp, int b, int q, int which) {
    return (((size_t)comp * A.nb + b) * A.npair + q) * 2 + which;
}

// left orbital indices handled by one workgroup (one wave each) and the
// number of such groups
template <int NORB>
struct AGroups {
    static constexpr int AG = NORB < 4 ? NORB : 4;
    static constexpr int NG = NORB / AG;
};
// orbital-pair groups of a leaf, each a workgroup with its own output slot
template <int NORB>
struct LeafGroups {
    static constexpr int LG = leaf_groups(NORB);
};

// ---------------------------------------------------------------------------
// Projection of rows [chunk*kch, +kch) of U (which = 0, rows merged so far) or
// V (which = 1) of one block and orbital pair onto the folded Sigma row, scaled
// by S; the chunk partials are summed by proj_reduce.
// Lane layout: lane = g * RP + rl covers rank rp + rl of a pass of RP ranks and
// row group g of LPR = 64 / RP groups; wave w takes the groups w*LPR .. +LPR, so
// the 4 waves interleave 4*LPR row groups and a wave's load of one step reads RP
// factor columns over LPR consecutive rows.  Each thread sums its rows for all
// NORB left orbitals; the row groups are then summed by shuffles inside the wave
// (log2(LPR) steps) and the waves through LDS.
template <int NORB, class FT, int RP, class Stage>
__device__ void fact_pass(const HistArgs& A, const FT* F, int ld, int i0, int i1, int rk, bool cj, const cd* xs,
                          const double* S, cd* out, cd* red, Stage stage) {
    constexpr int LPR = 64 / RP, G = 4 * LPR;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rl = lane % RP, g = wave * LPR + lane / RP;
    // the first four rows of the first pass are loaded while the Sigma rows are staged
    cd f0[4];
    {
        const FT* Fr = F + (size_t)min(rl, rk - 1) * ld;
#pragma unroll
        for (int u = 0; u < 4; ++u) f0[u] = to_cd(Fr[min(i0 + g + u * G, i1 - 1)]);
    }
    stage();
    __syncthreads();
    for (int rp = 0; rp < rk; rp += RP) {
        const int r = rp + rl;
        const bool rv = r < rk;
        const FT* Fr = F + (size_t)min(r, rk - 1) * ld;
        cd acc[NORB];
#pragma unroll
        for (int a = 0; a < NORB; ++a) acc[a] = mk(0.0, 0.0);
        // four rows per step with their loads issued together; indices are clamped so
        // that every load is in range and out-of-range terms are zeroed
        for (int i = i0 + g; i < i1; i += 4 * G) {
            cd f[4];
            if (rp == 0 && i == i0 + g) {
#pragma unroll
                for (int u = 0; u < 4; ++u) f[u] = f0[u];
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) f[u] = to_cd(Fr[min(i + u * G, i1 - 1)]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int iu = i + u * G;
                if (iu < i1 && rv) {
                    const cd fv = cj ? conj(f[u]) : f[u];
                    const cd* x = xs + (size_t)(iu - i0) * NORB;
#pragma unroll
                    for (int a = 0; a < NORB; ++a) fma_(acc[a], x[a], fv);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
#pragma unroll
            for (int off = RP; off < 64; off <<= 1) {
                acc[a].x += __shfl_xor(acc[a].x, off, 64);
                acc[a].y += __shfl_xor(acc[a].y, off, 64);
            }
        }
        __syncthreads();   // red is free (previous pass consumed)
        if (lane < RP)   // red[(a * 4 + wave) * RP + rl]: consecutive lanes, consecutive words
#pragma unroll
            for (int a = 0; a < NORB; ++a) red[((size_t)a * 4 + wave) * RP + rl] = acc[a];
        __syncthreads();
        if (wave == 0 && lane < RP && rv) {
            cd sum[NORB];
#pragma unroll
            for (int a = 0; a < NORB; ++a) sum[a] = red[((size_t)a * 4) * RP + rl];
            for (int ww = 1; ww < 4; ++ww)
#pragma unroll
                for (int a = 0; a < NORB; ++a) sum[a] = sum[a] + red[((size_t)a * 4 + ww) * RP + rl];
            const double sr = S[r];
#pragma unroll
            for (int a = 0; a < NORB; ++a) out[(size_t)a * A.RC + r] = sr * sum[a];
        }
    }
}

template <int NORB, class FT>
__device__ void fact_task(const HistArgs& A, const FactTask& t, unsigned char* smem) {
    const int comp = t.comp, b = t.b, q = t.q, which = t.which;
    if (comp == 0 && which == 0 && !A.wantR) return;
    if ((comp == 1 || which == 1) && !A.wantL) return;
    if (comp == 1 && A.adj) return;
    constexpr int npair = NORB * NORB;
    const int RC = A.RC;
    const int qr = q / NORB, qc = q % NORB;
    const int rk = rank_of(A, comp, b, q);
    if (rk == 0) return;
    const int* bk = A.blk + 5 * b;
    const int r0 = bk[1], r1 = bk[2], c0 = bk[3], c1 = bk[4];
    int len, base, ld;
    const FT* F;
    if (which == 0) {
        len = min(A.n0[comp] - r0, r1 - r0);
        base = r0;
        ld = r1 - r0;
        F = p_U<FT>(A, comp, b) + A.Uoff[b] + (size_t)q * RC * ld;
    } else {
        len = c1 - c0;
        base = c0;
        ld = c1 - c0;
        F = p_V<FT>(A, comp, b) + A.Voff[b] + (size_t)q * RC * ld;
    }
    const int kCH = A.kch;
    const int i0 = t.chunk * kCH, i1 = min(len, i0 + kCH);
    if (i0 >= i1) return;
    const int n = A.n;
    // folded Sigma entry multiplying row i of the factor, left orbital a
    auto xval = [&](int i, int a) -> cd {
        const int j = base + i;
        if (comp == 0 && which == 0) return w_end(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + qr];
        if (comp == 0) {
            if (A.adj) return p_sigL(A)[(size_t)j * npair + a * NORB + qc];   // Ibar(n, j)[a][qc]
            return -w_start(A.W, j) * conj(p_sigL(A)[(size_t)j * npair + qc * NORB + a]);
        }
        return interval_w(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + (which == 0 ? qc : qr)];
    };
    cd* xs = reinterpret_cast<cd*>(smem);   // kCH x NORB
    cd* red = xs + (size_t)kCH * NORB;       // 4 waves x 32 ranks x NORB
    auto stage = [&]() {
        for (int e = threadIdx.x; e < (i1 - i0) * NORB; e += NT) xs[e] = xval(i0 + e / NORB, e % NORB);
    };
    const double* S = p_S(A, comp, b) + ((size_t)b * npair + q) * RC;
    const size_t slot = proj_slot(A, comp, b, q, which);
    cd* out = p_part(A) + (size_t)(A.partoff[slot] + t.chunk) * NORB * RC;
    const bool cj = (comp == 1);
    if (rk <= 4) fact_pass<NORB, FT, 4>(A, F, ld, i0, i1, rk, cj, xs, S, out, red, stage);
    else if (rk <= 8) fact_pass<NORB, FT, 8>(A, F, ld, i0, i1, rk, cj, xs, S, out, red, stage);
    else if (rk <= 16) fact_pass<NORB, FT, 16>(A, F, ld, i0, i1, rk, cj, xs, S, out, red, stage);
    else fact_pass<NORB, FT, 32>(A, F, ld, i0, i1, rk, cj, xs, S, out, red, stage);
}

// ---------------------------------------------------------------------------
// Projections at norb = 4: one task per (block, factor, chunk, orbital index beta)
// takes the 4 orbital pairs whose folded Sigma entries carry the same beta: their
// common folded row X is staged once in LDS and wave w projects pair o = w alone.
// Lane layout of a wave: lane = g * RP + rl covers rank rp + rl of a pass of RP
// ranks and row group g of LPR = 64 / RP; a step takes four rows per lane with
// their loads issued together; the row groups are summed by shuffles, so a wave
// needs no barrier after the staging.  Surplus rank lanes compute on clamped
// (in-range) loads and are never written.
template <int NORB, class FT, int RP>
__device__ void fact_wave(const FT* F, int ld, int i0, int i1, int rk, bool cj, const cd* xs, const double* S,
                          cd* out, int RC) {
    constexpr int LPR = 64 / RP;
    const int lane = threadIdx.x & 63, rl = lane % RP, g = lane / RP;
    for (int rp = 0; rp < rk; rp += RP) {
        const int r = rp + rl;
        const FT* Fr = F + (size_t)min(r, rk - 1) * ld;
        cd acc[NORB];
#pragma unroll
        for (int a = 0; a < NORB; ++a) acc[a] = mk(0.0, 0.0);
        for (int i = i0 + g; i < i1; i += 4 * LPR) {
            cd f[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) f[u] = to_cd(Fr[min(i + u * LPR, i1 - 1)]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int iu = i + u * LPR;
                if (iu < i1) {
                    const cd fv = cj ? conj(f[u]) : f[u];
                    const cd* x = xs + (size_t)(iu - i0) * NORB;
#pragma unroll
                    for (int a = 0; a < NORB; ++a) fma_(acc[a], x[a], fv);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
#pragma unroll
            for (int off = RP; off < 64; off <<= 1) {
                acc[a].x += __shfl_xor(acc[a].x, off, 64);
                acc[a].y += __shfl_xor(acc[a].y, off, 64);
            }
        }
        if (g == 0 && r < rk) {
            const double sr = S[r];
#pragma unroll
            for (int a = 0; a < NORB; ++a) out[(size_t)a * RC + r] = sr * acc[a];
        }
    }
}

template <int NORB, class FT>
__device__ void fact_task_beta(const HistArgs& A, const FactTask& t, unsigned char* smem) {
    static_assert(NORB == 4, "one wave per orbital pair of a shared index");
    const int comp = t.comp, b = t.b, beta = t.q, which = t.which;
    if (comp == 0 && which == 0 && !A.wantR) return;
    if ((comp == 1 || which == 1) && !A.wantL) return;
    if (comp == 1 && A.adj) return;
    constexpr int npair = NORB * NORB;
    const int RC = A.RC;
    const int* bk = A.blk + 5 * b;
    const int r0 = bk[1], r1 = bk[2], c0 = bk[3], c1 = bk[4];
    int len, base, ld;
    const FT* F;
    if (which == 0) {
        len = min(A.n0[comp] - r0, r1 - r0);
        base = r0;
        ld = r1 - r0;
        F = p_U<FT>(A, comp, b) + A.Uoff[b];
    } else {
        len = c1 - c0;
        base = c0;
        ld = c1 - c0;
        F = p_V<FT>(A, comp, b) + A.Voff[b];
    }
    const int kCH = A.kch;
    const int i0 = t.chunk * kCH, i1 = min(len, i0 + kCH);
    if (i0 >= i1) return;
    const int n = A.n;
    cd* xs = reinterpret_cast<cd*>(smem);   // kCH x NORB
    for (int e = threadIdx.x; e < (i1 - i0) * NORB; e += NT) {
        const int i = e / NORB, a = e % NORB, j = base + i0 + i;
        cd v;
        if (comp == 0 && which == 0) v = w_end(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + beta];
        else if (comp == 0) v = A.adj ? p_sigL(A)[(size_t)j * npair + a * NORB + beta]
                                      : -w_start(A.W, j) * conj(p_sigL(A)[(size_t)j * npair + beta * NORB + a]);
        else v = interval_w(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + beta];
        xs[e] = v;
    }
    __syncthreads();
    const int o = threadIdx.x >> 6;
    const int q = (comp ^ which) ? o * NORB + beta : beta * NORB + o;
    const int rk = rank_of(A, comp, b, q);
    if (rk == 0) return;
    const FT* Fq = F + (size_t)q * RC * ld;
    const double* S = p_S(A, comp, b) + ((size_t)b * npair + q) * RC;
    cd* out = p_part(A) + (size_t)(A.partoff[proj_slot(A, comp, b, q, which)] + t.chunk) * NORB * RC;
    const bool cj = (comp == 1);
    if (rk <= 4) fact_wave<NORB, FT, 4>(Fq, ld, i0, i1, rk, cj, xs, S, out, RC);
    else if (rk <= 8) fact_wave<NORB, FT, 8>(Fq, ld, i0, i1, rk, cj, xs, S, out, RC);
    else if (rk <= 16) fact_wave<NORB, FT, 16>(Fq, ld, i0, i1, rk, cj, xs, S, out, RC);
    else fact_wave<NORB, FT, 32>(Fq, ld, i0, i1, rk, cj, xs, S, out, RC);
}

// ---------------------------------------------------------------------------
// Projections of the FP32-factor form at norb = 16 on the matrix cores.  For one
// block, component, factor and chunk of kch rows, the 16 orbital pairs whose
// folded Sigma entries carry the same orbital index beta share one folded row:
// with X[i][a] = x_{a,beta}(row i) the projection of pair q is the product
// Z_q = X^T F_q (16 left orbitals x rank), a complex 16 x 16 x rows product done
// as four real v_mfma_f32_16x16x4f32 chains (re.re, im.im, re.im, im.re) with
// FP32 inputs and FP32 accumulation.  X is staged once in LDS as complex float;
// each wave takes four pairs and streams their factor columns, the next 32-row
// tile's loads in flight while the current tile is multiplied.  Each tile's sum
// is added to the running FP32 sum with TwoSum compensation, so the chunk sum
// carries the rounding of one tile, not of the whole chunk.
// Lane layout of the 16x16x4 products: A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, D[i][j] in lane j + 16 (i / 4), register i % 4.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline v4f mfma_16x16x4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// s += v, the rounding error of the addition added to e (TwoSum)
__device__ inline void two_sum_acc(float& s, float& e, float v) {
    const float t = s + v;
    const float bp = t - s;
    e += (s - (t - bp)) + (v - bp);
    s = t;
}

constexpr int kXS = 16;   // LDS row stride of staged X in complex floats: the consecutive
                          // rows that one read touches fall in alternate bank halves
constexpr int kPT = 32;   // factor rows per tile

// Z(a, r) = S_r sum_i X[i][a] op(F[r*ld + i]) over rows [i0, i1) for one pair, op =
// conj for CONJ; written to out[a*RC + r] for r < rk.  The staged X rows past i1
// are zero and every factor index is clamped into [i0, i1) x [0, rk), so all
// loads are in range and the surplus terms vanish.
template <bool CONJ>
__device__ void fact_mfma_pair(const cf* F, int ld, int i0, int i1, int rk, const cf* xs, const double* S,
                               cd* out, int RC) {
    const int lane = threadIdx.x & 63, j = lane & 15, kk = lane >> 4;
    const int ntile = (i1 - i0 + kPT - 1) / kPT;
    const cf* Fj = F + (size_t)min(j, rk - 1) * ld;
    float sr[4] = {0.f, 0.f, 0.f, 0.f}, er[4] = {0.f, 0.f, 0.f, 0.f};
    float si[4] = {0.f, 0.f, 0.f, 0.f}, ei[4] = {0.f, 0.f, 0.f, 0.f};
    cf bc[8], bn[8];
    // K step s of tile t takes rows t*kPT + 4s + kk: one load instruction reads four
    // consecutive rows of each of the 16 columns
    auto load = [&](cf (&bb)[8], int t) {
        const int r = i0 + t * kPT + kk;
#pragma unroll
        for (int s = 0; s < 8; ++s) bb[s] = Fj[min(r + 4 * s, i1 - 1)];
    };
    load(bc, 0);
    for (int t = 0; t < ntile; ++t) {
        if (t + 1 < ntile) load(bn, t + 1);
        v4f rr = {0.f, 0.f, 0.f, 0.f}, ii = rr, ri = rr, ir = rr;
        const cf* xt = xs + (size_t)(t * kPT + kk) * kXS + j;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const cf x = xt[4 * s * kXS];
            rr = mfma_16x16x4(x.x, bc[s].x, rr);
            ii = mfma_16x16x4(x.y, bc[s].y, ii);
            ri = mfma_16x16x4(x.x, bc[s].y, ri);
            ir = mfma_16x16x4(x.y, bc[s].x, ir);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            two_sum_acc(sr[v], er[v], CONJ ? rr[v] + ii[v] : rr[v] - ii[v]);
            two_sum_acc(si[v], ei[v], CONJ ? ir[v] - ri[v] : ri[v] + ir[v]);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) bc[s] = bn[s];
    }
    if (j < rk) {
        const double sj = S[j];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            out[(size_t)(4 * kk + v) * RC + j] =
                sj * mk((double)sr[v] + (double)er[v], (double)si[v] + (double)ei[v]);
    }
}

// One task: block b, component comp, factor `which`, chunk, orbital index beta = t.q.
// The pairs sharing beta: q = beta*16 + o when the folded row takes the pair's row
// orbital (retarded U, lesser V), q = o*16 + beta when it takes the column orbital.
__device__ void fact_mfma_task(const HistArgs& A, const FactTask& t, unsigned char* smem) {
    constexpr int NORB = 16, npair = 256;
    const int comp = t.comp, b = t.b, beta = t.q, which = t.which;
    if (comp == 0 && which == 0 && !A.wantR) return;
    if ((comp == 1 || which == 1) && !A.wantL) return;
    if (comp == 1 && A.adj) return;
    const int RC = A.RC;
    const int* bk = A.blk + 5 * b;
    const int r0 = bk[1], r1 = bk[2], c0 = bk[3], c1 = bk[4];
    int len, base, ld;
    const cf* F;
    if (which == 0) {
        len = min(A.n0[comp] - r0, r1 - r0);
        base = r0;
        ld = r1 - r0;
        F = p_U<cf>(A, comp, b) + A.Uoff[b];
    } else {
        len = c1 - c0;
        base = c0;
        ld = c1 - c0;
        F = p_V<cf>(A, comp, b) + A.Voff[b];
    }
    const int kCH = A.kch;
    const int i0 = t.chunk * kCH, i1 = min(len, i0 + kCH);
    if (i0 >= i1) return;
    const int n = A.n, nrow = i1 - i0, nst = (nrow + kPT - 1) / kPT * kPT;
    cf* xs = reinterpret_cast<cf*>(smem);   // nst x kXS
    for (int e = threadIdx.x; e < nst * NORB; e += NT) {
        const int i = e >> 4, a = e & 15, jj = base + i0 + i;
        cd v = mk(0.0, 0.0);
        if (i < nrow) {
            if (comp == 0 && which == 0) v = w_end(A.W, n, jj) * p_sigRT(A)[(size_t)jj * npair + beta * NORB + a];
            else if (comp == 0) v = A.adj ? p_sigL(A)[(size_t)jj * npair + a * NORB + beta]
                                          : -w_start(A.W, jj) * conj(p_sigL(A)[(size_t)jj * npair + beta * NORB + a]);
            else v = interval_w(A.W, n, jj) * p_sigRT(A)[(size_t)jj * npair + beta * NORB + a];
        }
        xs[(size_t)i * kXS + a] = cf{(float)v.x, (float)v.y};
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const bool col_beta = (comp ^ which) != 0;
    for (int p = 0; p < 4; ++p) {
        const int o = 4 * wave + p;
        const int q = col_beta ? o * NORB + beta : beta * NORB + o;
        const int rk = rank_of(A, comp, b, q);
        if (rk == 0) continue;
        const cf* Fq = F + (size_t)q * RC * ld;
        const double* S = p_S(A, comp, b) + ((size_t)b * npair + q) * RC;
        cd* out = p_part(A) + (size_t)(A.partoff[proj_slot(A, comp, b, q, which)] + t.chunk) * NORB * RC;
        if (comp == 1) fact_mfma_pair<true>(Fq, ld, i0, i1, rk, xs, S, out, RC);
        else fact_mfma_pair<false>(Fq, ld, i0, i1, rk, xs, S, out, RC);
    }
}

// ---------------------------------------------------------------------------
// One leaf triangle and component; wave w handles the left orbital index
// a = 4*ag + w, lanes the leaf's columns m.  Each orbital pair's triangle is
// staged in LDS with coalesced loads; the column sum (rows j >= m) and the row
// dot (columns s <= m) of lane m run in one loop over LDS.
template <int NORB>
__device__ void leaf_task(const HistArgs& A, int leaf, int comp, int ag, int pg, unsigned char* smem) {
    if (comp == 1 && (!A.wantL || A.adj)) return;
    constexpr int npair = NORB * NORB, AG = AGroups<NORB>::AG;
    constexpr int PPG = npair / LeafGroups<NORB>::LG;   // orbital pairs per group
    const int n = A.n;
    const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
    const int lw = s1 - s0;
    const int nrow = min(s1, A.last[comp] + 1) - s0;   // stored rows (row n, or up to n-1 for a step solve)
    const cd* L = p_leaf(A, comp) + A.Loff[leaf];
    const long long tsz = tri(lw), tnow = tri(nrow);
    cd* T = reinterpret_cast<cd*>(smem);   // tri(64)
    cd* xa = T + tri(64);                  // 64 x AG
    cd* xb = xa + 64 * AG;                 // 64 x AG
    const int wave = threadIdx.x >> 6, mo = threadIdx.x & 63;
    const int a = ag * AG + wave;
    const bool act = wave < AG && mo < nrow;
    const bool doR = A.wantR, doL = A.wantL;
    cd accA[NORB], accB[NORB];
#pragma unroll
    for (int c = 0; c < NORB; ++c) accA[c] = accB[c] = mk(0.0, 0.0);
    // the next pair's triangle and Sigma entries are loaded into registers while
    // the current pair is computed (one triangle element per thread and pass)
    constexpr int TPT = (64 * 65 / 2 + NT - 1) / NT;   // triangle elements of a 64-row leaf per thread
    cd pT[TPT], pxa = mk(0.0, 0.0), pxb = mk(0.0, 0.0);
    auto fetch = [&](int q) {
        const int qr = q / NORB, qc = q % NORB;
        const cd* Lq = L + (size_t)q * tsz;
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const long long e = threadIdx.x + (long long)u * NT;
            pT[u] = e < tnow ? Lq[e] : mk(0.0, 0.0);
        }
        const int e = threadIdx.x;   // nrow * AG <= NT
        if (e < nrow * AG) {
            const int i = e / AG, aa = ag * AG + e % AG, j = s0 + i;
            if (comp == 0) {
                pxa = doR ? w_end(A.W, n, j) * p_sigR(A)[(size_t)j * npair + aa * NORB + qr] : mk(0.0, 0.0);
                pxb = !doL ? mk(0.0, 0.0)
                      : A.adj ? p_sigL(A)[(size_t)j * npair + aa * NORB + qc]
                              : -w_start(A.W, j) * conj(p_sigL(A)[(size_t)j * npair + qc * NORB + aa]);
            } else {
                pxa = interval_w(A.W, n, j) * p_sigR(A)[(size_t)j * npair + aa * NORB + qr];
                pxb = interval_w(A.W, n, j) * p_sigR(A)[(size_t)j * npair + aa * NORB + qc];
            }
        }
    };
    fetch(pg * PPG);
    for (int q = pg * PPG; q < (pg + 1) * PPG; ++q) {
        const int qr = q / NORB, qc = q % NORB;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const long long e = threadIdx.x + (long long)u * NT;
            if (e < tnow) T[e] = pT[u];
        }
        if ((int)threadIdx.x < nrow * AG) {
            xa[threadIdx.x] = pxa;
            xb[threadIdx.x] = pxb;
        }
        if (q + 1 < (pg + 1) * PPG) fetch(q + 1);
        __syncthreads();
        if (act) {
            cd colsum = mk(0.0, 0.0), rowdot = mk(0.0, 0.0);
            const cd* rowm = T + tri(mo);
            const int w = wave;
            if (comp == 0) {
                // column sum x(j) G^R(j, m), j = m..; row dot x2(s) G^R(m, s)^dagger, s <= m
                // the second lesser term is empty at m = 0; the adjoint row dot is not
                const bool rowok = doL && (A.adj || s0 + mo > 0);
                for (int t = 0; t < nrow; ++t) {
                    const int j = mo + t;
                    if (doR && j < nrow) fma_(colsum, xa[j * AG + w], T[tri(j) + mo]);
                    if (rowok && t <= mo) fmac_(rowdot, rowm[t], xb[t * AG + w]);
                }
                add_at(accA, qc, colsum);   // -> I^R column m
                add_at(accB, qr, rowdot);   // -> I^< (second term) row m
            } else {
                // row dot x1(s) G^<(s, m) for s <= m; column sum -x1(s) G^<(m, s)^dagger for s > m
                for (int t = 0; t < nrow; ++t) {
                    const int j = mo + 1 + t;
                    if (t <= mo) fma_(rowdot, xa[t * AG + w], rowm[t]);
                    if (j < nrow) fmac_(colsum, T[tri(j) + mo], xb[j * AG + w]);
                }
                add_at(accA, qc, rowdot);
                add_at(accA, qr, -colsum);
            }
        }
    }
    if (act) {
        const int m = s0 + mo;
#pragma unroll
        for (int c = 0; c < NORB; ++c) {
            const size_t o = ((size_t)pg * A.nt + m) * npair + a * NORB + c;
            if (comp == 0) {
                p_leafR(A)[o] = accA[c];
                p_leafLR(A)[o] = accB[c];
            } else {
                p_leafLL(A)[o] = accA[c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One leaf triangle, component and orbital pair (qr, qc) for NORB <= 4.  The
// triangle is loaded in one round trip (every thread's loads issued together)
// and staged in LDS as a packed strictly lower triangle (row r's entries left of
// the diagonal at tri(r - 1)): the diagonal entry (m, m) is only ever read by the
// thread that owns m and sums index j = m, which loads it into a register, so that
// the task's LDS (tri(63) + 128 NORB entries) leaves room for four workgroups per
// compute unit.  Lane m owns column and row m,
// wave w the summation indices = w (mod 4), and every thread carries all NORB left
// orbitals, so each staged element feeds NORB complex FMAs.  Outputs (slot, orbital
// entry) have one writer each; the combine sums the slots:
//   comp 0: column sum x(j)[a][qr] G^R(j,m), j >= m      -> leafR [qr][m][a][qc]
//           row dot x2(s)[a][qc] G^R(m,s)^*, s <= m       -> leafLR[qc][m][a][qr]
//   comp 1: row dot x1(s)[a][qr] G<(m,s), s <= m          -> leafLL[qr][m][a][qc]
//           column sum -x1(j)[a][qc] G<(j,m)^*, j > m     -> leafLL[NORB + qc][m][a][qr]
template <int NORB>
__device__ void leaf_pair_task(const HistArgs& A, int leaf, int comp, int q, unsigned char* smem) {
    static_assert(NORB <= 4, "one orbital pair per task");
    if (comp == 1 && (!A.wantL || A.adj)) return;
    constexpr int npair = NORB * NORB;
    const int qr = q / NORB, qc = q % NORB;
    const int n = A.n;
    const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
    const int lw = s1 - s0;
    const int nrow = min(s1, A.last[comp] + 1) - s0;   // stored rows (row n, or up to n-1 for a step solve)
    const cd* Lq = p_leaf(A, comp) + A.Loff[leaf] + (size_t)q * tri(lw);
    const long long tnow = tri(nrow);
    cd* T = reinterpret_cast<cd*>(smem);   // tri(63): (r, j < r) at tri(r - 1) + j
    cd* xa = T + tri(63);                  // 64 x NORB: Sigma entries with orbital qr
    cd* xb = xa + 64 * NORB;               // 64 x NORB: Sigma entries with orbital qc
    const int w = threadIdx.x >> 6, m = threadIdx.x & 63;
    // the diagonal entry (m, m), read by the wave whose summation indices j = w + 4t hit m
    const cd dg = ((m & 3) == w && m < nrow) ? Lq[tri(m) + m] : mk(0.0, 0.0);
    const bool doR = A.wantR, doL = A.wantL;
    const bool colOn = comp == 1 || doR;
    const bool rowOn = (comp == 1 || doL) && (comp == 1 || A.adj || s0 + m > 0);
    constexpr int TPT = (64 * 65 / 2 + NT - 1) / NT;   // triangle elements per thread
    {
        cd v[TPT];
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const long long e = threadIdx.x + (long long)u * NT;
            v[u] = e < tnow ? Lq[e] : mk(0.0, 0.0);
        }
        if ((int)threadIdx.x < 64 * NORB) {   // rows beyond the leaf's present rows are zero
            const int i = threadIdx.x / NORB, a = threadIdx.x % NORB, j = s0 + (i < nrow ? i : 0);
            cd va, vb;
            if (i >= nrow) {
                va = vb = mk(0.0, 0.0);
            } else if (comp == 0) {
                va = doR ? w_end(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + qr] : mk(0.0, 0.0);
                vb = !doL ? mk(0.0, 0.0)
                     : A.adj ? p_sigL(A)[(size_t)j * npair + a * NORB + qc]
                             : -w_start(A.W, j) * conj(p_sigL(A)[(size_t)j * npair + qc * NORB + a]);
            } else {
                const double wi = interval_w(A.W, n, j);
                va = wi * p_sigR(A)[(size_t)j * npair + a * NORB + qr];
                vb = wi * p_sigR(A)[(size_t)j * npair + a * NORB + qc];
            }
            xa[threadIdx.x] = va;
            xb[threadIdx.x] = vb;
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int e = (int)threadIdx.x + u * NT;
            // row r of element e (tri(r) <= e < tri(r + 1)): the float root is exact to
            // well within one for e < 2080, the two tests settle the boundaries
            int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            if ((r + 1) * (r + 2) / 2 <= e) ++r;
            if (r * (r + 1) / 2 > e) --r;
            if (e < tnow && e - r * (r + 1) / 2 < r) T[e - r] = v[u];   // strictly lower entries
        }
    }
    __syncthreads();
    cd accC[NORB], accW[NORB];   // column sums, row dots
#pragma unroll
    for (int a = 0; a < NORB; ++a) accC[a] = accW[a] = mk(0.0, 0.0);
    // Summation index j = w + 4t, t = 0..15: the column sum of column m takes row j and
    // the row dot of row m takes column j.  Both LDS reads are in bounds for every
    // j, m < 64 and are issued for every t; terms outside the triangle, the present rows
    // or the requested products are zeroed by selects (the x entries of absent rows are
    // zero), so the loop has a fixed trip count and no divergence.
    const int trm = m * (m - 1) / 2;
#pragma unroll 4
    for (int t = 0; t < 16; ++t) {
        const int j = w + 4 * t;
        const bool vc = colOn && m < nrow && j < nrow && (comp == 0 ? j >= m : j > m);
        const bool vr = rowOn && m < nrow && j <= m;
        // (j, m) for j > m and (m, j) for j < m; the indices stay below tri(63) for
        // every j, m < 64 except on the diagonal, which takes the register copy
        const cd tc0 = T[min(j * (j - 1) / 2 + m, (int)tri(63) - 1)];
        const cd tr0 = T[min(trm + j, (int)tri(63) - 1)];
        const cd tc = vc ? (j == m ? dg : tc0) : mk(0.0, 0.0);
        const cd tr = vr ? (j == m ? dg : tr0) : mk(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            if (comp == 0) {
                fma_(accC[a], xa[j * NORB + a], tc);
                fmac_(accW[a], tr, xb[j * NORB + a]);
            } else {
                fmac_(accC[a], tc, xb[j * NORB + a]);
                fma_(accW[a], xa[j * NORB + a], tr);
            }
        }
    }
    // sum the four waves' partial sums through LDS (the triangle is no longer read);
    // red[(k * 4 + wave) * 64 + lane]: consecutive lanes, consecutive 16-byte words
    cd* red = T;   // 2 NORB x 4 x 64
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
        red[((size_t)a * 4 + w) * 64 + m] = accC[a];
        red[((size_t)(NORB + a) * 4 + w) * 64 + m] = accW[a];
    }
    __syncthreads();
    if (w != 0 || m >= nrow) return;
    for (int ww = 1; ww < 4; ++ww)
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            accC[a] = accC[a] + red[((size_t)a * 4 + ww) * 64 + m];
            accW[a] = accW[a] + red[((size_t)(NORB + a) * 4 + ww) * 64 + m];
        }
    const size_t mo = (size_t)(s0 + m) * npair;
    const size_t sl = (size_t)A.nt * npair;   // one slot
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
        if (comp == 0) {
            if (doR) p_leafR(A)[qr * sl + mo + a * NORB + qc] = accC[a];
            if (doL) p_leafLR(A)[qc * sl + mo + a * NORB + qr] = accW[a];
        } else {
            p_leafLL(A)[qr * sl + mo + a * NORB + qc] = accW[a];
            p_leafLL(A)[(NORB + qc) * sl + mo + a * NORB + qr] = -accC[a];
        }
    }
}

// ---------------------------------------------------------------------------
// Tail rows for NORB <= 4: one task per component, 64-column chunk and orbital
// pair (qr, qc); the 32 x 64 tile (rows n0.. of the ring, columns of the chunk) is
// loaded in one round trip and staged in LDS with its column index XORed by
// (row & 15), so that lanes over columns and lanes over rows both spread over
// distinct banks.  Column sums: lane = column, wave = rows = w (mod 4); row dots:
// lane = (row, half of the columns), wave = 8 columns of that half.  Every thread
// carries all NORB left orbitals.  Outputs (one writer per slot entry):
//   comp 0: column sum x(j)[a][qr] G^R(j,m)        -> tailcol[qr][m][a][qc]
//           row dot x2(m)[a][qc] G^R(r,m)^*         -> tailpart[chunk][qc][r][a][qr]
//   comp 1: column sum -x1(j)[a][qc] G<(j,m)^*      -> tailcol[qc][m][a][qr]
//           row dot x1(m)[a][qr] G<(r,m)            -> tailpart[chunk][qr][r][a][qc]
template <int NORB>
__device__ void tail_pair_task(const HistArgs& A, int comp, int chunk, int q, unsigned char* smem) {
    static_assert(NORB <= 4, "one orbital pair per task");
    if (comp == 1 && (!A.wantL || A.adj)) return;
    constexpr int npair = NORB * NORB, TG = tail_groups(NORB);
    const int qr = q / NORB, qc = q % NORB;
    const int n = A.n;
    const int n0 = A.n0[comp], nrows = A.last[comp] - n0 + 1, ls = A.ls[comp];
    const int cbeg = chunk * kTailCH, ncol = min(kTailCH, ls - cbeg);
    cd* T = reinterpret_cast<cd*>(smem);       // 32 x 64, swizzled
    cd* xr = T + (size_t)kTailRows * kTailCH;  // 32 x NORB (row side)
    cd* xm = xr + (size_t)kTailRows * NORB;    // 64 x NORB (column side)
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool doR = A.wantR, doL = A.wantL;
    const cd* Tg = p_tail(A, comp);
    constexpr int EPT = kTailRows * kTailCH / NT;   // tile elements per thread
    {
        cd v[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = threadIdx.x + u * NT, i = e / kTailCH, mm = e % kTailCH;
            const int r = n0 + i;                                   // tail row
            const int lsr = r < A.nsplit[comp] ? A.lslo[comp] : ls; // its dense columns
            v[u] = (i < nrows && cbeg + mm < lsr) ? Tg[((size_t)(r % A.ring) * npair + q) * A.nt + cbeg + mm]
                                                 : mk(0.0, 0.0);
        }
        const int e = threadIdx.x;
        if (e < kTailRows * NORB) {   // row side; rows beyond the tail are zero
            const int i = e / NORB, a = e % NORB, j = n0 + i;
            xr[e] = i >= nrows ? mk(0.0, 0.0)
                    : comp == 0 ? (doR ? w_end(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + qr] : mk(0.0, 0.0))
                                : interval_w(A.W, n, j) * p_sigR(A)[(size_t)j * npair + a * NORB + qc];
        }
        if (e < kTailCH * NORB) {   // column side
            const int mm = e / NORB, a = e % NORB, m = cbeg + mm;
            cd vv = mk(0.0, 0.0);
            if (mm < ncol) {
                if (comp == 0) {
                    if (doL)
                        vv = A.adj ? p_sigL(A)[(size_t)m * npair + a * NORB + qc]
                                   : -w_start(A.W, m) * conj(p_sigL(A)[(size_t)m * npair + qc * NORB + a]);
                } else {
                    vv = interval_w(A.W, n, m) * p_sigR(A)[(size_t)m * npair + a * NORB + qr];
                }
            }
            xm[e] = vv;
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = threadIdx.x + u * NT, i = e / kTailCH, mm = e % kTailCH;
            T[i * kTailCH + (mm ^ (i & 15))] = v[u];
        }
    }
    __syncthreads();
    cd col[NORB], row[NORB];
#pragma unroll
    for (int a = 0; a < NORB; ++a) col[a] = row[a] = mk(0.0, 0.0);
    // column sums (lane = column, rows = w mod 4; rows beyond the tail are zero in the
    // tile and in xr, so the trip count is fixed)
#pragma unroll 4
    for (int i = w; i < kTailRows; i += 4) {
        const cd v = T[i * kTailCH + (lane ^ (i & 15))];
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            if (comp == 0) fma_(col[a], xr[i * NORB + a], v);
            else fmac_(col[a], v, xr[i * NORB + a]);
        }
    }
    // row dots (lane = row ri and column half part; wave = 8 columns of the half)
    const int ri = lane & 31, part = lane >> 5;
    {   // rows beyond the tail are zero in the tile
        const int mb = part * 32 + w * 8;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int mm = mb + u;
            const cd v = T[ri * kTailCH + (mm ^ (ri & 15))];
#pragma unroll
            for (int a = 0; a < NORB; ++a) {
                if (comp == 0) fmac_(row[a], v, xm[mm * NORB + a]);
                else fma_(row[a], xm[mm * NORB + a], v);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NORB; ++a) {   // the two column halves of each row dot
        row[a].x += __shfl_xor(row[a].x, 32, 64);
        row[a].y += __shfl_xor(row[a].y, 32, 64);
    }
    // sum over the waves through LDS (the tile is no longer read);
    // red[(k * 4 + wave) * 64 + lane]: consecutive lanes, consecutive 16-byte words
    cd* red = T;   // 2 NORB x 4 x 64
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
        red[((size_t)a * 4 + w) * 64 + lane] = col[a];
        red[((size_t)(NORB + a) * 4 + w) * 64 + lane] = row[a];
    }
    __syncthreads();
    if (w != 0) return;
    for (int ww = 1; ww < 4; ++ww)
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            col[a] = col[a] + red[((size_t)a * 4 + ww) * 64 + lane];
            row[a] = row[a] + red[((size_t)(NORB + a) * 4 + ww) * 64 + lane];
        }
    const size_t sl = (size_t)A.nt * npair;
    if (lane < ncol) {
        const size_t mo = (size_t)(cbeg + lane) * npair;
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            if (comp == 0) p_tailcol(A, 0)[qr * sl + mo + a * NORB + qc] = col[a];
            else p_tailcol(A, 1)[qc * sl + mo + a * NORB + qr] = -col[a];
        }
    }
    if (part == 0 && ri < nrows) {
        const int slot = comp == 0 ? qc : qr, c = comp == 0 ? qr : qc;
        cd* tp = p_tailpart(A, comp) + ((size_t)(chunk * TG + slot) * A.ring + ri) * npair + c;
#pragma unroll
        for (int a = 0; a < NORB; ++a) tp[a * NORB] = row[a];
    }
}

// ---------------------------------------------------------------------------
// Rows appended since the last panel merge (dense), columns [chunk*64, +64) of
// [0, ls): the column sums over those rows are complete here; the row dots are
// written per column chunk and summed by the combine.
template <int NORB>
__device__ void tail_task(const HistArgs& A, int comp, int ag, int chunk, int tg, unsigned char* smem) {
    if (comp == 1 && (!A.wantL || A.adj)) return;
    constexpr int npair = NORB * NORB, AG = AGroups<NORB>::AG;
    constexpr int TG = tail_groups(NORB), PPG = npair / TG;   // orbital pairs of this group
    const int n = A.n;
    const int n0 = A.n0[comp], nrows = A.last[comp] - n0 + 1, ls = A.ls[comp];
    const int cbeg = chunk * kTailCH, ncol = min(kTailCH, ls - cbeg);
    cd* T = reinterpret_cast<cd*>(smem);       // 32 x 64 (entries outside the tail rows are zero)
    cd* xr = T + (size_t)kTailRows * kTailCH;  // 32 x AG  (row-side Sigma)
    cd* xm = xr + (size_t)kTailRows * AG;      // 64 x AG  (column-side Sigma)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = ag * AG + wave;
    const bool wok = wave < AG;
    const bool doR = A.wantR, doL = A.wantL;
    const cd* Tg = p_tail(A, comp);
    cd col[NORB], row[NORB];
#pragma unroll
    for (int c = 0; c < NORB; ++c) col[c] = row[c] = mk(0.0, 0.0);
    const int ri = lane & 31, part = lane >> 5;   // row-dot mapping: row ri, 32 columns per part
    // the next pair's tile and Sigma entries are loaded into registers while the
    // current pair is computed
    constexpr int EPT = kTailRows * kTailCH / NT;   // tile elements per thread
    cd pT[EPT], pxr = mk(0.0, 0.0), pxm = mk(0.0, 0.0);
    auto fetch = [&](int q) {
        const int qr = q / NORB, qc = q % NORB;
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = threadIdx.x + u * NT, i = e / kTailCH, mm = e % kTailCH;
            const int r = n0 + i;                                   // tail row
            const int lsr = r < A.nsplit[comp] ? A.lslo[comp] : ls; // its dense columns
            pT[u] = (i < nrows && cbeg + mm < lsr)
                        ? Tg[((size_t)(r % A.ring) * npair + q) * A.nt + cbeg + mm] : mk(0.0, 0.0);
        }
        const int e = threadIdx.x;
        if (e < nrows * AG) {     // row side, nrows * AG <= NT
            const int i = e / AG, aa = ag * AG + e % AG, j = n0 + i;
            pxr = comp == 0 ? (doR ? w_end(A.W, n, j) * p_sigR(A)[(size_t)j * npair + aa * NORB + qr] : mk(0.0, 0.0))
                            : interval_w(A.W, n, j) * p_sigR(A)[(size_t)j * npair + aa * NORB + qc];
        }
        if (e < kTailCH * AG) {   // column side, 64 * AG <= NT
            const int mm = e / AG, aa = ag * AG + e % AG, m = cbeg + mm;
            cd v = mk(0.0, 0.0);
            if (mm < ncol) {
                if (comp == 0) {
                    if (doL)
                        v = A.adj ? p_sigL(A)[(size_t)m * npair + aa * NORB + qc]
                                  : -w_start(A.W, m) * conj(p_sigL(A)[(size_t)m * npair + qc * NORB + aa]);
                } else {
                    v = interval_w(A.W, n, m) * p_sigR(A)[(size_t)m * npair + aa * NORB + qr];
                }
            }
            pxm = v;
        }
    };
    fetch(tg * PPG);
    for (int q = tg * PPG; q < (tg + 1) * PPG; ++q) {
        const int qr = q / NORB, qc = q % NORB;
        __syncthreads();
        // the tile is stored with its column index XORed by (row & 15), so that the row
        // dots (lanes over rows) and the column sums (lanes over columns) both spread
        // over distinct LDS banks
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = threadIdx.x + u * NT, i = e / kTailCH, mm = e % kTailCH;
            T[i * kTailCH + (mm ^ (i & 15))] = pT[u];
        }
        if ((int)threadIdx.x < nrows * AG) xr[threadIdx.x] = pxr;
        if ((int)threadIdx.x < kTailCH * AG) xm[threadIdx.x] = pxm;
        if (q + 1 < (tg + 1) * PPG) fetch(q + 1);
        __syncthreads();
        if (wok) {
            // column sums (lane = column)
            cd cs = mk(0.0, 0.0);
            for (int i = 0; i < nrows; ++i) {
                const cd v = T[i * kTailCH + (lane ^ (i & 15))];
                if (comp == 0) fma_(cs, xr[i * AG + wave], v);
                else fmac_(cs, v, xr[i * AG + wave]);
            }
            if (comp == 0) {
                if (doR) add_at(col, qc, cs);       // x(j) G^R(j, m)
            } else {
                add_at(col, qr, -cs);               // -x1(j) G^<(m, j)^dagger
            }
            // row dots (lane = row ri, columns 32*part .. +32)
            cd rd = mk(0.0, 0.0);
            if (ri < nrows) {
                for (int mm = part * 32; mm < part * 32 + 32; ++mm) {
                    const cd v = T[ri * kTailCH + (mm ^ (ri & 15))];
                    if (comp == 0) fmac_(rd, v, xm[mm * AG + wave]);
                    else fma_(rd, xm[mm * AG + wave], v);
                }
            }
            if (comp == 0) add_at(row, qr, rd);     // x2(m) G^R(j, m)^dagger
            else add_at(row, qc, rd);               // x1(m) G^<(m, j)
        }
    }
    // add the two column parts of each row dot (lanes ri and ri + 32)
#pragma unroll
    for (int c = 0; c < NORB; ++c) {
        double re = row[c].x, im = row[c].y;
        re += __shfl_xor(re, 32, 64);
        im += __shfl_xor(im, 32, 64);
        row[c] = mk(re, im);
    }
    if (wok) {
        if (lane < ncol) {
#pragma unroll
            for (int c = 0; c < NORB; ++c)
                p_tailcol(A, comp)[((size_t)tg * A.nt + cbeg + lane) * npair + a * NORB + c] = col[c];
        }
        if (part == 0 && ri < nrows) {
            cd* tp = p_tailpart(A, comp) + ((size_t)(chunk * TG + tg) * A.ring + ri) * npair + a * NORB;
#pragma unroll
            for (int c = 0; c < NORB; ++c) tp[c] = row[c];
        }
    }
}

template <int NORB, class FT>
__global__ void __launch_bounds__(NT) hist_tasks(HistArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NG = AGroups<NORB>::NG;
    // longest tasks first: the tail tiles (all orbital pairs of a column chunk), then
    // the leaf triangles, then the many short projection chunks that fill in behind
    // them; every section starts at a multiple of 8, so workgroup id % 8 is the XCD
    // that xcd_group assumes
    int rel = blockIdx.x;
    if constexpr (NORB != 16) {   // norb 16: the dense pieces are the dense16 kernel's
    if (rel < A.ntailtask) {
        constexpr int TG = tail_groups(NORB);
        int g, mem;
        const int ng = A.ntailchunk[0] + A.ntailchunk[1];
        if constexpr (NORB <= 4) {
            if (!xcd_group(rel, ng, NORB * NORB, g, mem)) return;
            if (g < A.ntailchunk[0]) tail_pair_task<NORB>(A, 0, g, mem, smem);
            else tail_pair_task<NORB>(A, 1, g - A.ntailchunk[0], mem, smem);
        } else {
            if (!xcd_group(rel, ng, NG * TG, g, mem)) return;
            if (g < A.ntailchunk[0])
                tail_task<NORB>(A, 0, mem % NG, g, mem / NG, smem);
            else
                tail_task<NORB>(A, 1, mem % NG, g - A.ntailchunk[0], mem / NG, smem);
        }
        return;
    }
    rel -= A.ntailtask;
    if (rel < A.nleaftask) {
        constexpr int LG = LeafGroups<NORB>::LG;
        int g, mem;
        if constexpr (NORB <= 4) {
            if (!xcd_group(rel, 2 * A.nleaf, NORB * NORB, g, mem)) return;
            leaf_pair_task<NORB>(A, g >> 1, g & 1, mem, smem);
        } else {
            if (!xcd_group(rel, 2 * A.nleaf, NG * LG, g, mem)) return;
            leaf_task<NORB>(A, g >> 1, g & 1, mem % NG, mem / NG, smem);
        }
        return;
    }
    rel -= A.nleaftask;
    }
    int idx = rel;
    if constexpr (NORB == 4) {   // the four tasks of a chunk (consecutive in the list) on one XCD
        int g, mem;
        if (!xcd_group(rel, (A.nf[0] + A.nf[1]) / 4, 4, g, mem)) return;
        idx = 4 * g + mem;
    }
    if (idx >= A.nf[0] + A.nf[1]) return;
    const FactTask& t = idx < A.nf[0] ? A.ft[0][idx] : A.ft[1][idx - A.nf[0]];
    if constexpr (NORB == 4) fact_task_beta<NORB, FT>(A, t, smem);   // tasks per shared index
    else fact_task<NORB, FT>(A, t, smem);
}

// Matrix-core projections (norb 16, complex-float factors) in a kernel of their own, so
// that their register budget is not that of the leaf and tail tasks.
__global__ void __launch_bounds__(NT) proj_mfma(HistArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int rel = blockIdx.x;
    if (rel >= A.nf[0] + A.nf[1]) return;
    fact_mfma_task(A, rel < A.nf[0] ? A.ft[0][rel] : A.ft[1][rel - A.nf[0]], smem);
}

// ---------------------------------------------------------------------------
// Second phase of the tasks: (i) the sum of the chunk partials of every active
// projection, one thread per (slot, a, r) (slots of inactive blocks, ranks
// beyond the block's rank and components not asked for are neither written
// nor read by the combine); (ii) the sum over the column chunks of the row
// dots of every tail row, one wave per (component, row, orbital pair), lanes
// over the chunks and a fixed-order wave reduction.
inline long long proj_reduce_blocks(const HistArgs& A) {
    return (4LL * A.nb * A.npair * A.norb * A.RC + 255) / 256;
}

template <int NORB>
__global__ void __launch_bounds__(256) proj_reduce(HistArgs A) {
    const int RC = A.RC;
    const long long per = (long long)NORB * RC;
    const long long nblk = (4LL * A.nb * A.npair * per + 255) / 256;
    if ((long long)blockIdx.x >= nblk) {
        constexpr int npair = NORB * NORB;
        const long long w = ((long long)blockIdx.x - nblk) * 4 + (threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        const int q = (int)(w % npair);
        const int slot = (int)((w / npair) % A.ring);
        const int comp = (int)(w / ((long long)npair * A.ring));
        if (comp > 1 || !A.wantL || (comp == 1 && A.adj)) return;
        if (slot > A.last[comp] - A.n0[comp]) return;   // also: no tail rows at all
        const cd* tp = p_tailpart(A, comp) + (size_t)slot * npair + q;
        double re = 0.0, im = 0.0;
        for (int ch = lane; ch < A.ntailchunk[comp] * tail_groups(NORB); ch += 64) {   // chunks x pair groups
            const cd v = tp[(size_t)ch * A.ring * npair];
            re += v.x;
            im += v.y;
        }
        re = wsum64(re);
        im = wsum64(im);
        if (lane == 0) p_tailrow(A, comp)[(size_t)slot * npair + q] = mk(re, im);
        return;
    }
    const long long tid = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long slot = tid / per;
    if (slot >= 4LL * A.nb * A.npair) return;
    const int e = (int)(tid - slot * per);   // a * RC + r
    const int r = e % RC;
    const int which = (int)(slot & 1);
    const long long bq = slot >> 1;
    const int q = (int)(bq % A.npair);
    const int b = (int)((bq / A.npair) % A.nb);
    const int comp = (int)(bq / ((long long)A.npair * A.nb));
    if (comp == 0 && which == 0 && !A.wantR) return;
    if ((comp == 1 || which == 1) && !A.wantL) return;
    if (comp == 1 && A.adj) return;
    if (r >= rank_of(A, comp, b, q)) return;
    const int* bk = A.blk + 5 * b;
    const int r0 = bk[1];
    if (A.n0[comp] <= r0) return;
    const int len = which == 0 ? min(A.n0[comp] - r0, bk[2] - r0) : bk[4] - bk[3];
    const int nch = (len + A.kch - 1) / A.kch;
    const cd* p = p_part(A) + (size_t)A.partoff[slot] * per + e;
    cd s = mk(0.0, 0.0);
    for (int ch = 0; ch < nch; ++ch) s = s + p[(size_t)ch * per];
    p_proj(A)[(size_t)slot * per + e] = s;
}

// ---------------------------------------------------------------------------
// acc[a] (+|-)= op(F[r*ld]) z[a*RC + r] over the ranks r = rs, rs + RS, ... < rk,
// op = conj or identity.  The factor loads of a batch of eight ranks are issued
// together (indices clamped to rk - 1, surplus terms skipped) so that they
// overlap in flight.
template <int NORB, bool CONJ, bool NEG, int RS, class FT>
__device__ inline void expand_ranks(cd (&acc)[NORB], const FT* F, int ld, const cd* z, int RC, int rk, int rs) {
    constexpr int B = 8;
    for (int r0 = rs; r0 < rk; r0 += B * RS) {
        cd f[B];
#pragma unroll
        for (int u = 0; u < B; ++u) f[u] = to_cd(F[(size_t)min(r0 + u * RS, rk - 1) * ld]);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int r = r0 + u * RS;
            if (r >= rk) break;
            const cd fv = NEG ? -f[u] : f[u];
#pragma unroll
            for (int a = 0; a < NORB; ++a) {
                if (CONJ) fmac_(acc[a], fv, z[a * RC + r]);
                else fma_(acc[a], fv, z[a * RC + r]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Final sum of one output entry (column m, left orbital a, right orbital c) from
// its expansion sum y: the leaf and tail slots, the tail row dots, the band
// corrections of the Gregory weights, the factor h; part 0 writes I^R, part 1
// writes I^< (or, in adjoint mode, dL/dSigma^R(n, j = m)).
template <int NORB>
__device__ void finish_entry(const HistArgs& A, int m, int a, int c, int part, cd y) {
    constexpr int npair = NORB * NORB, LG = LeafGroups<NORB>::LG;
    const int n = A.n, k = A.W.k, kb = k + 1;
    const size_t sl = (size_t)A.nt * npair;
    const size_t o = (size_t)m * npair + a * NORB + c;
    if (A.adj) {
        // outL(j = m) = h [ w_end(n, j) y(j) + corrections ]; the corrections replace
        // the bulk weight of the terms m' = j - i, i <= k, by the exact interval weight
        const int j = m;
        const double we = w_end(A.W, n, j);
        for (int pg = 0; pg < LG; ++pg) y = y + p_leafLR(A)[pg * sl + o];
        if (A.last[0] >= A.n0[0] && j >= A.n0[0] && j <= A.last[0])
            y = y + p_tailrow(A, 0)[(size_t)(j - A.n0[0]) * npair + a * NORB + c];
        cd out = we * y;
        const int imax = j < k ? j : k;
        for (int i = 0; i <= imax; ++i) {
            const int mp = j - i, L = n - mp;
            const double wc = L >= k ? A.W.om[i] - 1.0 : A.W.nc[L][i] - we;
            const cd* ib = p_sigL(A) + (size_t)mp * npair + a * NORB;            // Ibar(n, m')[a][b]
            const cd* bd = p_band(A) + ((size_t)mp * kb + i) * npair + c * NORB;   // G^R(j, m')[c][b]
#pragma unroll 4
            for (int bb = 0; bb < NORB; ++bb) fmac_(out, bd[bb], wc * ib[bb]);
        }
        p_outL(A)[o] = A.h * out;
        return;
    }
    if (part == 0) {
        cd sR = y;
        for (int pg = 0; pg < LG; ++pg) sR = sR + p_leafR(A)[pg * sl + o];
        if (A.last[0] >= A.n0[0] && m < A.ls[0])
            for (int tg = 0; tg < tail_groups(NORB); ++tg) sR = sR + p_tailcol(A, 0)[tg * sl + o];
        // band correction: start weights (n-m >= k) or Newton-Cotes (n-m < k)
        const int L = n - m;
        if (L == 0) {
            p_outR(A)[o] = mk(0.0, 0.0);
            return;
        }
        // the newest term (j = n) is absent when row n is not stored (step solve)
        const int imax = min(L < k ? L : k, A.last[0] - m);
        for (int i = 0; i <= imax; ++i) {
            const double wc = L < k ? A.W.nc[L][i] - w_end(A.W, n, m + i) : A.W.om[i] - 1.0;
            const cd* sg = p_sigR(A) + (size_t)(m + i) * npair + a * NORB;
            const cd* bd = p_band(A) + ((size_t)m * kb + i) * npair + c;
#pragma unroll 4
            for (int bb = 0; bb < NORB; ++bb) fma_(sR, sg[bb], wc * bd[bb * NORB]);
        }
        p_outR(A)[o] = A.h * sR;
        return;
    }
    cd sL = y;
    for (int pg = 0; pg < LG; ++pg) sL = sL + p_leafLR(A)[pg * sl + o];
    for (int pg = 0; pg < leaf_ll_slots(NORB); ++pg) sL = sL + p_leafLL(A)[pg * sl + o];
    for (int comp = 0; comp < 2; ++comp) {
        if (A.last[comp] < A.n0[comp]) continue;   // no tail rows
        if (comp == 1 && m < A.ls[1])
            for (int tg = 0; tg < tail_groups(NORB); ++tg) sL = sL + p_tailcol(A, 1)[tg * sl + o];
        if (m >= A.n0[comp] && m <= A.last[comp])
            sL = sL + p_tailrow(A, comp)[(size_t)(m - A.n0[comp]) * npair + a * NORB + c];
    }
    // second lesser term: end weights (m >= k) or Newton-Cotes (m < k); the
    // interval is empty at m = 0 (no bulk term was added there either)
    // Sigma^<(n,s)[a][b] = -conj(sigL[s][b][a]);  G^R(m,s)^dagger[b][c] = conj(G^R(m,s)[c][b])
    const int imax = m == 0 ? -1 : (m < k ? m : k);
    for (int i = 0; i <= imax; ++i) {
        const int s = m - i;
        const double wc = m < k ? A.W.nc[m][s] - w_start(A.W, s) : A.W.om[i] - 1.0;
        const cd* slp = p_sigL(A) + (size_t)s * npair + a;
        const cd* bd = p_band(A) + ((size_t)s * kb + i) * npair + c * NORB;
#pragma unroll 4
        for (int bb = 0; bb < NORB; ++bb) fmac_(sL, slp[bb * NORB], mk(-wc, 0.0) * conj(bd[bb]));
    }
    p_outL(A)[o] = A.h * sL;
}

// ---------------------------------------------------------------------------
// Combine.  A wave handles MW consecutive columns m and one output orbital c
// (c = wave, wave + 4, ...); its G = GO * RS lane groups split the summed
// orbital index of the expansions (lane group g takes the orbitals g % GO,
// + GO, ...) and the ranks (r = g / GO, + RS, ...), so that a wave's serial
// chain of dependent factor loads is short and a step has many waves; the
// groups are summed by shuffles, and lane group g then adds the leaf, tail and
// band pieces of the outputs a = g, g+G, ... and writes them.
template <int NORB>
struct CombMap {
    static constexpr int GO = NORB < 4 ? NORB : 4;
    static constexpr int RS = NORB <= 4 ? 8 / GO : 1;
    static constexpr int G = GO * RS;
    static constexpr int MW = 64 / G;
    static constexpr int WAVES = NORB < 4 ? NORB : 4;
    static constexpr int NCI = NORB / WAVES;
};

template <int NORB, class FT>
__global__ void __launch_bounds__(64 * CombMap<NORB>::WAVES) hist_combine(HistArgs A) {
    using M = CombMap<NORB>;
    constexpr int npair = NORB * NORB, G = M::G, MW = M::MW, GO = M::GO, RS = M::RS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / MW, og = g % GO, rs = g / GO;
    const int m = blockIdx.x * MW + lane % MW;
    const int n = A.n;
    const bool live = m <= n;
    const int RC = A.RC;
    for (int ci = 0; ci < M::NCI; ++ci) {
        const int c = wave + M::WAVES * ci;
        cd accR[NORB], accL[NORB];
#pragma unroll
        for (int a = 0; a < NORB; ++a) accR[a] = accL[a] = mk(0.0, 0.0);
        if (live) {
            // the next level's block index is loaded while the current level is expanded
            int cv_next = A.cover[m];
            for (int l = 0; l < A.nlvl; ++l) {
                const int cv = cv_next;
                if (l + 1 < A.nlvl) cv_next = A.cover[(size_t)(l + 1) * A.nt + m];
                if (cv >= 0) {  // m is a column of block b: expand through V
                    const int b = cv;
                    const int r0 = A.blk[5 * b + 1], c0 = A.blk[5 * b + 3], c1 = A.blk[5 * b + 4];
                    const int ldV = c1 - c0;
                    if (A.wantR && A.n0[0] > r0) {
                        for (int o = og; o < NORB; o += GO) {
                            const int q = o * NORB + c;
                            const int rk = rank_of(A, 0, b, q);
                            const FT* Vq = p_V<FT>(A, 0, b) + A.Voff[b] + (size_t)q * RC * ldV + (m - c0);
                            const cd* z = p_proj(A) + proj_slot(A, 0, b, q, 0) * NORB * RC;
                            if (rk > 0) expand_ranks<NORB, true, false, RS>(accR, Vq, ldV, z, RC, rk, rs);
                        }
                    }
                    if (A.wantL && !A.adj && A.n0[1] > r0) {
                        for (int o = og; o < NORB; o += GO) {
                            const int q = c * NORB + o;
                            const int rk = rank_of(A, 1, b, q);
                            const FT* Vq = p_V<FT>(A, 1, b) + A.Voff[b] + (size_t)q * RC * ldV + (m - c0);
                            const cd* z = p_proj(A) + proj_slot(A, 1, b, q, 0) * NORB * RC;
                            if (rk > 0) expand_ranks<NORB, false, true, RS>(accL, Vq, ldV, z, RC, rk, rs);
                        }
                    }
                } else if (A.wantL) {  // m is a row of block b: expand through U
                    const int b = ~cv;
                    const int r0 = A.blk[5 * b + 1], r1 = A.blk[5 * b + 2];
                    const int ldU = r1 - r0;
                    if (m < A.n0[0]) {
                        for (int o = og; o < NORB; o += GO) {
                            const int q = c * NORB + o;
                            const int rk = rank_of(A, 0, b, q);
                            const FT* Uq = p_U<FT>(A, 0, b) + A.Uoff[b] + (size_t)q * RC * ldU + (m - r0);
                            const cd* z = p_proj(A) + proj_slot(A, 0, b, q, 1) * NORB * RC;
                            if (rk > 0) expand_ranks<NORB, true, false, RS>(accL, Uq, ldU, z, RC, rk, rs);
                        }
                    }
                    if (!A.adj && m < A.n0[1]) {
                        for (int o = og; o < NORB; o += GO) {
                            const int q = o * NORB + c;
                            const int rk = rank_of(A, 1, b, q);
                            const FT* Uq = p_U<FT>(A, 1, b) + A.Uoff[b] + (size_t)q * RC * ldU + (m - r0);
                            const cd* z = p_proj(A) + proj_slot(A, 1, b, q, 1) * NORB * RC;
                            if (rk > 0) expand_ranks<NORB, false, false, RS>(accL, Uq, ldU, z, RC, rk, rs);
                        }
                    }
                }
            }
        }
        // sum over the lane groups (every lane of the wave takes part)
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
#pragma unroll
            for (int sh = MW; sh < 64; sh <<= 1) {
                accR[a].x += __shfl_xor(accR[a].x, sh, 64);
                accR[a].y += __shfl_xor(accR[a].y, sh, 64);
                accL[a].x += __shfl_xor(accL[a].x, sh, 64);
                accL[a].y += __shfl_xor(accL[a].y, sh, 64);
            }
        }
        if (!live) continue;
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            if (a % G != g) continue;
            if (A.adj) {
                finish_entry<NORB>(A, m, a, c, 1, accL[a]);
            } else {
                if (A.wantR) finish_entry<NORB>(A, m, a, c, 0, accR[a]);
                if (A.wantL) finish_entry<NORB>(A, m, a, c, 1, accL[a]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Dense pieces at norb = 16 on the FP64 matrix cores (both factor forms: the leaf
// triangles and tail rows are FP64).  Every piece is, for one output orbital c, a
// complex product Y[a][x] = sum over (b', k) of X[a][(b', k)] op(T_{q(b')}[k][x])
// with the 16 left orbitals a as the M dimension: X is a folded Sigma entry at
// the summation row or column k, T the stored triangle or tail row of the pair
// q(b') = (b', c) or (c, b').  Each is done as four real v_mfma_f64_16x16x4f64
// chains over K steps of 4 (re.re, im.im, re.im, im.re), both operands loaded
// from memory by the lane that feeds them, out-of-range terms zeroed by selects
// on clamped (in-range) loads.
// Lane layout of the FP64 16x16x4 product: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[i][j] in lane j + 16 (i % 4), register i / 4.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma64_16x16x4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct CAcc {
    v4d rr, ii, ri, ir;
};
__device__ inline void cacc_zero(CAcc& z) {
    z.rr = v4d{0.0, 0.0, 0.0, 0.0};
    z.ii = z.rr;
    z.ri = z.rr;
    z.ir = z.rr;
}
__device__ inline void cacc_step(CAcc& z, cd a, cd b) {
    z.rr = mfma64_16x16x4(a.x, b.x, z.rr);
    z.ii = mfma64_16x16x4(a.y, b.y, z.ii);
    z.ri = mfma64_16x16x4(a.x, b.y, z.ri);
    z.ir = mfma64_16x16x4(a.y, b.x, z.ir);
}
// register v of the product: sum a b, or sum a conj(b) for CONJ
template <bool CONJ>
__device__ inline cd cacc_get(const CAcc& z, int v) {
    const double rr = z.rr[v], ii = z.ii[v], ri = z.ri[v], ir = z.ir[v];
    return CONJ ? mk(rr + ii, ir - ri) : mk(rr - ii, ri + ir);
}

// One leaf triangle, component and output orbital c.  Wave w owns the columns m of
// tile w (16w .. 16w + 15) for both products of the component, which balances
// the waves (the column sums of tile w run over rows j >= 16w, the row dots over
// columns t <= 16w + 15):
//   comp 0: column sum x(j)[a][b'] G^R_{b'c}(j,m), j >= m     -> leafR [0][m][a][c]
//           row dot x2(t)[a][b'] G^R_{cb'}(m,t)^*, t <= m     -> leafLR[0][m][a][c]
//   comp 1: row dot x1(t)[a][b'] G<_{b'c}(m,t), t <= m        -> leafLL[0][m][a][c]
//           column sum -x1(j)[a][b'] G<_{cb'}(j,m)^*, j > m   -> leafLL[1][m][a][c]
__device__ void leaf16_task(const HistArgs& A, int leaf, int comp, int c) {
    constexpr int NORB = 16, npair = 256;
    if (comp == 1 && (!A.wantL || A.adj)) return;
    const int n = A.n;
    const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
    const int lw = s1 - s0, nrow = min(s1, A.last[comp] + 1) - s0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, x = lane & 15, kk = lane >> 4;
    if (16 * wave >= nrow) return;
    const int m = 16 * wave + x;
    const cd* L = p_leaf(A, comp) + A.Loff[leaf];
    const cd* sRT = p_sigRT(A);
    const cd* sL = p_sigL(A);
    const bool colOn = comp == 1 || A.wantR;
    const bool rowOn = comp == 1 || A.wantL;
    CAcc col, row;
    cacc_zero(col);
    cacc_zero(row);
    // column sums: rows j = 16w + 4st + kk < nrow
    if (colOn) {
        const int ncs = (nrow - 16 * wave + 3) >> 2;
        for (int bp = 0; bp < NORB; ++bp) {
            const cd* T = L + (size_t)(comp == 0 ? bp * NORB + c : c * NORB + bp) * tri(lw);
#pragma unroll 4
            for (int st = 0; st < ncs; ++st) {
                const int j = 16 * wave + 4 * st + kk;
                const bool jv = j < nrow;
                const int jc = jv ? j : nrow - 1, jg = s0 + jc;
                const cd sg = sRT[(size_t)jg * npair + bp * NORB + x];
                const cd tv = T[tri(jc) + min(m, jc)];
                const double w = comp == 0 ? w_end(A.W, n, jg) : interval_w(A.W, n, jg);
                const bool bv = jv && m < nrow && (comp == 0 ? jc >= m : jc > m);
                cacc_step(col, jv ? w * sg : mk(0.0, 0.0), bv ? tv : mk(0.0, 0.0));
            }
        }
    }
    // row dots: columns t = 4st + kk <= min(16w + 15, nrow - 1)
    if (rowOn) {
        const int tend = min(16 * wave + 16, nrow);
        const int nrs = (tend + 3) >> 2;
        const bool mok = m < nrow && (comp == 1 || A.adj || s0 + m > 0);   // empty interval at m = 0
        const int mc = m < nrow ? m : nrow - 1;
        for (int bp = 0; bp < NORB; ++bp) {
            const cd* T = L + (size_t)(comp == 0 ? c * NORB + bp : bp * NORB + c) * tri(lw);
#pragma unroll 4
            for (int st = 0; st < nrs; ++st) {
                const int t = 4 * st + kk;
                const bool tv_ = t < tend;
                const int tc = tv_ ? t : tend - 1, tg = s0 + tc;
                cd xv;
                if (comp == 0) {
                    xv = A.adj ? sL[(size_t)tg * npair + x * NORB + bp]
                               : -w_start(A.W, tg) * conj(sL[(size_t)tg * npair + bp * NORB + x]);
                } else {
                    xv = interval_w(A.W, n, tg) * sRT[(size_t)tg * npair + bp * NORB + x];
                }
                const cd tv = T[tri(mc) + min(tc, mc)];
                const bool bv = tv_ && mok && tc <= m;
                cacc_step(row, tv_ ? xv : mk(0.0, 0.0), bv ? tv : mk(0.0, 0.0));
            }
        }
    }
    if (m >= nrow) return;
    const size_t sl = (size_t)A.nt * npair;
    const size_t mo = (size_t)(s0 + m) * npair + c;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int a = 4 * v + kk;
        if (comp == 0) {
            if (A.wantR) p_leafR(A)[mo + a * NORB] = cacc_get<false>(col, v);
            if (A.wantL) p_leafLR(A)[mo + a * NORB] = cacc_get<true>(row, v);
        } else {
            p_leafLL(A)[mo + a * NORB] = cacc_get<false>(row, v);
            p_leafLL(A)[sl + mo + a * NORB] = -cacc_get<true>(col, v);
        }
    }
}

// Tail rows at norb 16: component comp, output orbital c, columns [chunk*64, +64) of
// the dense tail.  Column sums: wave w owns column tile w, K over (b', tail row).
// Row dots: wave w owns tail-row tile w & 1 and the column half w >> 1, K over
// (b', column); the two halves are added through LDS.
//   comp 0: column sum x(j)[a][b'] G^R_{b'c}(j,m)          -> tailcol[0][m][a][c]
//           row dot x2(m)[a][b'] G^R_{cb'}(r,m)^*           -> tailpart[chunk][0][r][a][c]
//   comp 1: column sum -x1(j)[a][b'] G<_{cb'}(j,m)^*        -> tailcol[0][m][a][c]
//           row dot x1(m)[a][b'] G<_{b'c}(r,m)              -> tailpart[chunk][0][r][a][c]
__device__ void tail16_task(const HistArgs& A, int comp, int c, int chunk, unsigned char* smem) {
    constexpr int NORB = 16, npair = 256;
    if (comp == 1 && (!A.wantL || A.adj)) return;
    const int n = A.n, n0 = A.n0[comp], nrows = A.last[comp] - n0 + 1, ls = A.ls[comp];
    const int cbeg = chunk * kTailCH, ncol = min(kTailCH, ls - cbeg);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, x = lane & 15, kk = lane >> 4;
    const cd* Tg = p_tail(A, comp);
    const cd* sRT = p_sigRT(A);
    const cd* sL = p_sigL(A);
    const int nt = A.nt, ring = A.ring;
    const bool colOn = comp == 1 || A.wantR;
    const bool rowOn = comp == 1 || A.wantL;
    // dense columns of tail row i (relative to n0)
    auto lsr = [&](int i) { return n0 + i < A.nsplit[comp] ? A.lslo[comp] : ls; };
    // column sums
    CAcc col;
    cacc_zero(col);
    const int mcol = cbeg + 16 * wave + x;
    if (colOn && 16 * wave < ncol) {
        const int ncs = (nrows + 3) >> 2;
        const int mc = min(mcol, ls - 1);
        for (int bp = 0; bp < NORB; ++bp) {
            const int q = comp == 0 ? bp * NORB + c : c * NORB + bp;
#pragma unroll 4
            for (int st = 0; st < ncs; ++st) {
                const int i = 4 * st + kk;
                const bool iv = i < nrows;
                const int ic = iv ? i : nrows - 1, j = n0 + ic;
                const cd sg = sRT[(size_t)j * npair + bp * NORB + x];
                const double w = comp == 0 ? w_end(A.W, n, j) : interval_w(A.W, n, j);
                const cd tv = Tg[((size_t)(j % ring) * npair + q) * nt + mc];
                const bool bv = iv && mcol < cbeg + ncol && mcol < lsr(ic);
                cacc_step(col, iv ? w * sg : mk(0.0, 0.0), bv ? tv : mk(0.0, 0.0));
            }
        }
    }
    // row dots
    CAcc row;
    cacc_zero(row);
    const int rt = wave & 1, half = wave >> 1;
    const int ir = 16 * rt + x;   // this lane's tail row (B operand column)
    if (rowOn && 16 * rt < nrows) {
        const int irc = ir < nrows ? ir : nrows - 1, jr = n0 + irc;
        const int lim = min(cbeg + ncol, lsr(irc));
        const cd* Trow = Tg + (size_t)(jr % ring) * npair * nt;
        const int mb = cbeg + 32 * half;
        for (int bp = 0; bp < NORB; ++bp) {
            const int q = comp == 0 ? c * NORB + bp : bp * NORB + c;
            const cd* Tq = Trow + (size_t)q * nt;
#pragma unroll 4
            for (int st = 0; st < 8; ++st) {
                const int mm = mb + 4 * st + kk;
                const bool mv = mm < cbeg + ncol;
                const int mmc = mv ? mm : cbeg + ncol - 1;
                cd xv;
                if (comp == 0) {
                    xv = A.adj ? sL[(size_t)mmc * npair + x * NORB + bp]
                               : -w_start(A.W, mmc) * conj(sL[(size_t)mmc * npair + bp * NORB + x]);
                } else {
                    xv = interval_w(A.W, n, mmc) * sRT[(size_t)mmc * npair + bp * NORB + x];
                }
                const cd tv = Tq[min(mmc, ls - 1)];
                const bool bv = mv && ir < nrows && mmc < lim;
                cacc_step(row, mv ? xv : mk(0.0, 0.0), bv ? tv : mk(0.0, 0.0));
            }
        }
    }
    const size_t sl = (size_t)nt * npair;
    (void)sl;
    if (colOn && mcol < cbeg + ncol) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = 4 * v + kk;
            const size_t o = (size_t)mcol * npair + a * NORB + c;
            if (comp == 0) p_tailcol(A, 0)[o] = cacc_get<false>(col, v);
            else p_tailcol(A, 1)[o] = -cacc_get<true>(col, v);
        }
    }
    // the two column halves of the row dots: the upper half's waves hand theirs over
    cd* red = reinterpret_cast<cd*>(smem);   // [rt][v][lane]
    cd rv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) rv[v] = comp == 0 ? cacc_get<true>(row, v) : cacc_get<false>(row, v);
    if (half == 1)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((size_t)rt * 4 + v) * 64 + lane] = rv[v];
    __syncthreads();
    if (half == 0 && rowOn && ir < nrows) {
        cd* tp = p_tailpart(A, comp) + ((size_t)chunk * ring + ir) * npair + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) tp[(4 * v + kk) * NORB] = rv[v] + red[((size_t)rt * 4 + v) * 64 + lane];
    }
}

// Dense pieces at norb 16: tail tasks first (ntailtask: column chunks of both
// components x 16 output orbitals), then the leaves (2 * nleaf x 16); the 16 tasks
// of one chunk or leaf land on one XCD.
__global__ void __launch_bounds__(256) dense16(HistArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    int rel = blockIdx.x;
    int g, mem;
    if (rel < A.ntailtask) {
        if (!xcd_group(rel, A.ntailchunk[0] + A.ntailchunk[1], 16, g, mem)) return;
        if (g < A.ntailchunk[0]) tail16_task(A, 0, mem, g, smem);
        else tail16_task(A, 1, mem, g - A.ntailchunk[0], smem);
        return;
    }
    rel -= A.ntailtask;
    if (!xcd_group(rel, 2 * A.nleaf, 16, g, mem)) return;
    leaf16_task(A, g >> 1, g & 1, mem);
}

// ---------------------------------------------------------------------------
// Combine of the FP32-factor form at norb = 16 on the matrix cores.  A workgroup
// takes 16 consecutive columns m (a tile inside one leaf: every block boundary is
// a multiple of 16), wave w the output orbitals c = w, w+4, w+8, w+12.  For each
// level the tile's columns are columns (expansion through V) or rows (through U)
// of one block, and each expansion is the product
//   Y[a][m] (+|-)= sum over o, r of z_{q(o)}[a][r] op(F_{q(o)}[r][m])
// with A = z (16 orbitals a x 4 ranks, FP32 from the FP64 projections) and B =
// the factor rows of the tile's columns: four real 16x16x4 chains per 4 ranks.
// Each expansion (one block and component) is a K tile whose FP32 sum is added to
// the running sum with TwoSum compensation; the FP64 sum of the two then goes
// through the same leaf, tail and band pieces as every other form.

// one expansion into (s, e); rows of F whose column is not valid (colok) are zero
template <bool CONJ, bool NEG>
__device__ void expand_mfma(const HistArgs& A, int comp, int b, int which, bool q_row_c, int c, const cf* Fb,
                            int ld, int col, bool colok, float (&sr)[4], float (&er)[4], float (&si)[4],
                            float (&ei)[4]) {
    constexpr int NORB = 16;
    const int lane = threadIdx.x & 63, j = lane & 15, kk = lane >> 4;
    const int RC = A.RC;
    v4f rr = {0.f, 0.f, 0.f, 0.f}, ii = rr, ri = rr, ir = rr;
    // operands of pair o: ranks 4u + kk, u < 4, indices clamped to the capacity (the
    // rank mask is applied where they are used, so the loads do not wait for it)
    cd zc[4], zn[4];
    cf fc[4], fn[4];
    int rkc = 0, rkn = 0;
    auto fetch = [&](int o, cd (&z)[4], cf (&f)[4], int& rk) {
        const int q = q_row_c ? c * NORB + o : o * NORB + c;
        rk = rank_of(A, comp, b, q);
        const cf* F = Fb + (size_t)q * RC * ld + col;
        const cd* zq = p_proj(A) + proj_slot(A, comp, b, q, which) * NORB * RC + (size_t)j * RC;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = min(4 * u + kk, RC - 1);
            z[u] = zq[r];
            f[u] = F[(size_t)r * ld];
        }
    };
    fetch(0, zc, fc, rkc);
    for (int o = 0; o < NORB; ++o) {
        if (o + 1 < NORB) fetch(o + 1, zn, fn, rkn);
        const int nq = (rkc + 3) >> 2;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (u < nq) {
                const bool ok = 4 * u + kk < rkc;
                const float zr = ok ? (float)zc[u].x : 0.f, zi = ok ? (float)zc[u].y : 0.f;
                const float fr = colok ? fc[u].x : 0.f, fi = colok ? fc[u].y : 0.f;
                rr = mfma_16x16x4(zr, fr, rr);
                ii = mfma_16x16x4(zi, fi, ii);
                ri = mfma_16x16x4(zr, fi, ri);
                ir = mfma_16x16x4(zi, fr, ir);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            zc[u] = zn[u];
            fc[u] = fn[u];
        }
        rkc = rkn;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        float yr = CONJ ? rr[v] + ii[v] : rr[v] - ii[v];
        float yi = CONJ ? ir[v] - ri[v] : ri[v] + ir[v];
        if (NEG) {
            yr = -yr;
            yi = -yi;
        }
        two_sum_acc(sr[v], er[v], yr);
        two_sum_acc(si[v], ei[v], yi);
    }
}

__global__ void __launch_bounds__(256) combine_mfma(HistArgs A) {
    constexpr int NORB = 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, kk = lane >> 4;
    const int m0 = blockIdx.x * 16, m = m0 + j;
    const int n = A.n;
    if (m0 > n) return;
    for (int ci = 0; ci < 4; ++ci) {
        const int c = wave + 4 * ci;
        float Rsr[4] = {0.f, 0.f, 0.f, 0.f}, Rer[4] = {0.f, 0.f, 0.f, 0.f};
        float Rsi[4] = {0.f, 0.f, 0.f, 0.f}, Rei[4] = {0.f, 0.f, 0.f, 0.f};
        float Lsr[4] = {0.f, 0.f, 0.f, 0.f}, Ler[4] = {0.f, 0.f, 0.f, 0.f};
        float Lsi[4] = {0.f, 0.f, 0.f, 0.f}, Lei[4] = {0.f, 0.f, 0.f, 0.f};
        for (int l = 0; l < A.nlvl; ++l) {
            const int cv = A.cover[(size_t)l * A.nt + m0];
            if (cv >= 0) {   // the tile's columns are columns of block b: expand through V
                const int b = cv;
                const int r0 = A.blk[5 * b + 1], c0 = A.blk[5 * b + 3], c1 = A.blk[5 * b + 4];
                const int ld = c1 - c0, col = min(m - c0, ld - 1);
                if (A.wantR && A.n0[0] > r0)
                    expand_mfma<true, false>(A, 0, b, 0, false, c, p_V<cf>(A, 0, b) + A.Voff[b], ld, col, true,
                                             Rsr, Rer, Rsi, Rei);
                if (A.wantL && !A.adj && A.n0[1] > r0)
                    expand_mfma<false, true>(A, 1, b, 0, true, c, p_V<cf>(A, 1, b) + A.Voff[b], ld, col, true,
                                             Lsr, Ler, Lsi, Lei);
            } else if (A.wantL) {   // rows of block b: expand through U (merged rows only)
                const int b = ~cv;
                const int r0 = A.blk[5 * b + 1], r1 = A.blk[5 * b + 2];
                const int ld = r1 - r0, col = min(m - r0, ld - 1);
                if (m0 < A.n0[0])
                    expand_mfma<true, false>(A, 0, b, 1, true, c, p_U<cf>(A, 0, b) + A.Uoff[b], ld, col,
                                             m < A.n0[0], Lsr, Ler, Lsi, Lei);
                if (!A.adj && m0 < A.n0[1])
                    expand_mfma<false, false>(A, 1, b, 1, false, c, p_U<cf>(A, 1, b) + A.Uoff[b], ld, col,
                                              m < A.n0[1], Lsr, Ler, Lsi, Lei);
            }
        }
        if (m > n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = 4 * kk + v;
            const cd yL = mk((double)Lsr[v] + (double)Ler[v], (double)Lsi[v] + (double)Lei[v]);
            if (A.adj) {
                finish_entry<NORB>(A, m, a, c, 1, yL);
            } else {
                if (A.wantR)
                    finish_entry<NORB>(A, m, a, c, 0,
                                       mk((double)Rsr[v] + (double)Rer[v], (double)Rsi[v] + (double)Rei[v]));
                if (A.wantL) finish_entry<NORB>(A, m, a, c, 1, yL);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Gradient of a real loss with respect to the retarded factors of the current
// (frozen) state: the contributions of step n.  With x_n(j) the folded Sigma^R row
// and Ibar(n, m) the cotangent of I^R(n, m), the gradient of block b, pair
// q = (b', c), with respect to its entries is
//   Gbar(j, m) = h sum_n w^{(n-m)}_{j-m} sum_a conj(Sigma^R(n,j)[a][b']) Ibar(n,m)[a][c]
// (the transpose of Eq. KBER's history sum), and through G = U S V^H
//   Ubar = Gbar V S,   Vbar = Gbar^H U S,   Sbar = Re diag(U^H Gbar V).
// The bulk weight w_end(n, j) is folded into x_n, so the bulk parts need only the
// step's projections P0 = S_r (x_n U)[a][r] and P1 = S_r (Ibar_n V)[a][r]:
//   Ubar(j, r) += h sum_a conj(x_n(j)[a][b']) P1[a][r]
//   Vbar(m, r) += h sum_a conj(Ibar(n,m)[a][c]) P0[a][r]
//   Sbar(r)    += h sum_a Re(conj(P0[a][r]) P1[a][r]) / S_r^2
// The block entries within k of the diagonal (j - m <= k, the corner next to the
// leaf boundary), whose exact weight w^{(n-m)}_{j-m} differs from w_end(n, j), are
// added with the weight difference.  One thread per (pair, rank, U row | V row |
// S), so every output entry has one writer; the block is blockIdx.x / xper (a single
// object: grid.y = 1, which the accessors take as the object index).
template <int NORB>
__global__ void __launch_bounds__(256) fgrad_kernel(HistArgs A, int xper) {
    constexpr int npair = NORB * NORB;
    const int b = blockIdx.x / xper;
    const int* bk = A.blk + 5 * b;
    const int r0 = bk[1], r1 = bk[2], c0 = bk[3], c1 = bk[4];
    const int n = A.n;
    if (r0 > n || A.n0[0] <= r0) return;   // no merged row of the block at or below n
    const int ldU = r1 - r0, ldV = c1 - c0, RC = A.RC, k = A.W.k;
    const long long per = (long long)ldU + ldV + 1;
    const long long t = (long long)(blockIdx.x % xper) * 256 + threadIdx.x;
    if (t >= per * RC * npair) return;
    const int row = (int)(t % per);
    const int r = (int)((t / per) % RC);
    const int q = (int)(t / (per * RC));
    const int rk = rank_of(A, 0, b, q);
    if (r >= rk) return;
    const int qr = q / NORB, qc = q % NORB;
    const int jend = min(A.n0[0], n + 1);   // merged rows at or below n
    const long long buf = buf_of(A, 0, b);
    const cd* Uq = A.Ud + buf * A.bU + A.Uoff[b] + (size_t)q * RC * ldU + (size_t)r * ldU;
    const cd* Vq = A.Vd + buf * A.bV + A.Voff[b] + (size_t)q * RC * ldV + (size_t)r * ldV;
    const double Sr = p_S(A, 0, b)[((size_t)b * npair + q) * RC + r];
    const cd* P0 = p_proj(A) + proj_slot(A, 0, b, q, 0) * NORB * RC + r;
    const cd* P1 = p_proj(A) + proj_slot(A, 0, b, q, 1) * NORB * RC + r;
    const cd* sR = p_sigR(A);
    const cd* ib = p_sigL(A);   // Ibar(n, m)
    // corner term: h (w^{(n-m)}_{j-m} - w_end(n, j)) sum_a conj(Sigma(n,j)[a][b']) Ibar(n,m)[a][c]
    auto gcorner = [&](int j, int m) -> cd {
        const double dw = interval_w(A.W, n - m, j - m) - w_end(A.W, n, j);
        cd g = mk(0.0, 0.0);
        for (int a = 0; a < NORB; ++a) fmac_(g, sR[(size_t)j * npair + a * NORB + qr], ib[(size_t)m * npair + a * NORB + qc]);
        return (A.h * dw) * g;
    };
    if (row < ldU) {
        const int j = r0 + row;
        if (j >= jend) return;
        const double we = w_end(A.W, n, j);
        cd acc = mk(0.0, 0.0);
        for (int a = 0; a < NORB; ++a) fmac_(acc, sR[(size_t)j * npair + a * NORB + qr], P1[(size_t)a * RC]);
        acc = (A.h * we) * acc;
        for (int m = max(c0, j - k); m < c1; ++m) acc = acc + Sr * (gcorner(j, m) * Vq[m - c0]);
        cd* d = A.dU + A.Uoff[b] + (size_t)q * RC * ldU + (size_t)r * ldU + row;
        *d = *d + acc;
    } else if (row < ldU + ldV) {
        const int m = c0 + row - ldU;
        cd acc = mk(0.0, 0.0);
        for (int a = 0; a < NORB; ++a) fmac_(acc, ib[(size_t)m * npair + a * NORB + qc], P0[(size_t)a * RC]);
        acc = A.h * acc;
        for (int j = r0; j < min(m + k + 1, jend); ++j) acc = acc + Sr * (conj(gcorner(j, m)) * Uq[j - r0]);
        cd* d = A.dV + A.Voff[b] + (size_t)q * RC * ldV + (size_t)r * ldV + (m - c0);
        *d = *d + acc;
    } else {
        double acc = 0.0;
        for (int a = 0; a < NORB; ++a) {
            const cd p0 = P0[(size_t)a * RC], p1 = P1[(size_t)a * RC];
            acc += p0.x * p1.x + p0.y * p1.y;
        }
        acc *= A.h / (Sr * Sr);
        for (int j = r0; j < min(c1 + k, jend); ++j)
            for (int m = max(c0, j - k); m < c1; ++m) {
                const cd g = gcorner(j, m) * Vq[m - c0];
                acc += Uq[j - r0].x * g.x + Uq[j - r0].y * g.y;   // Re(conj(U) g)
            }
        A.dS[((size_t)b * npair + q) * RC + r] += acc;
    }
}

size_t tasks_smem(int norb, bool mfproj, int kc) {
    const int ag = norb < 4 ? norb : 4;
    size_t fact = mfproj ? (size_t)kc * kXS * sizeof(cf) : (size_t)(kc * norb + 4 * 32 * norb) * sizeof(cd);
    // per-pair leaf tasks (norb <= 4) stage the strictly lower triangle, the others all of it
    size_t leaf = (size_t)((norb <= 4 ? tri(63) : tri(64)) + 2 * 64 * ag) * sizeof(cd);
    size_t tail = (size_t)(kTailRows * kTailCH + (kTailRows + kTailCH) * ag) * sizeof(cd);
    size_t s = fact > leaf ? fact : leaf;
    return s > tail ? s : tail;
}

// sigRT[j][b][a] = sigR[j][a][b] for j <= n (norb 16): the matrix-core kernels read the
// 16 left orbitals a of one (j, b) as consecutive words
__global__ void __launch_bounds__(256) sig_transpose16(const cd* sigR, cd* sigRT, long long kIn, long long kInT) {
    const long long j = blockIdx.x;
    const int t = threadIdx.x;
    const cd v = sigR[(long long)blockIdx.y * kIn + j * 256 + t];
    sigRT[(long long)blockIdx.y * kInT + j * 256 + (t & 15) * 16 + (t >> 4)] = v;
}

template <int NORB, class FT>
hipError_t launch_t(const HistArgs& a, hipStream_t st, hipEvent_t* ev) {
    const bool mf = NORB == 16 && std::is_same<FT, cf>::value && a.mfproj;
    if (ev) hipEventRecord(ev[0], st);
    if constexpr (NORB == 16) {
        if (a.sigR) sig_transpose16<<<dim3(a.n + 1, a.nk), 256, 0, st>>>(a.sigR, a.sigRT, a.kIn, a.kInT);
        // projections (matrix-core kernel or the generic tasks), then the dense pieces
        if (mf && a.nf[0] + a.nf[1] > 0)
            proj_mfma<<<dim3(a.nf[0] + a.nf[1], a.nk), NT, (size_t)a.kch * kXS * sizeof(cf), st>>>(a);
        if (!mf && a.nfpad > 0) {
            HistArgs b = a;
            b.ntailtask = 0;
            b.nleaftask = 0;
            hist_tasks<NORB, FT><<<dim3(a.nfpad, a.nk), NT, tasks_smem(NORB, false, a.kch), st>>>(b);
        }
        if (a.ntailtask + a.nleaftask > 0)
            dense16<<<dim3(a.ntailtask + a.nleaftask, a.nk), 256, 8 * 64 * sizeof(cd), st>>>(a);
    } else {
        const int ntask = a.nfpad + a.nleaftask + a.ntailtask;
        if (ntask > 0) hist_tasks<NORB, FT><<<dim3(ntask, a.nk), NT, tasks_smem(NORB, false, a.kch), st>>>(a);
    }
    if (ev) hipEventRecord(ev[1], st);
    {
        const long long nb1 = proj_reduce_blocks(a), nb2 = (2LL * a.ring * NORB * NORB + 3) / 4;
        proj_reduce<NORB><<<dim3((unsigned)(nb1 + nb2), a.nk), 256, 0, st>>>(a);
    }
    if (ev) hipEventRecord(ev[2], st);
    using M = CombMap<NORB>;
    if (a.fgrad) {
        // threads of the largest block: (U rows + V rows + 1) x RC x pairs
        const long long mx = (long long)(a.nt + 1) * a.RC * NORB * NORB;
        const int xper = (int)((mx + 255) / 256);
        fgrad_kernel<NORB><<<dim3((unsigned)((long long)xper * a.nb), 1), 256, 0, st>>>(a, xper);
    } else if (mf && a.mfcomb) {
        combine_mfma<<<dim3((a.n + 16) / 16, a.nk), 256, 0, st>>>(a);
    } else {
        const int nblk = (a.n + 1 + M::MW - 1) / M::MW;
        hist_combine<NORB, FT><<<dim3(nblk, a.nk), 64 * M::WAVES, 0, st>>>(a);
    }
    if (ev) hipEventRecord(ev[3], st);
    return hipGetLastError();
}

template <int NORB>
hipError_t launch_n(const HistArgs& a, hipStream_t st, hipEvent_t* ev) {
    return a.f32 ? launch_t<NORB, cf>(a, st, ev) : launch_t<NORB, cd>(a, st, ev);
}

}  // namespace

hipError_t launch_history(const HistArgs& a, hipStream_t st, hipEvent_t* ev) {
    switch (a.norb) {
        case 1: return launch_n<1>(a, st, ev);
        case 2: return launch_n<2>(a, st, ev);
        case 4: return launch_n<4>(a, st, ev);
        case 8: return launch_n<8>(a, st, ev);
        case 16: return launch_n<16>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t history_init() {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f, int norb) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)tasks_smem(norb, false, kch_max(norb)));
    };
    set((const void*)hist_tasks<1, cd>, 1);
    set((const void*)hist_tasks<1, cf>, 1);
    set((const void*)hist_tasks<2, cd>, 2);
    set((const void*)hist_tasks<2, cf>, 2);
    set((const void*)hist_tasks<4, cd>, 4);
    set((const void*)hist_tasks<4, cf>, 4);
    set((const void*)hist_tasks<8, cd>, 8);
    set((const void*)hist_tasks<8, cf>, 8);
    set((const void*)hist_tasks<16, cd>, 16);
    set((const void*)hist_tasks<16, cf>, 16);
    return e;
}

}  // namespace hn
