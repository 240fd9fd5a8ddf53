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

namespace hn {

namespace {

constexpr int NT = 256;
constexpr int CH = kCH;

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

// ranks come from device memory: clamp them to the allocated capacity
__device__ inline int rank_of(const HistArgs& A, int comp, int b, int q) {
    const int r = A.rank[comp][(size_t)b * A.npair + q];
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
    static constexpr int LG = NORB == 1 ? 1 : 4;
};

// ---------------------------------------------------------------------------
// Projection of the whole U (which = 0, rows merged so far) or V (which = 1)
// of one block and orbital pair, by one workgroup (no cross-workgroup
// reduction, hence no device-scope fences).  Wave w takes the ranks
// r = w, w+4, ...; its lanes run over the rows; the Sigma rows are staged in
// LDS per kCH rows and shared by the four waves.
template <int NORB>
__device__ void fact_task(const HistArgs& A, const FactTask& t, unsigned char* smem) {
    const int comp = t.comp, b = t.b, q = t.q, which = t.which;
    if (comp == 0 && which == 0 && !A.wantR) return;
    if ((comp == 1 || which == 1) && !A.wantL) return;
    constexpr int npair = NORB * NORB;
    constexpr bool kStage = NORB <= 4;             // Sigma rows staged in LDS
    constexpr int RW = 4;                          // ranks per wave (rank capacity <= 16)
    const int RC = A.RC;
    const int qr = q / NORB, qc = q % NORB;
    const int rk = rank_of(A, comp, b, q);
    if (rk == 0) return;
    const int* bk = A.blk + 5 * b;
    const int r0 = bk[1], r1 = bk[2], c0 = bk[3], c1 = bk[4];
    int len, base, ld;
    const cd* F;
    if (which == 0) {
        len = min(A.n0[comp] - r0, r1 - r0);
        base = r0;
        ld = r1 - r0;
        F = A.U[comp] + A.Uoff[b] + (size_t)q * RC * ld;
    } else {
        len = c1 - c0;
        base = c0;
        ld = c1 - c0;
        F = A.V[comp] + A.Voff[b] + (size_t)q * RC * ld;
    }
    const int n = A.n;
    // folded Sigma entry multiplying row i of the factor, left orbital a
    auto xval = [&](int i, int a) -> cd {
        const int j = base + i;
        if (comp == 0 && which == 0) return w_end(A.W, n, j) * A.sigR[(size_t)j * npair + a * NORB + qr];
        if (comp == 0) return -w_start(A.W, j) * conj(A.sigL[(size_t)j * npair + qc * NORB + a]);
        return interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + a * NORB + (which == 0 ? qc : qr)];
    };
    cd* xs = reinterpret_cast<cd*>(smem);  // CH x NORB
    const bool cj = (comp == 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    cd acc[RW][NORB];
#pragma unroll
    for (int k = 0; k < RW; ++k)
#pragma unroll
        for (int a = 0; a < NORB; ++a) acc[k][a] = mk(0.0, 0.0);
    for (int i0 = 0; i0 < len; i0 += CH) {
        const int i1 = min(len, i0 + CH);
        if (kStage) {
            __syncthreads();
            for (int e = threadIdx.x; e < (i1 - i0) * NORB; e += NT) xs[e] = xval(i0 + e / NORB, e % NORB);
            __syncthreads();
        }
        for (int i = i0 + lane; i < i1; i += 64) {
            cd xv[NORB];
#pragma unroll
            for (int a = 0; a < NORB; ++a) xv[a] = kStage ? xs[(size_t)(i - i0) * NORB + a] : xval(i, a);
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int r = wave + 4 * k;
                if (r < rk) {
                    cd f = F[(size_t)r * ld + i];
                    if (cj) f = conj(f);
#pragma unroll
                    for (int a = 0; a < NORB; ++a) fma_(acc[k][a], xv[a], f);
                }
            }
        }
    }
    const double* S = A.S[comp] + ((size_t)b * npair + q) * RC;
    cd* out = A.proj + proj_slot(A, comp, b, q, which) * (size_t)NORB * RC;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const int r = wave + 4 * k;
        if (r >= rk) continue;   // wave-uniform
        const double sr = S[r];
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            const double re = wsum64(acc[k][a].x), im = wsum64(acc[k][a].y);
            if (lane == 0) out[(size_t)a * RC + r] = mk(sr * re, sr * im);
        }
    }
}

// ---------------------------------------------------------------------------
// One leaf triangle and component; wave w handles the left orbital index
// a = 4*ag + w, lanes the leaf's columns m.  Each orbital pair's triangle is
// staged in LDS with coalesced loads; the column sum (rows j >= m) and the row
// dot (columns s <= m) of lane m run in one loop over LDS.
template <int NORB>
__device__ void leaf_task(const HistArgs& A, int leaf, int comp, int ag, int pg, unsigned char* smem) {
    if (comp == 1 && !A.wantL) return;
    constexpr int npair = NORB * NORB, AG = AGroups<NORB>::AG;
    constexpr int PPG = npair / LeafGroups<NORB>::LG;   // orbital pairs per group
    const int n = A.n;
    const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
    const int lw = s1 - s0;
    const int nrow = min(s1, n + 1) - s0;
    const cd* L = A.leaf[comp] + A.Loff[leaf];
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
    for (int q = pg * PPG; q < (pg + 1) * PPG; ++q) {
        const int qr = q / NORB, qc = q % NORB;
        const cd* Lq = L + (size_t)q * tsz;
        __syncthreads();
        for (long long e = threadIdx.x; e < tnow; e += NT) T[e] = Lq[e];
        for (int e = threadIdx.x; e < nrow * AG; e += NT) {
            const int i = e / AG, aa = ag * AG + e % AG, j = s0 + i;
            if (comp == 0) {
                xa[e] = w_end(A.W, n, j) * A.sigR[(size_t)j * npair + aa * NORB + qr];
                xb[e] = doL ? -w_start(A.W, j) * conj(A.sigL[(size_t)j * npair + qc * NORB + aa]) : mk(0.0, 0.0);
            } else {
                xa[e] = interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + aa * NORB + qr];
                xb[e] = interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + aa * NORB + qc];
            }
        }
        __syncthreads();
        if (act) {
            cd colsum = mk(0.0, 0.0), rowdot = mk(0.0, 0.0);
            const cd* rowm = T + tri(mo);
            const int w = wave;
            if (comp == 0) {
                // column sum x(j) G^R(j, m), j = m..; row dot x2(s) G^R(m, s)^dagger, s <= m
                const bool rowok = doL && (s0 + mo > 0);   // second lesser term is empty at m = 0
                for (int t = 0; t < nrow; ++t) {
                    const int j = mo + t;
                    if (doR && j < nrow) fma_(colsum, xa[j * AG + w], T[tri(j) + mo]);
                    if (rowok && t <= mo) fmac_(rowdot, rowm[t], xb[t * AG + w]);
                }
                accA[qc] = accA[qc] + colsum;   // -> I^R column m
                accB[qr] = accB[qr] + rowdot;   // -> I^< (second term) row m
            } else {
                // row dot x1(s) G^<(s, m) for s <= m; column sum -x1(s) G^<(m, s)^dagger for s > m
                for (int t = 0; t < nrow; ++t) {
                    const int j = mo + 1 + t;
                    if (t <= mo) fma_(rowdot, xa[t * AG + w], rowm[t]);
                    if (j < nrow) fmac_(colsum, T[tri(j) + mo], xb[j * AG + w]);
                }
                accA[qc] = accA[qc] + rowdot;
                accA[qr] = accA[qr] - colsum;
            }
        }
    }
    if (act) {
        const int m = s0 + mo;
#pragma unroll
        for (int c = 0; c < NORB; ++c) {
            const size_t o = ((size_t)pg * A.nt + m) * npair + a * NORB + c;
            if (comp == 0) {
                A.leafR[o] = accA[c];
                A.leafLR[o] = accB[c];
            } else {
                A.leafLL[o] = accA[c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Rows appended since the last panel merge (dense), columns [chunk*64, +64) of
// [0, ls): the column sums over those rows are complete here; the row dots are
// written per column chunk and summed by the combine.
template <int NORB>
__device__ void tail_task(const HistArgs& A, int comp, int ag, int chunk, unsigned char* smem) {
    if (comp == 1 && !A.wantL) return;
    constexpr int npair = NORB * NORB, AG = AGroups<NORB>::AG;
    const int n = A.n;
    const int n0 = A.n0[comp], nrows = A.last[comp] - n0 + 1, ls = A.ls[comp];
    const int cbeg = chunk * kTailCH, ncol = min(kTailCH, ls - cbeg);
    cd* T = reinterpret_cast<cd*>(smem);       // P x 64
    cd* xr = T + (size_t)A.P * kTailCH;        // P x AG   (row-side Sigma)
    cd* xm = xr + (size_t)A.P * AG;            // 64 x AG  (column-side Sigma)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = ag * AG + wave;
    const bool wok = wave < AG;
    const bool doR = A.wantR, doL = A.wantL;
    const cd* Tg = A.tail[comp];
    cd col[NORB], row[NORB];
#pragma unroll
    for (int c = 0; c < NORB; ++c) col[c] = row[c] = mk(0.0, 0.0);
    const int ri = lane & 15, part = lane >> 4;   // row-dot mapping: row ri, 16 columns per part
    for (int q = 0; q < npair; ++q) {
        const int qr = q / NORB, qc = q % NORB;
        __syncthreads();
        for (int e = threadIdx.x; e < nrows * kTailCH; e += NT) {
            const int i = e / kTailCH, mm = e % kTailCH;
            T[e] = mm < ncol ? Tg[((size_t)i * npair + q) * A.nt + cbeg + mm] : mk(0.0, 0.0);
        }
        for (int e = threadIdx.x; e < nrows * AG; e += NT) {
            const int i = e / AG, aa = ag * AG + e % AG, j = n0 + i;
            xr[e] = comp == 0 ? w_end(A.W, n, j) * A.sigR[(size_t)j * npair + aa * NORB + qr]
                              : interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + aa * NORB + qc];
        }
        for (int e = threadIdx.x; e < kTailCH * AG; e += NT) {
            const int mm = e / AG, aa = ag * AG + e % AG, m = cbeg + mm;
            cd v = mk(0.0, 0.0);
            if (mm < ncol) {
                if (comp == 0) {
                    if (doL) v = -w_start(A.W, m) * conj(A.sigL[(size_t)m * npair + qc * NORB + aa]);
                } else {
                    v = interval_w(A.W, n, m) * A.sigR[(size_t)m * npair + aa * NORB + qr];
                }
            }
            xm[e] = v;
        }
        __syncthreads();
        if (wok) {
            // column sums (lane = column)
            cd cs = mk(0.0, 0.0);
            for (int i = 0; i < nrows; ++i) {
                if (comp == 0) fma_(cs, xr[i * AG + wave], T[i * kTailCH + lane]);
                else fmac_(cs, T[i * kTailCH + lane], xr[i * AG + wave]);
            }
            if (comp == 0) {
                if (doR) col[qc] = col[qc] + cs;     // x(j) G^R(j, m)
            } else {
                col[qr] = col[qr] - cs;              // -x1(j) G^<(m, j)^dagger
            }
            // row dots (lane = row ri, columns 16*part .. +16)
            cd rd = mk(0.0, 0.0);
            if (ri < nrows) {
                for (int mm = part * 16; mm < part * 16 + 16; ++mm) {
                    if (comp == 0) fmac_(rd, T[ri * kTailCH + mm], xm[mm * AG + wave]);
                    else fma_(rd, xm[mm * AG + wave], T[ri * kTailCH + mm]);
                }
            }
            if (comp == 0) row[qr] = row[qr] + rd;   // x2(m) G^R(j, m)^dagger
            else row[qc] = row[qc] + rd;             // x1(m) G^<(m, j)
        }
    }
    // reduce the four column parts of each row dot (lanes ri, ri+16, ri+32, ri+48)
#pragma unroll
    for (int c = 0; c < NORB; ++c) {
        double re = row[c].x, im = row[c].y;
        re += __shfl_xor(re, 16, 64);
        im += __shfl_xor(im, 16, 64);
        re += __shfl_xor(re, 32, 64);
        im += __shfl_xor(im, 32, 64);
        row[c] = mk(re, im);
    }
    if (wok) {
        if (lane < ncol) {
#pragma unroll
            for (int c = 0; c < NORB; ++c)
                A.tailcol[comp][(size_t)(cbeg + lane) * npair + a * NORB + c] = col[c];
        }
        if (part == 0 && ri < nrows) {
            cd* tp = A.tailpart[comp] + ((size_t)chunk * A.P + ri) * npair + a * NORB;
#pragma unroll
            for (int c = 0; c < NORB; ++c) tp[c] = row[c];
        }
    }
}

template <int NORB>
__global__ void __launch_bounds__(NT) hist_tasks(HistArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NG = AGroups<NORB>::NG;
    int id = blockIdx.x;
    if (id < A.nf[0]) {
        fact_task<NORB>(A, A.ft[0][id], smem);
        return;
    }
    id -= A.nf[0];
    if (id < A.nf[1]) {
        fact_task<NORB>(A, A.ft[1][id], smem);
        return;
    }
    id -= A.nf[1];
    if (id < A.nleaftask) {
        constexpr int LG = LeafGroups<NORB>::LG;
        int g, mem;
        if (!xcd_group(id, 2 * A.nleaf, NG * LG, g, mem)) return;
        leaf_task<NORB>(A, g >> 1, g & 1, mem % NG, mem / NG, smem);
        return;
    }
    id -= A.nleaftask;
    int g, ag;
    const int ng = A.ntailchunk[0] + A.ntailchunk[1];
    if (!xcd_group(id, ng, NG, g, ag)) return;
    if (g < A.ntailchunk[0])
        tail_task<NORB>(A, 0, ag, g, smem);
    else
        tail_task<NORB>(A, 1, ag, g - A.ntailchunk[0], smem);
}

// ---------------------------------------------------------------------------
// One thread per output (m, c); all left orbital indices a in registers.
template <int NORB>
__global__ void __launch_bounds__(64 * NORB) hist_combine(HistArgs A) {
    constexpr int npair = NORB * NORB;
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const int c = threadIdx.x >> 6;
    const int n = A.n;
    if (m > n) return;
    const int RC = A.RC;
    cd accR[NORB], accL[NORB];
#pragma unroll
    for (int a = 0; a < NORB; ++a) accR[a] = accL[a] = mk(0.0, 0.0);
    for (int l = 0; l < A.nlvl; ++l) {
        const int cv = A.cover[(size_t)l * A.nt + m];
        if (cv >= 0) {  // m is a column of block b: expand through V
            const int b = cv;
            const int r0 = A.blk[5 * b + 1], c0 = A.blk[5 * b + 3], c1 = A.blk[5 * b + 4];
            const int ldV = c1 - c0;
            if (A.wantR && A.n0[0] > r0) {
                for (int qr = 0; qr < NORB; ++qr) {
                    const int q = qr * NORB + c;
                    const int rk = rank_of(A, 0, b, q);
                    const cd* Vq = A.V[0] + A.Voff[b] + (size_t)q * RC * ldV + (m - c0);
                    const cd* z = A.proj + proj_slot(A, 0, b, q, 0) * NORB * RC;
                    for (int r = 0; r < rk; ++r) {
                        const cd v = Vq[(size_t)r * ldV];
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fmac_(accR[a], v, z[a * RC + r]);
                    }
                }
            }
            if (A.wantL && A.n0[1] > r0) {
                for (int qc = 0; qc < NORB; ++qc) {
                    const int q = c * NORB + qc;
                    const int rk = rank_of(A, 1, b, q);
                    const cd* Vq = A.V[1] + A.Voff[b] + (size_t)q * RC * ldV + (m - c0);
                    const cd* z = A.proj + proj_slot(A, 1, b, q, 0) * NORB * RC;
                    for (int r = 0; r < rk; ++r) {
                        const cd v = -Vq[(size_t)r * ldV];
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fma_(accL[a], v, z[a * RC + r]);
                    }
                }
            }
        } else if (A.wantL) {  // m is a row of block b: expand through U
            const int b = ~cv;
            const int r0 = A.blk[5 * b + 1], r1 = A.blk[5 * b + 2];
            const int ldU = r1 - r0;
            if (m < A.n0[0]) {
                for (int qc = 0; qc < NORB; ++qc) {
                    const int q = c * NORB + qc;
                    const int rk = rank_of(A, 0, b, q);
                    const cd* Uq = A.U[0] + A.Uoff[b] + (size_t)q * RC * ldU + (m - r0);
                    const cd* z = A.proj + proj_slot(A, 0, b, q, 1) * NORB * RC;
                    for (int r = 0; r < rk; ++r) {
                        const cd u = Uq[(size_t)r * ldU];
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fmac_(accL[a], u, z[a * RC + r]);
                    }
                }
            }
            if (m < A.n0[1]) {
                for (int qr = 0; qr < NORB; ++qr) {
                    const int q = qr * NORB + c;
                    const int rk = rank_of(A, 1, b, q);
                    const cd* Uq = A.U[1] + A.Uoff[b] + (size_t)q * RC * ldU + (m - r0);
                    const cd* z = A.proj + proj_slot(A, 1, b, q, 1) * NORB * RC;
                    for (int r = 0; r < rk; ++r) {
                        const cd u = Uq[(size_t)r * ldU];
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fma_(accL[a], u, z[a * RC + r]);
                    }
                }
            }
        }
    }
    const size_t mo = (size_t)m * npair;
    constexpr int LG = LeafGroups<NORB>::LG;
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
        const size_t o = mo + a * NORB + c;
        for (int pg = 0; pg < LG; ++pg) {
            const size_t op = (size_t)pg * A.nt * npair + o;
            if (A.wantR) accR[a] = accR[a] + A.leafR[op];
            if (A.wantL) accL[a] = accL[a] + A.leafLR[op] + A.leafLL[op];
        }
        if (A.wantR) {
            if (A.last[0] >= A.n0[0] && m < A.ls[0]) accR[a] = accR[a] + A.tailcol[0][o];
        }
        if (A.wantL) {
            for (int comp = 0; comp < 2; ++comp) {
                if (A.last[comp] < A.n0[comp]) continue;   // no tail rows
                if (comp == 1 && m < A.ls[1]) accL[a] = accL[a] + A.tailcol[1][o];
                if (m >= A.n0[comp] && m <= A.last[comp]) {
                    const cd* tp = A.tailpart[comp] + (size_t)(m - A.n0[comp]) * npair + a * NORB + c;
                    for (int ch = 0; ch < A.ntailchunk[comp]; ++ch)
                        accL[a] = accL[a] + tp[(size_t)ch * A.P * npair];
                }
            }
        }
    }
    const int k = A.W.k;
    const int kb = k + 1;
    if (A.wantR) {
        // band correction: start weights (n-m >= k) or Newton-Cotes (n-m < k)
        const int L = n - m;
        if (L == 0) {
#pragma unroll
            for (int a = 0; a < NORB; ++a) A.outR[mo + a * NORB + c] = mk(0.0, 0.0);
        } else {
            const int imax = L < k ? L : k;
            for (int i = 0; i <= imax; ++i) {
                const double wc = L < k ? A.W.nc[L][i] - w_end(A.W, n, m + i) : A.W.om[i] - 1.0;
                const cd* sg = A.sigR + (size_t)(m + i) * npair;
                const cd* bd = A.band + ((size_t)m * kb + i) * npair;
#pragma unroll
                for (int bb = 0; bb < NORB; ++bb) {
                    const cd g = wc * bd[bb * NORB + c];
#pragma unroll
                    for (int a = 0; a < NORB; ++a) fma_(accR[a], sg[a * NORB + bb], g);
                }
            }
#pragma unroll
            for (int a = 0; a < NORB; ++a) A.outR[mo + a * NORB + c] = A.h * accR[a];
        }
    }
    if (A.wantL) {
        // second lesser term: end weights (m >= k) or Newton-Cotes (m < k); the
        // interval is empty at m = 0 (no bulk term was added there either)
        // Sigma^<(n,s)[a][b] = -conj(sigL[s][b][a]);  G^R(m,s)^dagger[b][c] = conj(G^R(m,s)[c][b])
        const int imax = m == 0 ? -1 : (m < k ? m : k);
        for (int i = 0; i <= imax; ++i) {
            const int s = m - i;
            const double wc = m < k ? A.W.nc[m][s] - w_start(A.W, s) : A.W.om[i] - 1.0;
            const cd* sl = A.sigL + (size_t)s * npair;
            const cd* bd = A.band + ((size_t)s * kb + i) * npair;
#pragma unroll
            for (int bb = 0; bb < NORB; ++bb) {
                const cd g = mk(-wc, 0.0) * conj(bd[c * NORB + bb]);
#pragma unroll
                for (int a = 0; a < NORB; ++a) fmac_(accL[a], sl[bb * NORB + a], g);
            }
        }
#pragma unroll
        for (int a = 0; a < NORB; ++a) A.outL[mo + a * NORB + c] = A.h * accL[a];
    }
}

size_t tasks_smem(int norb) {
    const int ag = norb < 4 ? norb : 4;
    size_t fact = norb <= 4 ? (size_t)CH * norb * sizeof(cd) : 0;
    size_t leaf = (size_t)(tri(64) + 2 * 64 * ag) * sizeof(cd);
    size_t tail = (size_t)(16 * kTailCH + (16 + kTailCH) * ag) * sizeof(cd);
    size_t s = fact > leaf ? fact : leaf;
    return s > tail ? s : tail;
}

template <int NORB>
hipError_t launch_t(const HistArgs& a, hipStream_t st, hipEvent_t* ev) {
    const int ntask = a.nf[0] + a.nf[1] + a.nleaftask + a.ntailtask;
    if (ev) hipEventRecord(ev[0], st);
    if (ntask > 0) hist_tasks<NORB><<<ntask, NT, tasks_smem(NORB), st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    const int nblk = (a.n + 1 + 63) / 64;
    hist_combine<NORB><<<nblk, 64 * NORB, 0, st>>>(a);
    if (ev) hipEventRecord(ev[2], st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_history(const HistArgs& a, hipStream_t st, hipEvent_t* ev) {
    switch (a.norb) {
        case 1: return launch_t<1>(a, st, ev);
        case 2: return launch_t<2>(a, st, ev);
        case 4: return launch_t<4>(a, st, ev);
        case 8: return launch_t<8>(a, st, ev);
        case 16: return launch_t<16>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t history_init() {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f, int norb) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tasks_smem(norb));
    };
    set((const void*)hist_tasks<1>, 1);
    set((const void*)hist_tasks<2>, 2);
    set((const void*)hist_tasks<4>, 4);
    set((const void*)hist_tasks<8>, 8);
    set((const void*)hist_tasks<16>, 16);
    return e;
}

}  // namespace hn
