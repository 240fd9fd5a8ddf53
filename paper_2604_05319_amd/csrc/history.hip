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

// ---------------------------------------------------------------------------
template <int NORB>
__device__ void fact_task(const HistArgs& A, const FactTask& t, unsigned char* smem) {
    const int comp = t.comp, b = t.b, q = t.q, which = t.which, chunk = t.chunk;
    if (comp == 0 && which == 0 && !A.wantR) return;
    if ((comp == 1 || which == 1) && !A.wantL) return;
    const int npair = NORB * NORB, RC = A.RC;
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
    const int nchunks = (len + CH - 1) / CH;
    const int i0 = chunk * CH, i1 = min(len, i0 + CH);
    const int n = A.n;
    cd* xs = reinterpret_cast<cd*>(smem);  // CH x NORB
    for (int e = threadIdx.x; e < (i1 - i0) * NORB; e += NT) {
        const int i = e / NORB, a = e % NORB;
        const int j = base + i0 + i;
        cd v;
        if (comp == 0 && which == 0) {
            v = w_end(A.W, n, j) * A.sigR[(size_t)j * npair + a * NORB + qr];
        } else if (comp == 0) {
            v = -w_start(A.W, j) * conj(A.sigL[(size_t)j * npair + qc * NORB + a]);
        } else {
            v = interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + a * NORB + (which == 0 ? qc : qr)];
        }
        xs[e] = v;
    }
    __syncthreads();
    const bool cj = (comp == 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t slot = proj_slot(A, comp, b, q, which);
    cd* part = A.part + (A.partoff[slot] + chunk) * (size_t)NORB * RC;
    for (int rb = 0; rb < rk; rb += NT / 64) {
        const int r = rb + wave;
        cd acc[NORB];
#pragma unroll
        for (int a = 0; a < NORB; ++a) acc[a] = mk(0.0, 0.0);
        if (r < rk) {
            const cd* Fr = F + (size_t)r * ld;
            for (int i = i0 + lane; i < i1; i += 64) {
                cd f = Fr[i];
                if (cj) f = conj(f);
                const cd* xi = xs + (size_t)(i - i0) * NORB;
#pragma unroll
                for (int a = 0; a < NORB; ++a) fma_(acc[a], xi[a], f);
            }
        }
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            acc[a].x = wsum64(acc[a].x);
            acc[a].y = wsum64(acc[a].y);
        }
        if (lane == 0 && r < rk) {
#pragma unroll
            for (int a = 0; a < NORB; ++a) part[(size_t)a * RC + r] = acc[a];
        }
    }
    __threadfence();
    __syncthreads();
    __shared__ int s_last;
    if (threadIdx.x == 0) s_last = (atomicAdd(&A.cnt[slot], 1) == nchunks - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const double* S = A.S[comp] + ((size_t)b * npair + q) * RC;
    const cd* p0 = A.part + A.partoff[slot] * (size_t)NORB * RC;
    cd* out = A.proj + slot * (size_t)NORB * RC;
    for (int e = threadIdx.x; e < NORB * rk; e += NT) {
        const int a = e / rk, r = e % rk;
        cd s = mk(0.0, 0.0);
        for (int c = 0; c < nchunks; ++c) s = s + p0[((size_t)c * NORB + a) * RC + r];
        out[(size_t)a * RC + r] = S[r] * s;
    }
    if (threadIdx.x == 0) A.cnt[slot] = 0;
}

// ---------------------------------------------------------------------------
// One leaf triangle, one component, one left orbital index a; the four waves
// split the orbital pairs, lanes run over the leaf's columns m.
template <int NORB>
__device__ void leaf_task(const HistArgs& A, int leaf, int comp, int a, unsigned char* smem) {
    if (comp == 1 && !A.wantL) return;
    constexpr int npair = NORB * NORB;
    const int n = A.n;
    const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
    const int lw = s1 - s0;
    const int nrow = min(s1, n + 1) - s0;
    const cd* L = A.leaf[comp] + A.Loff[leaf];
    const long long tsz = tri(lw);
    cd* xa = reinterpret_cast<cd*>(smem);  // 64 x NORB
    cd* xb = xa + 64 * NORB;               // 64 x NORB
    cd* red = xb + 64 * NORB;              // 3 x 64 x NORB
    for (int e = threadIdx.x; e < nrow * NORB; e += NT) {
        const int i = e / NORB, bb = e % NORB, j = s0 + i;
        if (comp == 0) {
            xa[e] = w_end(A.W, n, j) * A.sigR[(size_t)j * npair + a * NORB + bb];
            // Sigma^< is only passed (and only read) when the lesser output is wanted
            xb[e] = A.wantL ? -w_start(A.W, j) * conj(A.sigL[(size_t)j * npair + bb * NORB + a])
                            : mk(0.0, 0.0);
        } else {
            xa[e] = interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + a * NORB + bb];
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, mo = threadIdx.x & 63;
    const bool act = mo < nrow;
    cd accA[NORB], accB[NORB];
#pragma unroll
    for (int c = 0; c < NORB; ++c) accA[c] = accB[c] = mk(0.0, 0.0);
    if (act) {
        for (int q = wave; q < npair; q += NT / 64) {
            const int qr = q / NORB, qc = q % NORB;
            const cd* Lq = L + (size_t)q * tsz;
            const cd* rowm = Lq + tri(mo);
            if (comp == 0) {
                if (A.wantR) {  // P1: column sums x(j) G^R(j, m)
                    cd s = mk(0.0, 0.0);
                    for (int j = mo; j < nrow; ++j) fma_(s, xa[j * NORB + qr], Lq[tri(j) + mo]);
                    accA[qc] = accA[qc] + s;
                }
                if (A.wantL && s0 + mo > 0) {  // row dots x2(s) G^R(m, s)^dagger (empty at m = 0)
                    cd s = mk(0.0, 0.0);
                    for (int k = 0; k <= mo; ++k) fmac_(s, rowm[k], xb[k * NORB + qc]);
                    accB[qr] = accB[qr] + s;
                }
            } else {
                cd s = mk(0.0, 0.0);  // row dots x1(s) G^<(s, m), s <= m
                for (int k = 0; k <= mo; ++k) fma_(s, xa[k * NORB + qr], rowm[k]);
                accA[qc] = accA[qc] + s;
                cd u = mk(0.0, 0.0);  // column sums x1(s) G^<(s, m), s > m
                for (int j = mo + 1; j < nrow; ++j) fmac_(u, Lq[tri(j) + mo], xa[j * NORB + qc]);
                accA[qr] = accA[qr] - u;
            }
        }
    }
    // reduce the four waves
    for (int pass = 0; pass < (comp == 0 ? 2 : 1); ++pass) {
        cd* acc = pass == 0 ? accA : accB;
        if (wave > 0) {
#pragma unroll
            for (int c = 0; c < NORB; ++c) red[((wave - 1) * 64 + mo) * NORB + c] = acc[c];
        }
        __syncthreads();
        if (wave == 0 && act) {
            const int m = s0 + mo;
            cd* dst = comp == 1 ? A.leafLL : (pass == 0 ? A.leafR : A.leafLR);
#pragma unroll
            for (int c = 0; c < NORB; ++c) {
                cd v = acc[c];
                for (int w = 0; w < NT / 64 - 1; ++w) v = v + red[(w * 64 + mo) * NORB + c];
                dst[(size_t)m * npair + a * NORB + c] = v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Rows appended since the last panel merge (dense), columns [0, ls):
// column sums into tailcol, row dots (partial per column chunk) into taildot.
template <int NORB>
__device__ void tail_task(const HistArgs& A, int comp, int a, int chunk, unsigned char* smem) {
    if (comp == 1 && !A.wantL) return;
    constexpr int npair = NORB * NORB;
    const int n = A.n;
    const int n0 = A.n0[comp], nrows = A.last[comp] - n0 + 1, ls = A.ls[comp];
    const int m = chunk * kTailCH + threadIdx.x;
    const bool act = m < ls;
    cd* xr = reinterpret_cast<cd*>(smem);  // P x NORB
    cd* red = xr + (size_t)A.P * NORB;     // 4 x NORB
    for (int e = threadIdx.x; e < nrows * NORB; e += NT) {
        const int i = e / NORB, bb = e % NORB, j = n0 + i;
        const double w = comp == 0 ? w_end(A.W, n, j) : interval_w(A.W, n, j);
        xr[e] = w * A.sigR[(size_t)j * npair + a * NORB + bb];
    }
    cd xm[NORB];
#pragma unroll
    for (int bb = 0; bb < NORB; ++bb) {
        xm[bb] = mk(0.0, 0.0);
        if (act) {
            if (comp == 0) {
                if (A.wantL) xm[bb] = -w_start(A.W, m) * conj(A.sigL[(size_t)m * npair + bb * NORB + a]);
            } else
                xm[bb] = interval_w(A.W, n, m) * A.sigR[(size_t)m * npair + a * NORB + bb];
        }
    }
    __syncthreads();
    const cd* T = A.tail[comp];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    cd col[NORB];
#pragma unroll
    for (int c = 0; c < NORB; ++c) col[c] = mk(0.0, 0.0);
    cd* tp = A.tailpart[comp] + ((size_t)a * A.ntailchunk[comp] + chunk) * A.P * NORB;
    for (int i = 0; i < nrows; ++i) {
        cd row[NORB];
#pragma unroll
        for (int c = 0; c < NORB; ++c) row[c] = mk(0.0, 0.0);
        if (act) {
#pragma unroll
            for (int q = 0; q < npair; ++q) {
                const int qr = q / NORB, qc = q % NORB;
                const cd t = T[((size_t)i * npair + q) * A.nt + m];
                if (comp == 0) {
                    if (A.wantR) fma_(col[qc], xr[i * NORB + qr], t);   // x(j) G^R(j, m)
                    if (A.wantL) fmac_(row[qr], t, xm[qc]);              // x2(m) G^R(j, m)^dagger
                } else {
                    fmac_(col[qr], t, -xr[i * NORB + qc]);               // -x1(j) G^<(m, j)^dagger
                    fma_(row[qc], xm[qr], t);                            // x1(m) G^<(m, j)
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NORB; ++c) {
            row[c].x = wsum64(row[c].x);
            row[c].y = wsum64(row[c].y);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < NORB; ++c) red[wave * NORB + c] = row[c];
        }
        __syncthreads();
        if (threadIdx.x < NORB) {
            cd v = mk(0.0, 0.0);
            for (int w = 0; w < NT / 64; ++w) v = v + red[w * NORB + threadIdx.x];
            tp[(size_t)i * NORB + threadIdx.x] = v;
        }
        __syncthreads();
    }
    if (act) {
#pragma unroll
        for (int c = 0; c < NORB; ++c) A.tailcol[comp][(size_t)m * npair + a * NORB + c] = col[c];
    }
    __threadfence();
    __syncthreads();
    __shared__ int s_last;
    const int nch = A.ntailchunk[comp];
    int* cnt = A.tailcnt + comp * NORB + a;
    if (threadIdx.x == 0) s_last = (atomicAdd(cnt, 1) == nch - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const cd* tp0 = A.tailpart[comp] + (size_t)a * nch * A.P * NORB;
    for (int e = threadIdx.x; e < nrows * NORB; e += NT) {
        const int i = e / NORB, c = e % NORB;
        cd v = mk(0.0, 0.0);
        for (int ch = 0; ch < nch; ++ch) v = v + tp0[((size_t)ch * A.P + i) * NORB + c];
        A.taildot[comp][((size_t)i * NORB + a) * NORB + c] = v;
    }
    if (threadIdx.x == 0) *cnt = 0;
}

template <int NORB>
__global__ void __launch_bounds__(NT) hist_tasks(HistArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
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
        int g, a;
        if (!xcd_group(id, 2 * A.nleaf, NORB, g, a)) return;
        leaf_task<NORB>(A, g >> 1, g & 1, a, smem);
        return;
    }
    id -= A.nleaftask;
    int g, a;
    const int ng = A.ntailchunk[0] + A.ntailchunk[1];
    if (!xcd_group(id, ng, NORB, g, a)) return;
    if (g < A.ntailchunk[0])
        tail_task<NORB>(A, 0, a, g, smem);
    else
        tail_task<NORB>(A, 1, a, g - A.ntailchunk[0], smem);
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
#pragma unroll
    for (int a = 0; a < NORB; ++a) {
        const size_t o = mo + a * NORB + c;
        if (A.wantR) {
            accR[a] = accR[a] + A.leafR[o];
            if (A.last[0] >= A.n0[0] && m < A.ls[0]) accR[a] = accR[a] + A.tailcol[0][o];
        }
        if (A.wantL) {
            accL[a] = accL[a] + A.leafLR[o] + A.leafLL[o];
            if (A.last[0] >= A.n0[0] && m >= A.n0[0] && m <= A.last[0])
                accL[a] = accL[a] + A.taildot[0][(size_t)(m - A.n0[0]) * npair + a * NORB + c];
            if (A.last[1] >= A.n0[1]) {
                if (m < A.ls[1]) accL[a] = accL[a] + A.tailcol[1][o];
                if (m >= A.n0[1] && m <= A.last[1])
                    accL[a] = accL[a] + A.taildot[1][(size_t)(m - A.n0[1]) * npair + a * NORB + c];
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
    size_t fact = (size_t)CH * norb * sizeof(cd);
    size_t leaf = (size_t)(2 * 64 + 3 * 64) * norb * sizeof(cd);
    size_t tail = (size_t)(32 + 4) * norb * sizeof(cd);
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
