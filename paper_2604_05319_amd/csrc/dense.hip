// Dense baseline on the same device: the same history integrals by direct
// summation over fully stored lower triangles (no compression).
//
// Both components are packed lower triangles per orbital pair
// (L[q][t1(t1+1)/2 + t2]).  Each stored entry enters the step twice, once in a
// column sum and once in a row dot (the retarded entry G^R(j,m) in I^R(n,m)
// and, conjugated, in the second lesser term; the lesser entry in both halves
// of the first lesser term).  A workgroup owns a band of 128 rows and a chunk of
// 64 columns; for each 32-row sub-band and orbital pair it stages the 32 x 64
// tile in LDS with coalesced loads (the next pair's tile in flight in registers)
// and computes both products from LDS: lanes over columns for the column sums,
// lanes over rows for the row dots, wave w the left orbital a = w, so each entry
// is read from HBM once.  Partial sums per 128-row band (columns) and per
// 64-column chunk (rows) are reduced by a second kernel, which also adds the
// band corrections of the Gregory weights.
#include "dense.h"

namespace hn {

namespace {

constexpr int TB = 128;   // rows per band (column-sum partials)
constexpr int TC = 64;    // columns per chunk (row-dot partials)
constexpr int TR = 32;    // rows per staged sub-tile
constexpr int NTD = 256;  // threads per workgroup (4 waves)
constexpr int EPT = TR * TC / NTD;   // tile elements per thread

// workgroup t -> (band Jb, chunk Mc) over the chunks that meet the lower triangle
// of band Jb (64 Mc <= 128 Jb + 127: 2 Jb + 2 chunks), bands in order
__device__ inline void band_chunk(int t, int& Jb, int& Mc) {
    int b = (int)((sqrt(4.0 * t + 1.0) - 1.0) * 0.5);
    while ((long long)(b + 1) * (b + 2) <= t) ++b;
    while ((long long)b * (b + 1) > t) --b;
    Jb = b;
    Mc = t - b * (b + 1);
}

template <int NORB>
__global__ void __launch_bounds__(NTD) dense_bands(DenseArgs A) {
    static_assert(NORB <= 4, "one left orbital per wave");
    constexpr int npair = NORB * NORB;
    extern __shared__ __align__(16) unsigned char smem[];
    cd* T = reinterpret_cast<cd*>(smem);   // TR x TC, column index XORed by (row & 15)
    cd* xr = T + TR * TC;                  // TR x npair: row-side Sigma of the sub-band
    cd* xc = xr + TR * npair;              // TC x npair: column-side Sigma of the chunk
    int Jb, Mc;
    band_chunk(blockIdx.x, Jb, Mc);
    const int J0 = Jb * TB, M0 = Mc * TC, n = A.n;
    if (J0 > n) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = wave;                       // left orbital of this wave (waves >= NORB idle)
    const bool wa = a < NORB;
    const int m = M0 + lane;                  // column of this lane (column sums)
    const int ri = lane & 31, half = lane >> 5;   // row dots: row ri, columns 32*half..+32
    for (int comp = 0; comp < 2; ++comp) {
        const cd* Lc = A.L[comp];
        __syncthreads();
        for (int e = threadIdx.x; e < TC * npair; e += NTD) {
            const int sl = e / npair, p = e % npair, aa = p / NORB, bb = p % NORB, s = M0 + sl;
            cd v = mk(0.0, 0.0);
            if (s <= n)
                v = comp == 0 ? -w_start(A.W, s) * conj(A.sigL[(size_t)s * npair + bb * NORB + aa])
                              : interval_w(A.W, n, s) * A.sigR[(size_t)s * npair + p];
            xc[e] = v;
        }
        cd col[NORB];
#pragma unroll
        for (int c = 0; c < NORB; ++c) col[c] = mk(0.0, 0.0);
        for (int sb = 0; sb < TB / TR; ++sb) {
            const int R0 = J0 + sb * TR;
            if (R0 > n || R0 + TR - 1 < M0) continue;   // beyond the step or above the diagonal
            __syncthreads();
            for (int e = threadIdx.x; e < TR * npair; e += NTD) {
                const int i = e / npair, p = e % npair, j = R0 + i;
                cd v = mk(0.0, 0.0);
                if (j <= n) v = (comp == 0 ? w_end(A.W, n, j) : interval_w(A.W, n, j)) * A.sigR[(size_t)j * npair + p];
                xr[e] = v;
            }
            cd row[NORB];
#pragma unroll
            for (int c = 0; c < NORB; ++c) row[c] = mk(0.0, 0.0);
            // tile of pair q: element e = threadIdx + u * NTD at (i = e / TC, l = e % TC); the
            // tiles of the next two pairs are in flight in registers while pair q is computed
            // (loads from clamped in-range indices; entries above the diagonal or the step
            // are zeroed when the tile is stored, so no load waits at issue)
            cd pA[EPT], pB[EPT];
            auto fetch = [&](cd (&pt)[EPT], int q) {
                const cd* Lq = Lc + (size_t)q * A.trin;
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const int e = threadIdx.x + u * NTD, i = e / TC, l = e % TC;
                    const int j = min(R0 + i, n), s = min(M0 + l, j);
                    pt[u] = Lq[tri(j) + s];
                }
            };
            fetch(pA, 0);
            if (npair > 1) fetch(pB, 1);
            for (int q = 0; q < npair; ++q) {
                const int qr = q / NORB, qc = q % NORB;
                __syncthreads();
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const int e = threadIdx.x + u * NTD, i = e / TC, l = e % TC;
                    const int j = R0 + i, s = M0 + l;
                    T[i * TC + (l ^ (i & 15))] = (j <= n && s <= j) ? pA[u] : mk(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < EPT; ++u) pA[u] = pB[u];
                if (q + 2 < npair) fetch(pB, q + 2);
                __syncthreads();
                if (!wa) continue;
                // column sums of column m over the sub-band's rows (comp 1: rows j > m only)
                cd cs = mk(0.0, 0.0);
#pragma unroll 8
                for (int i = 0; i < TR; ++i) {
                    cd v = T[i * TC + (lane ^ (i & 15))];
                    if (comp == 1 && R0 + i == m) v = mk(0.0, 0.0);
                    if (comp == 0) fma_(cs, xr[i * npair + a * NORB + qr], v);
                    else fmac_(cs, v, xr[i * npair + a * NORB + qc]);
                }
                // col[c] += cs for c = qc (comp 0) or -= for c = qr (comp 1), without a run-time
                // register index
#pragma unroll
                for (int c = 0; c < NORB; ++c) {
                    if (comp == 0 && c == qc) col[c] = col[c] + cs;
                    if (comp == 1 && c == qr) col[c] = col[c] - cs;
                }
                // row dots of row R0 + ri over the chunk's columns 32*half .. +32
                cd rd = mk(0.0, 0.0);
#pragma unroll 8
                for (int t = 0; t < 32; ++t) {
                    const int l = 32 * half + t;
                    const cd v = T[ri * TC + (l ^ (ri & 15))];
                    if (comp == 0) fmac_(rd, v, xc[l * npair + a * NORB + qc]);
                    else fma_(rd, xc[l * npair + a * NORB + qr], v);
                }
#pragma unroll
                for (int c = 0; c < NORB; ++c)
                    if (c == (comp == 0 ? qr : qc)) row[c] = row[c] + rd;
            }
            // row dots: add the two column halves; lanes 0..31 then hold the sub-band's rows
#pragma unroll
            for (int c = 0; c < NORB; ++c) {
                double re = row[c].x, im = row[c].y;
                re += __shfl_xor(re, 32, 64);
                im += __shfl_xor(im, 32, 64);
                row[c] = mk(re, im);
            }
            const int jr = R0 + ri;
            // the second lesser term is empty at m = 0 (row 0 of the retarded component)
            if (wa && half == 0 && jr <= n && !(comp == 0 && jr == 0)) {
                cd* dst = A.rowL + ((size_t)Mc * A.nt + jr) * npair + a * NORB;
#pragma unroll
                for (int c = 0; c < NORB; ++c) dst[c] = comp == 0 ? row[c] : dst[c] + row[c];
            } else if (wa && half == 0 && jr <= n && comp == 0) {
                cd* dst = A.rowL + ((size_t)Mc * A.nt + jr) * npair + a * NORB;
#pragma unroll
                for (int c = 0; c < NORB; ++c) dst[c] = mk(0.0, 0.0);
            }
        }
        if (wa && m <= n) {
            cd* dst = (comp == 0 ? A.colR : A.colL) + ((size_t)Jb * A.nt + m) * npair + a * NORB;
#pragma unroll
            for (int c = 0; c < NORB; ++c) dst[c] = col[c];
        }
    }
}

template <int NORB>
__global__ void dense_reduce(DenseArgs A) {
    constexpr int npair = NORB * NORB;
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const int c = threadIdx.x >> 6;
    const int n = A.n;
    if (m > n) return;
    const int bm = m / TB, bn = n / TB, cm = m / TC;
    cd accR[NORB], accL[NORB];
#pragma unroll
    for (int a = 0; a < NORB; ++a) accR[a] = accL[a] = mk(0.0, 0.0);
    for (int Jb = bm; Jb <= bn; ++Jb) {
        const cd* pr = A.colR + ((size_t)Jb * A.nt + m) * npair;
        const cd* pl = A.colL + ((size_t)Jb * A.nt + m) * npair;
#pragma unroll
        for (int a = 0; a < NORB; ++a) {
            accR[a] = accR[a] + pr[a * NORB + c];
            accL[a] = accL[a] + pl[a * NORB + c];
        }
    }
    for (int Mb = 0; Mb <= cm; ++Mb) {
        const cd* pr = A.rowL + ((size_t)Mb * A.nt + m) * npair;
#pragma unroll
        for (int a = 0; a < NORB; ++a) accL[a] = accL[a] + pr[a * NORB + c];
    }
    const int k = A.W.k;
    const size_t mo = (size_t)m * npair;
    const cd* LR = A.L[0];
    // I^R band correction
    const int L = n - m;
    if (L == 0) {
#pragma unroll
        for (int a = 0; a < NORB; ++a) A.outR[mo + a * NORB + c] = mk(0.0, 0.0);
    } else {
        const int imax = L < k ? L : k;
        for (int i = 0; i <= imax; ++i) {
            const double wc = L < k ? A.W.nc[L][i] - w_end(A.W, n, m + i) : A.W.om[i] - 1.0;
            const cd* sg = A.sigR + (size_t)(m + i) * npair;
#pragma unroll
            for (int bb = 0; bb < NORB; ++bb) {
                const cd g = wc * LR[(size_t)(bb * NORB + c) * A.trin + tri(m + i) + m];
#pragma unroll
                for (int a = 0; a < NORB; ++a) fma_(accR[a], sg[a * NORB + bb], g);
            }
        }
#pragma unroll
        for (int a = 0; a < NORB; ++a) A.outR[mo + a * NORB + c] = A.h * accR[a];
    }
    // second lesser term correction (empty interval at m = 0)
    const int imax = m == 0 ? -1 : (m < k ? m : k);
    for (int i = 0; i <= imax; ++i) {
        const int s = m - i;
        const double wc = m < k ? A.W.nc[m][s] - w_start(A.W, s) : A.W.om[i] - 1.0;
        const cd* sl = A.sigL + (size_t)s * npair;
#pragma unroll
        for (int bb = 0; bb < NORB; ++bb) {
            const cd g = mk(-wc, 0.0) * conj(LR[(size_t)(c * NORB + bb) * A.trin + tri(m) + s]);
#pragma unroll
            for (int a = 0; a < NORB; ++a) fmac_(accL[a], sl[bb * NORB + a], g);
        }
    }
#pragma unroll
    for (int a = 0; a < NORB; ++a) A.outL[mo + a * NORB + c] = A.h * accL[a];
}

size_t dense_smem(int norb) { return (size_t)(TR * TC + (TR + TC) * norb * norb) * sizeof(cd); }

template <int NORB>
hipError_t launch_dense_t(const DenseArgs& a, hipStream_t st, hipEvent_t* ev) {
    const int nbands = a.n / TB + 1;
    const int ntiles = nbands * (nbands + 1);   // 2 Jb + 2 chunks per band
    if (ev) hipEventRecord(ev[0], st);
    dense_bands<NORB><<<ntiles, NTD, dense_smem(NORB), st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    dense_reduce<NORB><<<(a.n + 1 + 63) / 64, 64 * NORB, 0, st>>>(a);
    if (ev) hipEventRecord(ev[2], st);
    return hipGetLastError();
}

}  // namespace

int dense_band_count(int nt) { return (nt + TB - 1) / TB; }
int dense_chunk_count(int nt) { return (nt + TC - 1) / TC; }

hipError_t dense_init() {
    hipError_t e = hipFuncSetAttribute((const void*)dense_bands<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dense_smem(1));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)dense_bands<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)dense_smem(2));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)dense_bands<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)dense_smem(4));
    return e;
}

hipError_t launch_dense_history(const DenseArgs& a, hipStream_t st, hipEvent_t* ev) {
    switch (a.norb) {
        case 1: return launch_dense_t<1>(a, st, ev);
        case 2: return launch_dense_t<2>(a, st, ev);
        case 4: return launch_dense_t<4>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hn
