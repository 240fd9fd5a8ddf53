// Dense baseline on the same device: the same history integrals by direct
// summation over fully stored lower triangles (no compression).
//
// Both components are packed lower triangles per orbital pair
// (L[q][t1(t1+1)/2 + t2]).  Each stored entry enters the step twice, once in a
// column sum and once in a row dot (the retarded entry G^R(j,m) in I^R(n,m)
// and, conjugated, in the second lesser term; the lesser entry in both halves
// of the first lesser term), so a tile kernel reads each entry of both
// triangles from HBM once and produces both: lanes run over the tile's columns
// for the column sums and over its rows for the row dots (the second pass hits
// L2).  Partial sums per 128-row / 128-column band are reduced by a second
// kernel, which also adds the band corrections of the Gregory weights.
#include "dense.h"

namespace hn {

namespace {

constexpr int TB = 128;   // tile size (rows and columns)
constexpr int NTD = 128;  // threads per tile workgroup (2 waves)

template <int NORB>
__global__ void __launch_bounds__(NTD) dense_tiles(DenseArgs A) {
    constexpr int npair = NORB * NORB;
    extern __shared__ __align__(16) unsigned char smem[];
    cd* xr = reinterpret_cast<cd*>(smem);  // TB x npair (rows of the tile)
    cd* xc = xr + TB * npair;              // TB x npair (columns of the tile)
    const int t = blockIdx.x;
    int Jb = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((long long)(Jb + 1) * (Jb + 2) / 2 <= t) ++Jb;
    while ((long long)Jb * (Jb + 1) / 2 > t) --Jb;
    const int Mb = t - Jb * (Jb + 1) / 2;
    const int J0 = Jb * TB, M0 = Mb * TB;
    const int n = A.n;
    const int jhi = min(J0 + TB, n + 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = M0 + wave * 64 + lane;   // column of this lane (column sums)
    const int jr = J0 + wave * 64 + lane;  // row of this lane (row dots)
    cd rowacc[NORB][NORB];
#pragma unroll
    for (int a = 0; a < NORB; ++a)
#pragma unroll
        for (int c = 0; c < NORB; ++c) rowacc[a][c] = mk(0.0, 0.0);

    for (int comp = 0; comp < 2; ++comp) {
        __syncthreads();
        for (int e = threadIdx.x; e < TB * npair; e += NTD) {
            const int i = e / npair, p = e % npair, a = p / NORB, bb = p % NORB;
            const int j = J0 + i, s = M0 + i;
            cd vr = mk(0.0, 0.0), vc = mk(0.0, 0.0);
            if (comp == 0) {
                if (j <= n) vr = w_end(A.W, n, j) * A.sigR[(size_t)j * npair + p];
                if (s <= n) vc = -w_start(A.W, s) * conj(A.sigL[(size_t)s * npair + bb * NORB + a]);
            } else {
                if (j <= n) vr = interval_w(A.W, n, j) * A.sigR[(size_t)j * npair + p];
                if (s <= n) vc = interval_w(A.W, n, s) * A.sigR[(size_t)s * npair + p];
            }
            xr[e] = vr;
            xc[e] = vc;
        }
        __syncthreads();
        const cd* Lc = A.L[comp];
        // column sums over the tile rows, column m
        cd colacc[NORB][NORB];
#pragma unroll
        for (int a = 0; a < NORB; ++a)
#pragma unroll
            for (int c = 0; c < NORB; ++c) colacc[a][c] = mk(0.0, 0.0);
        const bool cact = m <= n;
        const int jlo = max(J0, comp == 0 ? m : m + 1);
        if (cact) {
#pragma unroll
            for (int q = 0; q < npair; ++q) {
                const int qr = q / NORB, qc = q % NORB;
                const cd* Lq = Lc + (size_t)q * A.trin;
                for (int j = jlo; j < jhi; ++j) {
                    const cd v = Lq[tri(j) + m];
                    const cd* x = xr + (j - J0) * npair;
                    if (comp == 0) {
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fma_(colacc[a][qc], x[a * NORB + qr], v);
                    } else {
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fmac_(colacc[a][qr], v, -x[a * NORB + qc]);
                    }
                }
            }
            cd* dst = (comp == 0 ? A.colR : A.colL) + ((size_t)Jb * A.nt + m) * npair;
#pragma unroll
            for (int a = 0; a < NORB; ++a)
#pragma unroll
                for (int c = 0; c < NORB; ++c) dst[a * NORB + c] = colacc[a][c];
        }
        // row dots over the tile columns, row jr (the second lesser term is empty at m = 0)
        if (jr <= n && !(comp == 0 && jr == 0)) {
            const int shi = min(M0 + TB, jr + 1);
#pragma unroll
            for (int q = 0; q < npair; ++q) {
                const int qr = q / NORB, qc = q % NORB;
                const cd* row = Lc + (size_t)q * A.trin + tri(jr);
                for (int s = M0; s < shi; ++s) {
                    const cd v = row[s];
                    const cd* x = xc + (s - M0) * npair;
                    if (comp == 0) {
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fmac_(rowacc[a][qr], v, x[a * NORB + qc]);
                    } else {
#pragma unroll
                        for (int a = 0; a < NORB; ++a) fma_(rowacc[a][qc], x[a * NORB + qr], v);
                    }
                }
            }
        }
    }
    if (jr <= n) {
        cd* dst = A.rowL + ((size_t)Mb * A.nt + jr) * npair;
#pragma unroll
        for (int a = 0; a < NORB; ++a)
#pragma unroll
            for (int c = 0; c < NORB; ++c) dst[a * NORB + c] = rowacc[a][c];
    }
}

template <int NORB>
__global__ void dense_reduce(DenseArgs A) {
    constexpr int npair = NORB * NORB;
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const int c = threadIdx.x >> 6;
    const int n = A.n;
    if (m > n) return;
    const int bm = m / TB, bn = n / TB;
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
    for (int Mb = 0; Mb <= bm; ++Mb) {
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

size_t dense_smem(int norb) { return (size_t)2 * TB * norb * norb * sizeof(cd); }

template <int NORB>
hipError_t launch_dense_t(const DenseArgs& a, hipStream_t st, hipEvent_t* ev) {
    const int nbands = a.n / TB + 1;
    const int ntiles = nbands * (nbands + 1) / 2;
    if (ev) hipEventRecord(ev[0], st);
    dense_tiles<NORB><<<ntiles, NTD, dense_smem(NORB), st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    dense_reduce<NORB><<<(a.n + 1 + 63) / 64, 64 * NORB, 0, st>>>(a);
    if (ev) hipEventRecord(ev[2], st);
    return hipGetLastError();
}

}  // namespace

int dense_band_count(int nt) { return (nt + TB - 1) / TB; }

hipError_t dense_init() {
    hipError_t e = hipFuncSetAttribute((const void*)dense_tiles<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dense_smem(1));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)dense_tiles<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)dense_smem(2));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)dense_tiles<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
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
