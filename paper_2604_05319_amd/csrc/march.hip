// Rows of G^R in the paper's orientation (section "Kadanoff-Baym equations", Eq. KBER:
// the derivative in the relative time, the current G row times the compressed Sigma
// history; section "Hierarchical decomposition" for the storage).  For a row n the right
// form of the retarded equation,
//   -i d/dt' G(t_n, t') - G(t_n, t') eps(t') = int_{t'}^{t_n} G(t_n, s) Sigma(s, t') ds,
// needs no other row: G(n, n) = -i, the columns n-k..n-1 from one k-unknown system (the
// polynomial differentiation weights on the points n-k..n, as in the time step), then the
// columns m < n-k leftwards by backward differentiation on the points m..m+k of the row:
//   G(n,m) M_m = -(i/h) sum_{l>=1} a_l G(n,m+l) + h sum_{s>m} w^{(n-m)}_{s-m} G(n,s) Sigma(s,m),
//   M_m = i a_0/h - eps(t_m) - h omega_0 Sigma(m,m).
// The sum over s > m splits by where Sigma(s, m) is stored: the leaf triangle of m's leaf
// (rows of the same leaf, taken column by column as the march goes), the low-rank blocks
// whose column range holds m (rows of later leaves below the merged front: their part of
// the row is projected once, G(n, R_b) U_b S_b, when the march enters the block's column
// range, then expanded through V_b for every column of each leaf), the dense tail (later
// rows above the merged front), with the end weights w_end(n, s); the start weights of
// s = m+1..m+k are corrected on the dense band.  One workgroup of 64 threads per row.
#include "march.h"

namespace hn {
namespace {

constexpr int NTM = 64;
constexpr int RCMAX = 32;

// Gauss-Jordan with partial pivoting (no row exchanges) by the workgroup on the K x ld
// row-major matrix [A | B] in LDS; (A^{-1} B)[p][c] = T[prow[p]][K+c] / T[prow[p]][p]
__device__ void gj64(cd* T, int K, int ld, int* used, int* prow) {
    const int t = threadIdx.x;
    for (int r = t; r < K; r += NTM) used[r] = 0;
    __syncthreads();
    for (int p = 0; p < K; ++p) {
        double best = -1.0;
        int bi = K;
        for (int r = t; r < K; r += NTM) {
            const double v = used[r] ? -1.0 : norm2(T[r * ld + p]);
            if (v > best) {
                best = v;
                bi = r;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (t == 0) {
            prow[p] = bi;
            used[bi] = 1;
        }
        __syncthreads();
        const int q = prow[p];
        const cd d = T[q * ld + p];
        const double s = 1.0 / norm2(d);
        const cd inv = mk(d.x * s, -d.y * s);
        const int w = ld - p - 1;
        for (int e = t; e < K * w; e += NTM) {
            const int r = e / w, j = p + 1 + e % w;
            if (r != q) T[r * ld + j] = T[r * ld + j] - (T[r * ld + p] * inv) * T[q * ld + j];
        }
        __syncthreads();
    }
}

__device__ inline cd gj_sol(const cd* T, int K, int ld, const int* prow, int p, int c) {
    const int q = prow[p];
    const cd d = T[q * ld + p];
    const double s = 1.0 / norm2(d);
    return T[q * ld + K + c] * mk(d.x * s, -d.y * s);
}

// the end-weight fold of the row sums, 1 + (omega_{n-j} - 1)[n-j <= k], with omega staged
// in LDS: a per-lane index into the weights held in the kernel arguments would be a
// global-memory load at every use
__device__ inline double wend_lds(const double* om, int k, int n, int j) {
    const int d = n - j;
    return d <= k ? om[d] : 1.0;
}

// M_m^{-1} for one column per thread (the matrix of the left side of the column's
// equation, the same for every row): Gauss-Jordan with partial pivoting; the row
// exchanges are value selects, so that every register index is static.

template <int NORB>
__global__ void __launch_bounds__(256) march_minv(MarchArgs A, int mcount) {
    constexpr int npair = NORB * NORB;
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= mcount) return;
    const int kb = A.k + 1;
    const double d0 = A.S.a[0] / A.h, wh = A.h * A.W.om[0];
    cd M[NORB][NORB], X[NORB][NORB];
#pragma unroll
    for (int a = 0; a < NORB; ++a)
#pragma unroll
        for (int b = 0; b < NORB; ++b) {
            const int q = a * NORB + b;
            M[a][b] = mk(0.0, a == b ? d0 : 0.0) - A.eps[(size_t)m * npair + q] -
                      wh * A.band[(size_t)m * kb * npair + q];
            X[a][b] = mk(a == b ? 1.0 : 0.0, 0.0);
        }
#pragma unroll
    for (int p = 0; p < NORB; ++p) {
        int piv = p;
        double best = norm2(M[p][p]);
#pragma unroll
        for (int r = p + 1; r < NORB; ++r) {
            const double v = norm2(M[r][p]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
#pragma unroll
        for (int r = p + 1; r < NORB; ++r) {
            const bool sw = r == piv;
#pragma unroll
            for (int j = 0; j < NORB; ++j) {
                const cd mp = M[p][j], mr = M[r][j], xp = X[p][j], xr = X[r][j];
                M[p][j] = sw ? mr : mp;
                M[r][j] = sw ? mp : mr;
                X[p][j] = sw ? xr : xp;
                X[r][j] = sw ? xp : xr;
            }
        }
        const cd d = M[p][p];
        const double s = 1.0 / norm2(d);
        const cd inv = mk(d.x * s, -d.y * s);
#pragma unroll
        for (int j = 0; j < NORB; ++j) {
            M[p][j] = M[p][j] * inv;
            X[p][j] = X[p][j] * inv;
        }
#pragma unroll
        for (int r = 0; r < NORB; ++r) {
            if (r == p) continue;
            const cd f = M[r][p];
#pragma unroll
            for (int j = 0; j < NORB; ++j) {
                M[r][j] = M[r][j] - f * M[p][j];
                X[r][j] = X[r][j] - f * X[p][j];
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NORB; ++a)
#pragma unroll
        for (int b = 0; b < NORB; ++b) A.minv[(size_t)m * npair + a * NORB + b] = X[a][b];
}

template <int NORB>
__global__ void __launch_bounds__(NTM) row_march(MarchArgs A) {
    constexpr int npair = NORB * NORB;
    // leaf sum of a column: thread (jg, a, bo) takes the rows j = m+1+jg, +SG, .. of the
    // leaf and the left orbital a, for every output orbital c
    constexpr int SG = NTM / npair;
    constexpr int NU = (63 + SG - 1) / SG;   // rows per thread (a leaf has at most 64)
    constexpr int NBD = (5 + SG - 1) / SG;   // band offsets i = jg+1, jg+1+SG, .. <= k per thread
    constexpr int KMAX = 5 * NORB, LDMAX = KMAX + NORB;
    static_assert(KMAX * LDMAX <= 64 * npair, "the start system fits the leaf buffer");
    // FR: the start system, then per leaf the far-field sums of the columns not yet
    // marched and w_end(n, j) G(n, j) of the marched ones (slot j - s0)
    __shared__ cd FR[64 * npair];
    __shared__ cd ring[8 * npair];        // G(n, j) at slot j % 8: the k columns right of m
    __shared__ cd red[NTM * NORB];        // partial sums of the leaf and band terms
    __shared__ cd rhs[npair];
    __shared__ int used[KMAX], prow[KMAX];
    __shared__ double om[8];              // Gregory end weights omega_0..omega_k
    cd* T = FR;
    const int n = A.nhi - (int)blockIdx.x;   // longest rows first
    if (n < A.nlo) return;
    const int k = A.k, nt = A.nt, kb = k + 1;
    const double h = A.h;
    const int t = threadIdx.x, e = t % npair, c = e / NORB, bo = e % NORB;
    const int jg = t / npair;                  // (jg, a = c, bo) in the leaf-sum role
    cd* row = A.rows + (size_t)(n - A.nlo) * A.rowStride;
    cd* P = A.proj + (size_t)blockIdx.x * A.nlvl * NORB * npair * RCMAX;
    auto sig_band = [&](int j, int m, int q) { return A.band[((size_t)m * kb + (j - m)) * npair + q]; };
    auto epsm = [&](int m, int a, int b) { return A.eps[(size_t)m * npair + a * NORB + b]; };
    if (t < 6) om[t] = A.W.om[t];

    // ---- columns n-k..n-1 (unknowns Y[(u,a)][c] = G(n, n-k+u)[c][a]) and G(n, n) = -i
    {
        const int K = k * NORB, ld = K + NORB;
        for (int x = t; x < K * ld; x += NTM) {
            const int r = x / ld, col = x % ld, i = r / NORB, b = r % NORB, m = n - k + i;
            cd v;
            if (col < K) {
                const int u = col / NORB, a = col % NORB;
                v = mk(0.0, a == b ? -A.S.D[i][u] / h : 0.0);
                if (u == i) v = v - epsm(m, a, b);
                if (u >= i) v = v - (h * interval_w(A.W, k - i, u - i)) * sig_band(n - k + u, m, a * NORB + b);
            } else {
                const int cc = col - K;
                const cd sg = sig_band(n, m, cc * NORB + b);
                const double wh = h * interval_w(A.W, k - i, k - i);
                v = mk((cc == b ? A.S.D[i][k] / h : 0.0) + wh * sg.y, -wh * sg.x);
            }
            T[x] = v;
        }
        __syncthreads();
        gj64(T, K, ld, used, prow);
        for (int x = t; x < K * NORB; x += NTM) {
            const int r = x / NORB, cc = x % NORB, u = r / NORB, a = r % NORB;
            const cd y = gj_sol(T, K, ld, prow, r, cc);
            row[(size_t)(n - k + u) * npair + cc * NORB + a] = y;
            ring[((n - k + u) & 7) * npair + cc * NORB + a] = y;
        }
        for (int x = t; x < npair; x += NTM) {
            const cd v = mk(0.0, x / NORB == x % NORB ? -1.0 : 0.0);
            row[(size_t)n * npair + x] = v;
            ring[(n & 7) * npair + x] = v;
        }
        __syncthreads();
    }
    const int mlast = n - k - 1;
    if (mlast < 0) return;
    const int rows_merged_end = A.n0 < n + 1 ? A.n0 : n + 1;   // block rows j < this count
    const int leaf0 = A.rowLeaf[mlast];
    int leaf = leaf0;
    int m = mlast;
    while (m >= 0) {
        const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
        const int mhi = m;                    // the leaf's columns marched: s0..mhi
        // (i) projections of the blocks whose column range starts its march in this leaf:
        // P[cc][q][r] = S_r sum_j w_end(n, j) G(n, j)[cc][a] U_q(j, r), q = (a, bb).  One lane
        // per pair q and ranks r = lane % LPQ + LPQ s (each lane streams its U columns along
        // j, no sums across lanes); the block's weighted row entries are staged in FR 64 rows
        // at a time and read by every lane of a pair.
        {
            constexpr int LPQ = NTM / npair, NR = (RCMAX + LPQ - 1) / LPQ;
            const int q = t / LPQ, a = q / NORB, rl = t % LPQ;
            for (int l = 0; l < A.nlvl; ++l) {
                const int b = A.cover[(size_t)l * nt + s0];
                if (b < 0) continue;
                const int* bk = A.blk + 5 * b;
                const int r0 = bk[1], r1 = bk[2], c1 = bk[4];
                if (c1 != s1 && leaf != leaf0) continue;   // computed at an earlier leaf
                const int jend = min(r1, rows_merged_end);
                if (r0 >= jend) continue;                   // no merged rows: the far field skips it
                cd* Pl = P + (size_t)l * NORB * npair * RCMAX;
                const int cb = A.cur[b] & 1, ld = r1 - r0;
                const int rk = min(max(A.rank[cb * A.bRank + (size_t)b * npair + q], 0), A.RC);
                const cd* Uq = A.U + cb * A.bU + A.Uoff[b] + (size_t)q * A.RC * ld;
                cd acc[NORB][NR];
#pragma unroll
                for (int cc = 0; cc < NORB; ++cc)
#pragma unroll
                    for (int s2 = 0; s2 < NR; ++s2) acc[cc][s2] = mk(0.0, 0.0);
                for (int jb = r0; jb < jend; jb += 64) {
                    const int nj = min(64, jend - jb);
                    __syncthreads();   // the previous chunk is consumed
                    for (int x = t; x < nj * npair; x += NTM) {
                        const int jj = jb + x / npair;
                        FR[x] = wend_lds(om, k, n, jj) * row[(size_t)jj * npair + x % npair];
                    }
                    __syncthreads();
                    const cd* Uj = Uq + (jb - r0);
#pragma unroll 8
                    for (int i = 0; i < nj; ++i) {
                        cd xv[NORB];
#pragma unroll
                        for (int cc = 0; cc < NORB; ++cc) xv[cc] = FR[i * npair + cc * NORB + a];
#pragma unroll
                        for (int s2 = 0; s2 < NR; ++s2) {
                            const int r = rl + LPQ * s2;
                            if (r < rk) {
                                const cd uv = Uj[(size_t)r * ld + i];
#pragma unroll
                                for (int cc = 0; cc < NORB; ++cc) fma_(acc[cc][s2], xv[cc], uv);
                            }
                        }
                    }
                }
                const double* Sq = A.Sv + cb * A.bS + ((size_t)b * npair + q) * A.RC;
#pragma unroll
                for (int s2 = 0; s2 < NR; ++s2) {
                    const int r = rl + LPQ * s2;
                    if (r < rk)
#pragma unroll
                        for (int cc = 0; cc < NORB; ++cc) Pl[(cc * npair + q) * RCMAX + r] = Sq[r] * acc[cc][s2];
                }
            }
        }
        __syncthreads();
        // (ii) far field of the leaf's columns, one lane per column: the covering blocks (the
        // column's V rows, coalesced over the lanes, against the row's projections) and the
        // dense tail; into FR, and the leaf's columns right of the march (the start columns)
        // as row values with their end weights
        const int jtop = min(n, s1 - 1);
        {
            const int mm = s0 + t;
            const bool on = mm <= mhi;
            cd acc[npair];   // [cc][bb]
#pragma unroll
            for (int x = 0; x < npair; ++x) acc[x] = mk(0.0, 0.0);
            cd* Ps = FR;   // [cc][q][16]: projections of 16 ranks of the level, staged
            for (int l = 0; l < A.nlvl; ++l) {
                const int b = A.cover[(size_t)l * nt + s0];   // the same block for every column of the leaf
                if (b < 0) continue;
                const int* bk = A.blk + 5 * b;
                const int r0 = bk[1], c0 = bk[3], c1 = bk[4];
                if (r0 >= rows_merged_end) continue;
                const int cb = A.cur[b] & 1, ldv = c1 - c0;
                const cd* Pl = P + (size_t)l * NORB * npair * RCMAX;
                const int col = on ? mm - c0 : 0;
                int rkq[npair], rkmax = 0;
#pragma unroll
                for (int q = 0; q < npair; ++q) {
                    rkq[q] = min(max(A.rank[cb * A.bRank + (size_t)b * npair + q], 0), A.RC);
                    rkmax = max(rkmax, rkq[q]);
                }
                const cd* Vb = A.V + cb * A.bV + A.Voff[b] + col;
                for (int rs = 0; rs < rkmax; rs += 16) {
                    __syncthreads();   // the previous stage is consumed
                    for (int x = t; x < NORB * npair * 16; x += NTM) {
                        const int q = (x / 16) % npair, r = rs + x % 16;
                        int rq = 0;
#pragma unroll
                        for (int qq = 0; qq < npair; ++qq) rq = qq == q ? rkq[qq] : rq;
                        Ps[x] = r < rq ? Pl[(x / (16 * npair) * npair + q) * RCMAX + r] : mk(0.0, 0.0);
                    }
                    __syncthreads();
                    const int nr = min(16, rkmax - rs);
                    constexpr int RU = NORB == 4 ? 1 : 2;   // ranks per batch of loads
                    for (int r = 0; r < nr; r += RU) {
                        cd v[npair][RU];
#pragma unroll
                        for (int q = 0; q < npair; ++q)
#pragma unroll
                            for (int u = 0; u < RU; ++u) {
                                // beyond the pair's rank: a zero (the factor memory there is not
                                // written, and zero weights would not clear a non-finite value)
                                const int rr = max(min(rs + r + u, rkq[q] - 1), 0);
                                const cd raw = Vb[((size_t)q * A.RC + rr) * ldv];
                                v[q][u] = rs + r + u < rkq[q] ? raw : mk(0.0, 0.0);
                            }
#pragma unroll
                        for (int q = 0; q < npair; ++q)
#pragma unroll
                            for (int u = 0; u < RU; ++u)
#pragma unroll
                                for (int cc = 0; cc < NORB; ++cc)   // P conj(V)
                                    fmac_(acc[cc * NORB + q % NORB], v[q][u], Ps[(cc * npair + q) * 16 + min(r + u, 15)]);
                    }
                }
            }
            __syncthreads();   // the staged projections are consumed before FR is written
            if (on && mm < A.ls)   // tail rows n0..n (above the merged front) hold the columns < ls
                for (int j = A.n0; j <= n; ++j) {
                    const double w = wend_lds(om, k, n, j);
                    const cd* tj = A.tail + (size_t)(j % A.ring) * npair * nt + mm;   // [q] at q * nt
                    cd tv[npair];
#pragma unroll
                    for (int q = 0; q < npair; ++q) tv[q] = tj[(size_t)q * nt];
#pragma unroll
                    for (int cc = 0; cc < NORB; ++cc)
#pragma unroll
                        for (int a = 0; a < NORB; ++a) {
                            const cd g = w * row[(size_t)j * npair + cc * NORB + a];
#pragma unroll
                            for (int bb = 0; bb < NORB; ++bb) fma_(acc[cc * NORB + bb], g, tv[a * NORB + bb]);
                        }
                }
            if (on) {
#pragma unroll
                for (int x = 0; x < npair; ++x) FR[t * npair + x] = acc[x];
            } else if (mm <= jtop) {   // the leaf sums take FR with the end weight folded in
                const double we = wend_lds(om, k, n, mm);
#pragma unroll
                for (int x = 0; x < npair; ++x) FR[t * npair + x] = we * row[(size_t)mm * npair + x];
            }
        }
        // (iii) the leaf's columns, right to left.  Per column: the leaf rows j > m and the
        // band corrections (start weights of s = m+1..m+k) as partial sums per (jg, a),
        // their sum with the far field into the right side, then G(n, m) = rhs M_m^{-1}.
        // The column's Sigma entries and M_m^{-1} do not depend on the march: those of
        // column m-1 are loaded while column m is solved.
        const long long lw = s1 - s0, tl = lw * (lw + 1) / 2;
        const cd* Lf = A.leaf + A.Loff[leaf] + (size_t)(c * NORB + bo) * tl;   // (a = c, bo) triangle
        cd lc[NU], bc[NBD], mc[NORB];
        auto load_col = [&](int mm, cd (&lv)[NU], cd (&bv)[NBD], cd (&mv)[NORB]) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int j = mm + 1 + jg + SG * u;
                lv[u] = j <= jtop ? Lf[(((j - s0) * (j - s0 + 1)) >> 1) + (mm - s0)] : mk(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < NBD; ++u) {
                const int i = jg + 1 + SG * u;
                bv[u] = i <= k ? sig_band(mm + i, mm, c * NORB + bo) : mk(0.0, 0.0);
            }
#pragma unroll
            for (int a = 0; a < NORB; ++a) mv[a] = t < npair ? A.minv[(size_t)mm * npair + a * NORB + bo] : mk(0.0, 0.0);
        };
        load_col(m, lc, bc, mc);
        // vmcnt(0) (expcnt and lgkmcnt left at their maxima): the first column's loads are
        // complete on entering the loop, so that no wait inside it covers the loads in flight
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        for (; m >= s0; --m) {
            // partial sums: acc[cc] = sum_j w_end(n, j) G(n, j)[cc][a] Sigma(j, m)[a][bo]
            //                        + sum_i (omega_i - 1) G(n, m+i)[cc][a] Sigma(m+i, m)[a][bo]
            cd acc[NORB];
#pragma unroll
            for (int cc = 0; cc < NORB; ++cc) acc[cc] = mk(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int j = m + 1 + jg + SG * u;
                if (j <= jtop)   // FR holds w_end(n, j) G(n, j) (the end weight is 1 left of n-k)
#pragma unroll
                    for (int cc = 0; cc < NORB; ++cc) fma_(acc[cc], FR[(j - s0) * npair + cc * NORB + c], lc[u]);
            }
#pragma unroll
            for (int u = 0; u < NBD; ++u) {
                const int i = jg + 1 + SG * u;
                if (i <= k) {
                    const cd bv = (om[i] - 1.0) * bc[u];
#pragma unroll
                    for (int cc = 0; cc < NORB; ++cc) fma_(acc[cc], ring[((m + i) & 7) * npair + cc * NORB + c], bv);
                }
            }
            // the next column's loads fly while this column is solved
            cd ln[NU], bn[NBD], mn[NORB];
            if (m > s0) load_col(m - 1, ln, bn, mn);
            // red[(jg NORB + a) npair + cc NORB + bo]
#pragma unroll
            for (int cc = 0; cc < NORB; ++cc) red[(jg * NORB + c) * npair + cc * NORB + bo] = acc[cc];
            __syncthreads();
            if (t < npair) {
                cd s = FR[(m - s0) * npair + e];
                for (int r = 0; r < SG * NORB; ++r) s = s + red[r * npair + e];
                cd bd = mk(0.0, 0.0);
#pragma unroll
                for (int l = 1; l <= 5; ++l)
                    if (l <= k) bd = bd + A.S.a[l] * ring[((m + l) & 7) * npair + e];
                rhs[e] = mk(h * s.x + bd.y / h, h * s.y - bd.x / h);   // h s - (i/h) bd
            }
            __syncthreads();
            if (t < npair) {   // G(n, m)[c][bo] = sum_a rhs[c][a] M_m^{-1}[a][bo]
                cd x = mk(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < NORB; ++a) fma_(x, rhs[c * NORB + a], mc[a]);
                FR[(m - s0) * npair + e] = x;
                ring[(m & 7) * npair + e] = x;
            }
            __syncthreads();
            if (m > s0) {
#pragma unroll
                for (int u = 0; u < NU; ++u) lc[u] = ln[u];
#pragma unroll
                for (int u = 0; u < NBD; ++u) bc[u] = bn[u];
#pragma unroll
                for (int a = 0; a < NORB; ++a) mc[a] = mn[a];
            }
        }
        // the leaf's marched columns to the output row (read by the next leaves' projections
        // and tail sums)
        for (int x = t; x < (mhi - s0 + 1) * npair; x += NTM) row[(size_t)s0 * npair + x] = FR[x];
        __syncthreads();
        --leaf;
    }
}

}  // namespace

hipError_t launch_march_minv(const MarchArgs& a, int mcount, hipStream_t st) {
    if (mcount <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((mcount + 255) / 256);
    switch (a.norb) {
        case 1: march_minv<1><<<nb, 256, 0, st>>>(a, mcount); break;
        case 2: march_minv<2><<<nb, 256, 0, st>>>(a, mcount); break;
        case 4: march_minv<4><<<nb, 256, 0, st>>>(a, mcount); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_row_march(const MarchArgs& a, hipStream_t st) {
    if (a.nlo < a.k || a.nhi < a.nlo || a.RC > RCMAX || a.k > 5) return hipErrorInvalidValue;
    const int nrows = a.nhi - a.nlo + 1;
    switch (a.norb) {
        case 1: row_march<1><<<nrows, NTM, 0, st>>>(a); break;
        case 2: row_march<2><<<nrows, NTM, 0, st>>>(a); break;
        case 4: row_march<4><<<nrows, NTM, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hn
