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

template <int NORB>
__global__ void __launch_bounds__(NTM) row_march(MarchArgs A) {
    constexpr int npair = NORB * NORB, SG = NTM / npair;
    constexpr int KMAX = 5 * NORB, LDMAX = KMAX + NORB;
    __shared__ cd T[KMAX * LDMAX];
    __shared__ int used[KMAX], prow[KMAX];
    __shared__ cd F[64 * npair];     // far-field sums of the current leaf's columns
    __shared__ cd red[NTM];
    __shared__ cd rhs[npair];
    const int n = A.nlo + blockIdx.x;
    if (n > A.nhi) return;
    const int k = A.k, nt = A.nt, kb = k + 1;
    const double h = A.h;
    const int t = threadIdx.x, e = t % npair, g = t / npair, c = e / NORB, bo = e % NORB;
    cd* row = A.rows + (size_t)blockIdx.x * A.rowStride;
    cd* P = A.proj + (size_t)blockIdx.x * A.nlvl * NORB * npair * RCMAX;
    auto sig_band = [&](int j, int m, int q) { return A.band[((size_t)m * kb + (j - m)) * npair + q]; };
    auto epsm = [&](int m, int a, int b) { return A.eps[(size_t)m * npair + a * NORB + b]; };

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
            row[(size_t)(n - k + u) * npair + cc * NORB + a] = gj_sol(T, K, ld, prow, r, cc);
        }
        for (int x = t; x < npair; x += NTM) row[(size_t)n * npair + x] = mk(0.0, x / NORB == x % NORB ? -1.0 : 0.0);
        __syncthreads();
    }
    const int mlast = n - k - 1;
    if (mlast < 0) return;
    const int rows_merged_end = A.n0 < n + 1 ? A.n0 : n + 1;   // block rows j < this count
    int leaf = A.rowLeaf[mlast];
    int m = mlast;
    while (m >= 0) {
        const int s0 = A.leafs[2 * leaf], s1 = A.leafs[2 * leaf + 1];
        const int mhi = m;                    // the leaf's columns marched: s0..mhi
        // (i) projections of the blocks whose column range starts its march in this leaf
        for (int l = 0; l < A.nlvl; ++l) {
            const int b = A.cover[(size_t)l * nt + s0];
            if (b < 0) continue;
            const int* bk = A.blk + 5 * b;
            const int r0 = bk[1], r1 = bk[2], c1 = bk[4];
            if (c1 != s1 && leaf != A.rowLeaf[mlast]) continue;   // computed at an earlier leaf
            const int jend = min(r1, rows_merged_end);
            cd* Pl = P + (size_t)l * NORB * npair * RCMAX;
            const int cb = A.cur[b] & 1;
            for (int o = t; o < NORB * npair * RCMAX; o += NTM) {
                const int cc = o / (npair * RCMAX), q = (o / RCMAX) % npair, r = o % RCMAX;
                const int rk = min(max(A.rank[cb * A.bRank + (size_t)b * npair + q], 0), A.RC);
                cd acc = mk(0.0, 0.0);
                if (r < rk && r0 < jend) {
                    const int a = q / NORB, ld = r1 - r0;
                    const cd* Uq = A.U + cb * A.bU + A.Uoff[b] + ((size_t)q * A.RC + r) * ld;
                    for (int j = r0; j < jend; ++j)
                        acc = acc + w_end(A.W, n, j) * (row[(size_t)j * npair + cc * NORB + a] * Uq[j - r0]);
                    acc = A.Sv[cb * A.bS + ((size_t)b * npair + q) * A.RC + r] * acc;
                }
                Pl[o] = acc;
            }
        }
        __syncthreads();
        // (ii) far-field sums of the leaf's columns: covering blocks and the dense tail
        for (int x = t; x < (mhi - s0 + 1) * npair; x += NTM) {
            const int mm = s0 + x / npair, ee = x % npair, cc = ee / NORB, bb = ee % NORB;
            cd acc = mk(0.0, 0.0);
            for (int l = 0; l < A.nlvl; ++l) {
                const int b = A.cover[(size_t)l * nt + mm];
                if (b < 0) continue;
                const int* bk = A.blk + 5 * b;
                const int r0 = bk[1], c0 = bk[3], c1 = bk[4];
                if (r0 >= rows_merged_end) continue;
                const int cb = A.cur[b] & 1, ldv = c1 - c0;
                const cd* Pl = P + (size_t)l * NORB * npair * RCMAX;
                for (int a = 0; a < NORB; ++a) {
                    const int q = a * NORB + bb;
                    const int rk = min(max(A.rank[cb * A.bRank + (size_t)b * npair + q], 0), A.RC);
                    const cd* Vq = A.V + cb * A.bV + A.Voff[b] + (size_t)q * A.RC * ldv + (mm - c0);
                    for (int r = 0; r < rk; ++r)
                        fmac_(acc, Vq[(size_t)r * ldv], Pl[(cc * npair + q) * RCMAX + r]);   // P conj(V)
                }
            }
            if (mm < A.ls)   // tail rows n0..n (above the merged front) hold the columns < ls
                for (int j = A.n0; j <= n; ++j) {
                    const double w = w_end(A.W, n, j);
                    for (int a = 0; a < NORB; ++a)
                        acc = acc + w * (row[(size_t)j * npair + cc * NORB + a] *
                                         A.tail[((size_t)(j % A.ring) * npair + a * NORB + bb) * nt + mm]);
                }
            F[(mm - s0) * npair + ee] = acc;
        }
        __syncthreads();
        // (iii) the leaf's columns, right to left
        const long long lw = s1 - s0;
        const cd* Lf = A.leaf + A.Loff[leaf];
        const int jtop = min(n, s1 - 1);
        for (; m >= s0; --m) {
            cd acc = mk(0.0, 0.0);   // rows j of this leaf, j > m (thread group g takes j = m+1+g, +SG, ..)
            for (int j = m + 1 + g; j <= jtop; j += SG) {
                const double w = w_end(A.W, n, j);
                const long long tj = (long long)(j - s0) * (j - s0 + 1) / 2 + (m - s0);
                for (int a = 0; a < NORB; ++a)
                    acc = acc + w * (row[(size_t)j * npair + c * NORB + a] *
                                     Lf[(size_t)(a * NORB + bo) * (lw * (lw + 1) / 2) + tj]);
            }
            red[t] = acc;
            __syncthreads();
            if (g == 0) {
                cd s = F[(m - s0) * npair + e];
                for (int q = 0; q < SG; ++q) s = s + red[q * npair + e];
                for (int i = 1; i <= k; ++i)   // start weights of s = m+i on the band
                    for (int a = 0; a < NORB; ++a)
                        s = s + (A.W.om[i] - 1.0) * (row[(size_t)(m + i) * npair + c * NORB + a] *
                                                     sig_band(m + i, m, a * NORB + bo));
                cd bd = mk(0.0, 0.0);
                for (int l = 1; l <= k; ++l) bd = bd + A.S.a[l] * row[(size_t)(m + l) * npair + e];
                rhs[e] = mk(h * s.x + bd.y / h, h * s.y - bd.x / h);   // h s - (i/h) bd
            }
            __syncthreads();
            // X M_m = rhs  <=>  M_m^T X^T = rhs^T: [M^T | rhs^T] with M = i a_0/h - eps(m) - h omega_0 Sigma(m,m)
            for (int x = t; x < NORB * 2 * NORB; x += NTM) {
                const int r = x / (2 * NORB), col = x % (2 * NORB);
                cd v;
                if (col < NORB)   // M^T[r][col] = M[col][r]
                    v = mk(0.0, r == col ? A.S.a[0] / h : 0.0) - epsm(m, col, r) -
                        (h * A.W.om[0]) * sig_band(m, m, col * NORB + r);
                else
                    v = rhs[(col - NORB) * NORB + r];   // rhs^T[r][cc] = rhs[cc][r]
                T[x] = v;
            }
            __syncthreads();
            gj64(T, NORB, 2 * NORB, used, prow);
            if (t < npair)   // X[c][a] = Y[a][c]
                row[(size_t)m * npair + c * NORB + bo] = gj_sol(T, NORB, 2 * NORB, prow, bo, c);
            __syncthreads();
        }
        --leaf;
    }
}

}  // namespace

hipError_t launch_row_march(const MarchArgs& a, hipStream_t st) {
    if (a.nlo < a.k || a.nhi < a.nlo || a.RC > RCMAX) return hipErrorInvalidValue;
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
