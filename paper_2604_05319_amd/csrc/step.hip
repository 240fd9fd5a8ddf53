// Retarded time step: the two small solves that turn the history sum of step n
// (computed by the history kernels over the stored rows 0..n-1) into row n of G^R.
//
// Equation: the retarded Kadanoff-Baym equation (section "Kadanoff-Baym
// equations", Eq. KBER and its left-form counterpart) with G^R(t,t) = -i;
// the time derivative by backward differentiation, a_l = -D_{0l}, and the
// start of the row by the polynomial differentiation weights D_{ip} (appendix on
// the differentiation weights); the integrals by the interval weights of the
// section "Numerical integration".
//
//  * step_near (one workgroup per object, beside the history kernels): the matrix of the
//    left form,
//      M = (i a_0/h) 1 - eps(t_n) - h w^{(L)}_L Sigma(n,n),
//    is the same for every column m < n-k (L = n-m >= k+1 makes w^{(L)}_L the end weight
//    omega_0), so it is inverted once; then the right form at (t_n, t_m), m = n-k..n-1,
//    whose integral over [t_m, t_n] and t'-derivative only touch the entries
//    G(n, n-k..n): the k unknown norb x norb entries multiply known matrices from the
//    right, so the norb rows of G decouple and one k norb x k norb system with norb
//    right sides is solved.  Both by Gauss-Jordan elimination with partial pivoting in
//    LDS; M^{-1} and the k entries go to a scratch buffer.
//  * step_bulk, columns m < n-k: the left form
//      M G(n,m) = -(i/h) sum_{l=1..k} a_l G(n-l,m) + h sum_{j=m}^{n-1} w^{(L)}_{j-m} Sigma(n,j) G(j,m)
//    (the history sum comes in through the output row), one streaming pass: every
//    thread forms one entry of a column's right side, the block's right sides are
//    staged in LDS and multiplied by M^{-1}; one more workgroup copies the near-diagonal
//    entries from the scratch into the row and writes G(n, n) = -i.
//
// Both kernels are FP64.  A singular system (zero pivot) leaves non-finite entries.
#include "step.h"

namespace hn {
namespace {

constexpr int NT = 256;

// object blockIdx.y of a batch: its arrays start one stride per object further
#define OBJ ((long long)blockIdx.y)

// Gauss-Jordan elimination with partial pivoting by one workgroup on the K x ld
// row-major matrix T = [A | B] in LDS (A of K columns).  Rows are never exchanged:
// the pivot of column p is the not yet used row prow[p] with the largest |T(r, p)|,
// and every other row r loses T(r, p) / T(prow[p], p) times it in the columns right
// of p (a column left of the current one is not read again, so it is not cleared).
// Two barriers per column.  On return (A^{-1} B)[p][c] =
// T[prow[p]][K + c] / T[prow[p]][p].  used, prow: K ints of LDS each.
__device__ void gauss_jordan(cd* T, int K, int ld, int* used, int* prow) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int r = t; r < K; r += NT) used[r] = 0;
    __syncthreads();
    for (int p = 0; p < K; ++p) {
        if (wave == 0) {
            double best = -1.0;
            int bi = K;
            for (int r = lane; r < K; r += 64) {
                const double v = used[r] ? -1.0 : norm2(T[r * ld + p]);
                if (v > best) {
                    best = v;
                    bi = r;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {   // largest value, first row on ties
                const double ov = __shfl_xor(best, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                prow[p] = bi;
                used[bi] = 1;
            }
        }
        __syncthreads();
        const int q = prow[p];
        const cd d = T[q * ld + p];
        const double s = 1.0 / norm2(d);
        const cd inv = mk(d.x * s, -d.y * s);
        const int w = ld - p - 1;
        for (int e = t; e < K * w; e += NT) {   // T(r, p) is read here and written by no one
            const int r = e / w, j = p + 1 + e % w;
            if (r != q) T[r * ld + j] = T[r * ld + j] - (T[r * ld + p] * inv) * T[q * ld + j];
        }
        __syncthreads();
    }
}

// (A^{-1} B)[p][c] after gauss_jordan
__device__ inline cd gj_solution(const cd* T, int K, int ld, const int* prow, int p, int c) {
    const int q = prow[p];
    const cd d = T[q * ld + p];
    const double s = 1.0 / norm2(d);
    return T[q * ld + K + c] * mk(d.x * s, -d.y * s);
}

// M^{-1} into the scratch, then the near-diagonal system of the right form: with the unknowns
// Y[(u, a)][c] = G(n, n-k+u)[c][a], u = 0..k-1, and the equation of column
// m = n-k+i (interval length L = k-i) as the row block (i, b):
//   sum_{u,a} C_{u,i}[a][b] Y[(u,a)][c] = R_i[c][b],
//   C_{u,i} = -(i/h) D_{iu} 1 - [u = i] eps(t_m) - [u >= i] h w^{(L)}_{u-i} Sigma(t_{n-k+u}, t_m),
//   R_i     = (D_{ik}/h) 1 - i h w^{(L)}_L Sigma(t_n, t_m)       (from G(n, n) = -i)
template <int NORB>
__global__ void __launch_bounds__(NT) step_near(StepArgs A) {
    constexpr int npair = NORB * NORB, KMAX = 5 * NORB, LDMAX = KMAX + NORB;
    __shared__ cd T[KMAX * LDMAX];
    __shared__ int used[KMAX], prow[KMAX];
    const int n = A.n, k = A.k, K = k * NORB, ld = K + NORB;
    const double h = A.h;
    const cd* eps = A.eps + OBJ * A.kEps;
    const cd* sigR = A.sigR + OBJ * A.kSig;
    const cd* sigNear = A.sigNear + OBJ * A.kNear;
    cd* minv = A.scr + OBJ * (k + 1) * npair;
    cd* nearOut = minv + npair;
    {   // [M | 1], NORB x 2 NORB
        constexpr int l2 = 2 * NORB;
        const double wl = h * A.W.om[0];   // h w^{(L)}_L for L >= k+1
        for (int e = threadIdx.x; e < NORB * l2; e += NT) {
            const int r = e / l2, col = e % l2;
            cd v;
            if (col < NORB)
                v = mk(0.0, r == col ? A.S.a[0] / h : 0.0) - eps[(size_t)k * npair + r * NORB + col] -
                    wl * sigR[(size_t)n * npair + r * NORB + col];
            else
                v = mk(r == col - NORB ? 1.0 : 0.0, 0.0);
            T[e] = v;
        }
        __syncthreads();
        gauss_jordan(T, NORB, l2, used, prow);
        for (int e = threadIdx.x; e < npair; e += NT) minv[e] = gj_solution(T, NORB, l2, prow, e / NORB, e % NORB);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < K * ld; e += NT) {
        const int r = e / ld, col = e % ld, i = r / NORB, b = r % NORB;
        cd v;
        if (col < K) {
            const int u = col / NORB, a = col % NORB;
            v = mk(0.0, a == b ? -A.S.D[i][u] / h : 0.0);
            if (u == i) v = v - eps[(size_t)i * npair + a * NORB + b];
            if (u >= i)
                v = v - (h * interval_w(A.W, k - i, u - i)) * sigNear[((size_t)u * k + i) * npair + a * NORB + b];
        } else {
            const int c = col - K;
            const cd sg = sigR[(size_t)(n - k + i) * npair + c * NORB + b];
            const double wh = h * interval_w(A.W, k - i, k - i);
            v = mk((c == b ? A.S.D[i][k] / h : 0.0) + wh * sg.y, -wh * sg.x);
        }
        T[e] = v;
    }
    __syncthreads();
    gauss_jordan(T, K, ld, used, prow);
    for (int e = threadIdx.x; e < K * NORB; e += NT) {
        const int r = e / NORB, c = e % NORB, u = r / NORB, a = r % NORB;
        nearOut[(size_t)u * npair + c * NORB + a] = gj_solution(T, K, ld, prow, r, c);
    }
}

// columns m < n-k, NT / npair columns per workgroup (the last workgroup of the grid
// copies the near-diagonal entries and writes G(n, n)): thread (m, e) forms entry e = (b, a)
// of column m's right side (reading exactly the row entry it later overwrites with entry
// e = (c, a) of the solution; the barrier separates every read of the block's columns
// from every write)
template <int NORB>
__global__ void __launch_bounds__(NT) step_bulk(StepArgs A) {
    constexpr int npair = NORB * NORB, CPB = NT / npair;
    __shared__ cd Mi[npair];
    __shared__ cd R[CPB * npair];
    const int t = threadIdx.x;
    cd* row = A.row + OBJ * A.kRow;
    const cd* scr = A.scr + OBJ * (A.k + 1) * npair;
    if (blockIdx.x == gridDim.x - 1) {   // whole workgroup: no barrier below is reached
        for (int e = t; e < A.k * npair; e += NT) row[(size_t)(A.n - A.k) * npair + e] = scr[npair + e];
        for (int e = t; e < npair; e += NT) row[(size_t)A.n * npair + e] = mk(0.0, e / NORB == e % NORB ? -1.0 : 0.0);
        return;
    }
    if (t < npair) Mi[t] = scr[t];
    const long long m = (long long)blockIdx.x * CPB + t / npair;
    const int e = t % npair;
    const bool on = t < CPB * npair && m < A.n - A.k;
    const double ih = 1.0 / A.h;
    const size_t o = (size_t)m * npair + e;
    if (on) {
        cd s = mk(0.0, 0.0);
#pragma unroll
        for (int l = 1; l <= 5; ++l)
            if (l <= A.k) s = s + A.S.a[l] * A.prev[l - 1][OBJ * A.kPrev + o];
        const cd hist = row[o];
        R[t] = mk(hist.x + s.y * ih, hist.y - s.x * ih);   // hist - (i/h) s
    }
    __syncthreads();
    if (!on) return;
    const int c = e / NORB, a = e % NORB, base = t - e;
    cd y = mk(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < NORB; ++b) fma_(y, Mi[c * NORB + b], R[base + b * NORB + a]);
    row[o] = y;
}

// ---------------------------------------------------------------------------
// lesser step

constexpr int kSumChunk = 256;   // time points s per workgroup of lesser_sums

// M_L^{-1}, M_L = (i a_0/h) 1 - eps(t_n) - h w^{(n)}_n Sigma^R(n, n), into scr[0..npair)
template <int NORB>
__global__ void __launch_bounds__(NT) lesser_prep(LesserStepArgs A) {
    constexpr int npair = NORB * NORB, l2 = 2 * NORB;
    __shared__ cd T[NORB * l2];
    __shared__ int used[NORB], prow[NORB];
    const int n = A.n, k = A.k;
    const double wl = A.h * interval_w(A.W, n, n);
    const cd* sRn = A.sigRn[k - 1] + (size_t)n * npair;
    for (int e = threadIdx.x; e < NORB * l2; e += NT) {
        const int r = e / l2, col = e % l2;
        T[e] = col < NORB ? mk(0.0, r == col ? A.S.a[0] / A.h : 0.0) - A.eps[(size_t)k * npair + r * NORB + col] -
                                wl * sRn[r * NORB + col]
                          : mk(r == col - NORB ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    gauss_jordan(T, NORB, l2, used, prow);
    for (int e = threadIdx.x; e < npair; e += NT) A.scr[e] = gj_solution(T, NORB, l2, prow, e / NORB, e % NORB);
}

// columns m <= n-k: thread (m, e = (b, a)) forms entry e of the right side
//   I^<(n,m) - (i/h) sum_l a_l G^<(n-l, m),  G^<(n-l, m)[b][a] = -conj(prev[l-1][m][a][b])
//   below the diagonal, the stored equal-time value prev[l-1][m][b][a] itself on it (m = n-l),
// the block's right sides are staged in LDS; thread (m, (c, a)) then writes the slice entry
// G^<(t_m, t_n)[a][c] = -conj(G^<(n, m)[c][a]) with G^<(n, m) = M_L^{-1} rhs
template <int NORB>
__global__ void __launch_bounds__(NT) lesser_bulk(LesserStepArgs A) {
    constexpr int npair = NORB * NORB, CPB = NT / npair;
    __shared__ cd Mi[npair];
    __shared__ cd R[CPB * npair];
    const int t = threadIdx.x;
    if (t < npair) Mi[t] = A.scr[t];
    const long long m = (long long)blockIdx.x * CPB + t / npair;
    const int e = t % npair;
    const bool on = t < CPB * npair && m <= A.n - A.k;
    const double ih = 1.0 / A.h;
    if (on) {
        const int b = e / NORB, a = e % NORB;
        const size_t ot = (size_t)m * npair + a * NORB + b;   // transposed entry
        cd s = mk(0.0, 0.0);
#pragma unroll
        for (int l = 1; l <= 5; ++l)
            if (l <= A.k) {
                const cd v = m == A.n - l ? A.prev[l - 1][(size_t)m * npair + e] : -conj(A.prev[l - 1][ot]);
                s = s + A.S.a[l] * v;
            }
        const cd hist = A.slice[(size_t)m * npair + e];
        R[t] = mk(hist.x + s.y * ih, hist.y - s.x * ih);   // hist - (i/h) s
    }
    __syncthreads();
    if (!on) return;
    const int c = e / NORB, a = e % NORB, base = t - e;
    cd y = mk(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < NORB; ++b) fma_(y, Mi[c * NORB + b], R[base + b * NORB + a]);
    A.slice[(size_t)m * npair + a * NORB + c] = mk(-y.x, y.y);   // -conj
}

// partial sums, near column i = 1..k (m = n-k+i, grid y), time points s of chunk blockIdx.x:
//   h sum_{s <= n-k} w^{(m)}_s G^<(n,s) Sigma^A(s,m) + h sum_{s <= n} w^{(n)}_s G^R(n,s) Sigma^<(s,m)
// thread (s group g, entry e = (c, a)) accumulates entry e over its time points
template <int NORB>
__global__ void __launch_bounds__(NT) lesser_sums(LesserStepArgs A) {
    constexpr int npair = NORB * NORB, SG = NT / npair;
    __shared__ cd red[NT];
    const int n = A.n, k = A.k, i = blockIdx.y + 1, m = n - k + i;
    const int t = threadIdx.x, e = t % npair, g = t / npair, c = e / NORB, a = e % NORB;
    const cd* sRm = A.sigRn[i - 1];
    const int s0 = blockIdx.x * kSumChunk, s1 = min(s0 + kSumChunk, n + 1);
    cd acc = mk(0.0, 0.0);
    for (int s = s0 + g; s < s1; s += SG) {
        if (s <= n - k) {   // G^<(n,s)[c][b] = -conj(slice[s][b][c]);  Sigma^A(s,m)[b][a] = conj(Sigma^R(m,s)[a][b])
            const double w = A.h * interval_w(A.W, m, s);
            cd x = mk(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < NORB; ++b)
                x = x - conj(A.slice[(size_t)s * npair + b * NORB + c]) * conj(sRm[(size_t)s * npair + a * NORB + b]);
            acc = acc + w * x;
        }
        {   // Sigma^<(s,m): slice m at s (s <= m), else -conj(slice s at m)^T
            const double w = A.h * interval_w(A.W, n, s);
            cd x = mk(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < NORB; ++b) {
                const cd sl = s <= m ? A.sigLn[i - 1][(size_t)s * npair + b * NORB + a]
                                     : -conj(A.sigLn[s - (n - k) - 1][(size_t)m * npair + a * NORB + b]);
                fma_(x, A.GRn[(size_t)s * npair + c * NORB + b], sl);
            }
            acc = acc + w * x;
        }
    }
    red[t] = acc;
    __syncthreads();
    if (g == 0) {
        cd sum = mk(0.0, 0.0);
        for (int q = 0; q < SG; ++q) sum = sum + red[q * npair + e];
        A.part[((size_t)(i - 1) * A.nchunk + blockIdx.x) * npair + e] = sum;
    }
}

// the near system: unknowns Y[(p, a)][c] = G^<(n, n-k+p)[c][a], p = 1..k; equation of column
// m = n-k+i as the row block (i, b):
//   sum_{p,a} C_{p,i}[a][b] Y[(p,a)][c] = R_i[c][b],
//   C_{p,i} = -(i/h) D_{ip} 1 - [p = i] eps(t_m) - [p <= i] h w^{(m)}_{n-k+p} Sigma^A(n-k+p, m),
//   R_i     = (i/h) D_{i0} G^<(n, n-k) + (the partial sums of column i)
template <int NORB>
__global__ void __launch_bounds__(NT) lesser_near(LesserStepArgs A) {
    constexpr int npair = NORB * NORB, KMAX = 5 * NORB, LDMAX = KMAX + NORB;
    __shared__ cd T[KMAX * LDMAX];
    __shared__ int used[KMAX], prow[KMAX];
    const int n = A.n, k = A.k, K = k * NORB, ld = K + NORB;
    const double h = A.h;
    for (int e = threadIdx.x; e < K * ld; e += NT) {
        const int r = e / ld, col = e % ld, i = r / NORB + 1, b = r % NORB, m = n - k + i;
        cd v;
        if (col < K) {
            const int p = col / NORB + 1, a = col % NORB, s = n - k + p;
            v = mk(0.0, a == b ? -A.S.D[i][p] / h : 0.0);
            if (p == i) v = v - A.eps[(size_t)i * npair + a * NORB + b];
            if (p <= i)   // Sigma^A(s,m)[a][b] = conj(Sigma^R(m,s)[b][a])
                v = v - (h * interval_w(A.W, m, s)) * conj(A.sigRn[i - 1][(size_t)s * npair + b * NORB + a]);
        } else {
            const int c = col - K;
            // (i/h) D_{i0} G^<(n, n-k)[c][b],  G^<(n, n-k)[c][b] = -conj(slice[n-k][b][c])
            const cd g0 = A.slice[(size_t)(n - k) * npair + b * NORB + c];
            const double d = A.S.D[i][0] / h;
            v = mk(-d * g0.y, -d * g0.x);   // (i d) (-conj(g0))
            for (int q = 0; q < A.nchunk; ++q) v = v + A.part[((size_t)(i - 1) * A.nchunk + q) * npair + c * NORB + b];
        }
        T[e] = v;
    }
    __syncthreads();
    gauss_jordan(T, K, ld, used, prow);
    for (int e = threadIdx.x; e < K * NORB; e += NT) {
        const int r = e / NORB, c = e % NORB, p = r / NORB + 1, a = r % NORB, s = n - k + p;
        const cd y = gj_solution(T, K, ld, prow, r, c);   // G^<(n, s)[c][a]
        if (s < n)
            A.slice[(size_t)s * npair + a * NORB + c] = mk(-y.x, y.y);   // G^<(t_s, t_n)[a][c] = -conj
        else
            A.slice[(size_t)n * npair + c * NORB + a] = y;               // G^<(t_n, t_n) itself
    }
}

template <int NORB>
hipError_t launch_lesser_rest_t(const LesserStepArgs& a, hipStream_t st, hipEvent_t* ev) {
    constexpr int CPB = NT / (NORB * NORB);
    const int nb = a.n - a.k + 1;
    if (ev) hipEventRecord(ev[0], st);
    lesser_bulk<NORB><<<(nb + CPB - 1) / CPB, NT, 0, st>>>(a);
    lesser_sums<NORB><<<dim3(a.nchunk, a.k), NT, 0, st>>>(a);
    lesser_near<NORB><<<1, NT, 0, st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    return hipGetLastError();
}

template <int NORB>
hipError_t launch_near_t(const StepArgs& a, hipStream_t st, hipEvent_t* ev) {
    if (ev) hipEventRecord(ev[0], st);
    step_near<NORB><<<dim3(1, a.nk), NT, 0, st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    return hipGetLastError();
}

template <int NORB>
hipError_t launch_bulk_t(const StepArgs& a, hipStream_t st, hipEvent_t* ev) {
    constexpr int CPB = NT / (NORB * NORB);
    const int nb = a.n - a.k;
    if (ev) hipEventRecord(ev[0], st);
    step_bulk<NORB><<<dim3((nb + CPB - 1) / CPB + 1, a.nk), NT, 0, st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    return hipGetLastError();
}

bool step_args_ok(const StepArgs& a) {
    return a.k >= 1 && a.k <= 5 && a.n >= a.k && a.nk >= 1 && a.nk <= 65535;
}

}  // namespace

int lesser_sum_chunks(int n) { return (n + 1 + kSumChunk - 1) / kSumChunk; }

hipError_t launch_lesser_prep(const LesserStepArgs& a, hipStream_t st) {
    if (a.k < 1 || a.k > 5 || a.n < a.k) return hipErrorInvalidValue;
    switch (a.norb) {
        case 1: lesser_prep<1><<<1, NT, 0, st>>>(a); break;
        case 2: lesser_prep<2><<<1, NT, 0, st>>>(a); break;
        case 4: lesser_prep<4><<<1, NT, 0, st>>>(a); break;
        case 8: lesser_prep<8><<<1, NT, 0, st>>>(a); break;
        case 16: lesser_prep<16><<<1, NT, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lesser_rest(const LesserStepArgs& a, hipStream_t st, hipEvent_t* ev) {
    if (a.k < 1 || a.k > 5 || a.n < a.k || a.nchunk != lesser_sum_chunks(a.n)) return hipErrorInvalidValue;
    switch (a.norb) {
        case 1: return launch_lesser_rest_t<1>(a, st, ev);
        case 2: return launch_lesser_rest_t<2>(a, st, ev);
        case 4: return launch_lesser_rest_t<4>(a, st, ev);
        case 8: return launch_lesser_rest_t<8>(a, st, ev);
        case 16: return launch_lesser_rest_t<16>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_near(const StepArgs& a, hipStream_t st, hipEvent_t* ev) {
    if (!step_args_ok(a)) return hipErrorInvalidValue;
    switch (a.norb) {
        case 1: return launch_near_t<1>(a, st, ev);
        case 2: return launch_near_t<2>(a, st, ev);
        case 4: return launch_near_t<4>(a, st, ev);
        case 8: return launch_near_t<8>(a, st, ev);
        case 16: return launch_near_t<16>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_bulk(const StepArgs& a, hipStream_t st, hipEvent_t* ev) {
    if (!step_args_ok(a)) return hipErrorInvalidValue;
    switch (a.norb) {
        case 1: return launch_bulk_t<1>(a, st, ev);
        case 2: return launch_bulk_t<2>(a, st, ev);
        case 4: return launch_bulk_t<4>(a, st, ev);
        case 8: return launch_bulk_t<8>(a, st, ev);
        case 16: return launch_bulk_t<16>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hn
