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
//  * step_bulk, columns m < n-k (interval length L = n-m >= k+1): the left form,
//      M G(n,m) = -(i/h) sum_{l=1..k} a_l G(n-l,m) + h sum_{j=m}^{n-1} w^{(L)}_{j-m} Sigma(n,j) G(j,m),
//      M = (i a_0/h) 1 - eps(t_n) - h w^{(L)}_L Sigma(n,n).
//    Since L >= k+1, w^{(L)}_L is the end weight omega_0 for every such column: M is
//    the same matrix for the whole row, inverted once per workgroup (a 2 norb wide
//    Gauss-Jordan sweep in LDS) and applied to each column's right side.
//  * step_near, columns n-k..n-1: the right form at (t_n, t_m), whose integral
//    over [t_m, t_n] and t'-derivative only touch the entries G(n, n-k..n); the k
//    unknown norb x norb entries multiply known matrices from the right, so the
//    norb rows of G decouple and one k norb x k norb system with norb right sides
//    is solved (Gauss-Jordan with partial pivoting in LDS, one workgroup).
//
// Both kernels are FP64.  A singular system (zero pivot) leaves non-finite entries.
#include "step.h"

namespace hn {
namespace {

constexpr int NT = 256;

// Gauss-Jordan elimination with partial pivoting by one workgroup on the
// K x ld row-major matrix T in LDS, [A | B] with A of K columns: on return the
// columns K..ld-1 hold A^{-1} B.  fcol: K entries of LDS, piv: one int of LDS.
__device__ void gauss_jordan(cd* T, int K, int ld, cd* fcol, int* piv) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int p = 0; p < K; ++p) {
        if (wave == 0) {   // pivot row: the largest |A(r, p)|, r >= p (first one on ties)
            double best = -1.0;
            int bi = p;
            for (int r = p + lane; r < K; r += 64) {
                const double v = norm2(T[r * ld + p]);
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
            if (lane == 0) *piv = bi;
        }
        __syncthreads();
        const int q = *piv;
        if (q != p)   // the columns left of p are zero in both rows
            for (int j = p + t; j < ld; j += NT) {
                const cd x = T[p * ld + j];
                T[p * ld + j] = T[q * ld + j];
                T[q * ld + j] = x;
            }
        __syncthreads();
        const cd d = T[p * ld + p];
        const double s = 1.0 / norm2(d);
        const cd inv = mk(d.x * s, -d.y * s);
        for (int r = t; r < K; r += NT) fcol[r] = T[r * ld + p];
        __syncthreads();
        for (int j = p + t; j < ld; j += NT) T[p * ld + j] = T[p * ld + j] * inv;
        __syncthreads();
        // remove column p from every other row (columns left of p are not read again)
        const int w = ld - p;
        for (int e = t; e < K * w; e += NT) {
            const int r = e / w, j = p + e % w;
            if (r != p) T[r * ld + j] = T[r * ld + j] - fcol[r] * T[p * ld + j];
        }
        __syncthreads();
    }
}

// the near-diagonal system of the right form: with the unknowns
// Y[(u, a)][c] = G(n, n-k+u)[c][a], u = 0..k-1, and the equation of column
// m = n-k+i (interval length L = k-i) as the row block (i, b):
//   sum_{u,a} C_{u,i}[a][b] Y[(u,a)][c] = R_i[c][b],
//   C_{u,i} = -(i/h) D_{iu} 1 - [u = i] eps(t_m) - [u >= i] h w^{(L)}_{u-i} Sigma(t_{n-k+u}, t_m),
//   R_i     = (D_{ik}/h) 1 - i h w^{(L)}_L Sigma(t_n, t_m)       (from G(n, n) = -i)
template <int NORB>
__global__ void __launch_bounds__(NT) step_near(StepArgs A) {
    constexpr int npair = NORB * NORB, KMAX = 5 * NORB, LDMAX = KMAX + NORB;
    __shared__ cd T[KMAX * LDMAX];
    __shared__ cd fcol[KMAX];
    __shared__ int piv;
    const int n = A.n, k = A.k, K = k * NORB, ld = K + NORB;
    const double h = A.h;
    for (int e = threadIdx.x; e < K * ld; e += NT) {
        const int r = e / ld, col = e % ld, i = r / NORB, b = r % NORB;
        cd v;
        if (col < K) {
            const int u = col / NORB, a = col % NORB;
            v = mk(0.0, a == b ? -A.S.D[i][u] / h : 0.0);
            if (u == i) v = v - A.eps[(size_t)i * npair + a * NORB + b];
            if (u >= i)
                v = v - (h * interval_w(A.W, k - i, u - i)) * A.sigNear[((size_t)u * k + i) * npair + a * NORB + b];
        } else {
            const int c = col - K;
            const cd sg = A.sigR[(size_t)(n - k + i) * npair + c * NORB + b];
            const double wh = h * interval_w(A.W, k - i, k - i);
            v = mk((c == b ? A.S.D[i][k] / h : 0.0) + wh * sg.y, -wh * sg.x);
        }
        T[e] = v;
    }
    __syncthreads();
    gauss_jordan(T, K, ld, fcol, &piv);
    for (int e = threadIdx.x; e < K * NORB; e += NT) {
        const int r = e / NORB, c = e % NORB, u = r / NORB, a = r % NORB;
        A.row[(size_t)(n - k + u) * npair + c * NORB + a] = T[r * ld + K + c];
    }
    for (int e = threadIdx.x; e < npair; e += NT)
        A.row[(size_t)n * npair + e] = mk(0.0, e / NORB == e % NORB ? -1.0 : 0.0);
}

// columns m < n-k: thread (m, a) takes column a of the right side of column m
// (it reads and then overwrites exactly the entries [m][b][a], b = 0..norb-1, of the
// row) and applies M^{-1}
template <int NORB>
__global__ void __launch_bounds__(NT) step_bulk(StepArgs A) {
    constexpr int npair = NORB * NORB, ld = 2 * NORB;
    __shared__ cd T[NORB * ld];
    __shared__ cd fcol[NORB];
    __shared__ int piv;
    const int n = A.n, k = A.k;
    const double h = A.h;
    const double wl = h * A.W.om[0];   // h w^{(L)}_L for L >= k+1
    for (int e = threadIdx.x; e < NORB * ld; e += NT) {
        const int r = e / ld, col = e % ld;
        cd v;
        if (col < NORB) {
            v = mk(0.0, r == col ? A.S.a[0] / h : 0.0) - A.eps[(size_t)k * npair + r * NORB + col] -
                wl * A.sigR[(size_t)n * npair + r * NORB + col];
        } else {
            v = mk(r == col - NORB ? 1.0 : 0.0, 0.0);
        }
        T[e] = v;
    }
    __syncthreads();
    gauss_jordan(T, NORB, ld, fcol, &piv);   // T[:, NORB:] = M^{-1}
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    const int m = (int)(t / NORB), a = (int)(t % NORB);
    if (m >= n - k) return;
    const double ih = 1.0 / h;
    cd x[NORB];
#pragma unroll
    for (int b = 0; b < NORB; ++b) {
        const size_t o = (size_t)m * npair + b * NORB + a;
        cd s = mk(0.0, 0.0);
        for (int l = 1; l <= k; ++l) s = s + A.S.a[l] * A.prev[l - 1][o];
        const cd hist = A.row[o];
        x[b] = mk(hist.x + s.y * ih, hist.y - s.x * ih);   // hist - (i/h) s
    }
#pragma unroll
    for (int c = 0; c < NORB; ++c) {
        cd y = mk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < NORB; ++b) fma_(y, T[c * ld + NORB + b], x[b]);
        A.row[(size_t)m * npair + c * NORB + a] = y;
    }
}

template <int NORB>
hipError_t launch_step_t(const StepArgs& a, hipStream_t st, hipEvent_t* ev) {
    if (ev) hipEventRecord(ev[0], st);
    step_near<NORB><<<1, NT, 0, st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    const long long threads = (long long)(a.n - a.k) * NORB;
    if (threads > 0) step_bulk<NORB><<<(unsigned)((threads + NT - 1) / NT), NT, 0, st>>>(a);
    if (ev) hipEventRecord(ev[2], st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const StepArgs& a, hipStream_t st, hipEvent_t* ev) {
    if (a.k < 1 || a.k > 5 || a.n < a.k) return hipErrorInvalidValue;
    switch (a.norb) {
        case 1: return launch_step_t<1>(a, st, ev);
        case 2: return launch_step_t<2>(a, st, ev);
        case 4: return launch_step_t<4>(a, st, ev);
        case 8: return launch_step_t<8>(a, st, ev);
        case 16: return launch_step_t<16>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hn
