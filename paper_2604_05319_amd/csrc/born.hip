// Lattice second-Born self-energy of one time step, evaluated in real space
// (section "Driven 2D Hubbard example", Eq. BornApproxLG, and its "Implementation
// details": transform G_k -> G_r, local product, transform Sigma_r -> Sigma_k).
//
// With one band, t = t_n >= t' = t_j, and what the history stores (the retarded row
// G^R_k(t_n, t_j) and the lesser slice G^<_k(t_j, t_n)):
//   a_k = G^>_k(t_n, t_j) = G^R_k(t_n, t_j) - conj(G^<_k(t_j, t_n)),
//   b_k = G^<_k(t_n, t_j) = -conj(G^<_k(t_j, t_n)),
//   a_r, b_r = (1/N) sum_k e^{i k.r} (a_k, b_k),
// and, since G^{<,>}_{-r}(t', t) = -conj(G^{<,>}_r(t, t')) (the components' anti-Hermitian
// symmetry in site indices),
//   Sigma^>_r = U^2 a_r^2 (-conj(b_r)),   Sigma^<_r = U^2 b_r^2 (-conj(a_r)),
//   Sigma^R_k(t_n, t_j) = sum_r e^{-i k.r} (Sigma^>_r - Sigma^<_r),
//   Sigma^<_k(t_j, t_n) = -conj(sum_r e^{-i k.r} Sigma^<_r).
//
// One workgroup per tile of JT consecutive columns j: it reads, for every momentum,
// the tile's entries of both inputs (JT consecutive complex numbers per object and
// array) into LDS (rows padded to L+1 entries), then runs the 2D transforms as 1D line
// transforms in registers, each line split over a pair of lanes: to real space by
// decimation in time (each lane transforms the even or odd samples, one shuffle
// exchange combines them into the two halves of the output), back by decimation in
// frequency (halves combined first, then each lane transforms one parity of the
// output).  All rows (along y), then per column the transform of both arrays, the Born
// products with the partner pair's values and the transforms back, then all rows
// again; three barriers in all.  The half-length transforms are fully unrolled, their
// twiddles read from a compile-time table in constant memory (uniform across lanes).
// Consecutive tiles go to workgroups on the same XCD (workgroup b runs on XCD b mod 8),
// so the halves of a 128-byte line of one object's row are read through one L2.  FP64
// throughout; HBM-bound (2 N (n+1) complex entries read and 2 N (n+1) written per step).
#include "born.h"

namespace hn {
namespace {

constexpr int NT = 256;

template <int L>
struct BornShape {
    static constexpr int N = L * L;
    static constexpr int LOG = L == 2 ? 1 : L == 4 ? 2 : L == 8 ? 3 : L == 16 ? 4 : 5;
    // 2 JT transforms of N complex in 64 KB of LDS (two workgroups per compute unit)
    static constexpr int JT = (2048 / N) > 16 ? 16 : (2048 / N);
};

__host__ __device__ constexpr int rev_bits(int v, int log) {
    int r = 0;
    for (int i = 0; i < log; ++i) r |= ((v >> i) & 1) << (log - 1 - i);
    return r;
}

// sin and cos of x in [0, pi/4] by their Taylor series (compile time only)
constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int i = 1; i < 20; ++i) {
        t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        s += t;
    }
    return s;
}
constexpr double taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int i = 1; i < 20; ++i) {
        t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        s += t;
    }
    return s;
}
constexpr double kPi = 3.14159265358979323846;
// e^{2 pi i m / 32}, m = 0..15: the angle reduced to [0, pi/4] by the quadrant and
// octant symmetries, so that m = 0, 8 give (1, 0), (0, 1) exactly
constexpr double tw_re(int m) {
    const int r = m % 8;
    const double c = r <= 4 ? taylor_cos(kPi * r / 16) : taylor_sin(kPi * (8 - r) / 16);
    const double s = r <= 4 ? taylor_sin(kPi * r / 16) : taylor_cos(kPi * (8 - r) / 16);
    return m < 8 ? c : -s;
}
constexpr double tw_im(int m) {
    const int r = m % 8;
    const double c = r <= 4 ? taylor_cos(kPi * r / 16) : taylor_sin(kPi * (8 - r) / 16);
    const double s = r <= 4 ? taylor_sin(kPi * r / 16) : taylor_cos(kPi * (8 - r) / 16);
    return m < 8 ? s : c;
}
#define HN_TW(m) cd{tw_re(m), tw_im(m)}
__constant__ cd kTw32[16] = {HN_TW(0),  HN_TW(1),  HN_TW(2),  HN_TW(3),  HN_TW(4),  HN_TW(5),
                             HN_TW(6),  HN_TW(7),  HN_TW(8),  HN_TW(9),  HN_TW(10), HN_TW(11),
                             HN_TW(12), HN_TW(13), HN_TW(14), HN_TW(15)};
#undef HN_TW

// e^{s 2 pi i m / LEN}, s = +1 (INV) or -1, LEN a power of two <= 32
// (after unrolling, m and len are compile-time constants and the load a uniform one)
template <bool INV>
__device__ inline cd twiddle(int m, int len) {
    const cd w = kTw32[m * (32 / len)];
    return INV ? w : conj(w);
}

// in-register DFT of LEN points, x_k <- sum_m e^{s 2 pi i k m / LEN} x_m (radix 2, fully
// unrolled: every index is a compile-time constant)
template <int LEN, bool INV>
__device__ inline void fft_reg(cd (&x)[LEN]) {
    constexpr int LOG = LEN == 1 ? 0 : LEN == 2 ? 1 : LEN == 4 ? 2 : LEN == 8 ? 3 : 4;
#pragma unroll
    for (int i = 0; i < LEN; ++i) {
        const int j = rev_bits(i, LOG);
        if (j > i) {
            const cd t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
#pragma unroll
    for (int h = 1; h < LEN; h *= 2) {
#pragma unroll
        for (int g = 0; g < LEN; g += 2 * h) {
#pragma unroll
            for (int p = 0; p < h; ++p) {
                const cd u = x[g + p];
                const cd v = p == 0 ? x[g + p + h] : twiddle<INV>(p, 2 * h) * x[g + p + h];
                x[g + p] = u + v;
                x[g + p + h] = u - v;
            }
        }
    }
}

__device__ inline cd shfl1(cd v) { return mk(__shfl_xor(v.x, 1), __shfl_xor(v.y, 1)); }

// DFT of one L-point line (entries line[i * st]) split over a lane pair, lane hb of
// the pair: decimation in time, the lane's output entries hb L/2 + k, k < L/2, in x
template <int L, bool INV>
__device__ inline void line_dit(const cd* line, int st, int hb, cd (&x)[L / 2]) {
    constexpr int H = L / 2;
#pragma unroll
    for (int m = 0; m < H; ++m) x[m] = line[(2 * m + hb) * st];
    fft_reg<H, INV>(x);   // lane 0: E_k (even samples), lane 1: O_k (odd samples)
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const cd mine = hb ? twiddle<INV>(k, L) * x[k] : x[k];   // lane 1 sends w^k O_k, lane 0 E_k
        const cd other = shfl1(mine);
        x[k] = hb ? other - mine : mine + other;                 // X_{k+H} = E_k - w^k O_k, X_k = E_k + w^k O_k
    }
}

// the same DFT with the input split as halves (lane hb holds entries hb L/2 + m in x):
// decimation in frequency, the lane's output entries 2k + hb written to line[(2k + hb) * st]
template <int L, bool INV>
__device__ inline void line_dif(cd (&x)[L / 2], int hb, cd* line, int st) {
    constexpr int H = L / 2;
#pragma unroll
    for (int m = 0; m < H; ++m) {
        const cd other = shfl1(x[m]);
        // lane 0: x_m + x_{m+H}; lane 1: (x_m - x_{m+H}) w^m
        x[m] = hb ? twiddle<INV>(m, L) * (other - x[m]) : x[m] + other;
    }
    fft_reg<H, INV>(x);
#pragma unroll
    for (int k = 0; k < H; ++k) line[(2 * k + hb) * st] = x[k];
}

// transforms along y of every row of the 2 JT arrays (row t of array t / L is line t):
// lane pair t, output halves written back in place
template <int L, int JT, bool INV>
__device__ inline void rows_pass(cd* X) {
    constexpr int LP = L + 1, H = L / 2;
#pragma unroll 1
    for (int t = threadIdx.x; t < 4 * JT * L; t += NT) {   // 2 JT L lines, 2 lanes each
        const int line = t >> 1, hb = t & 1;
        cd* row = X + (size_t)line * LP;
        cd x[H];
        line_dit<L, INV>(row, 1, hb, x);
#pragma unroll
        for (int k = 0; k < H; ++k) row[hb * H + k] = x[k];
    }
}

template <int L>
__global__ void __launch_bounds__(NT) born_kernel(BornArgs A) {
    using S = BornShape<L>;
    constexpr int N = S::N, JT = S::JT, LP = L + 1, AS = L * LP, H = L / 2;
    __shared__ cd X[2 * JT * AS];   // arrays 0..JT-1: a (then Sigma^R), JT..2JT-1: b (then Sigma^<); [x][y]
    const int ntiles = (A.n + 1 + JT - 1) / JT;
    const int per = (ntiles + 7) / 8;
    const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int j0 = tile * JT;
    for (int e = threadIdx.x; e < JT * N; e += NT) {
        const int k = e / JT, jj = e % JT, j = j0 + jj;
        cd a = mk(0.0, 0.0), b = mk(0.0, 0.0);
        if (j <= A.n) {
            const cd r = A.GR[(size_t)k * A.inStride + j];
            const cd l = A.GL[(size_t)k * A.inStride + j];
            a = mk(r.x - l.x, r.y + l.y);   // r - conj(l)
            b = mk(-l.x, l.y);              // -conj(l)
        }
        const int o = (k / L) * LP + k % L;
        X[(size_t)jj * AS + o] = a;
        X[(size_t)(JT + jj) * AS + o] = b;
    }
    __syncthreads();
    rows_pass<L, JT, true>(X);
    __syncthreads();
    // columns: the four lanes 4c..4c+3 take column c = jj L + y of a (lanes 4c, 4c+1) and
    // of b (4c+2, 4c+3), a lane pair per column; after the transform to real space lane
    // t and lane t ^ 2 hold a and b at the same sites x, which the Born products need.
    // 4 JT L is a multiple of 4, so the four lanes are always active together.
    const double inv = 1.0 / N;
#pragma unroll 1
    for (int t = threadIdx.x; t < 4 * JT * L; t += NT) {
        const int c = t >> 2, which = (t >> 1) & 1, hb = t & 1, jj = c / L, y = c % L;
        cd* col = X + (size_t)(which * JT + jj) * AS + y;
        cd x[H];
        line_dit<L, true>(col, LP, hb, x);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const cd own = inv * x[i];
            const cd oth = mk(__shfl_xor(own.x, 2), __shfl_xor(own.y, 2));
            const cd ar = which ? oth : own, br = which ? own : oth;
            const cd sl = A.u2 * ((br * br) * mk(-ar.x, ar.y));   // U^2 b^2 (-conj a)
            if (which) {
                x[i] = sl;
            } else {
                const cd sg = A.u2 * ((ar * ar) * mk(-br.x, br.y));   // U^2 a^2 (-conj b)
                x[i] = sg - sl;
            }
        }
        line_dif<L, false>(x, hb, col, LP);
    }
    __syncthreads();
    rows_pass<L, JT, false>(X);
    __syncthreads();
    for (int e = threadIdx.x; e < JT * N; e += NT) {
        const int k = e / JT, jj = e % JT, j = j0 + jj;
        if (j > A.n) continue;
        const int o = (k / L) * LP + k % L;
        const cd sr = X[(size_t)jj * AS + o], sl = X[(size_t)(JT + jj) * AS + o];
        A.SR[(size_t)k * A.outStride + j] = sr;
        A.SL[(size_t)k * A.outStride + j] = mk(-sl.x, sl.y);   // -conj
    }
}

template <int L>
hipError_t launch_born_t(const BornArgs& a, hipStream_t st, hipEvent_t* ev) {
    constexpr int JT = BornShape<L>::JT;
    const int ntiles = (a.n + 1 + JT - 1) / JT;
    if (ev) hipEventRecord(ev[0], st);
    born_kernel<L><<<8 * ((ntiles + 7) / 8), NT, 0, st>>>(a);
    if (ev) hipEventRecord(ev[1], st);
    return hipGetLastError();
}

}  // namespace

int born_tile(int L) {
    switch (L) {
        case 2: return BornShape<2>::JT;
        case 4: return BornShape<4>::JT;
        case 8: return BornShape<8>::JT;
        case 16: return BornShape<16>::JT;
        case 32: return BornShape<32>::JT;
        default: return 0;
    }
}

hipError_t launch_born(const BornArgs& a, hipStream_t st, hipEvent_t* ev) {
    switch (a.L) {
        case 2: return launch_born_t<2>(a, st, ev);
        case 4: return launch_born_t<4>(a, st, ev);
        case 8: return launch_born_t<8>(a, st, ev);
        case 16: return launch_born_t<16>(a, st, ev);
        case 32: return launch_born_t<32>(a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hn
