// Internal declarations shared by the host code and the HIP kernels of the
// compressed history-integral library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace hn {

// ---------------------------------------------------------------------------
// complex double
struct cd {
    double x, y;
};

__host__ __device__ inline cd mk(double a, double b) { return cd{a, b}; }
__host__ __device__ inline cd operator+(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cd operator-(cd a) { return cd{-a.x, -a.y}; }
__host__ __device__ inline cd operator*(cd a, cd b) {
    return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline cd operator*(double s, cd a) { return cd{s * a.x, s * a.y}; }
__host__ __device__ inline cd conj(cd a) { return cd{a.x, -a.y}; }
__host__ __device__ inline double norm2(cd a) { return a.x * a.x + a.y * a.y; }
// acc += a * b
__host__ __device__ inline void fma_(cd& acc, cd a, cd b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__host__ __device__ inline void fmac_(cd& acc, cd a, cd b) {
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

__host__ __device__ inline long long tri(long long n) { return n * (n + 1) / 2; }

// complex float: the storage type of the low-rank factors in the FP32-factor form
struct cf {
    float x, y;
};
// factor element <-> complex double (the arithmetic type of every kernel)
__host__ __device__ inline cd to_cd(cd v) { return v; }
__host__ __device__ inline cd to_cd(cf v) { return cd{(double)v.x, (double)v.y}; }
template <class FT>
__host__ __device__ inline FT from_cd(cd v);
template <>
__host__ __device__ inline cd from_cd<cd>(cd v) { return v; }
template <>
__host__ __device__ inline cf from_cd<cf>(cd v) { return cf{(float)v.x, (float)v.y}; }

// ---------------------------------------------------------------------------
// quadrature weights passed by value to kernels
struct Weights {
    int k;
    double om[6];      // Gregory end weights omega_0..omega_k
    double nc[6][7];   // nc[L][i]: interval weights for 0 <= L < k (L = 0: empty)
};

// interval weight w^{(L)}_i, any L >= 0 (device and host)
__host__ __device__ inline double interval_w(const Weights& W, int L, int i) {
    if (L < W.k) return W.nc[L][i];
    double w = 1.0;
    if (i <= W.k) w += W.om[i] - 1.0;
    if (L - i <= W.k) w += W.om[L - i] - 1.0;
    return w;
}
// end-weight fold of the retarded row: 1 + (omega_{n-j} - 1)[n-j <= k]
__host__ __device__ inline double w_end(const Weights& W, int n, int j) {
    int d = n - j;
    return d <= W.k ? W.om[d] : 1.0;
}
// start-weight fold: 1 + (omega_s - 1)[s <= k]
__host__ __device__ inline double w_start(const Weights& W, int s) {
    return s <= W.k ? W.om[s] : 1.0;
}

// ---------------------------------------------------------------------------
// host plan: HODLR geometry
struct Geometry {
    int nt = 0, nlvl = 0, nb = 0, nleaf = 0;
    std::vector<int> level, r0, r1, c0, c1;   // per block
    std::vector<int> s0, s1;                  // per leaf
    std::vector<int> row_leaf;                // leaf index of each row
    std::vector<int> cover;                   // [l][m], l = 0..nlvl-1: b (column role) or ~b (row role)
    int max_leaf = 0, min_leaf = 0;
};

// weights of the retarded time step: backward differentiation a_l (f'(t_n) h ~
// sum_l a_l f(t_{n-l})) and the differentiation matrix D[i][p] of the degree-k
// interpolant through k+1 equispaced points (derivative at point i)
struct StepWeights {
    int k;
    double a[6];
    double D[6][6];
};
bool make_step_weights(int k, StepWeights& S, std::string& err);

bool build_geometry(int nt, int nlvl, Geometry& g, std::string& err);
bool make_weights(int k, Weights& W, std::string& err);
// exact-rational interval weights, for the public hnessi_weights
bool interval_weights_exact(int k, int L, std::vector<double>& w, std::string& err);

// ---------------------------------------------------------------------------
// constants of the device kernels
// factor rows per projection task: more rows for small norb, whose tasks carry
// fewer bytes per row (the Sigma rows of a task are staged in LDS, kch * norb entries)
__host__ __device__ constexpr int kch(int norb) { return norb <= 2 ? 1024 : (norb == 4 ? 512 : 256); }
// projection chunk rows a handle may be created with (hnessi_set_tile_shape), by norb:
// 256..1024 for norb <= 4, 128..256 for norb 8 and 16 (the staged Sigma rows of a
// chunk and the rank reduction share the task's LDS)
__host__ __device__ constexpr int kch_max(int norb) { return norb <= 4 ? 1024 : 256; }
inline bool kch_allowed(int norb, int rows) {
    return rows == 0 || (norb <= 4 ? (rows == 256 || rows == 512 || rows == 1024) : (rows == 128 || rows == 256));
}
constexpr int kTailCH = 64;   // columns per tail task
constexpr int kTailRows = 32; // tail rows at most: the panel being merged and the one being formed
// orbital-pair groups of the tail tasks (one workgroup and one partial slot each)
// Output slots of the dense pieces (leaf triangles and tail rows).  For norb <= 4
// every orbital pair is a task of its own and writes one orbital entry of one
// slot per output array (slot = the pair orbital summed over by the other
// tasks), so that each slot entry has exactly one writer; for norb 8 a task
// takes a group of pairs and the output has four slots; for norb 16 a task
// takes one output orbital and sums over all pairs that feed it (one slot, two
// for the lesser leaf output, whose two products sum over different orbitals).
__host__ __device__ constexpr int tail_groups(int norb) { return norb <= 4 ? norb : (norb == 16 ? 1 : 4); }
__host__ __device__ constexpr int leaf_groups(int norb) { return norb <= 4 ? norb : (norb == 16 ? 1 : 4); }
__host__ __device__ constexpr int leaf_ll_slots(int norb) { return norb <= 4 ? 2 * norb : (norb == 16 ? 2 : 4); }

}  // namespace hn
