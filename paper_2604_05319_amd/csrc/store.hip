// Appending a time step's row to the stored lower triangles.
//
// HODLR storage (section "Hierarchical decomposition"; the paper keeps the
// newest rows and the diagonal leaves dense and the finished off-diagonal
// parts compressed): row n of a component goes
//   - columns in the diagonal leaf of row n      -> that leaf's dense triangle,
//   - columns left of the leaf (block columns)   -> the dense tail slot of row n,
//     compressed later by the panel merge,
//   - retarded entries G^R(n, n-i), i <= k       -> the band used by the
//     quadrature end corrections.
// All dense storage is orbital-pair-major so that a kernel reading one pair
// streams contiguous memory.
#include "store.h"

namespace hn {

__device__ inline void append_hodlr_row(const AppendArgs& a) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)(a.n + 1) * a.npair;
    if (e >= total) return;
    const long long o = blockIdx.y;   // object of the batch
    const int j = (int)(e / a.npair), q = (int)(e % a.npair);
    const cd v = a.row[o * a.kRow + e];
    if (j >= a.ls) {
        a.leaf[o * a.kLeaf + (size_t)q * tri(a.lw) + tri(a.n - a.ls) + (j - a.ls)] = v;
    } else {
        a.tail[o * a.kTail + ((size_t)a.slot * a.npair + q) * a.nt + j] = v;
    }
    if (a.band && a.n - j <= a.k) a.band[o * a.kBand + ((size_t)j * (a.k + 1) + (a.n - j)) * a.npair + q] = v;
}

__global__ void append_hodlr_kernel(AppendArgs a) { append_hodlr_row(a); }

__global__ void append_hodlr2_kernel(AppendArgs a0, AppendArgs a1) {
    if (blockIdx.z == 0) append_hodlr_row(a0);
    else append_hodlr_row(a1);
}

__global__ void append_dense_kernel(cd* dst, const cd* row, int n, int npair, long long trin) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)(n + 1) * npair;
    if (e >= total) return;
    const int j = (int)(e / npair), q = (int)(e % npair);
    dst[(size_t)q * trin + tri(n) + j] = row[e];
}

hipError_t launch_append_hodlr(const AppendArgs& a, int nk, hipStream_t st) {
    const long long total = (long long)(a.n + 1) * a.npair;
    const int nb = (int)((total + 255) / 256);
    append_hodlr_kernel<<<dim3(nb, nk), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_append_hodlr2(const AppendArgs& a0, const AppendArgs& a1, int nk, hipStream_t st) {
    const long long total = (long long)(a0.n + 1) * a0.npair;
    const int nb = (int)((total + 255) / 256);
    append_hodlr2_kernel<<<dim3(nb, nk, 2), 256, 0, st>>>(a0, a1);
    return hipGetLastError();
}

hipError_t launch_append_dense(cd* dst, const cd* row, int n, int npair, long long trin,
                               hipStream_t st) {
    const long long total = (long long)(n + 1) * npair;
    const int nb = (int)((total + 255) / 256);
    append_dense_kernel<<<nb, 256, 0, st>>>(dst, row, n, npair, trin);
    return hipGetLastError();
}

}  // namespace hn
