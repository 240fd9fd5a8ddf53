// Truncated SVD of one dense block (section "Hierarchical decomposition":
// a finished block B is stored as U S V^dagger, keeping the singular values
// sigma >= eps_SVD, so that |B - U S V^dagger|_2 = sigma_{r+1} < eps_SVD).
//
// The block is factored with the same panel merges that build the HODLR
// blocks (TSQR of [V S, A_p^dagger], small SVD, truncation), P rows at a time,
// but every merge except the last drops only the singular values below
// delta * eps with delta = 5e-4 / (number of merges).  The dropped parts add
// up to less than 5e-4 * eps in the spectral norm, so the last merge, which
// truncates at eps, sees the singular values of the block to within
// 5e-4 * eps: its rank is the eps-rank of the block except for a singular
// value within 1e-3 * eps of eps, and the spectral error is below eps under
// the same condition.
#include <mutex>
#include <string>
#include <type_traits>

#include "alloc.h"
#include "merge.h"

namespace hn {

namespace {

constexpr int kCW = kWLarge;            // merge width of the block factorization
constexpr int kCP = 8;                  // rows per merge
constexpr int kCapInt = kCW - kCP;      // rank capacity of the intermediate factors
constexpr double kDropBudget = 5e-4;    // total intermediate drop, in units of eps

__global__ void compress_finish(const int* err, int* rank_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int ei = err[0], ef = err[1];
        if ((ei | ef) & 2) rank_out[0] = HNESSI_E_VALUE;
        else if (ei & 1) rank_out[0] = HNESSI_E_RANK;
    }
}

// device scratch of one factorization
struct CompressScratch {
    cd *Us, *Vs, *nodeR, *nodeQ, *chunkQ, *UK, *VR;
    double *Ss, *Sold;
    int *rks, *nodecnt, *rold, *err;   // err[0]: intermediate merges, err[1]: final merge
};

struct ScratchSizes {
    size_t Us, Vs, nodeR, nodeQ, chunkQ, UK, VR, Ss, Sold, rks, nodecnt, rold, err;
};

constexpr ScratchSizes scratch_sizes(int rows, int cols) {
    const size_t nch = (size_t)((cols + merge_ch(kCW) - 1) / merge_ch(kCW));
    ScratchSizes z{};
    z.Us = (size_t)rows * kCapInt;
    z.Vs = (size_t)cols * kCapInt;
    z.nodeR = (size_t)tree_nodes((int)nch) * kCW * kCW;
    z.nodeQ = (size_t)tree_nodes((int)nch) * node_q(kCW);
    z.chunkQ = nch * chunk_q(kCW);
    z.UK = z.VR = (size_t)kCW * kCW;
    z.Ss = kCapInt;
    z.Sold = kCW;
    z.rks = 1;
    z.nodecnt = (size_t)tree_nodes((int)nch);
    z.rold = 1;
    z.err = 2;
    return z;
}

int check_args(const void* A, int rows, int cols, int lda, double tol, int max_rank, const void* U,
               const double* S, const void* V, const int* rank_out) {
    if (!A || !U || !S || !V || !rank_out) return set_error(HNESSI_E_ARG, "NULL argument");
    if (rows < 1 || cols < 1 || lda < cols) return set_error(HNESSI_E_ARG, "bad matrix shape");
    if (!(tol > 0.0)) return set_error(HNESSI_E_ARG, "tol must be > 0");
    if (max_rank < 1 || max_rank > kCapInt)
        return set_error(HNESSI_E_ARG, "max_rank must be in 1.." + std::to_string(kCapInt));
    return HNESSI_OK;
}

// Enqueue the factorization on st; the scratch must be in place until st reaches its end.
int compress_run(const void* A, int rows, int cols, int lda, double tol, int max_rank, void* U, double* S,
                 void* V, int* rank_out, hipStream_t st, const CompressScratch& s) {
    const int nmerge = (rows + kCP - 1) / kCP;
    const int nch = (cols + merge_ch(kCW) - 1) / merge_ch(kCW);
    const double tol_int = tol * (kDropBudget / nmerge);
    hipError_t e = launch_fill_int(s.rks, 1, 0, st);
    if (e == hipSuccess) e = launch_fill_int(s.nodecnt, tree_nodes(nch), 0, st);
    if (e == hipSuccess) e = launch_fill_int(s.err, 2, 0, st);
    if (e == hipSuccess) e = launch_fill_int(rank_out, 1, 0, st);
    for (int i = 0; i < nmerge && e == hipSuccess; ++i) {
        const int p0 = i * kCP;
        const bool last = (i == nmerge - 1);
        MergeArgs a{};
        a.W = kCW;
        a.pp = rows - p0 < kCP ? rows - p0 : kCP;
        a.npair = 1;
        a.RCr = kCapInt;
        a.Ur = s.Us;
        a.Vr = s.Vs;
        a.Sr = s.Ss;
        a.rankr = s.rks;
        if (last) {   // the final merge truncates at eps into the caller's factors
            a.RC = max_rank;
            a.tol = tol;
            a.U = static_cast<cd*>(U);
            a.V = static_cast<cd*>(V);
            a.S = S;
            a.rank = rank_out;
            a.err = s.err + 1;
        } else {
            a.RC = kCapInt;
            a.tol = tol_int;
            a.U = s.Us;
            a.V = s.Vs;
            a.S = s.Ss;
            a.rank = s.rks;
            a.err = s.err;
        }
        a.src = static_cast<const cd*>(A) + (size_t)p0 * lda;
        a.src_row = lda;
        a.src_pair = 0;
        a.src_first = 0;
        a.src_ring = 1 << 30;   // rows of A in place: no wrap
        a.nodeR = s.nodeR;
        a.nodeQ = s.nodeQ;
        a.chunkQ = s.chunkQ;
        a.nodecnt = s.nodecnt;
        a.UK = s.UK;
        a.VR = s.VR;
        a.Sold = s.Sold;
        a.rold = s.rold;
        a.flip = 0;
        MergeBlk& B = a.blk[0];
        B.b = 0;
        B.c0 = 0;
        B.ncols = cols;
        B.ldU = rows;
        B.kb = p0;
        B.nchunks = nch;
        B.task_off = 0;
        B.utask_off = 0;
        B.nutask = (p0 + a.pp + 255) / 256;
        B.nnodes = tree_nodes(nch);
        B.node_base = 0;
        B.chunk_base = 0;
        B.Uoff = 0;
        B.Voff = 0;
        B.rd = 0;
        a.nblk = 1;
        a.ntask_v = nch;
        a.ntask_u = B.nutask;
        e = launch_merge(a, 1, st);
    }
    if (e == hipSuccess) {
        compress_finish<<<1, 64, 0, st>>>(s.err, rank_out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_error(HNESSI_E_DEVICE, std::string("compress_block: ") + hipGetErrorString(e));
    return HNESSI_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing: one file-scope device
// array, sized for blocks of at most kNoAllocRows x kNoAllocCols.  Host code
// never uses the array's name as an address: the device address of each GPU's
// copy comes from hipGetSymbolAddress on the first call with that device
// current and is kept per device.
constexpr int kNoAllocRows = 4096;
constexpr int kNoAllocCols = 4096;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t scratch_bytes(const ScratchSizes& z) {
    return align256(z.Us * sizeof(cd)) + align256(z.Vs * sizeof(cd)) + align256(z.nodeR * sizeof(cd)) +
           align256(z.nodeQ * sizeof(cd)) + align256(z.chunkQ * sizeof(cd)) + align256(z.UK * sizeof(cd)) +
           align256(z.VR * sizeof(cd)) + align256(z.Ss * sizeof(double)) + align256(z.Sold * sizeof(double)) +
           align256(z.rks * sizeof(int)) + align256(z.nodecnt * sizeof(int)) + align256(z.rold * sizeof(int)) +
           align256(z.err * sizeof(int));
}
constexpr size_t kNoAllocBytes = scratch_bytes(scratch_sizes(kNoAllocRows, kNoAllocCols));

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// carve the scratch of a rows x cols factorization out of base (256-byte aligned parts)
CompressScratch carve(unsigned char* base, int rows, int cols) {
    const ScratchSizes z = scratch_sizes(rows, cols);
    CompressScratch s{};
    size_t off = 0;
    auto take = [&](auto*& p, size_t count) {
        using T = std::remove_reference_t<decltype(*p)>;
        p = reinterpret_cast<T*>(base + off);
        off += align256(count * sizeof(T));
    };
    take(s.Us, z.Us);
    take(s.Vs, z.Vs);
    take(s.nodeR, z.nodeR);
    take(s.nodeQ, z.nodeQ);
    take(s.chunkQ, z.chunkQ);
    take(s.UK, z.UK);
    take(s.VR, z.VR);
    take(s.Ss, z.Ss);
    take(s.Sold, z.Sold);
    take(s.rks, z.rks);
    take(s.nodecnt, z.nodecnt);
    take(s.rold, z.rold);
    take(s.err, z.err);
    return s;
}

}  // namespace

}  // namespace hn

static __device__ __align__(256) unsigned char scratch[hn::kNoAllocBytes];

namespace hn {
namespace {

// device address of the current device's copy of `scratch`, looked up once per device
int scratch_address(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(HNESSI_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(HNESSI_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(HNESSI_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_dev[dev];
    return HNESSI_OK;
}

}  // namespace
}  // namespace hn

using namespace hn;

extern "C" {

int hnessi_compress_block(const void* A, int rows, int cols, int lda, double tol, int max_rank, void* U,
                          double* S, void* V, int* rank_out, void* stream) {
    int rc = check_args(A, rows, cols, lda, tol, max_rank, U, S, V, rank_out);
    if (rc != HNESSI_OK) return rc;
    rc = lib_init();
    if (rc != HNESSI_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const ScratchSizes z = scratch_sizes(rows, cols);
    DevAlloc al = DevAlloc::current(st);
    CompressScratch s{};
    if (dev_alloc(al, s.Us, z.Us, false) != HNESSI_OK || dev_alloc(al, s.Vs, z.Vs, false) != HNESSI_OK ||
        dev_alloc(al, s.nodeR, z.nodeR, false) != HNESSI_OK || dev_alloc(al, s.nodeQ, z.nodeQ, false) != HNESSI_OK ||
        dev_alloc(al, s.chunkQ, z.chunkQ, false) != HNESSI_OK || dev_alloc(al, s.UK, z.UK, false) != HNESSI_OK ||
        dev_alloc(al, s.VR, z.VR, false) != HNESSI_OK || dev_alloc(al, s.Ss, z.Ss, false) != HNESSI_OK ||
        dev_alloc(al, s.Sold, z.Sold, false) != HNESSI_OK || dev_alloc(al, s.rks, z.rks, false) != HNESSI_OK ||
        dev_alloc(al, s.nodecnt, z.nodecnt, false) != HNESSI_OK || dev_alloc(al, s.rold, z.rold, false) != HNESSI_OK ||
        dev_alloc(al, s.err, z.err, false) != HNESSI_OK) {
        al.release(true);
        return set_error(HNESSI_E_NOMEM, "compress_block: scratch allocation failed");
    }
    rc = compress_run(A, rows, cols, lda, tol, max_rank, U, S, V, rank_out, st, s);
    // stream-ordered release: the memory returns to the hook after st reaches this point
    al.release(true);
    return rc;
}

int hnessi_compress_block_noalloc(const void* A, int rows, int cols, int lda, double tol, int max_rank, void* U,
                                  double* S, void* V, int* rank_out, void* stream) {
    int rc = check_args(A, rows, cols, lda, tol, max_rank, U, S, V, rank_out);
    if (rc != HNESSI_OK) return rc;
    if (rows > kNoAllocRows || cols > kNoAllocCols)
        return set_error(HNESSI_E_ARG, "compress_block_noalloc: the block exceeds the static scratch (rows and "
                                       "cols must be at most " + std::to_string(kNoAllocRows) + ")");
    rc = lib_init();
    if (rc != HNESSI_OK) return rc;
    unsigned char* base = nullptr;
    rc = scratch_address(&base);
    if (rc != HNESSI_OK) return rc;
    return compress_run(A, rows, cols, lda, tol, max_rank, U, S, V, rank_out, (hipStream_t)stream,
                        carve(base, rows, cols));
}

}  // extern "C"
