// C ABI of the compressed history-integral library (see include/hnessi.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hnessi.h"
#include "alloc.h"
#include "born.h"
#include "common.h"
#include "dense.h"
#include "history.h"
#include "march.h"
#include "merge.h"
#include "step.h"
#include "store.h"

using namespace hn;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(HNESSI_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool g_init = false;

// the process-wide allocator hook (default: stream-ordered hipMallocAsync / hipFreeAsync)
void* default_alloc(size_t bytes, void* stream, void*) {
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, (hipStream_t)stream) != hipSuccess) return nullptr;
    return p;
}
void default_free(void* p, void* stream, void*) { (void)hipFreeAsync(p, (hipStream_t)stream); }
hnessi_alloc_fn g_alloc = default_alloc;
hnessi_free_fn g_free = default_free;
void* g_alloc_ctx = nullptr;
// projection chunk rows of handles created from now on, by norb (0: the built-in default)
std::mutex g_tile_mu;
int g_proj_rows[17] = {};

#define ALLOC(al, p, n, z)                                                                     \
    do {                                                                                       \
        if (dev_alloc((al), (p), (n), (z)) != HNESSI_OK)                                       \
            return fail(HNESSI_E_NOMEM, "device allocation of " + std::to_string((size_t)(n)) + \
                                            " elements failed");                              \
    } while (0)

int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

// HIP-event timing of kernel launches on the launch stream
struct Prof {
    int stride = 0;  // 0: off; otherwise time the launches of steps n % stride == 0
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int kind, n;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    hipEvent_t ev() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    bool capturing = false;   // a graph capture is open: no timing events
    bool want(int n) const { return !capturing && stride > 0 && n % stride == 0; }
    void clear() {
        recs.clear();
        used = 0;
    }
    void release() {
        for (hipEvent_t e : pool) hipEventDestroy(e);
        pool.clear();
        clear();
    }
    int read(int kind, int* steps, double* ms, int cap) {
        int cnt = 0;
        for (const Rec& r : recs) {
            if (r.kind != kind) continue;
            if (cnt < cap) {
                float t = 0.f;
                if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
                    return fail(HNESSI_E_DEVICE, "event timing failed");
                if (steps) steps[cnt] = r.n;
                if (ms) ms[cnt] = t;
            }
            ++cnt;
        }
        return cnt;
    }
};

}  // namespace

namespace hn {

int set_error(int code, const std::string& msg) { return fail(code, msg); }

int lib_init() {
    if (g_init) return HNESSI_OK;
    HIP_TRY(merge_init());
    HIP_TRY(history_init());
    HIP_TRY(dense_init());
    g_init = true;
    return HNESSI_OK;
}

DevAlloc DevAlloc::current(hipStream_t st) {
    DevAlloc a;
    a.fa = g_alloc;
    a.ff = g_free;
    a.ctx = g_alloc_ctx;
    a.st = st;
    return a;
}

void* DevAlloc::raw(size_t nbytes, bool zero) {
    void* q = fa(nbytes, (void*)st, ctx);
    if (!q) return nullptr;
    ptrs.push_back(q);
    bytes += nbytes;
    if (zero) {
        // zero fill by a kernel on the allocating stream
        if (launch_fill_int(static_cast<int*>(q), (long long)((nbytes + 3) / 4), 0, st) != hipSuccess) return nullptr;
    }
    return q;
}

void DevAlloc::release(bool on_stream) {
    for (void* q : ptrs) ff(q, on_stream ? (void*)st : nullptr, ctx);
    ptrs.clear();
    bytes = 0;
}

}  // namespace hn

struct hnessi_hodlr_s {
    int nt = 0, nlvl = 0, norb = 0, npair = 0, k = 0, P = 0, RC = 0, flags = 0;
    int nk = 1;  // objects of a batch (same geometry, independent data)
    // per-object element counts of the batched arrays (the stride between objects)
    long long oU = 0, oV = 0, oS = 0, oRank = 0, oLeaf = 0, oTail = 0, oBand = 0, oProj = 0, oPart = 0,
              oLeafOut = 0, oLeafOutLL = 0, oTailcol = 0, oTailpart = 0, oTailrow = 0, oNodeR = 0, oNodeQ = 0, oNodeCnt = 0, oProbW2 = 0,
              oProbW = 0, oProb = 0, oChunkQ = 0;
    double tol = 0.0;
    Weights W{};
    StepWeights SW{};   // weights of the retarded time step
    cd* step_scr = nullptr;    // the step's scratch ((k+1) npair entries per object), allocated by the first step
    cd* lstep_scr = nullptr;   // the lesser step's scratch, allocated by its first call
    cd* march_scr = nullptr;   // row march: projections of the rows of a launch and M_m^{-1}, allocated by its first call
    hipStream_t sstream = nullptr;   // the step's near-diagonal solves, beside the history kernels
    hipEvent_t ev_sfork = nullptr, ev_sjoin = nullptr;
    Geometry g;
    int MW = 0;           // merge width (kWSmall or kWLarge)
    DevAlloc al;
    hipEvent_t ev_last = nullptr;   // recorded after the work of every call on that call's stream
    // geometry on the device
    int* d_blk = nullptr;
    int* d_leaf = nullptr;
    int* d_cover = nullptr;
    int* d_rowleaf = nullptr;   // leaf index of each row
    long long* d_Uoff = nullptr;
    long long* d_Voff = nullptr;
    long long* d_Loff = nullptr;
    std::vector<long long> Uoff, Voff, Loff;
    // per component
    bool f32 = false;    // complex-float mirrors of the factors feed the history kernels
    bool mfproj = false; // norb 16, complex-float factors, rank capacity <= 16: projections
                         // on the matrix cores (task per block, factor, chunk, orbital beta)
    bool mfcomb = false; // and leaves starting at multiples of 16: matrix-core expansions
    int kch = 0;         // factor rows per projection chunk
    cd* U[2] = {};       // FP64 factors (merges, reconstruction)
    cd* V[2] = {};
    cf* U32[2] = {};     // mirrors, or nullptr
    cf* V32[2] = {};
    double* S[2] = {};
    int* rank[2] = {};
    cd* leaf[2] = {};
    cd* tail[2] = {};
    cd* band = nullptr;
    int last[2] = {-1, -1};
    int n0[2] = {0, 0};        // first row not in the current factor buffers
    int fstart[2] = {0, 0};    // first row of the panel being formed
    // Panel merges run on their own stream one panel behind: while panel [p0, p1) is
    // merged into the blocks' other factor buffer, the history kernels keep reading
    // the current buffer and treat the panel's rows as dense tail rows.
    long long bU = 0, bV = 0, bS = 0, bRank = 0;   // buffer 1 offset (elements)
    std::vector<int> cur[2];                        // per block: current buffer
    int* d_cur[2] = {};
    hipStream_t mstream[2] = {};   // per component: the two components' merges run concurrently
    hipEvent_t ev_app[2] = {}, ev_merge[2] = {};
    struct Pending {
        bool on = false;
        int p0 = 0, p1 = 0;
        std::vector<int> blocks;
    } pend[2];
    // projection tasks, sorted by activation row
    FactTask* d_ft[2] = {};
    std::vector<int> ft_act[2];
    long long* d_partoff = nullptr;
    // history scratch
    cd* part = nullptr;
    cd* proj = nullptr;
    cd* leafR = nullptr;
    cd* leafLR = nullptr;
    cd* leafLL = nullptr;
    cd* tailcol[2] = {};
    cd* tailpart[2] = {};
    cd* tailrow[2] = {};
    cd* sigRT = nullptr;   // norb 16: Sigma^R row with swapped orbital indices (per step)
    long long oSigRT = 0;
    // gradient of a loss with respect to the retarded factors (allocated on first use):
    // dU, dV laid out like one buffer of U, V; dS like one buffer of S
    cd* dU = nullptr;
    cd* dV = nullptr;
    double* dS = nullptr;
    // sweeps as graphs (HNESSI_FLAG_GRAPHS): launches between two panel ends are captured
    // from the launch stream (the merges fork to and join from their streams inside the
    // window) and replayed through one executable graph, updated window by window
    struct Graph {
        bool on = false;       // a sweep in graph mode is running (a capture is open)
        hipGraphExec_t exec = nullptr;
        long long windows = 0, instantiations = 0;
    } graph;
    int ntailchunk_max = 0;
    // merge scratch
    std::vector<long long> lvl_node_base;  // per level: first node of pair 0
    std::vector<int> lvl_nodes;            // per level: nodes per pair
    std::vector<long long> lvl_chunk_base; // per level: first chunk slot of pair 0
    // per component (the two components' merges run concurrently)
    cd* nodeR[2] = {};
    cd* nodeQ[2] = {};
    cd* chunkQ[2] = {};
    int* nodecnt[2] = {};
    cd* UK[2] = {};
    cd* VR[2] = {};
    double* Sold[2] = {};
    int* rold[2] = {};
    int* err = nullptr;
    Prof prof;
};

struct hnessi_dense_s {
    int nt = 0, norb = 0, npair = 0, k = 0;
    Weights W{};
    DevAlloc al;
    hipEvent_t ev_last = nullptr;
    long long trin = 0;
    cd* L[2] = {};
    cd* colR = nullptr;
    cd* colL = nullptr;
    cd* rowL = nullptr;
    int last[2] = {-1, -1};
    Prof prof;
};

extern "C" {

const char* hnessi_last_error(void) { return g_err.c_str(); }

int hnessi_set_tile_shape(int norb, int proj_rows) {
    if (!(norb == 1 || norb == 2 || norb == 4 || norb == 8 || norb == 16))
        return fail(HNESSI_E_ARG, "norb must be 1, 2, 4, 8 or 16");
    if (!kch_allowed(norb, proj_rows))
        return fail(HNESSI_E_ARG, "projection chunk rows: 0, 256, 512 or 1024 for norb <= 4; 0, 128 or 256 above");
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_proj_rows[norb] = proj_rows;
    return HNESSI_OK;
}

int hnessi_get_tile_shape(hnessi_hodlr_t H) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    return H->kch;
}

int hnessi_set_allocator(hnessi_alloc_fn alloc, hnessi_free_fn free_fn, void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(HNESSI_E_ARG, "allocator and free function must both be given or both be NULL");
    if (alloc) {
        g_alloc = alloc;
        g_free = free_fn;
        g_alloc_ctx = ctx;
    } else {
        g_alloc = default_alloc;
        g_free = default_free;
        g_alloc_ctx = nullptr;
    }
    return HNESSI_OK;
}

int hnessi_weights(int k, int L, double* w_host) {
    if (!w_host) return fail(HNESSI_E_ARG, "w_host is NULL");
    std::vector<double> w;
    std::string err;
    if (!interval_weights_exact(k, L, w, err)) return fail(HNESSI_E_ARG, err);
    std::memcpy(w_host, w.data(), w.size() * sizeof(double));
    return HNESSI_OK;
}

int hnessi_born_lattice(int L, int n, double U, const void* GR_rows, const void* GL_slices, long long in_stride,
                        void* SR_rows, void* SL_slices, long long out_stride, void* stream) {
    if (!(L == 2 || L == 4 || L == 8 || L == 16 || L == 32)) return fail(HNESSI_E_ARG, "L must be 2, 4, 8, 16 or 32");
    if (n < 0) return fail(HNESSI_E_RANGE, "n must be >= 0");
    if (!GR_rows || !GL_slices || !SR_rows || !SL_slices) return fail(HNESSI_E_ARG, "a pointer is NULL");
    if (in_stride < n + 1 || out_stride < n + 1) return fail(HNESSI_E_ARG, "object stride shorter than a row");
    if (!std::isfinite(U)) return fail(HNESSI_E_ARG, "U must be finite");
    int rc = lib_init();
    if (rc != HNESSI_OK) return rc;
    BornArgs a{};
    a.L = L;
    a.n = n;
    a.u2 = U * U;
    a.GR = static_cast<const cd*>(GR_rows);
    a.GL = static_cast<const cd*>(GL_slices);
    a.inStride = in_stride;
    a.SR = static_cast<cd*>(SR_rows);
    a.SL = static_cast<cd*>(SL_slices);
    a.outStride = out_stride;
    HIP_TRY(launch_born(a, (hipStream_t)stream));
    return HNESSI_OK;
}

int hnessi_step_weights(int k, double* a_host, double* D_host) {
    if (!a_host || !D_host) return fail(HNESSI_E_ARG, "an output is NULL");
    StepWeights S;
    std::string err;
    if (!make_step_weights(k, S, err)) return fail(HNESSI_E_ARG, err);
    for (int i = 0; i <= k; ++i) {
        a_host[i] = S.a[i];
        for (int p = 0; p <= k; ++p) D_host[i * (k + 1) + p] = S.D[i][p];
    }
    return HNESSI_OK;
}

}  // extern "C"

namespace {

// ev_last marks the end of the work a call enqueued on its stream
int mark(hnessi_hodlr_t H, hipStream_t st) {
    HIP_TRY(hipEventRecord(H->ev_last, st));
    return HNESSI_OK;
}

// wait for the work of the handle: its last call's stream and its merge stream
int wait_handle(hnessi_hodlr_t H) {
    if (H->ev_last) HIP_TRY(hipEventSynchronize(H->ev_last));
    for (int c = 0; c < 2; ++c)
        if (H->mstream[c]) HIP_TRY(hipStreamSynchronize(H->mstream[c]));
    if (H->sstream) HIP_TRY(hipStreamSynchronize(H->sstream));
    return HNESSI_OK;
}

void release_streams(hnessi_hodlr_t H) {
    for (int c = 0; c < 2; ++c)
        if (H->mstream[c]) hipStreamSynchronize(H->mstream[c]);
    for (int c = 0; c < 2; ++c) {
        if (H->ev_app[c]) hipEventDestroy(H->ev_app[c]);
        if (H->ev_merge[c]) hipEventDestroy(H->ev_merge[c]);
        H->ev_app[c] = H->ev_merge[c] = nullptr;
    }
    for (int c = 0; c < 2; ++c) {
        if (H->mstream[c]) hipStreamDestroy(H->mstream[c]);
        H->mstream[c] = nullptr;
    }
    if (H->sstream) {
        hipStreamSynchronize(H->sstream);
        hipStreamDestroy(H->sstream);
        H->sstream = nullptr;
    }
    if (H->ev_sfork) hipEventDestroy(H->ev_sfork);
    if (H->ev_sjoin) hipEventDestroy(H->ev_sjoin);
    H->ev_sfork = H->ev_sjoin = nullptr;
}

int create_impl(hnessi_hodlr_t* out, int nk, int nt, int nlvl, int norb, int k, double svd_tol, int panel,
                int max_rank, int flags, hipStream_t st) {
    if (!out) return fail(HNESSI_E_ARG, "out is NULL");
    *out = nullptr;
    if (nk < 1 || nk > 65535) return fail(HNESSI_E_ARG, "nk must be in 1..65535");
    if (flags & ~(HNESSI_FLAG_FP32_FACTORS | HNESSI_FLAG_GRAPHS)) return fail(HNESSI_E_ARG, "unknown flags");
    if (!(norb == 1 || norb == 2 || norb == 4 || norb == 8 || norb == 16))
        return fail(HNESSI_E_ARG, "norb must be 1, 2, 4, 8 or 16");
    if (!(svd_tol > 0.0)) return fail(HNESSI_E_ARG, "svd_tol must be > 0");
    if (panel < 1 || panel > 16) return fail(HNESSI_E_ARG, "panel must be in 1..16");
    if (max_rank < 1 || max_rank + panel > kWLarge)
        return fail(HNESSI_E_ARG, "need 1 <= max_rank and max_rank + panel <= " + std::to_string(kWLarge));
    int rc = lib_init();
    if (rc != HNESSI_OK) return rc;
    auto* H = new hnessi_hodlr_s();
    std::string err;
    if (!make_weights(k, H->W, err) || !make_step_weights(k, H->SW, err) || !build_geometry(nt, nlvl, H->g, err)) {
        delete H;
        return fail(HNESSI_E_ARG, err);
    }
    const Geometry& g = H->g;
    if (g.max_leaf > 64) {
        delete H;
        return fail(HNESSI_E_ARG, "leaves must hold at most 64 rows (increase nlvl)");
    }
    if (g.min_leaf < k + 1 || g.min_leaf < panel) {
        delete H;
        return fail(HNESSI_E_ARG, "leaves must hold at least k+1 rows and the panel");
    }
    H->nk = nk;
    H->nt = nt;
    H->nlvl = nlvl;
    H->norb = norb;
    H->npair = norb * norb;
    H->k = k;
    H->P = panel;
    H->RC = max_rank;
    H->flags = flags;
    H->f32 = (flags & HNESSI_FLAG_FP32_FACTORS) != 0;
    H->mfproj = H->f32 && norb == 16 && max_rank <= 16;
    {
        std::lock_guard<std::mutex> lk(g_tile_mu);
        H->kch = g_proj_rows[norb] ? g_proj_rows[norb] : kch(norb);
    }
    H->mfcomb = H->mfproj;
    for (int i = 0; i < H->g.nleaf; ++i) H->mfcomb = H->mfcomb && H->g.s0[i] % 16 == 0;
    H->tol = svd_tol;
    H->MW = merge_width(max_rank, panel);
    const int npair = H->npair, RC = H->RC, nb = g.nb, MW = H->MW;
    H->al = DevAlloc::current(st);
    DevAlloc& al = H->al;
    auto bail = [&](int code) {
        (void)hipStreamSynchronize(st);
        al.release(true);
        if (H->ev_last) hipEventDestroy(H->ev_last);
        delete H;
        return code;
    };
#define HALLOC(p, n, z)                                                                           \
    do {                                                                                          \
        if (dev_alloc(al, (p), (n), (z)) != HNESSI_OK)                                            \
            return bail(fail(HNESSI_E_NOMEM, "device allocation of " + std::to_string((size_t)(n)) + \
                                                 " elements failed"));                           \
    } while (0)
    // one allocation holding nk objects; o receives the per-object count
#define HALLOC_K(p, n, z, o)                             \
    do {                                                 \
        (o) = (long long)(n);                            \
        HALLOC(p, (size_t)(o) * nk, z);                  \
    } while (0)
    // geometry
    std::vector<int> blk(5 * std::max(nb, 1)), lf(2 * g.nleaf);
    H->Uoff.assign(nb, 0);
    H->Voff.assign(nb, 0);
    long long uo = 0, vo = 0;
    for (int b = 0; b < nb; ++b) {
        blk[5 * b] = g.level[b];
        blk[5 * b + 1] = g.r0[b];
        blk[5 * b + 2] = g.r1[b];
        blk[5 * b + 3] = g.c0[b];
        blk[5 * b + 4] = g.c1[b];
        H->Uoff[b] = uo;
        H->Voff[b] = vo;
        uo += (long long)npair * RC * (g.r1[b] - g.r0[b]);
        vo += (long long)npair * RC * (g.c1[b] - g.c0[b]);
    }
    H->Loff.assign(g.nleaf, 0);
    long long lo = 0;
    for (int i = 0; i < g.nleaf; ++i) {
        lf[2 * i] = g.s0[i];
        lf[2 * i + 1] = g.s1[i];
        H->Loff[i] = lo;
        lo += (long long)npair * tri(g.s1[i] - g.s0[i]);
    }
    HALLOC(H->d_blk, blk.size(), false);
    HALLOC(H->d_leaf, lf.size(), false);
    HALLOC(H->d_cover, g.cover.size(), false);
    HALLOC(H->d_rowleaf, g.row_leaf.size(), false);
    HALLOC(H->d_Uoff, std::max(nb, 1), false);
    HALLOC(H->d_Voff, std::max(nb, 1), false);
    HALLOC(H->d_Loff, g.nleaf, false);
    // factor and dense storage
    for (int c = 0; c < 2; ++c) {
        // two buffers per object: [object][buffer][...]
        H->bU = uo;
        H->bV = vo;
        H->bS = (long long)std::max(nb, 1) * npair * RC;
        H->bRank = (long long)std::max(nb, 1) * npair;
        HALLOC_K(H->U[c], 2 * uo, true, H->oU);
        HALLOC_K(H->V[c], 2 * vo, true, H->oV);
        if (H->f32) {
            HALLOC(H->U32[c], (size_t)2 * uo * nk, true);
            HALLOC(H->V32[c], (size_t)2 * vo * nk, true);
        }
        HALLOC_K(H->S[c], 2 * H->bS, true, H->oS);
        HALLOC_K(H->rank[c], 2 * H->bRank, true, H->oRank);
        HALLOC(H->d_cur[c], (size_t)std::max(nb, 1), true);
        H->cur[c].assign(std::max(nb, 1), 0);
        HALLOC_K(H->leaf[c], lo, true, H->oLeaf);
        HALLOC_K(H->tail[c], (size_t)kTailRows * npair * nt, true, H->oTail);
    }
    HALLOC_K(H->band, (size_t)nt * (k + 1) * npair, true, H->oBand);
    if (norb == 16) HALLOC_K(H->sigRT, (size_t)nt * npair, false, H->oSigRT);
    HALLOC_K(H->proj, (size_t)2 * std::max(nb, 1) * npair * 2 * norb * RC, true, H->oProj);
    // chunk partials of the projections: one slot per kch(norb) factor rows
    std::vector<long long> partoff((size_t)2 * std::max(nb, 1) * npair * 2, 0);
    long long ps = 0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < npair; ++q)
                for (int w = 0; w < 2; ++w) {
                    partoff[(((size_t)c * nb + b) * npair + q) * 2 + w] = ps;
                    ps += div_up(w == 0 ? g.r1[b] - g.r0[b] : g.c1[b] - g.c0[b], H->kch);
                }
    HALLOC(H->d_partoff, partoff.size(), false);
    HALLOC_K(H->part, (size_t)std::max(ps, 1LL) * norb * RC, true, H->oPart);
    const int leaf_slots = leaf_groups(norb);   // orbital-pair groups of the leaf tasks
    HALLOC_K(H->leafR, (size_t)leaf_slots * nt * npair, true, H->oLeafOut);
    HALLOC_K(H->leafLR, (size_t)leaf_slots * nt * npair, true, H->oLeafOut);
    HALLOC_K(H->leafLL, (size_t)leaf_ll_slots(norb) * nt * npair, true, H->oLeafOutLL);
    H->ntailchunk_max = div_up(nt, kTailCH);
    for (int c = 0; c < 2; ++c) {
        HALLOC_K(H->tailcol[c], (size_t)tail_groups(norb) * nt * npair, true, H->oTailcol);
        HALLOC_K(H->tailpart[c], (size_t)H->ntailchunk_max * tail_groups(norb) * kTailRows * npair, true,
                 H->oTailpart);
        HALLOC_K(H->tailrow[c], (size_t)kTailRows * npair, true, H->oTailrow);
    }
    // merge scratch: one block per level per panel
    H->lvl_node_base.assign(nlvl + 1, 0);
    H->lvl_nodes.assign(nlvl + 1, 0);
    H->lvl_chunk_base.assign(nlvl + 1, 0);
    long long nodes = 0, chunks = 0;
    for (int l = 1; l <= nlvl; ++l) {
        int maxc = 0;
        for (int b = 0; b < nb; ++b)
            if (g.level[b] == l) maxc = std::max(maxc, g.c1[b] - g.c0[b]);
        H->lvl_nodes[l] = tree_nodes(div_up(maxc, merge_ch(MW)));
        H->lvl_node_base[l] = nodes;
        nodes += (long long)npair * H->lvl_nodes[l];
        H->lvl_chunk_base[l] = chunks;
        chunks += (long long)npair * div_up(maxc, merge_ch(MW));
    }
    const long long nprob = (long long)std::max(nlvl, 1) * npair;
    for (int c = 0; c < 2; ++c) {
        HALLOC_K(H->nodeR[c], (size_t)std::max(nodes, 1LL) * MW * MW, false, H->oNodeR);
        HALLOC_K(H->nodeQ[c], (size_t)std::max(nodes, 1LL) * node_q(MW), false, H->oNodeQ);
        HALLOC_K(H->chunkQ[c], (size_t)std::max(chunks, 1LL) * chunk_q(MW), false, H->oChunkQ);
        HALLOC_K(H->nodecnt[c], (size_t)std::max(nodes, 1LL), true, H->oNodeCnt);
        HALLOC_K(H->UK[c], (size_t)nprob * MW * MW, false, H->oProbW2);
        HALLOC_K(H->VR[c], (size_t)nprob * MW * MW, false, H->oProbW2);
        HALLOC_K(H->Sold[c], (size_t)nprob * MW, false, H->oProbW);
        HALLOC_K(H->rold[c], (size_t)nprob, false, H->oProb);
    }
    HALLOC(H->err, 1, true);
    // projection task lists (sorted by the row that activates them)
    for (int c = 0; c < 2; ++c) {
        std::vector<FactTask> ts;
        // one task per shared orbital index instead of per pair: the matrix-core
        // projections of norb 16 and the wave-per-pair projections of norb 4
        const int ntq = (H->mfproj || norb == 4) ? norb : npair;
        if (norb == 4 && !H->mfproj) {
            // the four tasks of a chunk (one per shared index) next to each other: the
            // kernel places each such group on one XCD, whose L2 then fetches the
            // chunk's Sigma rows once
            for (int b = 0; b < nb; ++b) {
                for (int ch = 0; ch < div_up(g.r1[b] - g.r0[b], H->kch); ++ch)
                    for (int q = 0; q < ntq; ++q) ts.push_back(FactTask{c, b, q, 0, ch, g.r0[b] + ch * H->kch});
                for (int ch = 0; ch < div_up(g.c1[b] - g.c0[b], H->kch); ++ch)
                    for (int q = 0; q < ntq; ++q) ts.push_back(FactTask{c, b, q, 1, ch, g.r0[b]});
            }
        } else {
            for (int b = 0; b < nb; ++b)
                for (int q = 0; q < ntq; ++q) {
                    for (int ch = 0; ch < div_up(g.r1[b] - g.r0[b], H->kch); ++ch)
                        ts.push_back(FactTask{c, b, q, 0, ch, g.r0[b] + ch * H->kch});
                    for (int ch = 0; ch < div_up(g.c1[b] - g.c0[b], H->kch); ++ch)
                        ts.push_back(FactTask{c, b, q, 1, ch, g.r0[b]});
                }
        }
        std::stable_sort(ts.begin(), ts.end(),
                         [](const FactTask& x, const FactTask& y) { return x.act < y.act; });
        H->ft_act[c].resize(ts.size());
        for (size_t i = 0; i < ts.size(); ++i) H->ft_act[c][i] = ts[i].act;
        HALLOC(H->d_ft[c], ts.size(), false);
        if (!ts.empty() && hipMemcpyAsync(H->d_ft[c], ts.data(), ts.size() * sizeof(FactTask),
                                          hipMemcpyHostToDevice, st) != hipSuccess)
            return bail(fail(HNESSI_E_DEVICE, "copy of task table failed"));
        // the host tables are local: the copies complete before they go out of scope
        if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(HNESSI_E_DEVICE, "stream synchronization failed"));
    }
    auto h2d = [&](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
    };
    if (!h2d(H->d_blk, blk.data(), blk.size() * sizeof(int)) || !h2d(H->d_leaf, lf.data(), lf.size() * sizeof(int)) ||
        !h2d(H->d_cover, g.cover.data(), g.cover.size() * sizeof(int)) ||
        !h2d(H->d_rowleaf, g.row_leaf.data(), g.row_leaf.size() * sizeof(int)) ||
        !h2d(H->d_Uoff, H->Uoff.data(), nb * sizeof(long long)) ||
        !h2d(H->d_Voff, H->Voff.data(), nb * sizeof(long long)) ||
        !h2d(H->d_Loff, H->Loff.data(), g.nleaf * sizeof(long long)) ||
        !h2d(H->d_partoff, partoff.data(), partoff.size() * sizeof(long long)))
        return bail(fail(HNESSI_E_DEVICE, "copy of geometry failed"));
    // every allocation, fill and copy of this handle is ordered on st; the host tables
    // above are local, so the copies complete before create returns
    if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(HNESSI_E_DEVICE, "stream synchronization failed"));
    // the merge stream (default priority) and its events
    if (hipStreamCreateWithFlags(&H->mstream[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&H->mstream[1], hipStreamNonBlocking) != hipSuccess) {
        release_streams(H);
        return bail(fail(HNESSI_E_DEVICE, "stream creation failed"));
    }
    for (int c = 0; c < 2; ++c)
        if (hipEventCreateWithFlags(&H->ev_app[c], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&H->ev_merge[c], hipEventDisableTiming) != hipSuccess) {
            release_streams(H);
            return bail(fail(HNESSI_E_DEVICE, "event creation failed"));
        }
    if (hipEventCreateWithFlags(&H->ev_last, hipEventDisableTiming) != hipSuccess) {
        H->ev_last = nullptr;
        release_streams(H);
        return bail(fail(HNESSI_E_DEVICE, "event creation failed"));
    }
#undef HALLOC_K
#undef HALLOC
    *out = H;
    return HNESSI_OK;
}

}  // namespace

extern "C" {

int hnessi_hodlr_create(hnessi_hodlr_t* out, int nt, int nlvl, int norb, int k, double svd_tol,
                        int panel, int max_rank, int flags, void* stream) {
    return create_impl(out, 1, nt, nlvl, norb, k, svd_tol, panel, max_rank, flags, (hipStream_t)stream);
}

int hnessi_hodlr_create_batched(hnessi_hodlr_t* out, int nk, int nt, int nlvl, int norb, int k,
                                double svd_tol, int panel, int max_rank, int flags, void* stream) {
    return create_impl(out, nk, nt, nlvl, norb, k, svd_tol, panel, max_rank, flags, (hipStream_t)stream);
}

int hnessi_hodlr_nk(hnessi_hodlr_t H) { return H ? H->nk : fail(HNESSI_E_ARG, "handle is NULL"); }

int hnessi_hodlr_destroy(hnessi_hodlr_t H) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    const int rc = wait_handle(H);
    release_streams(H);
    H->prof.release();
    if (H->graph.exec) (void)hipGraphExecDestroy(H->graph.exec);
    H->al.release(false);
    if (H->ev_last) hipEventDestroy(H->ev_last);
    delete H;
    return rc;
}

int hnessi_hodlr_graph_stats(hnessi_hodlr_t H, long long* windows, long long* instantiations) {
    if (!H || !windows || !instantiations) return fail(HNESSI_E_ARG, "NULL argument");
    *windows = H->graph.windows;
    *instantiations = H->graph.instantiations;
    return HNESSI_OK;
}

int hnessi_hodlr_reset(hnessi_hodlr_t H, void* stream) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    hipStream_t st = (hipStream_t)stream;
    for (int c = 0; c < 2; ++c) {
        if (H->pend[c].on) HIP_TRY(hipStreamWaitEvent(st, H->ev_merge[c], 0));   // merge done first
        H->pend[c].on = false;
        HIP_TRY(launch_fill_int(H->rank[c], H->oRank * H->nk, 0, st));
        HIP_TRY(launch_fill_int(H->d_cur[c], (long long)H->cur[c].size(), 0, st));
        std::fill(H->cur[c].begin(), H->cur[c].end(), 0);
        H->last[c] = -1;
        H->n0[c] = 0;
        H->fstart[c] = 0;
    }
    HIP_TRY(launch_fill_int(H->err, 1, 0, st));
    return mark(H, st);
}

}  // extern "C"

namespace {

int merge_panel(hnessi_hodlr_t H, int c, int p0, int p1, hipStream_t st, std::vector<int>& blocks) {
    const Geometry& g = H->g;
    blocks.clear();
    MergeArgs a{};
    a.flip = 1;
    a.bU = H->bU;
    a.bV = H->bV;
    a.bS = H->bS;
    a.bRank = H->bRank;
    a.src_first = p0 % kTailRows;
    a.src_ring = kTailRows;
    a.pp = p1 - p0;
    a.npair = H->npair;
    a.W = H->MW;
    a.RC = H->RC;
    a.RCr = H->RC;
    a.tol = H->tol;
    a.Ur = H->U[c];
    a.Vr = H->V[c];
    a.Sr = H->S[c];
    a.rankr = H->rank[c];
    a.U = H->U[c];
    a.V = H->V[c];
    a.U32 = H->U32[c];
    a.V32 = H->V32[c];
    a.S = H->S[c];
    a.rank = H->rank[c];
    a.src = H->tail[c];
    a.src_row = (long long)H->npair * H->nt;
    a.src_pair = H->nt;
    a.nodeR = H->nodeR[c];
    a.nodeQ = H->nodeQ[c];
    a.chunkQ = H->chunkQ[c];
    a.kChunkQ = H->oChunkQ;
    a.nodecnt = H->nodecnt[c];
    a.UK = H->UK[c];
    a.VR = H->VR[c];
    a.Sold = H->Sold[c];
    a.rold = H->rold[c];
    a.err = H->err;
    a.kU = H->oU;
    a.kV = H->oV;
    a.kS = H->oS;
    a.kRank = H->oRank;
    a.kSrc = H->oTail;
    a.kNodeR = H->oNodeR;
    a.kNodeQ = H->oNodeQ;
    a.kNodeCnt = H->oNodeCnt;
    a.kProbW2 = H->oProbW2;
    a.kProbW = H->oProbW;
    a.kProb = H->oProb;
    int nv = 0, nu = 0, nblk = 0;
    for (int l = 0; l < H->nlvl; ++l) {
        int cv = g.cover[(size_t)l * H->nt + p0];
        if (cv >= 0) continue;
        int b = ~cv;
        if (nblk >= kMaxMergeBlk) return fail(HNESSI_E_ARG, "too many levels for one merge");
        MergeBlk& B = a.blk[nblk];
        B.b = b;
        B.c0 = g.c0[b];
        B.ncols = g.c1[b] - g.c0[b];
        B.ldU = g.r1[b] - g.r0[b];
        B.kb = p0 - g.r0[b];
        B.nchunks = div_up(B.ncols, merge_ch(H->MW));
        B.task_off = nv;
        B.utask_off = nu;
        B.nutask = div_up(B.kb + a.pp, 256);
        B.nnodes = H->lvl_nodes[g.level[b]];
        B.node_base = H->lvl_node_base[g.level[b]];
        B.chunk_base = H->lvl_chunk_base[g.level[b]];
        B.Uoff = H->Uoff[b];
        B.Voff = H->Voff[b];
        B.rd = H->cur[c][b];
        blocks.push_back(b);
        nv += H->npair * B.nchunks;
        nu += H->npair * B.nutask;
        ++nblk;
    }
    if (nblk == 0) return HNESSI_OK;
    a.nblk = nblk;
    a.ntask_v = nv;
    a.ntask_u = nu;
    const bool timed = H->prof.stride > 0 && !H->prof.capturing;
    hipEvent_t e0 = timed ? H->prof.ev() : nullptr, e1 = timed ? H->prof.ev() : nullptr;
    if (e0) hipEventRecord(e0, st);
    HIP_TRY(launch_merge(a, H->nk, st));
    if (e1) {
        hipEventRecord(e1, st);
        H->prof.recs.push_back({2, p1 - 1, e0, e1});
    }
    return HNESSI_OK;
}

bool panel_ends(hnessi_hodlr_t H, int c, int n) {
    if (n + 1 >= H->nt) return true;
    if (n + 1 - H->fstart[c] >= H->P) return true;
    return H->g.row_leaf[n + 1] != H->g.row_leaf[n];
}

// Make the in-flight merge of component c current for the work queued on st
// after this call: st waits for the merge, the merged blocks switch buffers and
// the panel's rows leave the dense tail.
int finish_pending(hnessi_hodlr_t H, int c, hipStream_t st) {
    auto& pd = H->pend[c];
    if (!pd.on) return HNESSI_OK;
    HIP_TRY(hipStreamWaitEvent(st, H->ev_merge[c], 0));
    HIP_TRY(launch_flip(H->d_cur[c], pd.blocks.data(), (int)pd.blocks.size(), st));
    for (int b : pd.blocks) H->cur[c][b] ^= 1;
    H->n0[c] = pd.p1;
    pd.on = false;
    return HNESSI_OK;
}

// Finish every in-flight merge (queries of the stored state): each component's
// pending flip is enqueued on its own merge stream, which the caller then waits for.
int drain(hnessi_hodlr_t H) {
    for (int c = 0; c < 2; ++c) {
        int rc = finish_pending(H, c, H->mstream[c]);
        if (rc != HNESSI_OK) return rc;
    }
    return HNESSI_OK;
}

// Retarded-only calls (history_R, its adjoint, the factor gradient) also accept a
// step n below the last appended row: they then evaluate step n over the stored
// (frozen) state, which holds the compressed G^R of every row so far: the merged
// rows at or below n through the factors, rows n0..n from the tail, no row above n.
// implicit (retarded history only): step n = last appended row + 1, whose row is not
// stored, so the sum runs over j = m..n-1 (the history term of a step solve).
int do_history(hnessi_hodlr_t H, int n, const void* sigR, const void* sigL, double h, void* outR,
               void* outL, bool wantR, bool wantL, hipStream_t st, long long in_stride = 0,
               long long out_stride = 0, bool adj = false, bool fgrad = false, bool implicit = false) {
    if (n < 0 || n >= H->nt) return fail(HNESSI_E_RANGE, "n outside the grid");
    if (!sigR && (!adj || fgrad)) return fail(HNESSI_E_ARG, "sigR_row is NULL");
    if (wantR && !outR && !fgrad) return fail(HNESSI_E_ARG, "output is NULL");
    if (wantL && (!sigL || (!outL && !fgrad))) return fail(HNESSI_E_ARG, "input or output is NULL");
    const bool ronly = !wantL || adj;
    if (implicit) {
        // retarded: rows 0..n-1 stored; lesser: lesser rows 0..n-1 and retarded rows to n-1 or n
        const bool okR = wantR && !wantL && n == H->last[0] + 1;
        const bool okL = wantL && !wantR && n == H->last[1] + 1 && H->last[0] >= n - 1 && H->last[0] <= n;
        if (adj || fgrad || !(okR || okL))
            return fail(HNESSI_E_ORDER, "the step solve needs rows 0..n-1 appended and row n not");
    } else if (n > H->last[0] || (n < H->last[0] && !ronly)) {
        return fail(HNESSI_E_ORDER, "retarded row n has not been appended (or later rows have)");
    }
    if (wantL && !adj && !implicit && H->last[1] != n)
        return fail(HNESSI_E_ORDER, "lesser row n has not been appended (or later rows have)");
    const bool frozen = n < H->last[0];
    if (frozen) {
        // the in-flight merge of the retarded component becomes current first
        int rc = finish_pending(H, 0, st);
        if (rc != HNESSI_OK) return rc;
    }
    const Geometry& g = H->g;
    HistArgs A{};
    A.n = n;
    for (int c = 0; c < 2; ++c) {
        A.n0[c] = H->n0[c];
        A.last[c] = H->last[c];
        if (frozen && c == 0) {
            A.n0[0] = std::min(H->n0[0], n + 1);
            A.last[0] = n;
        }
        A.ls[c] = 0;
        A.ntailchunk[c] = 0;
        A.nf[c] = 0;
        bool use = (c == 0) || (wantL && !adj);
        if (!use) continue;
        A.nf[c] = (int)(std::lower_bound(H->ft_act[c].begin(), H->ft_act[c].end(), A.n0[c]) -
                        H->ft_act[c].begin());
        // tail rows n0..last: those of the panel still being merged (before nsplit) hold
        // columns [0, lslo), the later ones [0, ls)
        A.nsplit[c] = H->pend[c].on ? H->pend[c].p1 : A.n0[c];
        if (A.last[c] >= A.n0[c]) {
            A.lslo[c] = g.s0[g.row_leaf[A.n0[c]]];
            A.ls[c] = A.nsplit[c] <= A.last[c] ? g.s0[g.row_leaf[A.nsplit[c]]] : A.lslo[c];
            A.ntailchunk[c] = div_up(A.ls[c], kTailCH);
        }
    }
    A.nt = H->nt;
    A.norb = H->norb;
    A.npair = H->npair;
    A.RC = H->RC;
    A.nlvl = H->nlvl;
    A.nb = g.nb;
    A.P = H->P;
    A.wantR = wantR;
    A.wantL = wantL;
    A.adj = adj;
    A.h = h;
    A.W = H->W;
    A.sigR = static_cast<const cd*>(sigR);
    A.sigL = static_cast<const cd*>(sigL);
    for (int c = 0; c < 2; ++c) {
        A.U[c] = H->f32 ? (const void*)H->U32[c] : (const void*)H->U[c];
        A.V[c] = H->f32 ? (const void*)H->V32[c] : (const void*)H->V[c];
        A.S[c] = H->S[c];
        A.rank[c] = H->rank[c];
        A.leaf[c] = H->leaf[c];
        A.tail[c] = H->tail[c];
        A.ft[c] = H->d_ft[c];
        A.tailcol[c] = H->tailcol[c];
        A.tailpart[c] = H->tailpart[c];
        A.tailrow[c] = H->tailrow[c];
    }
    A.band = H->band;
    A.blk = H->d_blk;
    A.leafs = H->d_leaf;
    A.cover = H->d_cover;
    A.Uoff = H->d_Uoff;
    A.Voff = H->d_Voff;
    A.Loff = H->d_Loff;
    A.partoff = H->d_partoff;
    // norb 4: groups of four projection tasks share an XCD (blocks of 32 workgroups)
    A.nfpad = H->norb == 4 ? div_up(A.nf[0] + A.nf[1], 32) * 32 : div_up(A.nf[0] + A.nf[1], 8) * 8;
    A.nleaf = g.row_leaf[n] + 1;
    const int ngroups = H->norb <= 4 ? 1 : H->norb / 4;   // left-orbital groups of 4 waves
    // dense-piece tasks per leaf and per tail chunk: one per orbital pair for norb <= 4,
    // left-orbital groups x pair groups for norb 8, one per output orbital for norb 16
    const int per_piece = H->norb <= 4 ? H->npair : ngroups * 4;
    A.nleaftask = div_up(2 * A.nleaf, 8) * 8 * per_piece;
    A.ntailtask = div_up(A.ntailchunk[0] + A.ntailchunk[1], 8) * 8 * per_piece;
    if (fgrad) {   // the projections only
        A.nleaftask = 0;
        A.ntailtask = 0;
        A.fgrad = 1;
        A.Ud = H->U[0];
        A.Vd = H->V[0];
        A.dU = H->dU;
        A.dV = H->dV;
        A.dS = H->dS;
    }
    A.part = H->part;
    A.proj = H->proj;
    A.leafR = H->leafR;
    A.leafLR = H->leafLR;
    A.leafLL = H->leafLL;
    A.outR = static_cast<cd*>(outR);
    A.outL = static_cast<cd*>(outL);
    A.nk = H->nk;
    A.f32 = H->f32;
    A.kch = H->kch;
    A.mfproj = H->mfproj;
    A.mfcomb = H->mfcomb;
    A.ring = kTailRows;
    A.bU = H->bU;
    A.bV = H->bV;
    A.bS = H->bS;
    A.bRank = H->bRank;
    A.cur[0] = H->d_cur[0];
    A.cur[1] = H->d_cur[1];
    A.kIn = in_stride;
    A.kOut = out_stride;
    A.kU = H->oU;
    A.kV = H->oV;
    A.kS = H->oS;
    A.kRank = H->oRank;
    A.kLeaf = H->oLeaf;
    A.kTail = H->oTail;
    A.kBand = H->oBand;
    A.sigRT = H->sigRT;
    A.kInT = H->oSigRT;
    A.kProj = H->oProj;
    A.kPart = H->oPart;
    A.kLeafOut = H->oLeafOut;
    A.kLeafOutLL = H->oLeafOutLL;
    A.kTailcol = H->oTailcol;
    A.kTailpart = H->oTailpart;
    A.kTailrow = H->oTailrow;
    if (H->prof.want(n)) {
        hipEvent_t ev[4] = {H->prof.ev(), H->prof.ev(), H->prof.ev(), H->prof.ev()};
        HIP_TRY(launch_history(A, st, ev));
        H->prof.recs.push_back({0, n, ev[0], ev[1]});
        H->prof.recs.push_back({3, n, ev[1], ev[2]});
        H->prof.recs.push_back({1, n, ev[2], ev[3]});
    } else {
        HIP_TRY(launch_history(A, st));
    }
    return HNESSI_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// the append arguments of row n of component c
AppendArgs append_args(hnessi_hodlr_t H, int c, int n, const void* row, long long k_stride) {
    const Geometry& g = H->g;
    const int leaf = g.row_leaf[n];
    AppendArgs a{};
    a.row = static_cast<const cd*>(row);
    a.n = n;
    a.npair = H->npair;
    a.nt = H->nt;
    a.k = H->k;
    a.ls = g.s0[leaf];
    a.lw = g.s1[leaf] - g.s0[leaf];
    a.slot = n % kTailRows;
    a.leaf = H->leaf[c] + H->Loff[leaf];
    a.tail = H->tail[c];
    a.band = c == HNESSI_RET ? H->band : nullptr;
    a.kRow = k_stride;
    a.kLeaf = H->oLeaf;
    a.kTail = H->oTail;
    a.kBand = H->oBand;
    return a;
}

int check_append(hnessi_hodlr_t H, int c, int n, const void* row) {
    if (c != HNESSI_RET && c != HNESSI_LES) return fail(HNESSI_E_ARG, "component must be RET or LES");
    if (!row) return fail(HNESSI_E_ARG, "row is NULL");
    if (n < 0 || n >= H->nt) return fail(HNESSI_E_RANGE, "n outside the grid");
    if (n != H->last[c] + 1) return fail(HNESSI_E_ORDER, "rows must be appended in order");
    return HNESSI_OK;
}

// this panel's merge (rows fstart..n of component c) is launched on the merge stream
int launch_panel(hnessi_hodlr_t H, int c, int n, hipStream_t st) {
    const int p0 = H->fstart[c], p1 = n + 1;
    int rc = HNESSI_OK;
    // this panel's merge runs on the merge stream after the work queued so far on st
    // and writes the blocks' other buffers; until the next panel ends, the history
    // kernels read the panel's rows from the dense tail
    HIP_TRY(hipEventRecord(H->ev_app[c], st));
    HIP_TRY(hipStreamWaitEvent(H->mstream[c], H->ev_app[c], 0));
    auto& pd = H->pend[c];
    rc = merge_panel(H, c, p0, p1, H->mstream[c], pd.blocks);
    if (rc != HNESSI_OK) return rc;
    HIP_TRY(hipEventRecord(H->ev_merge[c], H->mstream[c]));
    pd.on = true;
    pd.p0 = p0;
    pd.p1 = p1;
    H->fstart[c] = p1;
    return HNESSI_OK;
}

// after row n of component c is appended: when it completes a panel, the previous
// panel's merge becomes current and this panel's merge is launched
int after_append(hnessi_hodlr_t H, int c, int n, hipStream_t st) {
    H->last[c] = n;
    if (!panel_ends(H, c, n)) return HNESSI_OK;
    // the previous panel's merge becomes current for everything queued from here on
    int rc = finish_pending(H, c, st);
    return rc != HNESSI_OK ? rc : launch_panel(H, c, n, st);
}

// Close the open capture on st, run it through the handle's executable graph (updated
// in place when the window has the same shape as the last one, instantiated anew
// otherwise) and, with reopen, open the next window.
int graph_window(hnessi_hodlr_t H, hipStream_t st, bool reopen = true) {
    hipGraph_t g = nullptr;
    H->graph.on = false;
    HIP_TRY(hipStreamEndCapture(st, &g));
    bool ok = false;
    if (H->graph.exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res;
        ok = hipGraphExecUpdate(H->graph.exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!ok) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(H->graph.exec);
            H->graph.exec = nullptr;
        }
    }
    if (!ok) {
        if (hipGraphInstantiate(&H->graph.exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            H->graph.exec = nullptr;
            return fail(HNESSI_E_DEVICE, "graph instantiation failed");
        }
        ++H->graph.instantiations;
    }
    (void)hipGraphDestroy(g);
    HIP_TRY(hipGraphLaunch(H->graph.exec, st));
    ++H->graph.windows;
    if (reopen) {
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        H->graph.on = true;
    }
    return HNESSI_OK;
}

int append_impl(hnessi_hodlr_t H, int c, int n, const void* row, long long k_stride, hipStream_t st) {
    int rc = check_append(H, c, n, row);
    if (rc != HNESSI_OK) return rc;
    HIP_TRY(launch_append_hodlr(append_args(H, c, n, row, k_stride), H->nk, st));
    return after_append(H, c, n, st);
}

// rows n of both components in one launch
int append2_impl(hnessi_hodlr_t H, int n, const void* rowR, const void* rowL, long long k_stride, hipStream_t st) {
    int rc = check_append(H, HNESSI_RET, n, rowR);
    if (rc == HNESSI_OK) rc = check_append(H, HNESSI_LES, n, rowL);
    if (rc != HNESSI_OK) return rc;
    HIP_TRY(launch_append_hodlr2(append_args(H, HNESSI_RET, n, rowR, k_stride),
                                 append_args(H, HNESSI_LES, n, rowL, k_stride), H->nk, st));
    if (!H->graph.on) {
        rc = after_append(H, HNESSI_RET, n, st);
        if (rc != HNESSI_OK) return rc;
        return after_append(H, HNESSI_LES, n, st);
    }
    // graph windows: both components' panels end at the same rows; the previous merges
    // are joined, the window's graph is launched, and the next window opens with the
    // new merges
    H->last[0] = H->last[1] = n;
    if (!panel_ends(H, HNESSI_RET, n)) return HNESSI_OK;
    for (int c = 0; c < 2; ++c) {
        rc = finish_pending(H, c, st);
        if (rc != HNESSI_OK) return rc;
    }
    rc = graph_window(H, st);
    if (rc != HNESSI_OK) return rc;
    for (int c = 0; c < 2; ++c) {
        rc = launch_panel(H, c, n, st);
        if (rc != HNESSI_OK) return rc;
    }
    return HNESSI_OK;
}

int single_only(hnessi_hodlr_t H) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    if (H->nk != 1) return fail(HNESSI_E_ARG, "batched handle: use the _batched calls");
    return HNESSI_OK;
}

int batched_stride(hnessi_hodlr_t H, long long stride, long long need) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    if (H->nk > 1 && stride < need) return fail(HNESSI_E_ARG, "object stride smaller than one object's data");
    return HNESSI_OK;
}

}  // namespace

extern "C" {

int hnessi_hodlr_append_row(hnessi_hodlr_t H, int c, int n, const void* row, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = append_impl(H, c, n, row, 0, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_hodlr_append_row_batched(hnessi_hodlr_t H, int c, int n, const void* rows, long long k_stride,
                                    void* stream) {
    int rc = batched_stride(H, k_stride, (long long)(n + 1) * (H ? H->npair : 0));
    if (rc != HNESSI_OK) return rc;
    rc = append_impl(H, c, n, rows, k_stride, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_history_R(hnessi_hodlr_t H, int n, const void* sigR_row, double h, void* out, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = do_history(H, n, sigR_row, nullptr, h, out, nullptr, true, false, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// one step of every object: strides in complex entries from one object's array to the next
int step_impl(hnessi_hodlr_t H, int n, const void* eps, long long eps_stride, const void* sigR_rows,
              long long in_stride, const void* sig_near, long long near_stride, const void* const* prev_rows,
              long long prev_stride, double h, void* rows_out, long long out_stride, hipStream_t st) {
    const int k = H->k;
    const long long np = H->npair;
    if (n < 0 || n >= H->nt) return fail(HNESSI_E_RANGE, "n outside the grid");
    if (n < k) return fail(HNESSI_E_RANGE, "the step needs n >= k (the first k rows are a start-up)");
    if (!eps || !sigR_rows || !sig_near || !prev_rows || !rows_out) return fail(HNESSI_E_ARG, "a pointer is NULL");
    if (!(h > 0.0)) return fail(HNESSI_E_ARG, "h must be > 0");
    if (H->nk > 1 && (eps_stride < (k + 1) * np || in_stride < (n + 1) * np || near_stride < (long long)k * k * np ||
                      prev_stride < (n - k) * np || out_stride < (n + 1) * np))
        return fail(HNESSI_E_ARG, "object stride smaller than one object's data");
    StepArgs a{};
    for (int l = 0; l < k; ++l) {
        if (!prev_rows[l]) return fail(HNESSI_E_ARG, "a previous row is NULL");
        a.prev[l] = static_cast<const cd*>(prev_rows[l]);
    }
    if (!H->step_scr) {
        if (dev_alloc(H->al, H->step_scr, (size_t)((k + 1) * np * H->nk), false) != HNESSI_OK) {
            H->step_scr = nullptr;
            return fail(HNESSI_E_NOMEM, "device allocation of the step scratch failed");
        }
        HIP_TRY(hipStreamSynchronize(H->al.st));
    }
    if (!H->sstream) {   // default priority, like every stream of the library
        if (hipStreamCreateWithFlags(&H->sstream, hipStreamNonBlocking) != hipSuccess) {
            H->sstream = nullptr;
            return fail(HNESSI_E_DEVICE, "stream creation failed");
        }
        if (hipEventCreateWithFlags(&H->ev_sfork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&H->ev_sjoin, hipEventDisableTiming) != hipSuccess)
            return fail(HNESSI_E_DEVICE, "event creation failed");
    }
    // an order check before anything is enqueued (the history call repeats it)
    if (n != H->last[0] + 1) return fail(HNESSI_E_ORDER, "the step solve needs rows 0..n-1 appended and row n not");
    a.n = n;
    a.k = k;
    a.norb = H->norb;
    a.h = h;
    a.W = H->W;
    a.S = H->SW;
    a.eps = static_cast<const cd*>(eps);
    a.sigR = static_cast<const cd*>(sigR_rows);
    a.sigNear = static_cast<const cd*>(sig_near);
    a.row = static_cast<cd*>(rows_out);
    a.scr = H->step_scr;
    a.nk = H->nk;
    a.kEps = eps_stride;
    a.kSig = in_stride;
    a.kNear = near_stride;
    a.kPrev = prev_stride;
    a.kRow = out_stride;
    const bool timed = H->prof.want(n);
    // the near-diagonal solves on the side stream, after the work queued so far on st
    // (and after the previous step's bulk kernel, the scratch's last reader)
    HIP_TRY(hipEventRecord(H->ev_sfork, st));
    HIP_TRY(hipStreamWaitEvent(H->sstream, H->ev_sfork, 0));
    if (timed) {
        hipEvent_t ev[2] = {H->prof.ev(), H->prof.ev()};
        HIP_TRY(launch_step_near(a, H->sstream, ev));
        H->prof.recs.push_back({4, n, ev[0], ev[1]});
    } else {
        HIP_TRY(launch_step_near(a, H->sstream));
    }
    HIP_TRY(hipEventRecord(H->ev_sjoin, H->sstream));
    // the history sum over the stored rows, into the output rows (on st, beside them)
    int rc = do_history(H, n, sigR_rows, nullptr, h, rows_out, nullptr, true, false, st, in_stride, out_stride,
                        false, false, true);
    // joined also when the history call failed, so that no work of this call is left behind
    HIP_TRY(hipStreamWaitEvent(st, H->ev_sjoin, 0));
    if (rc != HNESSI_OK) return rc;
    if (timed) {
        hipEvent_t ev[2] = {H->prof.ev(), H->prof.ev()};
        HIP_TRY(launch_step_bulk(a, st, ev));
        H->prof.recs.push_back({5, n, ev[0], ev[1]});
    } else {
        HIP_TRY(launch_step_bulk(a, st));
    }
    return HNESSI_OK;
}

}  // namespace

extern "C" {

int hnessi_step_R(hnessi_hodlr_t H, int n, const void* eps, const void* sigR_row, const void* sig_near,
                  const void* const* prev_rows, double h, void* row_out, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = step_impl(H, n, eps, 0, sigR_row, 0, sig_near, 0, prev_rows, 0, h, row_out, 0, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_step_lesser(hnessi_hodlr_t H, int n, const void* eps, const void* const* sigR_rows,
                       const void* const* sigL_slices, const void* GR_row, const void* const* prev_slices, double h,
                       void* slice_out, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    const int k = H->k;
    const long long np = H->npair;
    hipStream_t st = (hipStream_t)stream;
    if (n < 0 || n >= H->nt) return fail(HNESSI_E_RANGE, "n outside the grid");
    if (n < k) return fail(HNESSI_E_RANGE, "the step needs n >= k (the first k rows are a start-up)");
    if (!eps || !sigR_rows || !sigL_slices || !GR_row || !prev_slices || !slice_out)
        return fail(HNESSI_E_ARG, "a pointer is NULL");
    if (!(h > 0.0)) return fail(HNESSI_E_ARG, "h must be > 0");
    LesserStepArgs a{};
    for (int l = 0; l < k; ++l) {
        if (!sigR_rows[l] || !sigL_slices[l] || !prev_slices[l]) return fail(HNESSI_E_ARG, "a row pointer is NULL");
        a.sigRn[l] = static_cast<const cd*>(sigR_rows[l]);
        a.sigLn[l] = static_cast<const cd*>(sigL_slices[l]);
        a.prev[l] = static_cast<const cd*>(prev_slices[l]);
    }
    if (n != H->last[1] + 1 || H->last[0] < n - 1 || H->last[0] > n)
        return fail(HNESSI_E_ORDER, "the lesser step needs lesser rows 0..n-1 appended (row n not) and retarded rows to n-1");
    const int nch_max = lesser_sum_chunks(H->nt - 1);
    if (!H->lstep_scr) {
        if (dev_alloc(H->al, H->lstep_scr, (size_t)((1 + k) * np + (long long)k * nch_max * np), false) != HNESSI_OK) {
            H->lstep_scr = nullptr;
            return fail(HNESSI_E_NOMEM, "device allocation of the lesser step scratch failed");
        }
        HIP_TRY(hipStreamSynchronize(H->al.st));
    }
    if (!H->sstream) {
        if (hipStreamCreateWithFlags(&H->sstream, hipStreamNonBlocking) != hipSuccess) {
            H->sstream = nullptr;
            return fail(HNESSI_E_DEVICE, "stream creation failed");
        }
        if (hipEventCreateWithFlags(&H->ev_sfork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&H->ev_sjoin, hipEventDisableTiming) != hipSuccess)
            return fail(HNESSI_E_DEVICE, "event creation failed");
    }
    a.n = n;
    a.k = k;
    a.norb = H->norb;
    a.h = h;
    a.W = H->W;
    a.S = H->SW;
    a.eps = static_cast<const cd*>(eps);
    a.GRn = static_cast<const cd*>(GR_row);
    a.slice = static_cast<cd*>(slice_out);
    a.scr = H->lstep_scr;
    a.part = H->lstep_scr + (1 + k) * np;
    a.nchunk = lesser_sum_chunks(n);
    // M_L^{-1} on the side stream, beside the history kernels
    HIP_TRY(hipEventRecord(H->ev_sfork, st));
    HIP_TRY(hipStreamWaitEvent(H->sstream, H->ev_sfork, 0));
    HIP_TRY(launch_lesser_prep(a, H->sstream));
    HIP_TRY(hipEventRecord(H->ev_sjoin, H->sstream));
    // I^<(n, m) over the stored rows (the first integral without its s = n term), into the output
    rc = do_history(H, n, sigR_rows[k - 1], sigL_slices[k - 1], h, nullptr, slice_out, false, true, st, 0, 0, false,
                    false, true);
    HIP_TRY(hipStreamWaitEvent(st, H->ev_sjoin, 0));
    if (rc != HNESSI_OK) return rc;
    if (H->prof.want(n)) {
        hipEvent_t ev[2] = {H->prof.ev(), H->prof.ev()};
        HIP_TRY(launch_lesser_rest(a, st, ev));
        H->prof.recs.push_back({6, n, ev[0], ev[1]});
    } else {
        HIP_TRY(launch_lesser_rest(a, st));
    }
    return mark(H, st);
}

int hnessi_row_march_R(hnessi_hodlr_t H, int n_lo, int n_hi, const void* eps, double h, void* rows_out,
                       long long row_stride, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    const int k = H->k;
    if (!(H->norb == 1 || H->norb == 2 || H->norb == 4)) return fail(HNESSI_E_ARG, "the row march takes norb 1, 2 or 4");
    if (H->RC > 32) return fail(HNESSI_E_ARG, "the row march takes a rank capacity of at most 32");
    if (n_lo < k || n_hi < n_lo || n_hi >= H->nt) return fail(HNESSI_E_RANGE, "rows must satisfy k <= n_lo <= n_hi < nt");
    if (n_hi > H->last[0]) return fail(HNESSI_E_ORDER, "Sigma^R rows up to n_hi must be appended");
    if (!eps || !rows_out) return fail(HNESSI_E_ARG, "a pointer is NULL");
    if (row_stride < (long long)(n_hi + 1) * H->npair) return fail(HNESSI_E_ARG, "row_stride shorter than row n_hi");
    if (!(h > 0.0)) return fail(HNESSI_E_ARG, "h must be > 0");
    // rows per launch: every row of the grid when the projection scratch stays within
    // 2 GiB, so that one launch holds all rows (longest first); the scratch also holds
    // M_m^{-1} of every column
    const long long per_row = (long long)H->nlvl * H->norb * H->npair * 32;
    const long long cap_rows = std::max(1024LL, (2LL << 30) / (per_row * (long long)sizeof(hn::cd)));
    const int march_rows = (int)std::min<long long>(cap_rows, (long long)H->nt - k);
    if (!H->march_scr) {
        const size_t cnt = (size_t)(per_row * march_rows) + (size_t)H->nt * H->npair;
        if (dev_alloc(H->al, H->march_scr, cnt, false) != HNESSI_OK) {
            H->march_scr = nullptr;
            return fail(HNESSI_E_NOMEM, "device allocation of the row-march scratch failed");
        }
        HIP_TRY(hipStreamSynchronize(H->al.st));
    }
    hipStream_t st = (hipStream_t)stream;
    // every merge finished: the stored state is frozen (tail rows n0..last hold columns [0, ls))
    rc = drain(H);
    if (rc != HNESSI_OK) return rc;
    for (int c = 0; c < 2; ++c) HIP_TRY(hipStreamSynchronize(H->mstream[c]));
    const Geometry& g = H->g;
    MarchArgs a{};
    a.nt = H->nt;
    a.norb = H->norb;
    a.npair = H->npair;
    a.RC = H->RC;
    a.k = k;
    a.nlvl = H->nlvl;
    a.ring = kTailRows;
    a.n0 = H->n0[0];
    a.ls = H->n0[0] <= H->last[0] ? g.s0[g.row_leaf[H->n0[0]]] : 0;
    a.h = h;
    a.W = H->W;
    a.S = H->SW;
    a.U = H->U[0];
    a.V = H->V[0];
    a.Sv = H->S[0];
    a.rank = H->rank[0];
    a.cur = H->d_cur[0];
    a.bU = H->bU;
    a.bV = H->bV;
    a.bS = H->bS;
    a.bRank = H->bRank;
    a.Uoff = H->d_Uoff;
    a.Voff = H->d_Voff;
    a.Loff = H->d_Loff;
    a.blk = H->d_blk;
    a.leafs = H->d_leaf;
    a.rowLeaf = H->d_rowleaf;
    a.cover = H->d_cover;
    a.leaf = H->leaf[0];
    a.tail = H->tail[0];
    a.band = H->band;
    a.eps = static_cast<const cd*>(eps);
    a.rowStride = row_stride;
    a.proj = H->march_scr;
    a.minv = H->march_scr + (size_t)(per_row * march_rows);
    HIP_TRY(launch_march_minv(a, n_hi - k, st));   // columns 0..n_hi-k-1
    for (int hi = n_hi; hi >= n_lo; hi -= march_rows) {   // the longest rows first
        a.nhi = hi;
        a.nlo = std::max(n_lo, hi - march_rows + 1);
        a.rows = static_cast<cd*>(rows_out) + (size_t)(a.nlo - n_lo) * row_stride;
        HIP_TRY(launch_row_march(a, st));
    }
    return mark(H, st);
}

int hnessi_step_R_batched(hnessi_hodlr_t H, int n, const void* eps, long long eps_stride, const void* sigR_rows,
                          long long in_stride, const void* sig_near, long long near_stride,
                          const void* const* prev_rows, long long prev_stride, double h, void* rows_out,
                          long long out_stride, void* stream) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    int rc = step_impl(H, n, eps, eps_stride, sigR_rows, in_stride, sig_near, near_stride, prev_rows, prev_stride, h,
                       rows_out, out_stride, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_history_lesser(hnessi_hodlr_t H, int n, const void* sigR_row, const void* sigL_slice,
                          double h, void* out, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = do_history(H, n, sigR_row, sigL_slice, h, nullptr, out, false, true, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_history_step(hnessi_hodlr_t H, int n, const void* sigR_row, const void* sigL_slice,
                        double h, void* outR, void* outL, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = do_history(H, n, sigR_row, sigL_slice, h, outR, outL, true, true, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_history_R_adjoint(hnessi_hodlr_t H, int n, const void* ibar_row, double h, void* out, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = do_history(H, n, nullptr, ibar_row, h, nullptr, out, false, true, (hipStream_t)stream, 0, 0, true);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_factor_grad_reset(hnessi_hodlr_t H, void* stream);

int hnessi_history_R_factor_grad(hnessi_hodlr_t H, int n, const void* sigR_row, const void* ibar_row, double h,
                                 void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!H->dU) {
        // allocated on the handle's stream (ordered there), then cleared on st
        DevAlloc& al = H->al;
        if (dev_alloc(al, H->dU, (size_t)H->bU, false) != HNESSI_OK ||
            dev_alloc(al, H->dV, (size_t)H->bV, false) != HNESSI_OK ||
            dev_alloc(al, H->dS, (size_t)H->bS, false) != HNESSI_OK) {
            H->dU = nullptr;
            return fail(HNESSI_E_NOMEM, "device allocation of the factor gradients failed");
        }
        HIP_TRY(hipStreamSynchronize(al.st));
        rc = hnessi_factor_grad_reset(H, stream);
        if (rc != HNESSI_OK) return rc;
    }
    rc = do_history(H, n, sigR_row, ibar_row, h, nullptr, nullptr, true, true, st, 0, 0, true, true);
    return rc != HNESSI_OK ? rc : mark(H, st);
}

int hnessi_factor_grad_reset(hnessi_hodlr_t H, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    if (!H->dU) return HNESSI_OK;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_fill_int(reinterpret_cast<int*>(H->dU), 4 * H->bU, 0, st));
    HIP_TRY(launch_fill_int(reinterpret_cast<int*>(H->dV), 4 * H->bV, 0, st));
    HIP_TRY(launch_fill_int(reinterpret_cast<int*>(H->dS), 2 * H->bS, 0, st));
    return mark(H, st);
}

int hnessi_history_step_batched(hnessi_hodlr_t H, int n, const void* sigR_rows, const void* sigL_slices,
                                long long in_stride, double h, void* outR, void* outL, long long out_stride,
                                void* stream) {
    const long long need = (long long)(n + 1) * (H ? H->npair : 0);
    int rc = batched_stride(H, in_stride, need);
    if (rc == HNESSI_OK) rc = batched_stride(H, out_stride, need);
    if (rc != HNESSI_OK) return rc;
    rc = do_history(H, n, sigR_rows, sigL_slices, h, outR, outL, true, true, (hipStream_t)stream, in_stride,
                    out_stride);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

}  // extern "C"

namespace {

int sweep_steps(hnessi_hodlr_t H, int n_begin, int n_end, const void* GR, const void* GL, const void* SR,
                const void* SL, long long k_stride, double h, void* IR, void* IL, hipStream_t st) {
    const size_t np = H->npair;
    for (int n = n_begin; n < n_end; ++n) {
        const size_t off = (size_t)tri(n) * np;
        int rc = append2_impl(H, n, static_cast<const cd*>(GR) + off, static_cast<const cd*>(GL) + off, k_stride, st);
        if (rc != HNESSI_OK) return rc;
        rc = do_history(H, n, static_cast<const cd*>(SR) + off, static_cast<const cd*>(SL) + off, h,
                        static_cast<cd*>(IR) + off, static_cast<cd*>(IL) + off, true, true, st, k_stride, k_stride);
        if (rc != HNESSI_OK) return rc;
    }
    return HNESSI_OK;
}

int sweep_impl(hnessi_hodlr_t H, int n_begin, int n_end, const void* GR, const void* GL, const void* SR,
               const void* SL, long long k_stride, double h, void* IR, void* IL, hipStream_t st) {
    if (!GR || !GL || !SR || !SL || !IR || !IL) return fail(HNESSI_E_ARG, "NULL array");
    if (n_begin < 0 || n_end > H->nt || n_begin > n_end) return fail(HNESSI_E_RANGE, "bad sweep range");
    if (!(H->flags & HNESSI_FLAG_GRAPHS) || n_begin == n_end)
        return sweep_steps(H, n_begin, n_end, GR, GL, SR, SL, k_stride, h, IR, IL, st);
    if (!st) return fail(HNESSI_E_ARG, "graph sweeps need a stream other than the NULL stream");
    // merges launched before the sweep are joined outside the capture
    for (int c = 0; c < 2; ++c) {
        int rc = finish_pending(H, c, st);
        if (rc != HNESSI_OK) return rc;
    }
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    H->graph.on = true;
    H->prof.capturing = true;
    int rc = sweep_steps(H, n_begin, n_end, GR, GL, SR, SL, k_stride, h, IR, IL, st);
    // the last window joins its merges before the capture closes
    for (int c = 0; c < 2 && rc == HNESSI_OK; ++c) rc = finish_pending(H, c, st);
    if (rc == HNESSI_OK) rc = graph_window(H, st, false);
    if (H->graph.on) {   // an error left the capture open: discard it
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
    }
    H->graph.on = false;
    H->prof.capturing = false;
    return rc;
}

}  // namespace

extern "C" {

int hnessi_sweep(hnessi_hodlr_t H, int n_begin, int n_end, const void* GR, const void* GL,
                 const void* SR, const void* SL, double h, void* IR, void* IL, void* stream) {
    int rc = single_only(H);
    if (rc != HNESSI_OK) return rc;
    rc = sweep_impl(H, n_begin, n_end, GR, GL, SR, SL, 0, h, IR, IL, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_sweep_batched(hnessi_hodlr_t H, int n_begin, int n_end, const void* GR, const void* GL,
                         const void* SR, const void* SL, long long k_stride, double h, void* IR, void* IL,
                         void* stream) {
    int rc = batched_stride(H, k_stride, tri(H ? H->nt : 0) * (H ? H->npair : 0));
    if (rc != HNESSI_OK) return rc;
    rc = sweep_impl(H, n_begin, n_end, GR, GL, SR, SL, k_stride, h, IR, IL, (hipStream_t)stream);
    return rc != HNESSI_OK ? rc : mark(H, (hipStream_t)stream);
}

int hnessi_hodlr_status(hnessi_hodlr_t H, void* stream) {
    if (!H) return fail(HNESSI_E_ARG, "handle is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int rc = drain(H);
    if (rc == HNESSI_OK) rc = wait_handle(H);
    if (rc != HNESSI_OK) return rc;
    int e = 0;
    HIP_TRY(hipMemcpy(&e, H->err, sizeof(int), hipMemcpyDeviceToHost));
    if (e & 2) return fail(HNESSI_E_VALUE, "a truncation met non-finite data (NaN or Inf in the rows)");
    if (e & 1) return fail(HNESSI_E_RANK, "a truncation needed more than max_rank singular values");
    return HNESSI_OK;
}

int hnessi_hodlr_get(hnessi_hodlr_t H, int c, int t1, int t2, void* out_host) {
    if (!H || !out_host) return fail(HNESSI_E_ARG, "NULL argument");
    if (H->nk != 1) return fail(HNESSI_E_ARG, "batched handle: reconstruction is for single objects");
    if (c != HNESSI_RET && c != HNESSI_LES) return fail(HNESSI_E_ARG, "component must be RET or LES");
    if (t2 < 0 || t2 > t1 || t1 > H->last[c]) return fail(HNESSI_E_RANGE, "(t1, t2) outside the stored region");
    int rc = wait_handle(H);
    if (rc != HNESSI_OK) return rc;
    const Geometry& g = H->g;
    const int npair = H->npair;
    std::vector<cd> out(npair);
    const int leaf = g.row_leaf[t1];
    const int ls = g.s0[leaf];
    if (t2 >= ls) {
        const int lw = g.s1[leaf] - ls;
        for (int q = 0; q < npair; ++q)
            HIP_TRY(hipMemcpy(&out[q], H->leaf[c] + H->Loff[leaf] + (size_t)q * tri(lw) + tri(t1 - ls) + (t2 - ls),
                              sizeof(cd), hipMemcpyDeviceToHost));
    } else if (t1 >= H->n0[c]) {
        const int slot = t1 % kTailRows;
        for (int q = 0; q < npair; ++q)
            HIP_TRY(hipMemcpy(&out[q], H->tail[c] + ((size_t)slot * npair + q) * H->nt + t2, sizeof(cd),
                              hipMemcpyDeviceToHost));
    } else {
        int b = -1;
        for (int l = 0; l < H->nlvl; ++l) {
            int c1 = g.cover[(size_t)l * H->nt + t1], c2 = g.cover[(size_t)l * H->nt + t2];
            if (c1 < 0 && c2 == ~c1) { b = c2; break; }
        }
        if (b < 0) return fail(HNESSI_E_RANGE, "no block holds (t1, t2)");
        const int RC = H->RC;
        const int ldU = g.r1[b] - g.r0[b], ldV = g.c1[b] - g.c0[b];
        const int bf = H->cur[c][b];   // the block's current buffer
        std::vector<int> rk(npair);
        HIP_TRY(hipMemcpy(rk.data(), H->rank[c] + bf * H->bRank + (size_t)b * npair, npair * sizeof(int),
                          hipMemcpyDeviceToHost));
        std::vector<double> S(RC);
        for (int q = 0; q < npair; ++q) {
            cd acc = mk(0.0, 0.0);
            HIP_TRY(hipMemcpy(S.data(), H->S[c] + bf * H->bS + ((size_t)b * npair + q) * RC, RC * sizeof(double),
                              hipMemcpyDeviceToHost));
            for (int r = 0; r < rk[q]; ++r) {
                cd u, v;
                HIP_TRY(hipMemcpy(&u, H->U[c] + bf * H->bU + H->Uoff[b] + ((size_t)q * RC + r) * ldU + (t1 - g.r0[b]),
                                  sizeof(cd), hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(&v, H->V[c] + bf * H->bV + H->Voff[b] + ((size_t)q * RC + r) * ldV + (t2 - g.c0[b]),
                                  sizeof(cd), hipMemcpyDeviceToHost));
                acc = acc + S[r] * (u * conj(v));
            }
            out[q] = acc;
        }
    }
    std::memcpy(out_host, out.data(), npair * sizeof(cd));
    return HNESSI_OK;
}

// block b, pair q of component c (or, with grad, the factor gradients of the
// retarded component) to the host; returns the rank
static int factors_to_host(hnessi_hodlr_t H, int c, int b, int q, void* U_host, double* S_host, void* V_host,
                           bool grad) {
    if (!H || !U_host || !S_host || !V_host) return fail(HNESSI_E_ARG, "NULL argument");
    if (H->nk != 1) return fail(HNESSI_E_ARG, "batched handle: factors are read for single objects");
    if (c != HNESSI_RET && c != HNESSI_LES) return fail(HNESSI_E_ARG, "component must be RET or LES");
    const Geometry& g = H->g;
    if (b < 0 || b >= g.nb || q < 0 || q >= H->npair) return fail(HNESSI_E_RANGE, "block or pair out of range");
    if (grad && !H->dU) return fail(HNESSI_E_ORDER, "no factor gradient has been accumulated");
    int rc = drain(H);
    if (rc == HNESSI_OK) rc = wait_handle(H);
    if (rc != HNESSI_OK) return rc;
    const int RC = H->RC, npair = H->npair;
    const int ldU = g.r1[b] - g.r0[b], ldV = g.c1[b] - g.c0[b];
    const long long bf = H->cur[c][b];
    int rk = 0;
    HIP_TRY(hipMemcpy(&rk, H->rank[c] + bf * H->bRank + (size_t)b * npair + q, sizeof(int), hipMemcpyDeviceToHost));
    rk = std::max(0, std::min(rk, RC));
    const size_t uo = (size_t)H->Uoff[b] + (size_t)q * RC * ldU, vo = (size_t)H->Voff[b] + (size_t)q * RC * ldV;
    const size_t so = ((size_t)b * npair + q) * RC;
    const cd* Us = grad ? H->dU + uo : H->U[c] + bf * H->bU + uo;
    const cd* Vs = grad ? H->dV + vo : H->V[c] + bf * H->bV + vo;
    const double* Ss = grad ? H->dS + so : H->S[c] + bf * H->bS + so;
    if (rk > 0) {
        HIP_TRY(hipMemcpy(U_host, Us, (size_t)rk * ldU * sizeof(cd), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(V_host, Vs, (size_t)rk * ldV * sizeof(cd), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(S_host, Ss, (size_t)rk * sizeof(double), hipMemcpyDeviceToHost));
    }
    return rk;
}

int hnessi_hodlr_factors(hnessi_hodlr_t H, int c, int block, int pair, void* U_host, double* S_host, void* V_host) {
    return factors_to_host(H, c, block, pair, U_host, S_host, V_host, false);
}

int hnessi_factor_grad_get(hnessi_hodlr_t H, int block, int pair, void* dU_host, double* dS_host, void* dV_host) {
    return factors_to_host(H, HNESSI_RET, block, pair, dU_host, dS_host, dV_host, true);
}

int hnessi_hodlr_ranks(hnessi_hodlr_t H, int c, int* ranks_host, int capacity) {
    if (!H || !ranks_host) return fail(HNESSI_E_ARG, "NULL argument");
    if (c != HNESSI_RET && c != HNESSI_LES) return fail(HNESSI_E_ARG, "component must be RET or LES");
    const int per = H->g.nb * H->npair;
    const long long total = (long long)per * H->nk;
    if (capacity < total) return fail(HNESSI_E_ARG, "capacity too small");
    int rc = drain(H);
    if (rc == HNESSI_OK) rc = wait_handle(H);
    if (rc != HNESSI_OK) return rc;
    std::vector<int> both((size_t)2 * per);
    for (int o = 0; o < H->nk && per > 0; ++o) {
        HIP_TRY(hipMemcpy(both.data(), H->rank[c] + (size_t)o * H->oRank, per * sizeof(int), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(both.data() + per, H->rank[c] + (size_t)o * H->oRank + H->bRank, per * sizeof(int),
                          hipMemcpyDeviceToHost));
        for (int b = 0; b < H->g.nb; ++b)
            for (int q = 0; q < H->npair; ++q)
                ranks_host[(size_t)o * per + (size_t)b * H->npair + q] =
                    both[(size_t)H->cur[c][b] * per + (size_t)b * H->npair + q];
    }
    return (int)total;
}

int hnessi_hodlr_blocks(hnessi_hodlr_t H, int* tab_host, int capacity) {
    if (!H || !tab_host) return fail(HNESSI_E_ARG, "NULL argument");
    const Geometry& g = H->g;
    if (capacity < 5 * g.nb) return fail(HNESSI_E_ARG, "capacity too small");
    for (int b = 0; b < g.nb; ++b) {
        tab_host[5 * b] = g.level[b];
        tab_host[5 * b + 1] = g.r0[b];
        tab_host[5 * b + 2] = g.r1[b];
        tab_host[5 * b + 3] = g.c0[b];
        tab_host[5 * b + 4] = g.c1[b];
    }
    return g.nb;
}

int hnessi_hodlr_leaves(hnessi_hodlr_t H, int* tab_host, int capacity) {
    if (!H || !tab_host) return fail(HNESSI_E_ARG, "NULL argument");
    const Geometry& g = H->g;
    if (capacity < 2 * g.nleaf) return fail(HNESSI_E_ARG, "capacity too small");
    for (int i = 0; i < g.nleaf; ++i) {
        tab_host[2 * i] = g.s0[i];
        tab_host[2 * i + 1] = g.s1[i];
    }
    return g.nleaf;
}

size_t hnessi_hodlr_bytes(hnessi_hodlr_t H) { return H ? H->al.bytes : 0; }

int hnessi_hodlr_profile(hnessi_hodlr_t H, int stride) {
    if (!H || stride < 0) return fail(HNESSI_E_ARG, "bad argument");
    int rc = wait_handle(H);
    if (rc != HNESSI_OK) return rc;
    H->prof.clear();
    H->prof.stride = stride;
    return HNESSI_OK;
}

int hnessi_hodlr_profile_read(hnessi_hodlr_t H, int kind, int* steps_host, double* ms_host, int capacity) {
    if (!H || kind < 0 || kind > 6) return fail(HNESSI_E_ARG, "bad argument");
    return H->prof.read(kind, steps_host, ms_host, capacity);
}

// ---------------------------------------------------------------------------
int hnessi_dense_create(hnessi_dense_t* out, int nt, int norb, int k, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!out) return fail(HNESSI_E_ARG, "out is NULL");
    *out = nullptr;
    if (!(norb == 1 || norb == 2 || norb == 4)) return fail(HNESSI_E_ARG, "dense storage supports norb 1, 2, 4");
    if (nt < 2) return fail(HNESSI_E_ARG, "nt must be >= 2");
    int rc = lib_init();
    if (rc != HNESSI_OK) return rc;
    auto* D = new hnessi_dense_s();
    std::string err;
    if (!make_weights(k, D->W, err)) {
        delete D;
        return fail(HNESSI_E_ARG, err);
    }
    D->nt = nt;
    D->norb = norb;
    D->npair = norb * norb;
    D->k = k;
    D->trin = tri(nt);
    const int nbands = dense_band_count(nt);
    D->al = DevAlloc::current(st);
    auto bail = [&](int code) {
        (void)hipStreamSynchronize(st);
        D->al.release(true);
        if (D->ev_last) hipEventDestroy(D->ev_last);
        delete D;
        return code;
    };
    auto nomem = [&]() { return bail(fail(HNESSI_E_NOMEM, "device allocation failed")); };
    for (int c = 0; c < 2; ++c)
        if (dev_alloc(D->al, D->L[c], (size_t)D->npair * D->trin, false) != HNESSI_OK) return nomem();
    if (dev_alloc(D->al, D->colR, (size_t)nbands * nt * D->npair, false) != HNESSI_OK ||
        dev_alloc(D->al, D->colL, (size_t)nbands * nt * D->npair, false) != HNESSI_OK ||
        dev_alloc(D->al, D->rowL, (size_t)dense_chunk_count(nt) * nt * D->npair, false) != HNESSI_OK)
        return nomem();
    if (hipEventCreateWithFlags(&D->ev_last, hipEventDisableTiming) != hipSuccess) {
        D->ev_last = nullptr;
        return bail(fail(HNESSI_E_DEVICE, "event creation failed"));
    }
    if (hipEventRecord(D->ev_last, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return bail(fail(HNESSI_E_DEVICE, "stream synchronization failed"));
    *out = D;
    return HNESSI_OK;
}

int hnessi_dense_destroy(hnessi_dense_t D) {
    if (!D) return fail(HNESSI_E_ARG, "handle is NULL");
    const hipError_t e = D->ev_last ? hipEventSynchronize(D->ev_last) : hipSuccess;
    D->prof.release();
    D->al.release(false);
    if (D->ev_last) hipEventDestroy(D->ev_last);
    delete D;
    return e == hipSuccess ? HNESSI_OK : fail(HNESSI_E_DEVICE, "event synchronization failed");
}

int hnessi_dense_reset(hnessi_dense_t D, void* stream) {
    (void)stream;
    if (!D) return fail(HNESSI_E_ARG, "handle is NULL");
    D->last[0] = D->last[1] = -1;
    return HNESSI_OK;
}

int hnessi_dense_append_row(hnessi_dense_t D, int c, int n, const void* row, void* stream) {
    if (!D || !row) return fail(HNESSI_E_ARG, "NULL argument");
    if (c != HNESSI_RET && c != HNESSI_LES) return fail(HNESSI_E_ARG, "component must be RET or LES");
    if (n < 0 || n >= D->nt) return fail(HNESSI_E_RANGE, "n outside the grid");
    if (n != D->last[c] + 1) return fail(HNESSI_E_ORDER, "rows must be appended in order");
    HIP_TRY(launch_append_dense(D->L[c], static_cast<const cd*>(row), n, D->npair, D->trin, (hipStream_t)stream));
    D->last[c] = n;
    HIP_TRY(hipEventRecord(D->ev_last, (hipStream_t)stream));
    return HNESSI_OK;
}

int hnessi_dense_history_step(hnessi_dense_t D, int n, const void* sigR_row, const void* sigL_slice,
                              double h, void* outR, void* outL, void* stream) {
    if (!D || !sigR_row || !sigL_slice || !outR || !outL) return fail(HNESSI_E_ARG, "NULL argument");
    if (n < 0 || n >= D->nt) return fail(HNESSI_E_RANGE, "n outside the grid");
    if (D->last[0] != n || D->last[1] != n) return fail(HNESSI_E_ORDER, "rows 0..n of both components are needed");
    DenseArgs a{};
    a.n = n;
    a.nt = D->nt;
    a.norb = D->norb;
    a.h = h;
    a.W = D->W;
    a.sigR = static_cast<const cd*>(sigR_row);
    a.sigL = static_cast<const cd*>(sigL_slice);
    a.L[0] = D->L[0];
    a.L[1] = D->L[1];
    a.trin = D->trin;
    a.colR = D->colR;
    a.colL = D->colL;
    a.rowL = D->rowL;
    a.outR = static_cast<cd*>(outR);
    a.outL = static_cast<cd*>(outL);
    if (D->prof.want(n)) {
        hipEvent_t ev[3] = {D->prof.ev(), D->prof.ev(), D->prof.ev()};
        HIP_TRY(launch_dense_history(a, (hipStream_t)stream, ev));
        D->prof.recs.push_back({0, n, ev[0], ev[1]});
        D->prof.recs.push_back({1, n, ev[1], ev[2]});
    } else {
        HIP_TRY(launch_dense_history(a, (hipStream_t)stream));
    }
    HIP_TRY(hipEventRecord(D->ev_last, (hipStream_t)stream));
    return HNESSI_OK;
}

int hnessi_dense_sweep(hnessi_dense_t D, int n_begin, int n_end, const void* GR, const void* GL,
                       const void* SR, const void* SL, double h, void* IR, void* IL, void* stream) {
    if (!D) return fail(HNESSI_E_ARG, "handle is NULL");
    if (!GR || !GL || !SR || !SL || !IR || !IL) return fail(HNESSI_E_ARG, "NULL array");
    if (n_begin < 0 || n_end > D->nt || n_begin > n_end) return fail(HNESSI_E_RANGE, "bad sweep range");
    const size_t np = D->npair;
    for (int n = n_begin; n < n_end; ++n) {
        const size_t off = (size_t)tri(n) * np;
        int rc = hnessi_dense_append_row(D, HNESSI_RET, n, static_cast<const cd*>(GR) + off, stream);
        if (rc != HNESSI_OK) return rc;
        rc = hnessi_dense_append_row(D, HNESSI_LES, n, static_cast<const cd*>(GL) + off, stream);
        if (rc != HNESSI_OK) return rc;
        rc = hnessi_dense_history_step(D, n, static_cast<const cd*>(SR) + off, static_cast<const cd*>(SL) + off, h,
                                       static_cast<cd*>(IR) + off, static_cast<cd*>(IL) + off, stream);
        if (rc != HNESSI_OK) return rc;
    }
    return HNESSI_OK;
}

size_t hnessi_dense_bytes(hnessi_dense_t D) { return D ? D->al.bytes : 0; }

int hnessi_dense_profile(hnessi_dense_t D, int stride) {
    if (!D || stride < 0) return fail(HNESSI_E_ARG, "bad argument");
    HIP_TRY(hipEventSynchronize(D->ev_last));
    D->prof.clear();
    D->prof.stride = stride;
    return HNESSI_OK;
}

int hnessi_dense_profile_read(hnessi_dense_t D, int kind, int* steps_host, double* ms_host, int capacity) {
    if (!D || kind < 0 || kind > 1) return fail(HNESSI_E_ARG, "bad argument");
    return D->prof.read(kind, steps_host, ms_host, capacity);
}

}  // extern "C"
