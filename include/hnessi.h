/*
 * hnessi.h - compressed history integrals of Kadanoff-Baym time stepping on one
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * What is computed (H-NESSi paper, arXiv 2604.05319):
 *   Two-time functions are stored as lower triangles on the grid t_j = j h
 *   (section "Green's functions and Keldysh components"):
 *       retarded  L^R[t1][t2] = C^R(t1, t2),  t1 >= t2
 *       lesser    L^<[t1][t2] = C^<(t2, t1),  t1 >= t2
 *   each entry an norb x norb complex matrix, orbital indices innermost and
 *   row-major.  Row n of a component is (n+1) x norb x norb complex128.
 *   The finished off-diagonal parts are kept as hierarchical (HODLR) blocks,
 *   each orbital pair of each block as a truncated SVD U S V^dagger with the
 *   singular values below eps_SVD dropped (sections "Hierarchical
 *   decomposition" and "Multiorbital compression"); diagonal leaves and the
 *   rows not yet compressed are kept dense.
 *   At step n the history integrals (right-hand sides of the retarded and
 *   lesser Kadanoff-Baym equations, section "Kadanoff-Baym equations", with
 *   Gregory quadrature of order k, appendix "Integral and derivative
 *   approximations") are, for every m <= n:
 *       I^R(n,m) = h sum_{j=m..n} w^{(n-m)}_{j-m} Sigma^R(n,j) G^R(j,m)
 *       I^<(n,m) = h sum_{s=0..n} w^{(n)}_s Sigma^R(n,s) G^<(s,m)
 *                + h sum_{s=0..m} w^{(m)}_s Sigma^<(n,s) G^A(s,m)
 *   with G^<(s,m) = -[G^<(m,s)]^dagger, G^A(s,m) = [G^R(m,s)]^dagger and
 *   Sigma^<(n,s) = -[Sigma^<(s,n)]^dagger (the paper's symmetry relations).
 *   The interval weights w^{(L)} are unit inside and carry the Gregory end
 *   weights omega_0..omega_k (partial sums of the (k+1)-step Adams-Moulton
 *   coefficients) at both ends for L >= k, and are the closed Newton-Cotes
 *   weights for 1 <= L < k; w^{(0)} = 0.
 *
 * Conventions for every call:
 *   - Data pointers marked "device" are device pointers (e.g. from contiguous
 *     complex128 torch tensors); "host" pointers are host memory.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls enqueue work on
 *     it and return without waiting, unless documented otherwise.
 *   - Argument, ordering and range errors are detected on the host before any
 *     work is enqueued; the call then returns a negative hnessi_status and
 *     hnessi_last_error() describes it.  Device-side conditions (rank cap
 *     reached, non-finite data in a truncation) set flags read by
 *     hnessi_hodlr_status().
 *   - A handle is not thread-safe; use one host thread per handle.
 *   - The caller owns all inputs and outputs; a handle owns its own device
 *     storage (factors, leaves, tail rows, band, scratch), obtained through
 *     the allocator hook (hnessi_set_allocator) on the stream of the call
 *     that creates it.
 *   - Calls that wait (destroy, get, ranks, status, profile) wait for the
 *     work of their own handle only: the stream of the handle's last call and
 *     its internal merge stream, never the whole device.
 */
#ifndef HNESSI_H
#define HNESSI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hnessi_hodlr_s* hnessi_hodlr_t;
typedef struct hnessi_dense_s* hnessi_dense_t;

typedef enum { HNESSI_RET = 0, HNESSI_LES = 1 } hnessi_comp;

typedef enum {
    HNESSI_OK = 0,
    HNESSI_E_ARG = -1,     /* invalid argument (null pointer, size out of range)          */
    HNESSI_E_ORDER = -2,   /* rows appended out of order, or history before the row exists */
    HNESSI_E_RANGE = -3,   /* time index outside the grid or the stored region            */
    HNESSI_E_NOMEM = -4,   /* device allocation failed                                    */
    HNESSI_E_DEVICE = -5,  /* a HIP runtime call failed                                   */
    HNESSI_E_RANK = -6,    /* a truncation needed more than max_rank singular values      */
    HNESSI_E_VALUE = -7    /* a truncation met non-finite data (NaN or Inf in the rows)   */
} hnessi_status;

/* Flags for hnessi_hodlr_create. */
#define HNESSI_FLAG_NONE 0
/* The history kernels read complex-float mirrors of the low-rank factors U
 * and V (half the factor bytes of every step), the precision split whose
 * error amplification the paper discusses next to the choice of eps_SVD.  The
 * merges keep working on the FP64 factors and refresh both copies, so FP32
 * rounding never enters a truncation (it would otherwise show up as singular
 * values near 6e-8 * sigma_max, above an absolute eps_SVD); leaves, dense
 * rows, band, singular values and all arithmetic stay FP64.  The added
 * relative error of I is about 1e-7, below 1e-5. */
#define HNESSI_FLAG_FP32_FACTORS 1
/* hnessi_sweep / hnessi_sweep_batched run as HIP graphs: the launches between two
 * panel ends (appends, history kernels, the panel merges forked to and joined from
 * their streams) are captured from the launch stream and replayed through one
 * executable graph of the handle, updated in place window by window (instantiated
 * anew when a window's shape differs).  The stream must not be the NULL stream.
 * Results are identical to the launch-by-launch sweep.  (Section "Implementation
 * details" runs one launch per k point and time step; here every momentum of a
 * lattice is one object of a batched handle.) */
#define HNESSI_FLAG_GRAPHS 2

/* Message for the last failing call on this host thread (never NULL). */
const char* hnessi_last_error(void);

/* ---------------------------------------------------------------------------
 * Device memory.  The paper's storage class owns the memory of its
 * compressed representation (section "The herm_matrix_hodlr class"); here
 * every device allocation of the library (handle storage and the scratch of
 * hnessi_compress_block) goes through one process-wide hook, so that a
 * caching allocator (e.g. PyTorch's) can serve it.
 *   alloc(bytes, stream, ctx)  returns a device pointer usable in stream order
 *                              on `stream`, or NULL on failure (the call that
 *                              allocates then returns HNESSI_E_NOMEM);
 *   free(ptr, stream, ctx)     returns ptr; `stream` is the allocating stream
 *                              when the release is stream-ordered, or NULL
 *                              after the library has waited for all work
 *                              that uses ptr.
 * hnessi_set_allocator(NULL, NULL, NULL) restores the default,
 * hipMallocAsync / hipFreeAsync.  A handle keeps the hook it was created with
 * and returns its memory through it.  Not thread-safe with respect to calls
 * that allocate.  HNESSI_E_ARG if exactly one of the two functions is NULL.
 * ------------------------------------------------------------------------- */
typedef void* (*hnessi_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*hnessi_free_fn)(void* ptr, void* stream, void* ctx);
int hnessi_set_allocator(hnessi_alloc_fn alloc, hnessi_free_fn free_fn, void* ctx);

/* Tile shape of handles created after this call, for one norb: the factor rows
 * of one projection task of the history kernels (and of one partial slot), 0 for
 * the built-in default (1024 for norb <= 2, 512 for norb 4, 256 above).  Allowed:
 * 256, 512, 1024 for norb <= 4; 128, 256 for norb 8 and 16; other values give
 * HNESSI_E_ARG.  Results do not depend on it beyond the order of floating-point
 * sums; it exists for the project's autotuner, which times the candidates on the
 * target workload and records its choice.  Process-wide, thread-safe. */
int hnessi_set_tile_shape(int norb, int proj_rows);

/* The projection chunk rows a handle was created with. */
int hnessi_get_tile_shape(hnessi_hodlr_t H);

/* Interval quadrature weights w^{(L)}_i, i = 0..L, for Gregory order k (1..5),
 * written to w_host[0..L] (host).  Appendix "Integral and derivative
 * approximations".  Returns HNESSI_E_ARG for k outside 1..5 or L < 0. */
int hnessi_weights(int k, int L, double* w_host);

/* Lattice second-Born self-energy of one time step (section "Driven 2D Hubbard
 * example", Eq. BornApproxLG, evaluated in real space as its "Implementation
 * details" describe: G_k -> G_r, local product, Sigma_r -> Sigma_k):
 *   Sigma^>_r(t,t') = U^2 G^>_r(t,t')^2 G^<_{-r}(t',t),
 *   Sigma^<_r(t,t') = U^2 G^<_r(t,t')^2 G^>_{-r}(t',t),
 * one band on the L x L square lattice (L = 2, 4, 8, 16 or 32), momenta
 * k = 2 pi (kx, ky)/L and sites r = (x, y) both x-major, G_r = (1/L^2) sum_k
 * e^{i k.r} G_k, Sigma_k = sum_r e^{-i k.r} Sigma_r.  Row t = t_n, t' = t_j,
 * j = 0..n; the greater and lesser values follow from the stored ones by the
 * definitions of the components (G^R = G^> - G^< for t >= t', anti-Hermitian
 * greater and lesser functions).
 * Device arrays of complex128; object (momentum) k starts k * stride entries after
 * the array's start, entry j of its row at +j:
 *   GR_rows    G^R_k(t_n, t_j)           GL_slices  G^<_k(t_j, t_n)   (in_stride)
 *   SR_rows    Sigma^R_k(t_n, t_j)       SL_slices  Sigma^<_k(t_j, t_n) (out_stride)
 * i.e. the retarded row and the lesser slice in the orientations of
 * hnessi_hodlr_append_row and of the history calls, so the outputs are the Sigma
 * inputs of step n of a batched lattice handle.  The outputs may alias the inputs
 * only exactly (SR_rows == GR_rows, SL_slices == GL_slices, equal strides);
 * otherwise they must not overlap them.  Errors: L not allowed, a NULL pointer, a
 * stride below n+1 or a non-finite U (HNESSI_E_ARG); n < 0 (HNESSI_E_RANGE).
 * Enqueued on stream; the call does not wait for the device. */
int hnessi_born_lattice(int L, int n, double U, const void* GR_rows, const void* GL_slices,
                        long long in_stride, void* SR_rows, void* SL_slices,
                        long long out_stride, void* stream);

/* One time step of the lesser component (section "Kadanoff-Baym equations", Eq. KBEL
 * without the mixed term, in its left form and in the conjugate-transposed right form):
 * the new lesser slice G^<(t_s, t_n), s = 0..n, into slice_out (device, (n+1)*norb*norb
 * complex128, the orientation of hnessi_hodlr_append_row), from the stored lesser rows
 * 0..n-1 and the retarded row n.  Not appended: the caller appends it.
 *   columns m <= n-k of the row G^<(t_n, t_m): the left form, t-derivative by the
 *     backward differentiation weights (every point below the diagonal), the two history
 *     integrals over the stored rows (hnessi_history_lesser without the s = n term of
 *     the first, which is taken to the left): one norb x norb solve per column;
 *   columns n-k+1..n (the equal-time entry included): the right form at (t_n, t_m), its
 *     t'-derivative by the differentiation weights D_ip on the points n-k..n of the row,
 *     the integrals over [0, t_m] and [0, t_n]: one system for the k entries.  (A column
 *     derivative up to the diagonal, with points above it from the row being solved, is
 *     unstable.)
 * Arguments (device pointers unless stated, complex128, orbital matrices row-major):
 *   eps          k+1 matrices eps(t_{n-k+i}), i = 0..k
 *   sigR_rows    host array of k device pointers: Sigma^R row n-k+u at [u-1] (u = 1..k),
 *                Sigma^R(t_{n-k+u}, t_s) at [s]; [k-1] is the current row n
 *   sigL_slices  host array of k device pointers: Sigma^< slice n-k+u at [u-1],
 *                Sigma^<(t_s, t_{n-k+u}) at [s]; [k-1] is the current slice n
 *   GR_row       the retarded row n, G^R(t_n, t_s), s = 0..n (hnessi_step_R's output)
 *   prev_slices  host array of k device pointers: lesser slice n-l at [l-1]
 *   h            time step (> 0)
 * Needs lesser rows 0..n-1 appended, lesser row n not, and retarded rows up to n-1 or n
 * (HNESSI_E_ORDER); n < k: HNESSI_E_RANGE; a batched handle, a NULL pointer or h <= 0:
 * HNESSI_E_ARG.  A singular system leaves non-finite entries; the call does not wait for
 * the device; slice_out must not overlap the inputs. */
int hnessi_step_lesser(hnessi_hodlr_t H, int n, const void* eps, const void* const* sigR_rows,
                       const void* const* sigL_slices, const void* GR_row,
                       const void* const* prev_slices, double h, void* slice_out, void* stream);

/* Rows n_lo..n_hi of G^R in the paper's orientation (section "Kadanoff-Baym
 * equations", Eq. KBER: the derivative in the relative time, the current G row times
 * the compressed Sigma history).  H holds the Sigma^R rows (appended as its retarded
 * component, up to n_hi at least).  Every row solves its own problem: the right form
 *   -i d/dt' G(t_n, t') - G(t_n, t') eps(t') = int_{t'}^{t_n} G(t_n, s) Sigma(s, t') ds
 * marched from G(n, n) = -i leftwards along the row, the first k columns by the
 * k-unknown start of hnessi_step_R, then backward differentiation weights (appendix
 * "Integral and derivative approximations") on the points m..m+k of the row and the
 * Gregory interval weights over [t_m, t_n], the sum over the Sigma history taken from
 * the compressed storage (leaf triangles, low-rank blocks through projections of the
 * row's finished part, the dense tail) -- sequential within a row, one workgroup per
 * row, all rows of the call in one launch, the longest first.  Waits for the handle's merges
 * (the stored state must be complete).  The first call allocates a scratch that the handle
 * keeps: nlvl * norb^3 * 32 complex entries per row for min(nt - k, rows within 2 GiB) rows
 * (larger calls run in several launches), and nt * norb^2 entries for the inverses of the
 * columns' left-side matrices.
 *   eps       device, eps(t_j) for j = 0..n_hi (nt matrices may be passed)
 *   rows_out  device, row n at rows_out + (n - n_lo) * row_stride complex entries,
 *             G^R(t_n, t_m) at [m][a][b], m = 0..n
 * norb must be 1, 2 or 4 and the rank capacity at most 32 (HNESSI_E_ARG); a batched
 * handle, a NULL pointer, a row stride below (n_hi+1)*norb^2 or h <= 0: HNESSI_E_ARG;
 * rows outside k..nt-1: HNESSI_E_RANGE; Sigma rows not appended: HNESSI_E_ORDER. */
int hnessi_row_march_R(hnessi_hodlr_t H, int n_lo, int n_hi, const void* eps, double h,
                       void* rows_out, long long row_stride, void* stream);

/* Weights of the retarded time step (hnessi_step_R) for order k (1..5), host
 * outputs: a_host[0..k] the backward differentiation weights a_l = -D_{0l}
 * (f'(t_n) h ~ sum_l a_l f(t_{n-l})) and D_host[i*(k+1) + p], i, p = 0..k, the
 * derivative at point i of the degree-k interpolant through the equispaced
 * points 0..k (unit spacing), appendix "Integral and derivative
 * approximations".  Returns HNESSI_E_ARG for k outside 1..5 or a NULL output. */
int hnessi_step_weights(int k, double* a_host, double* D_host);

/* ---------------------------------------------------------------------------
 * HODLR-compressed storage of the retarded and lesser components
 * (the paper's herm_matrix_hodlr for its R and < parts).
 * ------------------------------------------------------------------------- */

/* Create a handle for nt time steps (the constructor of the paper's
 * herm_matrix_hodlr, section "The herm_matrix_hodlr class", with the
 * partitioning parameters of section "Hierarchical decomposition").
 *   nlvl     number of hierarchical levels; level l holds 2^(l-1) off-diagonal
 *            blocks of about nt/2^l rows; the 2^nlvl diagonal leaves are kept
 *            dense.  The smallest leaf must hold at least k+1 rows and the
 *            panel; every leaf at most 64 rows.
 *   norb     orbital dimension: 1, 2, 4, 8 or 16 (norb^2 separately
 *            compressed orbital pairs, section "Multiorbital compression").
 *   k        Gregory order, 1..5 (section "Numerical integration").
 *   svd_tol  absolute truncation threshold eps_SVD > 0: singular values
 *            sigma >= svd_tol are kept.
 *   panel    rows per compression panel P (1..16); a panel also ends at
 *            every leaf start, so it need not divide the leaf size.
 *   max_rank rank capacity per block and orbital pair; max_rank + panel <= 48
 *            (the width of the small SVD solved at each merge).
 *   flags    HNESSI_FLAG_NONE, or HNESSI_FLAG_FP32_FACTORS and/or HNESSI_FLAG_GRAPHS.
 *   stream   every allocation, fill and copy of the handle is ordered on it;
 *            the call returns once they are complete.
 * On success *out is set.  HNESSI_E_ARG for an argument out of range,
 * HNESSI_E_NOMEM when the allocator hook fails (nothing is leaked). */
int hnessi_hodlr_create(hnessi_hodlr_t* out, int nt, int nlvl, int norb, int k,
                        double svd_tol, int panel, int max_rank, int flags, void* stream);

/* Wait for the handle's work (its last call's stream and its merge stream),
 * then return its memory through the hook it was created with. */
int hnessi_hodlr_destroy(hnessi_hodlr_t H);

/* Graph windows replayed by the handle's sweeps so far and how many of them needed a
 * new instantiation (HNESSI_FLAG_GRAPHS; both zero otherwise). */
int hnessi_hodlr_graph_stats(hnessi_hodlr_t H, long long* windows, long long* instantiations);

/* Forget all rows and the device status flags (start a new sweep from
 * n = 0); storage is kept.  Enqueued on stream. */
int hnessi_hodlr_reset(hnessi_hodlr_t H, void* stream);

/* Append row n of component c (device pointer, (n+1)*norb*norb complex128);
 * the current-timestep set of Tab. getset followed by the once-per-step
 * update_blocks of section "The herm_matrix_hodlr class":
 *   HNESSI_RET: G^R(t_n, t_j), j = 0..n
 *   HNESSI_LES: G^<(t_s, t_n), s = 0..n   (the paper's stored lesser slice)
 * n must equal the previous row of that component plus one (HNESSI_E_ORDER);
 * n outside the grid: HNESSI_E_RANGE; NULL row: HNESSI_E_ARG.
 * When the row completes a panel, the panel is merged into the truncated SVDs
 * of the blocks it belongs to (incremental TSVD update, section "Hierarchical
 * decomposition").  The input may be reused once the stream reaches the call. */
int hnessi_hodlr_append_row(hnessi_hodlr_t H, int c, int n, const void* row, void* stream);

/* I^R(n, m), m = 0..n, into out (device, (n+1)*norb*norb complex128): the
 * history integral of the retarded Kadanoff-Baym equation (Eq. KBER, section
 * "Kadanoff-Baym equations") in the form with the current Sigma^R row on the
 * left, Gregory weights of the appendix "Integral and derivative
 * approximations".  sigR_row: Sigma^R(t_n, t_j), j = 0..n (device).
 * Needs retarded rows 0..n appended (HNESSI_E_ORDER otherwise); with later
 * rows appended, step n is evaluated over the stored (frozen) state, see
 * hnessi_history_R_adjoint.  NULL pointers: HNESSI_E_ARG. */
int hnessi_history_R(hnessi_hodlr_t H, int n, const void* sigR_row, double h,
                     void* out, void* stream);

/* One time step of the retarded Kadanoff-Baym equation (section "Kadanoff-Baym
 * equations", Eq. KBER and its left form, G^R(t,t) = -i): row n of G^R from the
 * stored rows 0..n-1, written to row_out (device, (n+1)*norb*norb complex128,
 * G^R(t_n, t_m) at [m][a][b]).  The row is not appended: the caller appends it
 * (hnessi_hodlr_append_row), or calls again with a new Sigma^R first (a
 * self-consistent iteration at fixed n).
 *   columns m < n-k: the left form, the t-derivative by the backward
 *     differentiation weights a_l = -D_{0l} of the appendix "Integral and
 *     derivative approximations", the history sum over the stored rows with the
 *     Gregory interval weights (the hnessi_history_R sum without its newest term,
 *     which is taken to the left side): one norb x norb solve per column;
 *   columns n-k..n-1: the right form at (t_n, t_m), its t'-derivative by the
 *     polynomial differentiation weights D_{ip} of the same appendix on the points
 *     n-k..n and its integral over [t_m, t_n] on the same points: one linear system
 *     for those k entries.
 * Arguments (device pointers, complex128, orbital matrices row-major [a][b]):
 *   eps        k+1 matrices eps(t_{n-k+i}), i = 0..k
 *   sigR_row   Sigma^R(t_n, t_j), j = 0..n
 *   sig_near   k*k matrices at [u*k + i]: Sigma^R(t_{n-k+u}, t_{n-k+i}) for
 *              0 <= i <= u < k (the entries with u < i are not read)
 *   prev_rows  host array of k device pointers: prev_rows[l-1] holds row n-l of
 *              G^R, G^R(t_{n-l}, t_m) at [m][a][b] (columns m < n-k are read)
 *   h          time step (> 0)
 * The first k rows (the start-up of the paper's bootstrapping) are the caller's:
 * n < k gives HNESSI_E_RANGE.  Needs retarded rows 0..n-1 appended and row n not
 * (HNESSI_E_ORDER), a handle of one object (HNESSI_E_ARG for a batch), no NULL
 * pointer and h > 0 (HNESSI_E_ARG).  A singular system (a zero pivot) leaves
 * non-finite entries in row_out; the call does not wait for the device.
 * row_out must not overlap the inputs. */
int hnessi_step_R(hnessi_hodlr_t H, int n, const void* eps, const void* sigR_row,
                  const void* sig_near, const void* const* prev_rows, double h,
                  void* row_out, void* stream);

/* I^<(n, m), m = 0..n, into out (device): the two history integrals of the
 * lesser Kadanoff-Baym equation (Eq. KBEL, section "Kadanoff-Baym equations";
 * the mixed imaginary-time term is not part of this call), Gregory weights as
 * above.  sigL_slice: Sigma^<(t_s, t_n), s = 0..n (device, the stored
 * orientation of the current lesser slice, Tab. getset).  Needs both
 * components appended up to row n exactly (HNESSI_E_ORDER). */
int hnessi_history_lesser(hnessi_hodlr_t H, int n, const void* sigR_row,
                          const void* sigL_slice, double h, void* out, void* stream);

/* Adjoint (vector-Jacobian product) of hnessi_history_R with respect to the
 * Sigma^R row, for gradients of losses of I^R (adjoint form of the retarded
 * equation's history term; the paper differentiates nothing, the operation is
 * the transpose of the discrete sum of Eq. KBER's history integral):
 *   out(j) = h sum_{m=0..j} w^{(n-m)}_{j-m} Ibar(n, m) G^R(t_j, t_m)^dagger,  j = 0..n,
 * i.e. <Ibar, I^R> = <out, Sigma^R(n, .)> for the real inner product
 * Re sum tr(A^dagger B).  ibar_row: device (n+1)*norb*norb complex128, the
 * cotangent of I^R(n, m), m = 0..n; out: device, same size.  Needs the
 * retarded row n appended (HNESSI_E_ORDER otherwise); reads only the
 * retarded component.
 * Frozen state: like hnessi_history_R and hnessi_history_R_factor_grad, this call
 * also takes any n below the last appended retarded row and then evaluates step
 * n over the stored state (the compressed G^R of all rows appended so far, rows
 * above n excluded), so a backward pass needs no replay of the appends and
 * merges.  For n < last the call first completes the retarded component's
 * in-flight panel merge on stream. */
int hnessi_history_R_adjoint(hnessi_hodlr_t H, int n, const void* ibar_row, double h, void* out,
                             void* stream);

/* Gradient of a real loss with respect to the retarded HODLR factors of the
 * stored state, step n's contribution (the transpose of Eq. KBER's discrete
 * history sum, section "Hierarchical decomposition" for G = U S V^H per block and
 * orbital pair): with Gbar(j, m) = h sum_n w^{(n-m)}_{j-m} Sigma^R(n,j)^dagger
 * Ibar(n, m) the gradient with respect to the entries of block b, pair
 * q = (b', c), this call adds
 *   dU += Gbar V S,   dV += Gbar^dagger U S,   dS += Re diag(U^dagger Gbar V)
 * over the merged rows j <= n of every block (rows still in the dense tail carry
 * no factor).  sigR_row: Sigma^R(n, j), j = 0..n; ibar_row: the cotangent of
 * I^R(n, m), m = 0..n (device, (n+1)*norb*norb complex128 each).  The sums over
 * n accumulate in device buffers of the handle, allocated (and cleared) by the
 * first call; hnessi_factor_grad_reset clears them and hnessi_factor_grad_get
 * reads them.  Gradients are taken in torch's convention for complex tensors
 * (dL/dRe + i dL/dIm); S is real.  n may be below the last appended row
 * (frozen state, see hnessi_history_R_adjoint), which is how a backward pass
 * calls it: the factors are those of the handle when the call runs.  Single
 * objects only (HNESSI_E_ARG for batched handles); HNESSI_E_NOMEM if the first
 * call cannot allocate the buffers (one more copy of a buffer of U, V and S). */
int hnessi_history_R_factor_grad(hnessi_hodlr_t H, int n, const void* sigR_row, const void* ibar_row,
                                 double h, void* stream);

/* Clear the factor-gradient buffers (no-op before the first
 * hnessi_history_R_factor_grad), ordered on stream. */
int hnessi_factor_grad_reset(hnessi_hodlr_t H, void* stream);

/* Accumulated factor gradients of retarded block `block` (the row of
 * hnessi_hodlr_blocks), orbital pair `pair` = b' * norb + c, to host memory:
 * dU_host: rank columns of (r1 - r0) rows, column r at dU_host[r * (r1 - r0) + i]
 * (complex128); dV_host likewise with c1 - c0 rows; dS_host: rank values.
 * Returns the rank of the pair's current factors (the number of columns
 * written), HNESSI_E_ORDER before any accumulation.  Synchronizes with the
 * handle's work. */
int hnessi_factor_grad_get(hnessi_hodlr_t H, int block, int pair, void* dU_host, double* dS_host,
                           void* dV_host);

/* The current TSVD factors U, S, V of block `block`, pair `pair` of component
 * comp (section "Hierarchical decomposition": G = U S V^H on the block's rows
 * and columns, Tab. getcompress for reading the compressed storage), to host
 * memory in the layout of hnessi_factor_grad_get; rows of U at or above the
 * merge frontier are not yet part of the factors.  Returns the rank.
 * Completes in-flight merges and synchronizes with the handle's work. */
int hnessi_hodlr_factors(hnessi_hodlr_t H, int comp, int block, int pair, void* U_host, double* S_host,
                         void* V_host);

/* Both integrals of step n (Eqs. KBER and KBEL as for hnessi_history_R and
 * hnessi_history_lesser) in one pass over the stored data: each stored
 * factor is used for every product it enters.  outR / outL as above; errors
 * as for the two calls. */
int hnessi_history_step(hnessi_hodlr_t H, int n, const void* sigR_row, const void* sigL_slice,
                        double h, void* outR, void* outL, void* stream);

/* A whole sweep n = n_begin..n_end-1 driven natively (the time-stepping loop
 * of section "Timestepping and SVD updates" with the known rows of a
 * synthetic G): for each n, append G^R row n and G^< row n, then
 * hnessi_history_step.  All arrays are device packed lower triangles, row n
 * at element offset n(n+1)/2 (times norb^2):
 *   GR, GL  rows of the two components as for append_row;
 *   SR, SL  Sigma^R rows and Sigma^< slices as for the history calls;
 *   IR, IL  outputs I^R(n, .), I^<(n, .).
 * n_begin must be the next row to append. */
int hnessi_sweep(hnessi_hodlr_t H, int n_begin, int n_end, const void* GR, const void* GL,
                 const void* SR, const void* SL, double h, void* IR, void* IL, void* stream);

/* Device-side status (the paper's library throws when a call cannot honour
 * its contract, section "The herm_matrix_hodlr class"; here the device
 * conditions are flags), after synchronizing `stream` and the handle's
 * merges: HNESSI_OK; HNESSI_E_RANK
 * if any truncation needed more than max_rank singular values (the excess
 * ones were dropped and the eps_SVD guarantee does not hold); HNESSI_E_VALUE
 * if a truncation met non-finite data (those directions were dropped).  The
 * flags stay set until hnessi_hodlr_reset. */
int hnessi_hodlr_status(hnessi_hodlr_t H, void* stream);

/* ---------------------------------------------------------------------------
 * Batched objects: the k-point lattice form (sections "Driven 2D Hubbard
 * example" and "Implementation details", where every momentum k carries its
 * own Green's function and self-energy, the Dyson steps of different k are
 * independent and are distributed over threads and ranks).
 *
 * One handle holds nk objects of one geometry (nt, nlvl, norb, k, svd_tol,
 * panel, max_rank), advanced together: every call acts on all nk objects in
 * the same kernel launches (grid dimension y = object).  Ranks, factors and
 * truncations are per object.  Device arrays are object-major: object o's
 * data starts o * stride complex128 elements after object 0's; a stride must
 * be at least one object's data (HNESSI_E_ARG otherwise).  The single-object
 * calls (append_row, history_*, sweep, get) return HNESSI_E_ARG on a batched
 * handle; status, reset, ranks (nk * nb * norb^2 entries, object-major),
 * blocks, leaves, bytes and profiling work on both.
 * ------------------------------------------------------------------------- */

/* nk objects (momenta) in 1..65535; other arguments and errors as for
 * hnessi_hodlr_create. */
int hnessi_hodlr_create_batched(hnessi_hodlr_t* out, int nk, int nt, int nlvl, int norb, int k,
                                double svd_tol, int panel, int max_rank, int flags, void* stream);

/* Number of objects (momenta) of the handle (1 for hnessi_hodlr_create). */
int hnessi_hodlr_nk(hnessi_hodlr_t H);

/* hnessi_hodlr_append_row for every object (Tab. getset and update_blocks
 * per momentum): object o's row at rows + o*k_stride. */
int hnessi_hodlr_append_row_batched(hnessi_hodlr_t H, int c, int n, const void* rows, long long k_stride,
                                    void* stream);

/* hnessi_history_step for every object (Eqs. KBER and KBEL per momentum):
 * inputs of object o at sigR_rows +
 * o*in_stride and sigL_slices + o*in_stride, outputs at outR + o*out_stride
 * and outL + o*out_stride. */
int hnessi_history_step_batched(hnessi_hodlr_t H, int n, const void* sigR_rows, const void* sigL_slices,
                                long long in_stride, double h, void* outR, void* outL, long long out_stride,
                                void* stream);

/* hnessi_step_R for every object (the retarded time step per momentum, each object
 * with its own eps and Sigma^R): object o's arrays start o * stride complex entries
 * after the given pointers -- eps (k+1 matrices) at eps_stride, the Sigma^R row at
 * in_stride, the k*k near-diagonal Sigma^R matrices at near_stride, each previous row
 * prev_rows[l-1] at prev_stride, the output row at out_stride.  On a handle of more
 * than one object a stride smaller than one object's data (k+1, n+1, k*k, n-k and n+1
 * matrices) gives HNESSI_E_ARG; other errors as for hnessi_step_R. */
int hnessi_step_R_batched(hnessi_hodlr_t H, int n, const void* eps, long long eps_stride,
                          const void* sigR_rows, long long in_stride, const void* sig_near,
                          long long near_stride, const void* const* prev_rows, long long prev_stride,
                          double h, void* rows_out, long long out_stride, void* stream);

/* hnessi_sweep for every object (the time-stepping loop per momentum):
 * the six packed triangles of object o start
 * at o*k_stride elements (k_stride >= nt(nt+1)/2 * norb^2). */
int hnessi_sweep_batched(hnessi_hodlr_t H, int n_begin, int n_end, const void* GR, const void* GL,
                         const void* SR, const void* SL, long long k_stride, double h, void* IR, void* IL,
                         void* stream);

/* Value of component c at (t1, t2), t1 >= t2, t1 <= last appended row,
 * reconstructed from whichever storage holds it (dense leaf, dense row, or
 * truncated SVD), into out_host (norb*norb complex128): the general get of
 * Tab. getcompress, valid for any point up to the current timestep.
 * Waits for the handle's work.  HNESSI_E_RANGE outside the stored region;
 * HNESSI_E_ARG on a batched handle. */
int hnessi_hodlr_get(hnessi_hodlr_t H, int c, int t1, int t2, void* out_host);

/* Ranks of component c (the eps-ranks of section "Hierarchical
 * decomposition", one per orbital pair, section "Multiorbital compression"):
 * ranks_host[b*norb*norb + q] for block b (in the order of
 * hnessi_hodlr_blocks) and orbital pair q.  Waits for the handle's work and
 * its pending merges.  Returns the number of entries written, or a negative
 * status (HNESSI_E_ARG when capacity is too small). */
int hnessi_hodlr_ranks(hnessi_hodlr_t H, int c, int* ranks_host, int capacity);

/* Block table of the partitioning (section "Hierarchical decomposition"):
 * for block b, rows [r0, r1) and columns [c0, c1), level in 1..nlvl;
 * tab_host[5*b + {0..4}] = level, r0, r1, c0, c1.  Host only.
 * Returns the number of blocks (or a negative status). */
int hnessi_hodlr_blocks(hnessi_hodlr_t H, int* tab_host, int capacity);

/* Leaf table (the dense diagonal triangles of section "Hierarchical
 * decomposition"): tab_host[2*i + {0,1}] = s0, s1.  Returns the number of
 * leaves. */
int hnessi_hodlr_leaves(hnessi_hodlr_t H, int* tab_host, int capacity);

/* Device bytes held by the handle (factor capacity, leaves, tail, band,
 * scratch): the memory footprint the paper compares with dense storage
 * (section "Driven 2D Hubbard example"). */
size_t hnessi_hodlr_bytes(hnessi_hodlr_t H);

/* Kernel timing with HIP events recorded on the launch stream (measurement,
 * the per-part timings of section "Timing results").
 * stride > 0: from now on time the history kernels of every step n with
 * n % stride == 0, and every panel merge; stride = 0 stops.  Clears earlier
 * records (waits for the handle's work). */
int hnessi_hodlr_profile(hnessi_hodlr_t H, int stride);

/* Synchronizes the recorded events; for kernel kind 0 (projection / leaf /
 * tail tasks), 1 (combine), 2 (panel merge, both of its kernels), 3 (sum of
 * the projection chunk partials), 4 (time step: near-diagonal system), 5
 * (time step: columns m < n-k) or 6 (lesser step after its history) returns the
 * number of timed launches and writes, for the first `capacity` of them, the
 * step n (host int) and the duration in ms (host double).  Either output
 * pointer may be NULL. */
int hnessi_hodlr_profile_read(hnessi_hodlr_t H, int kind, int* steps_host, double* ms_host, int capacity);

/* ---------------------------------------------------------------------------
 * Truncated SVD of one dense block (section "Hierarchical decomposition":
 * B ~ U S V^dagger keeping the singular values >= eps_SVD, so that
 * |B - U S V^dagger|_2 < eps_SVD).
 * A (device, rows x cols complex128, row-major with leading dimension lda)
 * ~ U diag(S) V^dagger with the absolute threshold tol > 0:
 *   U: device, column-major rows x max_rank (column r at U + r*rows)
 *   S: device, max_rank doubles, non-increasing (zero beyond the rank)
 *   V: device, column-major cols x max_rank
 *   rank_out: device int, the kept rank r; then S[r-1] >= tol and
 *             |A - U S V^dagger|_2 < tol, except when a singular value of A
 *             lies within 1e-3 * tol of tol (it may then be kept or dropped).
 *             More than max_rank values >= tol: the largest max_rank are kept
 *             and *rank_out == max_rank.  Negative values report a failure
 *             found on the device: HNESSI_E_VALUE (non-finite entries in A) or
 *             HNESSI_E_RANK (an intermediate merge needed more than 40 values).
 * 1 <= max_rank <= 40.  The rows are merged 8 at a time; every merge but the
 * last drops only values below 5e-4 * tol / (number of merges), the last
 * truncates at tol.  Fully asynchronous on `stream`: the scratch comes from
 * the allocator hook and is returned to it in stream order.  Argument errors:
 * HNESSI_E_ARG; hook failure: HNESSI_E_NOMEM. */
int hnessi_compress_block(const void* A, int rows, int cols, int lda, double tol, int max_rank,
                          void* U, double* S, void* V, int* rank_out, void* stream);

/* hnessi_compress_block for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same factorization and results, with the scratch taken from
 * a static device array of about 18 MB that each GPU the library runs on
 * holds until the process ends.  It calls no allocation routine and no
 * allocator hook.  rows and cols must be at most 4096 (HNESSI_E_ARG beyond);
 * other arguments and errors as for hnessi_compress_block.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialized by the caller. */
int hnessi_compress_block_noalloc(const void* A, int rows, int cols, int lda, double tol, int max_rank,
                                  void* U, double* S, void* V, int* rank_out, void* stream);

/* ---------------------------------------------------------------------------
 * Dense storage (the uncompressed baseline on the same device, the role of
 * the NESSi solver in the paper's comparisons, sections "Timing results" and
 * "Driven 2D Hubbard example"): both components as full packed lower
 * triangles, the same history integrals (Eqs. KBER and KBEL) by direct
 * summation, one read of every stored entry per step.  Arguments, layouts and
 * errors as for the HODLR calls of the same name; norb is 1, 2 or 4.
 * ------------------------------------------------------------------------- */
/* Allocates 2 * norb^2 * nt(nt+1)/2 complex128 through the hook on stream. */
int hnessi_dense_create(hnessi_dense_t* out, int nt, int norb, int k, void* stream);
/* Waits for the handle's last call, then frees. */
int hnessi_dense_destroy(hnessi_dense_t D);
/* Forget all rows. */
int hnessi_dense_reset(hnessi_dense_t D, void* stream);
/* Row n of component c, as hnessi_hodlr_append_row (stored, never compressed). */
int hnessi_dense_append_row(hnessi_dense_t D, int c, int n, const void* row, void* stream);
/* I^R(n, .) and I^<(n, .) as hnessi_history_step. */
int hnessi_dense_history_step(hnessi_dense_t D, int n, const void* sigR_row,
                              const void* sigL_slice, double h, void* outR, void* outL,
                              void* stream);
/* A sweep as hnessi_sweep. */
int hnessi_dense_sweep(hnessi_dense_t D, int n_begin, int n_end, const void* GR, const void* GL,
                       const void* SR, const void* SL, double h, void* IR, void* IL,
                       void* stream);
/* Device bytes held (the dense memory footprint of the paper's comparisons). */
size_t hnessi_dense_bytes(hnessi_dense_t D);
/* Event timing of the dense kernels as for the HODLR handle: kind 0 = tile
 * kernel, 1 = reduction. */
int hnessi_dense_profile(hnessi_dense_t D, int stride);
int hnessi_dense_profile_read(hnessi_dense_t D, int kind, int* steps_host, double* ms_host, int capacity);

#ifdef __cplusplus
}
#endif

#endif /* HNESSI_H */
