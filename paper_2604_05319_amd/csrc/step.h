// Retarded time step (the Volterra step solve of the retarded Kadanoff-Baym
// equation): argument struct and launcher.
#pragma once

#include "common.h"

namespace hn {

// One step n >= k of G^R with rows 0..n-1 known.  Columns m < n-k come from the
// left form of the equation (t-derivative by backward differentiation, the history
// sum without its newest term, which moves to the left side); columns n-k..n-1 from
// the right form (t'-derivative of the degree-k interpolant through n-k..n, the
// integral over [t_m, t_n] on the same points), one linear system for the k
// unknown entries; G^R(n, n) = -i.
struct StepArgs {
    int n, k, norb;
    double h;
    Weights W;          // interval weights w^{(L)}_i
    StepWeights S;      // backward differentiation a_l, differentiation matrix D
    const cd* eps;      // [k+1][npair]: eps(t_{n-k+i}), row-major [a][b]
    const cd* sigR;     // [n+1][npair]: Sigma^R(n, j)
    const cd* sigNear;  // [k][k][npair]: (u, i) -> Sigma^R(t_{n-k+u}, t_{n-k+i}), i <= u
    const cd* prev[5];  // prev[l-1]: row n-l of G^R, G^R(n-l, m) at [m][npair]
    cd* row;            // in: h sum_{j=m}^{n-1} w^{(n-m)}_{j-m} Sigma^R(n,j) G^R(j,m) for m < n-k
                        // out: G^R(n, m), m = 0..n
    cd* scr;            // scratch of (k+1) npair entries per object: M^{-1} of the left form,
                        // then the near-diagonal entries G(n, n-k+u) at [1 + u][c][a] (written
                        // by the near-diagonal kernel, read by the bulk kernel)
    // batched objects (grid dimension y): element strides from one object's data to the
    // next (0 for one object)
    int nk;
    long long kEps, kSig, kNear, kPrev, kRow;
};

// One lesser step n >= k with lesser rows 0..n-1 and the retarded row n known: columns
// m <= n-k from the left form of the lesser equation (t-derivative by backward
// differentiation, the history sums without the newest term of the first), columns
// n-k+1..n (the equal-time entry included) from its right form on row n's points n-k..n
// (the integrals over [0, t_m] and [0, t_n]), one linear system for the k unknowns.
// Output in the stored orientation: slice[s] = G^<(t_s, t_n).
struct LesserStepArgs {
    int n, k, norb;
    double h;
    Weights W;
    StepWeights S;
    const cd* eps;        // [k+1][npair]: eps(t_{n-k+i})
    const cd* sigRn[5];   // sigRn[u-1]: Sigma^R row n-k+u (u = 1..k), Sigma^R(t_{n-k+u}, t_s) at [s]
    const cd* sigLn[5];   // sigLn[u-1]: Sigma^< slice n-k+u, Sigma^<(t_s, t_{n-k+u}) at [s]
    const cd* GRn;        // G^R(t_n, t_s), s <= n
    const cd* prev[5];    // prev[l-1]: lesser slice n-l, G^<(t_s, t_{n-l}) at [s]
    cd* slice;            // in: I^<(t_n, t_m) without the s = n term of the first integral, m <= n-k
                          // out: G^<(t_s, t_n), s = 0..n
    cd* scr;              // (1 + k) npair: M^{-1}, then per near column the known sum
    cd* part;             // [k][chunk][npair] partial sums of the near columns' integrals
    int nchunk;           // chunks of lesser_sums
};
int lesser_sum_chunks(int n);
hipError_t launch_lesser_prep(const LesserStepArgs& a, hipStream_t st);
hipError_t launch_lesser_rest(const LesserStepArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);

// The near-diagonal kernel needs no history sum, so it can run beside the history
// kernels; the bulk kernel (after them) also copies its results into the row and writes
// G(n, n).  ev: nullptr, or two events recorded around the launch on its stream.
hipError_t launch_step_near(const StepArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);
hipError_t launch_step_bulk(const StepArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);

}  // namespace hn
