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

// The near-diagonal kernel needs no history sum, so it can run beside the history
// kernels; the bulk kernel (after them) also copies its results into the row and writes
// G(n, n).  ev: nullptr, or two events recorded around the launch on its stream.
hipError_t launch_step_near(const StepArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);
hipError_t launch_step_bulk(const StepArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);

}  // namespace hn
