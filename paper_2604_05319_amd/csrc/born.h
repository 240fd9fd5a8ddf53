// Lattice second-Born self-energy of one time step: argument struct and launcher.
#pragma once

#include "common.h"

namespace hn {

// One band on the L x L square lattice; object k (momentum, x-major) of every array
// starts k * stride complex entries after the array's start.  Row entries j = 0..n.
struct BornArgs {
    int L, n;
    double u2;          // U^2
    const cd* GR;       // G^R_k(t_n, t_j)
    const cd* GL;       // G^<_k(t_j, t_n)  (stored lesser slice)
    long long inStride;
    cd* SR;             // Sigma^R_k(t_n, t_j)
    cd* SL;             // Sigma^<_k(t_j, t_n)
    long long outStride;
};

int born_tile(int L);   // time columns per workgroup
hipError_t launch_born(const BornArgs& a, hipStream_t st, hipEvent_t* ev = nullptr);

}  // namespace hn
