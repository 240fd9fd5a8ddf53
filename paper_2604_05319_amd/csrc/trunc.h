// Truncation step of a merge: ordering of the singular values of the small
// core and the kept rank under the absolute eps_SVD rule (section
// "Hierarchical decomposition": values below the threshold are dropped).
//
// Plain functions usable on the host and the device, so that the handling of
// non-finite data can be tested on the CPU.  Every index they return lies in
// range whatever the input holds:
//   - a key that is NaN, infinite or above 1e300 (non-finite data in the rows)
//     becomes -1, which sorts last and is never kept, and is reported;
//   - the descending order breaks ties by index, so the positions of the ne
//     keys are a permutation of 0..ne-1;
//   - the kept rank is clamped to the capacity, and an excess is reported.
#pragma once

#if defined(__HIPCC__)
#define HN_HD __host__ __device__
#else
#define HN_HD
#endif

namespace hn {

// Sort key of a singular value; *bad is set for a non-finite one.
HN_HD inline double trunc_key(double s, bool* bad) {
    if (!(s <= 1e300)) {   // NaN compares false
        *bad = true;
        return -1.0;
    }
    if (s < 0.0) return -1.0;   // never produced by a norm; kept out of range anyway
    return s;
}

// Position of key i in the descending order of key[0..ne-1] (ties by index).
HN_HD inline int trunc_position(const double* key, int ne, int i) {
    int pos = 0;
    for (int j = 0; j < ne; ++j) pos += (key[j] > key[i]) || (key[j] == key[i] && j < i);
    return pos;
}

// Number of keys >= tol in key order perm[0..ne-1], clamped to cap; *over is
// set when more than cap values reach tol.
HN_HD inline int trunc_rank(const double* key, const int* perm, int ne, double tol, int cap, bool* over) {
    int r = 0;
    for (int i = 0; i < ne; ++i) {
        int p = perm[i];
        p = p < 0 ? 0 : (p >= ne ? ne - 1 : p);
        r += (key[p] >= tol) ? 1 : 0;
    }
    if (r > cap) {
        *over = true;
        r = cap;
    }
    return r < 0 ? 0 : r;
}

}  // namespace hn
