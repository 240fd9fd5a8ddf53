// Host test of the merge truncation step (paper_2604_05319_amd/csrc/trunc.h):
// singular values that are NaN, infinite, huge, negative, tied or ordinary must
// give a valid permutation and a kept rank inside [0, cap], with non-finite
// input and capacity overflow reported.  Built with g++ and run under
// AddressSanitizer / UndefinedBehaviorSanitizer by tests/test_host_trunc.py.
#include <cmath>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "../../paper_2604_05319_amd/csrc/trunc.h"

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);     \
            ++failures;                                                 \
        }                                                               \
    } while (0)

// the device code's steps: keys, positions (one per index), kept rank
static int run(const std::vector<double>& sig, double tol, int cap, bool& bad, bool& over, std::vector<int>& perm) {
    const int ne = (int)sig.size();
    std::vector<double> key(ne);
    bad = false;
    over = false;
    for (int i = 0; i < ne; ++i) key[i] = hn::trunc_key(sig[i], &bad);
    perm.assign(ne, -1);
    for (int i = 0; i < ne; ++i) {
        const int pos = hn::trunc_position(key.data(), ne, i);
        CHECK(pos >= 0 && pos < ne);
        if (pos >= 0 && pos < ne) {
            CHECK(perm[pos] == -1);   // no two indices share a position
            perm[pos] = i;
        }
    }
    for (int p : perm) CHECK(p >= 0 && p < ne);
    // descending keys along the permutation
    for (int i = 1; i < ne; ++i) CHECK(key[perm[i - 1]] >= key[perm[i]]);
    const int r = hn::trunc_rank(key.data(), perm.data(), ne, tol, cap, &over);
    CHECK(r >= 0 && r <= cap);
    return r;
}

int main() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    bool bad, over;
    std::vector<int> perm;
    // ordinary values, one exactly at tol (kept), one below
    {
        std::vector<double> s = {0.5, 2.0, 1e-10, 3e-11, 1.0};
        int r = run(s, 1e-10, 8, bad, over, perm);
        CHECK(r == 4 && !bad && !over);
        CHECK(perm[0] == 1 && perm[1] == 4 && perm[2] == 0 && perm[3] == 2 && perm[4] == 3);
    }
    // non-finite and huge values sort last, are never kept, and are reported
    {
        std::vector<double> s = {nan, 1.0, inf, -inf, 2e300, 0.25, nan};
        int r = run(s, 1e-12, 8, bad, over, perm);
        CHECK(bad && !over);
        CHECK(r == 2);
        CHECK(perm[0] == 1 && perm[1] == 5);
    }
    // all NaN: rank 0, still a permutation
    {
        std::vector<double> s(9, nan);
        int r = run(s, 1e-12, 4, bad, over, perm);
        CHECK(bad && r == 0);
    }
    // ties keep index order
    {
        std::vector<double> s = {1.0, 1.0, 1.0, 0.0};
        int r = run(s, 0.5, 8, bad, over, perm);
        CHECK(r == 3 && perm[0] == 0 && perm[1] == 1 && perm[2] == 2 && perm[3] == 3);
    }
    // capacity overflow is clamped and reported
    {
        std::vector<double> s = {5, 4, 3, 2, 1};
        int r = run(s, 0.5, 3, bad, over, perm);
        CHECK(r == 3 && over && !bad);
    }
    // trunc_rank clamps a corrupted permutation entry instead of reading out of range
    {
        std::vector<double> key = {1.0, 0.5};
        std::vector<int> p = {7, -3};
        bool o = false;
        int r = hn::trunc_rank(key.data(), p.data(), 2, 0.1, 8, &o);
        CHECK(r == 2);
    }
    // random mixtures
    std::mt19937_64 g(1234);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int t = 0; t < 2000; ++t) {
        const int ne = 1 + (int)(u(g) * 64);
        std::vector<double> s(ne);
        int nfin = 0;
        for (double& x : s) {
            const double c = u(g);
            x = c < 0.1 ? nan : c < 0.15 ? inf : c < 0.2 ? 1e301 : c < 0.3 ? 1e-12 : std::pow(10.0, -12.0 * u(g));
        }
        const double tol = 1e-8;
        for (double x : s) nfin += (x <= 1e300 && x >= tol);
        const int cap = 1 + (int)(u(g) * 40);
        int r = run(s, tol, cap, bad, over, perm);
        CHECK(r == (nfin < cap ? nfin : cap));
        CHECK(over == (nfin > cap));
    }
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("trunc host test ok\n");
    return 0;
}
