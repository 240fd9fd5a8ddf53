// Host plan: HODLR geometry and quadrature weights.
//
// Geometry (section "Hierarchical decomposition"): the lower triangle of an
// nt x nt two-time matrix is split recursively; at every split of a diagonal
// interval [a, b) at mid = a + (b - a)/2 the off-diagonal block rows [mid, b)
// x columns [a, mid) belongs to the next level, and the two halves are split
// again.  Level l (1..nlvl) holds 2^(l-1) blocks; the 2^nlvl diagonal
// intervals left after nlvl splits are the dense leaves.
//
// Weights (appendix "Integral and derivative approximations"): the (k+1)-step
// Adams-Moulton coefficients are the polynomial integration weights of the
// degree-(k+1) interpolant through points 0..k+1 integrated over [k, k+1];
// the Gregory end weights are their partial sums from the newest point; the
// interval weights add the two end corrections to unit weights (intervals of
// at least k steps) or are closed Newton-Cotes weights (shorter intervals).
// All of this is done in exact rational arithmetic and rounded once.
#include <cstdint>
#include <functional>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"

namespace hn {

namespace {

// exact rationals on __int128 with reduction; sizes here stay tiny (k <= 5)
struct Q {
    __int128 p = 0, q = 1;
    Q() = default;
    Q(long long a) : p(a), q(1) {}
    Q(__int128 a, __int128 b) : p(a), q(b) { norm(); }
    static __int128 gcd(__int128 a, __int128 b) {
        if (a < 0) a = -a;
        if (b < 0) b = -b;
        while (b) { __int128 t = a % b; a = b; b = t; }
        return a;
    }
    void norm() {
        if (q < 0) { p = -p; q = -q; }
        __int128 g = gcd(p, q);
        if (g > 1) { p /= g; q /= g; }
    }
    Q operator+(const Q& o) const { return Q(p * o.q + o.p * q, q * o.q); }
    Q operator-(const Q& o) const { return Q(p * o.q - o.p * q, q * o.q); }
    Q operator*(const Q& o) const { return Q(p * o.p, q * o.q); }
    Q operator/(const Q& o) const { return Q(p * o.q, q * o.p); }
    bool zero() const { return p == 0; }
    double to_double() const { return (double)p / (double)q; }
};

Q qpow(long long base, int e) {
    Q r(1);
    for (int i = 0; i < e; ++i) r = r * Q(base);
    return r;
}

// P = M^{-1}, M_{ja} = j^a (0 <= j, a <= deg), by Gauss-Jordan over Q
std::vector<std::vector<Q>> vandermonde_inverse(int deg) {
    int n = deg + 1;
    std::vector<std::vector<Q>> a(n, std::vector<Q>(2 * n));
    for (int j = 0; j < n; ++j) {
        for (int c = 0; c < n; ++c) a[j][c] = qpow(j, c);
        a[j][n + j] = Q(1);
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        while (a[piv][col].zero()) ++piv;
        std::swap(a[piv], a[col]);
        Q pv = a[col][col];
        for (auto& v : a[col]) v = v / pv;
        for (int r = 0; r < n; ++r) {
            if (r == col || a[r][col].zero()) continue;
            Q f = a[r][col];
            for (int c = 0; c < 2 * n; ++c) a[r][c] = a[r][c] - f * a[col][c];
        }
    }
    // rows of a now hold M^{-1}: (M^{-1})_{j', l} = a[j'][n + l]; here j' indexes the power a
    std::vector<std::vector<Q>> P(n, std::vector<Q>(n));
    for (int pw = 0; pw < n; ++pw)
        for (int l = 0; l < n; ++l) P[pw][l] = a[pw][n + l];
    return P;
}

// I_{m n l} = sum_a P_{a l} (n^{a+1} - m^{a+1}) / (a + 1)
std::vector<Q> poly_int(int deg, int m, int n) {
    auto P = vandermonde_inverse(deg);
    std::vector<Q> w(deg + 1);
    for (int l = 0; l <= deg; ++l) {
        Q s(0);
        for (int a = 0; a <= deg; ++a)
            s = s + P[a][l] * (qpow(n, a + 1) - qpow(m, a + 1)) / Q(a + 1);
        w[l] = s;
    }
    return w;
}

std::vector<Q> gregory(int k) {
    auto b = poly_int(k + 1, k, k + 1);  // b_0 .. b_{k+1}
    std::vector<Q> om(k + 1);
    Q acc(0);
    for (int i = 0; i <= k; ++i) {
        acc = acc + b[k + 1 - i];
        om[i] = acc;
    }
    return om;
}

std::vector<Q> interval_q(int k, int L) {
    if (L == 0) return {Q(0)};
    if (L < k) return poly_int(L, 0, L);
    auto om = gregory(k);
    std::vector<Q> w(L + 1, Q(1));
    for (int i = 0; i <= k; ++i) {
        w[i] = w[i] + om[i] - Q(1);
        w[L - i] = w[L - i] + om[i] - Q(1);
    }
    return w;
}

}  // namespace

// D_{m l} = sum_{a >= 1} P_{a l} a m^{a-1}: derivative at point m of the degree-deg
// interpolant through points 0..deg (unit spacing)
std::vector<Q> poly_diff(int deg, int m) {
    auto P = vandermonde_inverse(deg);
    std::vector<Q> d(deg + 1);
    for (int l = 0; l <= deg; ++l) {
        Q s(0);
        for (int a = 1; a <= deg; ++a) s = s + P[a][l] * Q(a) * qpow(m, a - 1);
        d[l] = s;
    }
    return d;
}

bool make_step_weights(int k, StepWeights& S, std::string& err) {
    if (k < 1 || k > 5) { err = "order k must be in 1..5"; return false; }
    S = StepWeights{};
    S.k = k;
    for (int i = 0; i <= k; ++i) {
        auto d = poly_diff(k, i);
        for (int l = 0; l <= k; ++l) S.D[i][l] = d[l].to_double();
    }
    for (int l = 0; l <= k; ++l) S.a[l] = -S.D[0][l];   // backward differentiation: a_l = -D_{0 l}
    return true;
}

bool interval_weights_exact(int k, int L, std::vector<double>& w, std::string& err) {
    if (k < 1 || k > 5) { err = "Gregory order k must be in 1..5"; return false; }
    if (L < 0) { err = "interval length must be >= 0"; return false; }
    auto q = interval_q(k, L);
    w.resize(q.size());
    for (size_t i = 0; i < q.size(); ++i) w[i] = q[i].to_double();
    return true;
}

bool make_weights(int k, Weights& W, std::string& err) {
    if (k < 1 || k > 5) { err = "Gregory order k must be in 1..5"; return false; }
    W = Weights{};
    W.k = k;
    auto om = gregory(k);
    for (int i = 0; i <= k; ++i) W.om[i] = om[i].to_double();
    for (int L = 0; L < k; ++L) {
        auto w = interval_q(k, L);
        for (int i = 0; i <= L; ++i) W.nc[L][i] = w[i].to_double();
    }
    return true;
}

bool build_geometry(int nt, int nlvl, Geometry& g, std::string& err) {
    if (nt < 2) { err = "nt must be >= 2"; return false; }
    if (nlvl < 0 || nlvl > 20 || (nt >> nlvl) < 1) { err = "nlvl out of range for nt"; return false; }
    g = Geometry{};
    g.nt = nt;
    g.nlvl = nlvl;
    std::function<void(int, int, int)> rec = [&](int a, int b, int lvl) {
        if (lvl == nlvl) {
            g.s0.push_back(a);
            g.s1.push_back(b);
            return;
        }
        int mid = a + (b - a) / 2;
        g.level.push_back(lvl + 1);
        g.r0.push_back(mid);
        g.r1.push_back(b);
        g.c0.push_back(a);
        g.c1.push_back(mid);
        rec(a, mid, lvl + 1);
        rec(mid, b, lvl + 1);
    };
    rec(0, nt, 0);
    g.nb = (int)g.level.size();
    g.nleaf = (int)g.s0.size();
    g.row_leaf.assign(nt, -1);
    g.max_leaf = 0;
    g.min_leaf = nt;
    for (int i = 0; i < g.nleaf; ++i) {
        for (int r = g.s0[i]; r < g.s1[i]; ++r) g.row_leaf[r] = i;
        g.max_leaf = std::max(g.max_leaf, g.s1[i] - g.s0[i]);
        g.min_leaf = std::min(g.min_leaf, g.s1[i] - g.s0[i]);
    }
    g.cover.assign((size_t)std::max(nlvl, 1) * nt, 0);
    for (int b = 0; b < g.nb; ++b) {
        int l = g.level[b] - 1;
        for (int m = g.c0[b]; m < g.c1[b]; ++m) g.cover[(size_t)l * nt + m] = b;
        for (int m = g.r0[b]; m < g.r1[b]; ++m) g.cover[(size_t)l * nt + m] = ~b;
    }
    return true;
}

}  // namespace hn
