// Host-side helper of the s-step GMRES basis: Leja-ordered shifts.
// Header-only, plain C++ (no HIP), so that the CPU tests can compile it on
// its own.
#pragma once

#include <cmath>
#include <vector>

namespace rich {

// Leja order of k of the n points pts: the first of largest modulus, each
// next one maximising the product of its distances to those already taken
// (as a sum of logarithms).  Writes min(k, n) points.
inline int leja_order(const double *pts, int n, int k, double *out) {
    if (k > n) k = n;
    if (k <= 0) return 0;
    std::vector<double> lsum(n, 0.0);
    std::vector<char> used(n, 0);
    int best = 0;
    for (int g = 1; g < n; g++)
        if (std::fabs(pts[g]) > std::fabs(pts[best])) best = g;
    for (int t = 0; t < k; t++) {
        if (t > 0) {
            best = -1;
            double bv = -INFINITY;
            for (int g = 0; g < n; g++) {
                if (used[g]) continue;
                lsum[g] += std::log(std::fabs(pts[g] - out[t - 1]) + 1e-300);
                if (best < 0 || lsum[g] > bv) {
                    bv = lsum[g];
                    best = g;
                }
            }
        }
        used[best] = 1;
        out[t] = pts[best];
    }
    return k;
}

// k Leja points of the interval [a, b], taken from a grid of 4097 points
// (the first at the end of larger modulus).  b <= a gives k copies of a.
inline void leja_points(double a, double b, int k, double *out) {
    constexpr int NPT = 4097;
    if (!(b > a)) {
        for (int t = 0; t < k; t++) out[t] = a;
        return;
    }
    std::vector<double> grid(NPT);
    for (int g = 0; g < NPT; g++) grid[g] = a + (b - a) * g / (NPT - 1);
    leja_order(grid.data(), NPT, k, out);
}

}  // namespace rich
