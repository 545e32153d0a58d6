// Host check of the grid search (batched two-point probes from a
// uniform-grid guess) against std::lower_bound and std::upper_bound on
// uniform, jittered and strongly non-uniform grids, and of the batched
// predicate search against a plain scan.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "xrdvi_device.h"

int main() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long bad = 0, checks = 0;
    for (int g = 0; g < 300; ++g) {
        const int n = 1 + (int)(U(rng) * 3000);
        std::vector<double> x(n);
        const int kind = g % 3;
        double v = 10.0;
        for (int i = 0; i < n; ++i) {
            if (kind == 0) x[i] = 10.0 + i * 0.02;                        // uniform
            else if (kind == 1) x[i] = 10.0 + i * 0.02 + 0.004 * U(rng);  // jitter
            else { v += 1e-4 + std::pow(U(rng), 4.0); x[i] = v; }         // ragged
        }
        for (int i = 1; i < n; ++i)
            if (!(x[i] > x[i - 1])) x[i] = std::nextafter(x[i - 1], 1e300);
        const double x0 = x[0];
        const double inv = n > 1 ? (n - 1) / (x[n - 1] - x[0]) : 0.0;
        for (int q = 0; q < 400; ++q) {
            double val;
            const double r = U(rng);
            if (r < 0.3) val = x[(size_t)(U(rng) * n) % n];               // on a point
            else if (r < 0.95) val = x[0] - 1.0 + (x[n - 1] - x[0] + 2.0) * U(rng);
            else if (r < 0.97) val = std::numeric_limits<double>::infinity();
            else if (r < 0.99) val = -std::numeric_limits<double>::infinity();
            else val = std::nan("");
            const int2 pr = xrdvi::grid_range(x.data(), n, x0, inv, val, val);
            int rlo = (int)(std::lower_bound(x.begin(), x.end(), val) - x.begin());
            int rhi = (int)(std::upper_bound(x.begin(), x.end(), val) - x.begin());
            // NaN compares false with everything: both bounds are 0 (the
            // window plan then gives an empty window)
            if (std::isnan(val)) rlo = rhi = 0;
            checks += 2;
            if (pr.x != rlo || pr.y != rhi) {
                if (bad < 5) std::printf("n=%d kind=%d v=%.17g: %d %d vs %d %d\n", n, kind, val, pr.x, pr.y, rlo, rhi);
                ++bad;
            }
        }
    }
    // batched searches of a monotone predicate from any probe position (the
    // tile plan's searches over peak positions) against a plain scan
    for (int g = 0; g < 2000; ++g) {
        const int n = (int)(U(rng) * 200);
        std::vector<double> p(n);
        double v = 0.0;
        for (int j = 0; j < n; ++j) { v += (U(rng) < 0.1) ? 0.0 : U(rng); p[j] = v; }
        const int a = n ? (int)(U(rng) * n) : 0;
        const int b = a + (int)(U(rng) * (n - a + 1));
        for (int q = 0; q < 20; ++q) {
            const double key = -1.0 + (v + 2.0) * U(rng);
            const int j0 = -5 + (int)(U(rng) * (n + 10));
            auto pred = [&](double pv) { return pv >= key; };
            int ref = a;
            while (ref < b && !pred(p[ref])) ++ref;
            const double *pp = n ? p.data() : &key;
            const int got4 = xrdvi::probe_result(pp, a, b, xrdvi::probe_at<4>(pp, a, b, j0), pred);
            const int got2 = xrdvi::probe_result(pp, a, b, xrdvi::probe_at<2>(pp, a, b, j0), pred);
            checks += 2;
            if (got4 != ref || got2 != ref) {
                if (bad < 5) std::printf("n=%d [%d,%d) j0=%d: %d %d vs %d\n", n, a, b, j0, got4, got2, ref);
                ++bad;
            }
        }
    }
    std::printf("%ld checks, %ld mismatches\n", checks, bad);
    return bad != 0;
}
