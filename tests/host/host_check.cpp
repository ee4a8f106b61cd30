// Checks of the library's host-only planning and dense algebra (tk_host.cpp),
// built with the address and undefined-behaviour sanitizers by
// tests/test_host_sanitized.py.  Prints "ok" and returns 0 when every check
// holds; prints the failing check and returns 1 otherwise.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "tk_host.hpp"

using namespace tk;

static int failures = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            std::printf("FAIL %s: ", #cond);      \
            std::printf(__VA_ARGS__);             \
            std::printf("\n");                    \
            ++failures;                           \
        }                                         \
    } while (0)

static int64_t units_of(int q, int64_t n) { return q == 2 ? n : host_binom(n + (q - 2) - 1, q - 2); }

static void check_pass_plans()
{
    for (int q : {2, 4, 6, 8})
        for (int64_t n : {1, 2, 63, 64, 65, 128, 129, 192, 193, 256})
            for (int64_t waves : {1, 3, 64, 2048}) {
                if (q == 8 && n > 65) continue;
                const std::vector<int64_t> p = make_plan_host(q, n, waves);
                const int64_t units = units_of(q, n);
                CHECK((int64_t)p.size() == waves + 1, "q=%d n=%lld waves=%lld", q, (long long)n, (long long)waves);
                CHECK(p.front() == 0 && p.back() == units, "q=%d n=%lld ends", q, (long long)n);
                for (size_t i = 1; i < p.size(); ++i)
                    CHECK(p[i] >= p[i - 1] && p[i] <= units, "q=%d n=%lld monotone at %zu", q, (long long)n, i);
            }
}

static void check_hess_plans()
{
    for (int m : {2, 4, 6})
        for (int64_t n : {1, 2, 63, 64, 65, 128, 129, 192, 193, 256}) {
            if (m == 6 && n > 129) continue;
            const HostPlan h = make_host_plan(n, m);
            const int MP = m - 2;
            // row tiles partition [0, n) and hold at most kHessL upper-triangle entries
            int k = 0;
            for (int t = 0; t < h.ntiles(); ++t) {
                const int k0 = h.tiles[2 * t], k1 = h.tiles[2 * t + 1];
                CHECK(k0 == k && k1 > k0, "m=%d n=%lld tile %d", m, (long long)n, t);
                int64_t L = 0;
                for (int r = k0; r < k1; ++r) L += n - r;
                CHECK(L <= kHessL, "m=%d n=%lld tile %d size", m, (long long)n, t);
                k = k1;
                // the tile's items cover the units ending at or below its last row, in order
                const int64_t units = MP == 0 ? 1 : host_binom(k1 + MP - 1, MP);
                int64_t u = 0;
                for (int it = h.tile_items[t]; it < h.tile_items[t + 1]; ++it) {
                    CHECK(h.items[3 * it] == t && h.items[3 * it + 1] == u && h.items[3 * it + 2] > u,
                          "m=%d n=%lld item %d", m, (long long)n, it);
                    u = h.items[3 * it + 2];
                }
                CHECK(u == units, "m=%d n=%lld tile %d units", m, (long long)n, t);
            }
            CHECK(k == n, "m=%d n=%lld tiles end", m, (long long)n);
            CHECK((int64_t)h.tab.size() == (n + kTB) * kTB, "m=%d table", m);
            if (MP >= 2) {
                CHECK(h.rplan.front() == 0 && h.rplan.back() == host_binom(n + MP - 1, MP), "m=%d rplan ends", m);
                for (size_t i = 1; i < h.rplan.size(); ++i) CHECK(h.rplan[i] > h.rplan[i - 1], "m=%d rplan", m);
                CHECK(h.xs >= 1 && h.nq == host_binom(n + MP - 2, MP - 1), "m=%d cross plan", m);
            }
        }
}

static void check_spd_inverse()
{
    std::mt19937_64 rng(7);
    std::normal_distribution<double> N(0.0, 1.0);
    for (int n : {1, 2, 3, 5, 64, 65, 257}) {
        // A = G G^T + n I: symmetric positive definite, condition number modest
        std::vector<double> G((size_t)n * n), A((size_t)n * n);
        for (double &g : G) g = N(rng);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = (i == j) ? n : 0.0;
                for (int k = 0; k < n; ++k) s += G[(size_t)i * n + k] * G[(size_t)j * n + k];
                A[(size_t)i * n + j] = s;
            }
        std::vector<double> Ai = A;
        CHECK(spd_inverse(Ai, n), "n=%d spd", n);
        double err = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * Ai[(size_t)k * n + j];
                err = std::fmax(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
                CHECK(Ai[(size_t)i * n + j] == Ai[(size_t)j * n + i], "n=%d symmetric (%d,%d)", n, i, j);
            }
        CHECK(err < 1e-10, "n=%d |A A^-1 - I| = %g", n, err);
    }
    // indefinite and singular matrices are refused
    std::vector<double> B = {1.0, 2.0, 2.0, 1.0};
    CHECK(!spd_inverse(B, 2), "indefinite accepted");
    std::vector<double> Z = {1.0, 1.0, 1.0, 1.0};
    CHECK(!spd_inverse(Z, 2), "singular accepted");
    std::vector<double> Nn = {std::nan(""), 0.0, 0.0, 1.0};
    CHECK(!spd_inverse(Nn, 2), "NaN pivot accepted");
}

int main()
{
    check_pass_plans();
    check_hess_plans();
    check_spd_inverse();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
