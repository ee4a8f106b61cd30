// Host-only planning and small dense linear algebra (see tk_host.hpp).
#include "tk_host.hpp"

#include <algorithm>
#include <cmath>

namespace tk {

int64_t host_binom(int64_t a, int b)
{
    if (b < 0 || a < b) return 0;
    int64_t c = 1;
    for (int i = 1; i <= b; ++i) c = c * (a - b + i) / i;   // C(a-b+i, i), exact at every step
    return c;
}

namespace {
// Modelled cost of one row (fixed part plus one term per 64-column block it
// touches) and of one unit (fixed part).  The weights approximate the
// instruction counts of the kernel; only their ratios matter.
constexpr double kCostRow = 6.0, kCostBlock = 8.0, kCostBatch = 4.0, kCostUnit = 60.0;

}  // namespace

std::vector<int64_t> make_plan_host(int q, int64_t n, int64_t waves)
{
    const int nb = (int)((n + kWave - 1) / kWave);
    // cost of the rows k in [k0, n) of a unit whose leading indices end at k0
    std::vector<double> tail(n + 1, 0.0);
    for (int64_t k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + kCostRow + kCostBlock * (nb - (k >> 6));
    std::vector<int64_t> plan(waves + 1, 0);
    if (q == 2) {
        double total = tail[0];
        int64_t w = 1;
        double acc = 0.0;
        for (int64_t k = 0; k < n && w < waves; ++k) {
            acc += kCostRow + kCostBlock * (nb - (k >> 6));
            while (w < waves && acc >= total * (double)w / (double)waves) plan[w++] = k + 1;
        }
        while (w <= waves) plan[w++] = n;
        plan[waves] = n;
        return plan;
    }
    const int qp = q - 2;
    auto unit_cost = [&](int k0) {
        const double rows = (double)(n - k0);
        return tail[k0] + kCostBatch * std::ceil(rows / 4.0) + kCostUnit;
    };
    // units in nested-loop order; only the last index matters for the cost
    std::vector<int> t(qp, 0);
    double total = 0.0;
    int64_t units = 0;
    while (true) {
        total += unit_cost(t[qp - 1]);
        ++units;
        int pos = qp - 1;
        while (pos >= 0 && t[pos] == n - 1) --pos;
        if (pos < 0) break;
        t[pos] += 1;
        for (int i = pos + 1; i < qp; ++i) t[i] = t[pos];
    }
    std::fill(t.begin(), t.end(), 0);
    int64_t w = 1, u = 0;
    double acc = 0.0;
    while (u < units && w < waves) {
        acc += unit_cost(t[qp - 1]);
        ++u;
        while (w < waves && acc >= total * (double)w / (double)waves) plan[w++] = u;
        int pos = qp - 1;
        while (pos >= 0 && t[pos] == n - 1) --pos;
        if (pos < 0) break;
        t[pos] += 1;
        for (int i = pos + 1; i < qp; ++i) t[i] = t[pos];
    }
    while (w <= waves) plan[w++] = units;
    plan[waves] = units;
    return plan;
}


HostPlan make_host_plan(int64_t n, int m)
{
    HostPlan h;
    const int MP = m - 2;
    const int nb = (int)((n + kWave - 1) / kWave);
    // row tiles of at most kHessL upper-triangle entries
    std::vector<int64_t> work;
    double wtot = 0;
    for (int k = 0; k < n;) {
        const int k0 = k;
        int64_t L = 0;
        while (k < n && L + (n - k) <= kHessL) L += n - k++;
        h.tiles.push_back(k0);
        h.tiles.push_back(k);
        const int64_t units = MP == 0 ? 1 : host_binom(k + MP - 1, MP);
        work.push_back(units * ((L + kWave - 1) / kWave + 6));
        wtot += (double)work.back();
    }
    h.tile_items.push_back(0);
    for (int t = 0; t < h.ntiles(); ++t) {
        const int k1 = h.tiles[2 * t + 1];
        const int64_t units = MP == 0 ? 1 : host_binom(k1 + MP - 1, MP);
        int64_t it = (int64_t)std::llround((double)work[t] / wtot * kHessItems);
        it = std::max<int64_t>(1, std::min(it, units));
        const int64_t chunk = (units + it - 1) / it;
        for (int64_t u = 0; u < units; u += chunk) {
            h.items.push_back(t);
            h.items.push_back(u);
            h.items.push_back(std::min(units, u + chunk));
        }
        h.tile_items.push_back(h.nitems());
    }
    h.tab.assign((size_t)(n + kTB) * kTB, 0);
    for (int64_t a = 0; a < n + kTB; ++a)
        for (int b = 0; b < kTB; ++b) h.tab[(size_t)a * kTB + b] = host_binom(a, b);
    if (MP >= 2) {
        // unit plan balanced on modelled cost: per batch of 8 rows, the
        // loads of the column blocks it touches plus the reduction
        std::vector<double> cost_d(n);
        for (int d = 0; d < n; ++d) {
            double c = 16.0;
            for (int kb = d; kb < n; kb += 8) c += 8.0 * (nb - (kb >> 6)) + 12.0;
            cost_d[d] = c;
        }
        const int64_t units = host_binom(n + MP - 1, MP);
        double total = 0;   // units ending in d: C(d + MP - 1, MP - 1)
        for (int d = 0; d < n; ++d) total += cost_d[d] * (double)host_binom(d + MP - 1, MP - 1);
        const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(kHessRWaves, units));
        h.rplan.push_back(0);
        std::vector<int> P(MP, 0);
        double cum = 0;
        int64_t w = 1;
        for (int64_t u = 0; u < units && w < waves; ++u) {
            // cut before unit u once the units before it reach the next share
            if (cum >= total * (double)w / (double)waves && u > h.rplan.back()) {
                h.rplan.push_back(u);
                ++w;
            }
            cum += cost_d[P[MP - 1]];
            int p = MP - 1;
            while (p >= 0 && P[p] + 1 >= n) --p;
            if (p >= 0) {
                const int v = P[p] + 1;
                for (int q = p; q < MP; ++q) P[q] = v;
            }
        }
        h.rplan.push_back(units);
        h.nq = host_binom(n + MP - 2, MP - 1);
        const int64_t xs = (kHessXWaves + n - 1) / n;
        h.xs = (int)std::max<int64_t>(1, std::min<int64_t>(xs, h.nq));
    }
    return h;
}


// a . b over [k0, k1) with four independent partial sums (the host compiler
// may not reassociate a single chain; four chains keep its FP units busy)
double dot4(const double *a, const double *b, int k0, int k1)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = k0;
    for (; k + 3 < k1; k += 4) {
        s0 += a[k] * b[k];
        s1 += a[k + 1] * b[k + 1];
        s2 += a[k + 2] * b[k + 2];
        s3 += a[k + 3] * b[k + 3];
    }
    for (; k < k1; ++k) s0 += a[k] * b[k];
    return (s0 + s1) + (s2 + s3);
}

// Inverse of a symmetric positive definite matrix (row-major, n x n) through
// its Cholesky factor A = L L^T: W = L^{-1} by forward substitution, then
// A^{-1} = W^T W.  Returns false when a pivot is not positive.
bool spd_inverse(std::vector<double> &A, int n)
{
    std::vector<double> L((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        const double *Lj = &L[(size_t)j * n];
        const double d = A[(size_t)j * n + j] - dot4(Lj, Lj, 0, j);
        if (!(d > 0) || !std::isfinite(d)) return false;
        const double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            const double *Li = &L[(size_t)i * n];
            L[(size_t)i * n + j] = (A[(size_t)i * n + j] - dot4(Li, Lj, 0, j)) / ljj;
        }
    }
    // column c of W: W[c][c] = 1/L[c][c], W[i][c] = -(sum_{c<=k<i} L[i][k] W[k][c]) / L[i][i];
    // kept transposed (Wt[c][i] = W[i][c]) so the inner sums run over contiguous memory
    std::vector<double> Wt((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        double *wc = &Wt[(size_t)c * n];
        wc[c] = 1.0 / L[(size_t)c * n + c];
        for (int i = c + 1; i < n; ++i) {
            const double *Li = &L[(size_t)i * n];
            wc[i] = -dot4(Li, wc, c, i) / Li[i];
        }
    }
    // (W^T W)[r][c] = sum_{k >= max(r,c)} W[k][r] W[k][c] = Wt[r] . Wt[c] over k >= max(r, c)
    for (int r = 0; r < n; ++r)
        for (int c = 0; c <= r; ++c) {
            const double t = dot4(&Wt[(size_t)r * n], &Wt[(size_t)c * n], r, n);
            A[(size_t)r * n + c] = t;
            A[(size_t)c * n + r] = t;
        }
    return true;
}

}  // namespace tk
