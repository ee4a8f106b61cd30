// Host-only planning and small dense linear algebra of the library: plain
// C++ (no HIP), so that it also builds and runs under the address and
// undefined-behaviour sanitizers on a machine without a GPU.
#pragma once

#include <cstdint>
#include <vector>

#include "tk_limits.hpp"

namespace tk {

// C(a, b) for 0 <= b <= 16, exact in int64 for every size the library accepts.
int64_t host_binom(int64_t a, int b);

// Balanced work plan of one contraction pass over an order-q array of n
// points: waves + 1 boundaries (units for q >= 4, rows for q == 2), cut so
// that every wave gets the same modelled cost.
std::vector<int64_t> make_plan_host(int q, int64_t n, int64_t waves);

// Work plan of the Hessian kernels for an order-m tensor over n points.
struct HostPlan {
    std::vector<int> tiles;         // [ntiles][2]
    std::vector<int> tile_items;    // [ntiles + 1]
    std::vector<int64_t> items;     // [nitems][3]
    std::vector<int64_t> rplan;     // [rwaves + 1]
    std::vector<int64_t> tab;       // [(n + kTB) * kTB]
    int64_t nq = 0;
    int xs = 0;
    int ntiles() const { return (int)tiles.size() / 2; }
    int nitems() const { return (int)items.size() / 3; }
    int rwaves() const { return rplan.empty() ? 0 : (int)rplan.size() - 1; }
};
HostPlan make_host_plan(int64_t n, int m);

// a . b over [k0, k1) with four independent partial sums.
double dot4(const double *a, const double *b, int k0, int k1);

// Inverse of a symmetric positive definite matrix (row-major, n x n) in
// place, through its Cholesky factor; false when a pivot is not positive.
bool spd_inverse(std::vector<double> &A, int n);

}  // namespace tk
