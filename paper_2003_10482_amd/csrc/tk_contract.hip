// Host side of the packed contraction: work plans, grid sizes, launch
// dispatch, and the final fixed-order reduction of the per-workgroup column
// sums.  The pass kernels themselves are in tk_pass.hpp, instantiated per
// accumulation mode in tk_pass_{dd,f64,f32}.hip.
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tk_common.hpp"
#include "tk_contract.hpp"
#include "tk_host.hpp"

namespace tk {

// Final pass: g[b][l] = sum over passes and workgroups of the partials, in a
// fixed order (compensated).  A block of 1024 threads takes 8 columns of one
// vector: 128 slots per column, each with four independent compensated
// chains (partials w, w + 128, w + 256, w + 384 of each stride of 512), so a
// per-vector partial count of a few thousand costs a few dependent load
// rounds; the slots then meet in a fixed tree.
__global__ void __launch_bounds__(1024) reduce_partials_kernel(ReduceParams p)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    constexpr int cols = 8, slots = 128;
    __shared__ double sh_hi[cols * slots], sh_lo[cols * slots];
    const int lane_col = threadIdx.x % cols;
    const int slot = threadIdx.x / cols;
    const int b = blockIdx.y;
    const int l = blockIdx.x * cols + lane_col;
    DD s4[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    if (l < p.n) {
        for (int ps = 0; ps < p.npass; ++ps) {
            const double *src = p.part[ps] + 2 * ((int64_t)b * p.groups[ps]) * p.n;
            const int G = p.groups[ps];
            for (int w0 = slot; w0 < G; w0 += 4 * slots) {
                d2 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int w = w0 + slots * u;
                    v[u] = w < G ? *reinterpret_cast<const d2 *>(src + 2 * ((int64_t)w * p.n + l)) : d2{0.0, 0.0};
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    double t, e;
                    two_sum(s4[u].hi, v[u][0], t, e);
                    s4[u].hi = t;
                    s4[u].lo += e + v[u][1];
                }
            }
        }
    }
    const DD s = dd_add(dd_add(s4[0], s4[1]), dd_add(s4[2], s4[3]));
    sh_hi[threadIdx.x] = s.hi;
    sh_lo[threadIdx.x] = s.lo;
    __syncthreads();
    for (int stride = slots / 2; stride >= 1; stride >>= 1) {
        if (slot < stride) {
            DD a{sh_hi[threadIdx.x], sh_lo[threadIdx.x]};
            DD c{sh_hi[threadIdx.x + stride * cols], sh_lo[threadIdx.x + stride * cols]};
            DD r = dd_add(a, c);
            sh_hi[threadIdx.x] = r.hi;
            sh_lo[threadIdx.x] = r.lo;
        }
        __syncthreads();
    }
    if (slot == 0 && l < p.n) {
        const double v = sh_hi[threadIdx.x] + sh_lo[threadIdx.x];
        p.out[(int64_t)b * p.n + l] = v;
    }
}

// ------------------------------------------------------------ work plans ----
// (make_plan_host is in tk_host.cpp.)
namespace {
std::mutex g_plan_mu;
std::map<std::tuple<int, int, int64_t, int>, int64_t *> g_plans;
std::mutex g_hplan_mu;
std::map<std::tuple<int, int64_t, int>, std::vector<int64_t>> g_hplans;
}  // namespace

const std::vector<int64_t> &pass_plan_host(int q, int64_t n, int groups)
{
    // entries of the map are never erased or modified once made, so the
    // returned vector (and its data) stays valid for the life of the process
    std::lock_guard<std::mutex> lk(g_hplan_mu);
    const auto key = std::make_tuple(q, n, groups);
    auto it = g_hplans.find(key);
    if (it != g_hplans.end()) return it->second;
    return g_hplans.emplace(key, make_plan_host(q, n, (int64_t)groups * 4)).first->second;
}

const int64_t *pass_plan(int q, int64_t n, int groups, int *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = 1;
        return nullptr;
    }
    const auto key = std::make_tuple(dev, q, n, groups);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
    const std::vector<int64_t> &h = pass_plan_host(q, n, groups);
    int64_t *d = nullptr;
    if (hipMalloc((void **)&d, h.size() * sizeof(int64_t)) != hipSuccess ||
        hipMemcpy(d, h.data(), h.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
        *err = 1;
        return nullptr;
    }
    g_plans[key] = d;
    return d;
}

// Number of workgroups of one pass over an order-q array of `count` entries.
int pass_groups(int q, int64_t n, int64_t count, int resident, int64_t tiles)
{
    if (q == 2) {   // waves split the rows of the single unit: a few rows per wave
        int64_t g = (n + 15) / 16;
        return (int)(g < 1 ? 1 : g);
    }
    // at least about 4K entries per wave; the tiles of vectors (grid rows)
    // together fill the resident slots once
    int64_t g = (count + 4 * 4096 - 1) / (4 * 4096);
    // one tile of vectors: four rounds of the resident workgroups, so the
    // dispatcher evens out waves that run slower than their modelled share
    // (measured at n = 256, m = 4: compensated pass -15 %, directional
    // derivative -11 %, plain pass within noise); several tiles already give
    // the dispatcher that freedom (and four rounds slowed a tile of 8 by 10 %)
    int64_t cap = (tiles <= 1 ? 4 : 1) * (int64_t)resident / (tiles < 1 ? 1 : tiles);
    if (cap < 64) cap = 64;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

namespace {
std::mutex g_occ_mu;
std::map<std::tuple<int, int, int, int, int, int, int>, int> g_occ;
}  // namespace

int pass_resident(int q, int in_kind, int mode, int hv, int bt, int64_t n)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int nb = (int)((n + kWave - 1) / kWave);
    const auto key = std::make_tuple(dev, q, in_kind, mode, hv, bt, nb);
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        auto it = g_occ.find(key);
        if (it != g_occ.end()) return it->second;
    }
    PairParams pp{};
    int per_cu = 0;
    pp.n = (int)n;
    pp.B = bt;
    pp.occ_query = &per_cu;
    if (launch_pass(q, in_kind, mode, hv, bt, pp, 1, nullptr) != hipSuccess || per_cu <= 0) per_cu = 1;
    const int r = per_cu * cus;
    std::lock_guard<std::mutex> lk(g_occ_mu);
    g_occ[key] = r;
    return r;
}

hipError_t launch_pass(int q, int in_kind, int mode, int hv, int bt, const PairParams &pp,
                       int groups, hipStream_t st)
{
    // in_kind: 0 double, 1 float, 2 bf16, 3 DD intermediate;
    // hv: 0 value only, 1 tangent of alpha, 2 tangent of alpha and of the array
    if (mode == ACC_DD) return launch_pass_dd(q, in_kind, hv, bt, pp, groups, st);
    if (mode == ACC_PLAIN64) return launch_pass_f64(q, in_kind, hv, bt, pp, groups, st);
    if (mode == ACC_PLAIN32) return launch_pass_f32(q, in_kind, hv, bt, pp, groups, st);
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceParams &rp, int64_t B, hipStream_t st)
{
    dim3 grid((rp.n + 7) / 8, (unsigned)B);
    hipLaunchKernelGGL(reduce_partials_kernel, grid, dim3(1024), 0, st, rp);
    return hipGetLastError();
}

}  // namespace tk
