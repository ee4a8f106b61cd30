// Hessian J = (m-1) K . alpha^{m-2} of the contraction in two reads of the
// packed tensor, for the preconditioner of the dual solve.
//
// Grouping the packed tuples t = P ∪ {k, l} by their leading (m-2)-tuple P
// (a "unit": rows k = P_last .. n-1, entries l >= k, one contiguous
// triangle), the Hessian of the first dual term is the Hessian of
//     F(alpha) = sum_P N(P) alpha^P q_P(alpha),   q_P = 1/2 alpha^T S_P alpha,
// with N(P) = (m-2)!/prod(multiplicities) the orderings of P and S_P the
// symmetric matrix of the unit's triangle: S_kl = K_{P,k,l}, except the
// unit's first row (k = d = P_last, whose index repeats the run of rho equal
// values ending P), divided by rho+1 off the diagonal and scaled by
// 2/((rho+1)(rho+2)) on it.  (These are the multiplicity weights of the
// packed tuple, as in the contraction of Section 4.)  Then
//     H = sum_P N [ alpha^P S_P + grad(alpha^P) r_P^T + r_P grad(alpha^P)^T
//                   + q_P hess(alpha^P) ],        r_P = S_P alpha,
// and J = (m-1) H.  Three kernels:
//   tri   : U = sum_P N alpha^P S_P, the first term.  Output rows are cut into
//           tiles of <= kHessL upper-triangle entries; every unit that reaches
//           a tile contributes one contiguous chunk of its triangle, so the
//           kernel is a streaming weighted sum of chunks (one FMA per entry)
//           with lanes owning fixed tile positions;
//   unit  : r_P and q_P for every unit (a second streaming read);
//   cross : Y_x = sum_{P containing x} N d(alpha^P)/d alpha_x r_P plus half
//           the last term, row by row (sums over the units that contain x);
// and J = (m-1) (U + U^T - diag U + Y + Y^T) with fixed reduction orders, so
// the result is bitwise reproducible.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tk_hess.hpp"
#include "tk_host.hpp"

namespace tk {
namespace {


__host__ __device__ inline int64_t tri(int64_t L) { return L * (L + 1) / 2; }

template <typename TIn>
__device__ __forceinline__ double ldd(const TIn *p, int64_t i)
{
    return (double)Storage<TIn>::load(p, i);
}

// rank_tuple with the binomials read from a table (tab[a * kTB + b] = C(a, b)).
template <int Q>
__device__ __forceinline__ int64_t rank_tab(const int *t, int n, const int64_t *__restrict__ tab)
{
    int64_t r = 0;
    int lo = 0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const int rest = Q - p - 1;
        r += tab[(n - lo + rest) * kTB + rest + 1] - tab[(n - t[p] + rest) * kTB + rest + 1];
        lo = t[p];
    }
    return r;
}

// First entry of unit P in the packed array: rank of the m-tuple (P, d, d).
template <int MP>
__device__ __forceinline__ int64_t unit_offset(const int *P, int n, const int64_t *__restrict__ tab)
{
    int t[MP + 2];
    const int d = MP > 0 ? P[MP > 0 ? MP - 1 : 0] : 0;
#pragma unroll
    for (int i = 0; i < MP; ++i) t[i] = P[i];
    t[MP] = d;
    t[MP + 1] = d;
    return rank_tab<MP + 2>(t, n, tab);
}

// Lexicographic successor of a sorted tuple over [0, lim) (unchanged at the end).
template <int Q>
__device__ __forceinline__ void next_sorted(int *P, int lim)
{
    bool done = false;
#pragma unroll
    for (int p = Q - 1; p >= 0; --p) {
        if (!done && P[p] + 1 < lim) {
            const int v = P[p] + 1;
#pragma unroll
            for (int q = p; q < Q; ++q) P[q] = v;
            done = true;
        }
    }
}

// N(P) * alpha^P and the first-row weights of unit P.
template <int MP>
__device__ __forceinline__ void unit_coef(const int *P, const double *__restrict__ alpha, double &c, double &f1,
                                          double &f0)
{
    double prod = 1.0, den = 1.0, fact = 1.0;
    int run = 0;
#pragma unroll
    for (int i = 0; i < MP; ++i) {
        run = (i > 0 && P[i] == P[i - 1]) ? run + 1 : 1;
        den *= (double)run;
        fact *= (double)(i + 1);
        prod *= alpha[P[i]];
    }
    c = fact / den * prod;
    f1 = 1.0 / (double)(run + 1);
    f0 = 2.0 / (double)((run + 1) * (run + 2));
}

// ---------------------------------------------------------------- tile sums --
// Work item w: tile items[3w] (rows tiles[2t] .. tiles[2t+1]-1), units
// items[3w+1] .. items[3w+2]-1 in the lexicographic order of the sorted
// (m-2)-tuples over [0, k1) (the units whose triangles reach the tile).
template <int MP, typename TIn>
__global__ __launch_bounds__(256) void hess_tri_kernel(const TIn *__restrict__ K, const double *__restrict__ alpha,
                                                        int n, const int *__restrict__ tiles,
                                                        const int64_t *__restrict__ items, int nitems,
                                                        const int64_t *__restrict__ tab, double *__restrict__ part)
{
    const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int lane = threadIdx.x & 63;
    if (w >= nitems) return;
    const int t = (int)items[3 * w];
    const int64_t u0 = items[3 * w + 1], u1 = items[3 * w + 2];
    const int k0 = tiles[2 * t], k1 = tiles[2 * t + 1];
    const int L = (k1 - k0) * (2 * n - k0 - k1 + 1) / 2;
    int off[kHessJT];
#pragma unroll
    for (int j = 0; j < kHessJT; ++j) off[j] = min(lane + kWave * j, L - 1);
    double acc[kHessJT];
#pragma unroll
    for (int j = 0; j < kHessJT; ++j) acc[j] = 0.0;

    int P[MP > 0 ? MP : 1];
    unrank_tuple<MP>(u0, k1, P);
    int64_t uoff = unit_offset<MP>(P, n, tab);
    for (int64_t u = u0; u < u1; ++u) {
        const int d = MP > 0 ? P[MP > 0 ? MP - 1 : 0] : 0;
        double c, f1, f0;
        unit_coef<MP>(P, alpha, c, f1, f0);
        if (d < k0) {
            // every tile row is a regular row of this unit: one weight
            const TIn *src = K + uoff + (int64_t)(k0 - d) * (2 * n - d - k0 + 1) / 2;
            double v[kHessJT];
#pragma unroll
            for (int j = 0; j < kHessJT; ++j) v[j] = ldd(src, off[j]);
#pragma unroll
            for (int j = 0; j < kHessJT; ++j) acc[j] = fma(c, v[j], acc[j]);
        } else {
            // the unit starts inside the tile (k0 <= d < k1): positions before
            // its first row are skipped, the first row carries its weights
            const int s = (d - k0) * (2 * n - k0 - d + 1) / 2;
            const int rowend = s + (n - d);
            const TIn *src = K + uoff;
#pragma unroll
            for (int j = 0; j < kHessJT; ++j) {
                const int pos = lane + kWave * j;
                const bool valid = pos >= s && pos < L;
                const double v = ldd(src, valid ? pos - s : 0);
                const double wgt = pos == s ? f0 : (pos < rowend ? f1 : 1.0);
                acc[j] = fma(valid ? c * wgt : 0.0, v, acc[j]);
            }
        }
        if (MP == 0) break;
        if (d + 1 < k1) {   // the next unit follows this one in memory
            uoff += tri(n - d);
            P[MP > 0 ? MP - 1 : 0] = d + 1;
        } else {
            next_sorted<MP>(P, k1);
            uoff = unit_offset<MP>(P, n, tab);
        }
    }
    double *dst = part + (int64_t)w * kHessL;
#pragma unroll
    for (int j = 0; j < kHessJT; ++j) {
        const int pos = lane + kWave * j;
        if (pos < L) dst[pos] = acc[j];
    }
}

// U (packed upper triangle, row-major) = sum of the items' partial tiles in item order.
__global__ __launch_bounds__(256) void hess_tri_reduce(const double *__restrict__ part,
                                                        const int *__restrict__ tiles,
                                                        const int *__restrict__ tile_items, int n,
                                                        double *__restrict__ U)
{
    const int t = blockIdx.y;
    const int k0 = tiles[2 * t], k1 = tiles[2 * t + 1];
    const int L = (k1 - k0) * (2 * n - k0 - k1 + 1) / 2;
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= L) return;
    // eight independent partial sums keep eight loads in flight per thread
    // (the sum order is fixed, so the result stays reproducible)
    const int i0 = tile_items[t], i1 = tile_items[t + 1];
    double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = i0;
    for (; i + 8 <= i1; i += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += part[(int64_t)(i + u) * kHessL + pos];
#pragma unroll
    for (int u = 0; u < 7; ++u)
        if (i + u < i1) s8[u] += part[(int64_t)(i + u) * kHessL + pos];
    const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    U[(int64_t)k0 * (2 * n - k0 + 1) / 2 + pos] = s;
}

// ------------------------------------------------------------------ units --
// r_P = S_P alpha (n - d values per unit, stored at the unit's first row in
// the order of the sorted (m-1)-tuples) and q_P = alpha . r_P / 2, for the
// units plan[w] .. plan[w+1]-1.  Lanes own columns l = 64 b + lane; column
// sums stay in registers, row sums of 8 rows at a time come out of a
// transposed shuffle reduction.  One wave per workgroup.
template <int MP, typename TIn>
__global__ __launch_bounds__(64) void hess_unit_kernel(const TIn *__restrict__ K, const double *__restrict__ alpha,
                                                        int n, const int64_t *__restrict__ plan,
                                                        const int64_t *__restrict__ tab, double *__restrict__ R,
                                                        double *__restrict__ qv)
{
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t u0 = plan[w], u1 = plan[w + 1];
    __shared__ double rs[kMaxPoints];
    double aL[kMaxBlocks];
#pragma unroll
    for (int b = 0; b < kMaxBlocks; ++b) {
        const int l = kWave * b + lane;
        aL[b] = l < n ? alpha[l] : 0.0;
    }
    int P[MP > 0 ? MP : 1];
    unrank_tuple<MP>(u0, n, P);
    int64_t uoff = unit_offset<MP>(P, n, tab);
    int64_t rbase;
    {
        int t[MP + 1];
#pragma unroll
        for (int i = 0; i < MP; ++i) t[i] = P[i];
        t[MP] = MP > 0 ? P[MP > 0 ? MP - 1 : 0] : 0;
        rbase = rank_tab<MP + 1>(t, n, tab);
    }
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
    for (int64_t u = u0; u < u1; ++u) {
        const int d = MP > 0 ? P[MP > 0 ? MP - 1 : 0] : 0;
        double c, f1, f0;
        unit_coef<MP>(P, alpha, c, f1, f0);
        double col[kMaxBlocks];
#pragma unroll
        for (int b = 0; b < kMaxBlocks; ++b) col[b] = 0.0;
        int64_t roff = uoff;   // first entry of row kb
        for (int kb = d; kb < n; kb += 8) {
            // rows of the batch; rows past n repeat row n-1 with zero weight
            int64_t ro[8];
            int kk[8];
            double ak[8];
            {
                int64_t o = roff;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int k = kb + r;
                    kk[r] = k < n ? k : n - 1;
                    ro[r] = o;
                    if (k < n - 1) o += n - k;
                    ak[r] = k < n ? alpha[kk[r]] : 0.0;
                }
                roff = o;   // first entry of row kb + 8 when that row exists
            }
            double rp[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) rp[r] = 0.0;
            const int bmin = kb >> 6;
#pragma unroll
            for (int b = 0; b < kMaxBlocks; ++b) {
                if (b < bmin || kWave * b >= n) continue;
                const int l = kWave * b + lane;
                double v[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int pos = l - kk[r];
                    const int ix = pos < 0 ? 0 : (l < n ? pos : n - 1 - kk[r]);
                    v[r] = ldd(K + ro[r], ix);
                }
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int k = kb + r;
                    const int pos = l - k;
                    const bool valid = k < n && pos >= 0 && l < n;
                    const double wgt = k == d ? (pos == 0 ? f0 : f1) : 1.0;
                    const double vv = valid ? v[r] * wgt : 0.0;
                    rp[r] = fma(vv, aL[b], rp[r]);
                    col[b] = fma(pos > 0 ? vv : 0.0, ak[r], col[b]);
                }
            }
            // transposed reduction: lanes 8r..8r+7 end with the sum of row kb + r
            double s4[4], s2[2], s1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double send = h5 ? rp[i] : rp[i + 4];
                const double keep = h5 ? rp[i + 4] : rp[i];
                s4[i] = keep + __shfl_xor(send, 32);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const double send = h4 ? s4[i] : s4[i + 2];
                const double keep = h4 ? s4[i + 2] : s4[i];
                s2[i] = keep + __shfl_xor(send, 16);
            }
            {
                const double send = h3 ? s2[0] : s2[1];
                const double keep = h3 ? s2[1] : s2[0];
                s1 = keep + __shfl_xor(send, 8);
            }
            s1 += __shfl_xor(s1, 4);
            s1 += __shfl_xor(s1, 2);
            s1 += __shfl_xor(s1, 1);
            if ((lane & 7) == 0) {
                const int k = kb + (lane >> 3);
                if (k < n) rs[k] = s1;
            }
        }
        __syncthreads();
        double qa = 0.0;
#pragma unroll
        for (int b = 0; b < kMaxBlocks; ++b) {
            const int l = kWave * b + lane;
            if (l >= d && l < n) {
                const double rv = col[b] + rs[l];
                R[rbase + (l - d)] = rv;
                qa = fma(rv, aL[b], qa);
            }
        }
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1) qa += __shfl_xor(qa, sh);
        if (lane == 0) qv[u] = 0.5 * qa;
        __syncthreads();
        if (MP == 0) break;
        uoff += tri(n - d);   // units are contiguous in lexicographic order
        rbase += n - d;
        next_sorted<MP>(P, n);
    }
}

// ------------------------------------------------------------------ cross --
// Y[s][x][.] for the (m-3)-tuples Q (sorted, over [0, n)) numbered
// nq*s/S .. nq*(s+1)/S - 1: the unit P = Q ∪ {x} contributes
//     N(P) e_x alpha^Q r_P            (e_x: multiplicity of x in P)
// to row x, and half its share N q_P e_x e_y(Q) alpha^{Q-y} of the last term
// to column y of row x for every distinct y in Q.
template <int MP>
__global__ __launch_bounds__(64) void hess_cross_kernel(const double *__restrict__ alpha, int n,
                                                         const double *__restrict__ R,
                                                         const double *__restrict__ qv,
                                                         const int64_t *__restrict__ tab, int64_t nq, int S,
                                                         double *__restrict__ Y)
{
    constexpr int MQ = MP - 1;
    const int s = blockIdx.x, x = blockIdx.y;
    const int lane = threadIdx.x;
    const int64_t q0 = nq * s / S, q1 = nq * (s + 1) / S;
    double acc[kMaxBlocks];
#pragma unroll
    for (int b = 0; b < kMaxBlocks; ++b) acc[b] = 0.0;
    int Q[MQ];
    unrank_tuple<MQ>(q0, n, Q);
    for (int64_t qi = q0; qi < q1; ++qi) {
        int pos = 0, ex = 1;
#pragma unroll
        for (int i = 0; i < MQ; ++i) {
            pos += Q[i] <= x;
            ex += Q[i] == x;
        }
        int P[MP + 1];
#pragma unroll
        for (int p = 0; p < MP; ++p)
            P[p] = p < pos ? Q[p < MQ ? p : MQ - 1] : (p == pos ? x : Q[p > 0 ? p - 1 : 0]);
        double den = 1.0, fact = 1.0, aQ = 1.0;
        int run = 0;
#pragma unroll
        for (int i = 0; i < MP; ++i) {
            run = (i > 0 && P[i] == P[i - 1]) ? run + 1 : 1;
            den *= (double)run;
            fact *= (double)(i + 1);
        }
#pragma unroll
        for (int i = 0; i < MQ; ++i) aQ *= alpha[Q[i]];
        const double N = fact / den;
        const int d = P[MP - 1];
        const int64_t u = rank_tab<MP>(P, n, tab);
        P[MP] = d;
        const int64_t rbase = rank_tab<MP + 1>(P, n, tab);
        const double coef = N * (double)ex * aQ;
#pragma unroll
        for (int b = 0; b < kMaxBlocks; ++b) {
            if (kWave * b >= n) continue;
            const int l = kWave * b + lane;
            const bool valid = l >= d && l < n;
            acc[b] = fma(valid ? coef : 0.0, R[rbase + (valid ? l - d : 0)], acc[b]);
        }
        const double qu = qv[u];
#pragma unroll
        for (int i = 0; i < MQ; ++i) {
            if (i > 0 && Q[i] == Q[i - 1]) continue;
            const int y = Q[i];
            int ey = 0;
            double prod = 1.0;
#pragma unroll
            for (int j = 0; j < MQ; ++j) {
                ey += Q[j] == y;
                if (j != i) prod *= alpha[Q[j]];
            }
            const double c2 = 0.5 * N * qu * (double)ex * (double)ey * prod;
#pragma unroll
            for (int b = 0; b < kMaxBlocks; ++b) acc[b] += (kWave * b + lane == y) ? c2 : 0.0;
        }
        next_sorted<MQ>(Q, n);
    }
#pragma unroll
    for (int b = 0; b < kMaxBlocks; ++b) {
        const int l = kWave * b + lane;
        if (l < n) Y[((int64_t)s * n + x) * n + l] = acc[b];
    }
}

// J = scale * (U_sym + sum_s (Y_s + Y_s^T)).
__global__ __launch_bounds__(256) void hess_combine(const double *__restrict__ U, const double *__restrict__ Y,
                                                     int S, int n, double scale, double *__restrict__ J)
{
    const int i = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int a = i < j ? i : j, b = i < j ? j : i;
    double v = U[(int64_t)a * (2 * n - a + 1) / 2 + (b - a)];
    for (int s = 0; s < S; ++s)
        v += Y[((int64_t)s * n + i) * n + j] + Y[((int64_t)s * n + j) * n + i];
    J[(int64_t)i * n + j] = scale * v;
}

// ------------------------------------------------------------------- plans --
// (HostPlan and make_host_plan are in tk_host.cpp.)
std::mutex g_hess_mu;
std::map<std::tuple<int64_t, int>, HostPlan> g_host_plans;

const HostPlan &host_plan(int64_t n, int m)
{
    std::lock_guard<std::mutex> lk(g_hess_mu);
    const auto key = std::make_tuple(n, m);
    auto it = g_host_plans.find(key);
    if (it == g_host_plans.end()) it = g_host_plans.emplace(key, make_host_plan(n, m)).first;
    return it->second;
}

struct DevPlan {
    int *tiles = nullptr, *tile_items = nullptr;
    int64_t *items = nullptr, *rplan = nullptr, *tab = nullptr;
};
std::map<std::tuple<int, int64_t, int>, DevPlan> g_dev_plans;

template <typename T>
bool upload(T **dst, const std::vector<T> &src)
{
    if (src.empty()) return true;
    if (hipMalloc((void **)dst, src.size() * sizeof(T)) != hipSuccess) return false;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

const DevPlan *dev_plan(int64_t n, int m, const HostPlan &h)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_hess_mu);
    const auto key = std::make_tuple(dev, n, m);
    auto it = g_dev_plans.find(key);
    if (it != g_dev_plans.end()) return &it->second;
    DevPlan d;
    if (!upload(&d.tiles, h.tiles) || !upload(&d.tile_items, h.tile_items) || !upload(&d.items, h.items) ||
        !upload(&d.rplan, h.rplan) || !upload(&d.tab, h.tab))
        return nullptr;
    return &(g_dev_plans[key] = d);
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct HessBuffers {
    double *U, *part, *R, *q, *Y;
};

size_t carve_ws(int64_t n, int m, const HostPlan &h, void *work, HessBuffers *b)
{
    const int MP = m - 2;
    size_t sz[5] = {al256((size_t)tri(n) * 8), al256((size_t)h.nitems() * kHessL * 8), 0, 0, 0};
    if (MP >= 2) {
        sz[2] = al256((size_t)packed_count(n, m - 1) * 8);
        sz[3] = al256((size_t)packed_count(n, m - 2) * 8);
        sz[4] = al256((size_t)h.xs * n * n * 8);
    }
    if (b) {
        unsigned char *w = reinterpret_cast<unsigned char *>(work);
        double **p[5] = {&b->U, &b->part, &b->R, &b->q, &b->Y};
        size_t used = 0;
        for (int i = 0; i < 5; ++i) {
            *p[i] = sz[i] ? reinterpret_cast<double *>(w + used) : nullptr;
            used += sz[i];
        }
    }
    return sz[0] + sz[1] + sz[2] + sz[3] + sz[4];
}

template <int MP, typename TIn>
hipError_t launch_mp(const TIn *K, int64_t n, const double *alpha, double *J, const HostPlan &h, const DevPlan &d,
                     const HessBuffers &b, hipStream_t st)
{
    const int ni = h.nitems();
    const double tensor_bytes = (double)packed_count(n, MP + 2) * (double)sizeof(TIn);
    TimedLaunch tl = timing_begin(3, tensor_bytes, st);
    hess_tri_kernel<MP, TIn><<<(ni + 3) / 4, 256, 0, st>>>(K, alpha, (int)n, d.tiles, d.items, ni, d.tab, b.part);
    timing_end(tl, st);
    hess_tri_reduce<<<dim3(kHessL / 256, h.ntiles()), 256, 0, st>>>(b.part, d.tiles, d.tile_items, (int)n, b.U);
    int S = 0;
    if constexpr (MP >= 2) {
        tl = timing_begin(4, tensor_bytes, st);
        hess_unit_kernel<MP, TIn><<<h.rwaves(), 64, 0, st>>>(K, alpha, (int)n, d.rplan, d.tab, b.R, b.q);
        timing_end(tl, st);
        hess_cross_kernel<MP><<<dim3(h.xs, (unsigned)n), 64, 0, st>>>(alpha, (int)n, b.R, b.q, d.tab, h.nq, h.xs,
                                                                      b.Y);
        S = h.xs;
    }
    hess_combine<<<dim3((unsigned)((n + 255) / 256), (unsigned)n), 256, 0, st>>>(b.U, b.Y, S, (int)n,
                                                                                  (double)(MP + 1), J);
    return hipGetLastError();
}

template <typename TIn>
hipError_t launch_t(const TIn *K, int64_t n, int m, const double *alpha, double *J, const HostPlan &h,
                    const DevPlan &d, const HessBuffers &b, hipStream_t st)
{
    switch (m) {
    case 2: return launch_mp<0, TIn>(K, n, alpha, J, h, d, b, st);
    case 4: return launch_mp<2, TIn>(K, n, alpha, J, h, d, b, st);
    case 6: return launch_mp<4, TIn>(K, n, alpha, J, h, d, b, st);
    case 8: return launch_mp<6, TIn>(K, n, alpha, J, h, d, b, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t hessian_ws(int64_t n, int m)
{
    return carve_ws(n, m, host_plan(n, m), nullptr, nullptr);
}

int run_hessian(const void *K, int dtype, int64_t n, int m, const double *alpha, double *J, void *work,
                size_t work_bytes, hipStream_t st, int *passes)
{
    const HostPlan &h = host_plan(n, m);
    HessBuffers b{};
    const size_t need = carve_ws(n, m, h, work, &b);
    if (work_bytes < need)
        return fail(TK_ENOMEM, "Hessian workspace of %zu bytes, %zu needed", work_bytes, need);
    const DevPlan *d = dev_plan(n, m, h);
    if (!d) return fail(TK_EHIP, "could not upload the Hessian work plan");
    hipError_t e;
    if (dtype == TK_F64)
        e = launch_t(static_cast<const double *>(K), n, m, alpha, J, h, *d, b, st);
    else if (dtype == TK_F32)
        e = launch_t(static_cast<const float *>(K), n, m, alpha, J, h, *d, b, st);
    else
        e = launch_t(static_cast<const uint16_t *>(K), n, m, alpha, J, h, *d, b, st);
    if (e != hipSuccess) return fail(TK_EHIP, "Hessian kernels: %s", hipGetErrorString(e));
    if (passes) *passes = m == 2 ? 1 : 2;
    return TK_OK;
}

}  // namespace tk
