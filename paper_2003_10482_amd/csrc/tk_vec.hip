// Small batched FP64 vector kernels used by the dual solve (gfx950).  Every
// reduction is a fixed tree with compensated (double-double) partial sums, so
// the solver's scalars are reproducible and accurate to about 2^-100.
#include "tk_common.hpp"
#include <algorithm>

#include "tk_vec.hpp"

namespace tk {

namespace {

__device__ DD block_sum_dd(DD v, DD *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = dd_add(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    DD r = sh[0];
    __syncthreads();
    return r;
}

// grad_b = g_b + lam_b alpha_b - y_b ; stats_b = [alpha.g, alpha.alpha, y.alpha, grad.grad]
// (y_b = y + b * y_stride: one response shared by all problems, or one each)
__global__ void __launch_bounds__(256) grad_kernel(const double *__restrict__ g, const double *__restrict__ alpha,
                                                   const double *__restrict__ y, int64_t y_stride, Coefs lam,
                                                   double *__restrict__ grad, double *__restrict__ stats,
                                                   int64_t n)
{
    __shared__ DD sh[256];
    const int b = blockIdx.x;
    const double l = lam.c[b];
    DD s_ag{0, 0}, s_aa{0, 0}, s_ya{0, 0}, s_gg{0, 0};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        const double a = alpha[j], gv = g[j], yv = y[(int64_t)b * y_stride + i];
        // grad = g + lam a - y, formed with one rounding of the exact sum
        DD t{0, 0};
        dd_fma(t, l, a);
        DD u = dd_add(t, DD{gv, 0.0});
        u = dd_add(u, DD{-yv, 0.0});
        const double gr = u.hi + u.lo;
        grad[j] = gr;
        dd_fma(s_ag, a, gv);
        dd_fma(s_aa, a, a);
        dd_fma(s_ya, yv, a);
        dd_fma(s_gg, gr, gr);
    }
    DD r0 = block_sum_dd(s_ag, sh), r1 = block_sum_dd(s_aa, sh), r2 = block_sum_dd(s_ya, sh),
       r3 = block_sum_dd(s_gg, sh);
    if (threadIdx.x == 0) {
        stats[b * 4 + 0] = r0.hi + r0.lo;
        stats[b * 4 + 1] = r1.hi + r1.lo;
        stats[b * 4 + 2] = r2.hi + r2.lo;
        stats[b * 4 + 3] = r3.hi + r3.lo;
    }
}

// Logistic loss (the dual's separable term through the loss's Fenchel
// conjugate): with p = lam_b y_i alpha_i,
//   grad_b = g_b + y (log p - log(1 - p)),  hdiag_b = lam_b / (p (1 - p)),
//   stats_b = [alpha.g, alpha.alpha, S, grad.grad],  S = sum p log p + (1 - p) log(1 - p),
// so that D = alpha.g / m + S / lam_b; S = +inf when some p lies outside (0, 1).
__global__ void __launch_bounds__(256) grad_logistic_kernel(const double *__restrict__ g,
                                                            const double *__restrict__ alpha,
                                                            const double *__restrict__ y, int64_t y_stride,
                                                            Coefs lam, double *__restrict__ grad,
                                                            double *__restrict__ hdiag,
                                                            double *__restrict__ stats, int64_t n)
{
    __shared__ DD sh[256];
    const int b = blockIdx.x;
    const double l = lam.c[b];
    DD s_ag{0, 0}, s_aa{0, 0}, s_S{0, 0}, s_gg{0, 0};
    double outside = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        const double a = alpha[j], gv = g[j], yv = y[(int64_t)b * y_stride + i];
        const double p = l * yv * a;
        double gr, h, sv;
        if (p > 0.0 && p < 1.0) {
            const double lp = log(p), lq = log1p(-p);
            gr = gv + yv * (lp - lq);
            h = l / (p * (1.0 - p));
            sv = p * lp + (1.0 - p) * lq;
        } else {
            gr = gv;
            h = l;
            sv = 0.0;
            outside = 1.0;
        }
        grad[j] = gr;
        hdiag[j] = h;
        dd_fma(s_ag, a, gv);
        dd_fma(s_aa, a, a);
        s_S = dd_add(s_S, DD{sv, 0.0});
        dd_fma(s_gg, gr, gr);
    }
    DD r0 = block_sum_dd(s_ag, sh), r1 = block_sum_dd(s_aa, sh), r2 = block_sum_dd(s_S, sh),
       r3 = block_sum_dd(s_gg, sh), r4 = block_sum_dd(DD{outside, 0.0}, sh);
    if (threadIdx.x == 0) {
        stats[b * 4 + 0] = r0.hi + r0.lo;
        stats[b * 4 + 1] = r1.hi + r1.lo;
        stats[b * 4 + 2] = r4.hi > 0 ? INFINITY : r2.hi + r2.lo;
        stats[b * 4 + 3] = r3.hi + r3.lo;
    }
}

// Largest step t with lam_b y_i (alpha_i + t x_i) inside [0, 1] for every i
// (the logistic dual's domain): out_b = min over i of -p/dp (dp < 0) or
// (1 - p)/dp (dp > 0), +inf when no component moves.
__global__ void __launch_bounds__(256) step_cap_kernel(const double *__restrict__ alpha, const double *__restrict__ x,
                                                       const double *__restrict__ y, int64_t y_stride, Coefs lam,
                                                       double *__restrict__ out, int64_t n)
{
    __shared__ double sh[256];
    const int b = blockIdx.x;
    const double l = lam.c[b];
    double t = INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        const double yv = y[(int64_t)b * y_stride + i];
        const double p = l * yv * alpha[j], dp = l * yv * x[j];
        if (dp < 0) t = fmin(t, -p / dp);
        else if (dp > 0) t = fmin(t, (1.0 - p) / dp);
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = sh[0];
}

// alpha_b = y_b / (2 lam_b): the centre of the logistic dual's domain (p = 1/2)
__global__ void __launch_bounds__(256) logistic_start_kernel(const double *__restrict__ y, int64_t y_stride,
                                                             Coefs lam, double *__restrict__ alpha, int64_t n)
{
    const int b = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        alpha[(int64_t)b * n + i] = y[(int64_t)b * y_stride + i] / (2.0 * lam.c[b]);
}

// flag |= (y_i not in {-1, +1}) for the logistic loss's labels
__global__ void labels_kernel(const double *__restrict__ y, int64_t len, int *__restrict__ flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        if (!(y[i] == 1.0 || y[i] == -1.0)) atomicOr(flag, 1);
}

// count_b = number of j with cur[b][j] != prev[b][j]; then prev = cur
__global__ void __launch_bounds__(256) mask_diff_kernel(const uint8_t *__restrict__ cur, uint8_t *__restrict__ prev,
                                                        int64_t d, int *__restrict__ count)
{
    __shared__ int sh[256];
    const int b = blockIdx.x;
    int c = 0;
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
        const int64_t k = (int64_t)b * d + j;
        c += cur[k] != prev[k];
        prev[k] = cur[k];
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[b] = sh[0];
}

// out_b = x_b . y_b (both [B][n]; y_stride 0 broadcasts one vector)
__global__ void __launch_bounds__(256) dot_kernel(const double *__restrict__ x, const double *__restrict__ y,
                                                  int64_t y_stride, double *__restrict__ out, int64_t n)
{
    __shared__ DD sh[256];
    const int b = blockIdx.x;
    DD s{0, 0};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dd_fma(s, x[(int64_t)b * n + i], y[(int64_t)b * y_stride + i]);
    DD r = block_sum_dd(s, sh);
    if (threadIdx.x == 0) out[b] = r.hi + r.lo;
}

// z_b = a_b x_b + c_b y_b   (z may alias x or y)
__global__ void __launch_bounds__(256) lin2_kernel(const double *x, const double *y, Coefs a, Coefs c,
                                                   double *z, int64_t n)
{
    const int b = blockIdx.y;
    const double ab = a.c[b], cb = c.c[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        z[j] = __builtin_fma(ab, x[j], cb * y[j]);
    }
}

// Hd_b += lam_b d_b (or diag_b * d_b when diag is given) ; out_b = d_b . Hd_b
__global__ void __launch_bounds__(256) shift_dot_kernel(const double *__restrict__ dvec, double *__restrict__ hd,
                                                        Coefs lam, const double *__restrict__ diag,
                                                        double *__restrict__ out, int64_t n)
{
    __shared__ DD sh[256];
    const int b = blockIdx.x;
    DD s{0, 0};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        const double v = __builtin_fma(diag ? diag[j] : lam.c[b], dvec[j], hd[j]);
        hd[j] = v;
        dd_fma(s, dvec[j], v);
    }
    DD r = block_sum_dd(s, sh);
    if (threadIdx.x == 0) out[b] = r.hi + r.lo;
}

// x_b += a_b d_b ; r_b -= a_b Hd_b ; out_b = r_b . r_b
__global__ void __launch_bounds__(256) cg_update_kernel(double *__restrict__ x, double *__restrict__ r,
                                                        const double *__restrict__ dvec,
                                                        const double *__restrict__ hd, Coefs a,
                                                        double *__restrict__ out, int64_t n)
{
    __shared__ DD sh[256];
    const int b = blockIdx.x;
    const double ab = a.c[b];
    DD s{0, 0};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        x[j] = __builtin_fma(ab, dvec[j], x[j]);
        const double rv = __builtin_fma(-ab, hd[j], r[j]);
        r[j] = rv;
        dd_fma(s, rv, rv);
    }
    DD q = block_sum_dd(s, sh);
    if (threadIdx.x == 0) out[b] = q.hi + q.lo;
}

// elementwise v = u^(p) * s  (u, s [B][d] or broadcast), used by the dMSE gradient
__global__ void pow_mul_kernel(const double *__restrict__ u, const double *__restrict__ s, int p,
                               double *__restrict__ out, int64_t len)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
        double pw = 1.0;
        for (int e = 0; e < p; ++e) pw *= u[i];
        out[i] = pw * s[i];
    }
}

__global__ void sub_kernel(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ out,
                           int64_t len)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - b[i];
}

__global__ void nonfinite_kernel(const double *__restrict__ x, int64_t len, int *__restrict__ flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) atomicOr(flag, 1);
}

inline unsigned grid_for(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : g > 1024 ? 1024 : g);
}

// z_b = A_b x_b for symmetric row-major A_b [n][n]: one wave per output row,
// lanes over the row, a shuffle reduction at the end.
__global__ void __launch_bounds__(256) symv_kernel(const double *__restrict__ A, const double *__restrict__ x,
                                                   double *__restrict__ z, int n)
{
    const int b = blockIdx.y;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *Ar = A + ((int64_t)b * n + row) * n;
    const double *xb = x + (int64_t)b * n;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s = __builtin_fma(Ar[j], xb[j], s);
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) s += __shfl_xor(s, sh);
    if (lane == 0) z[(int64_t)b * n + row] = s;
}

// Sum over the 1024 threads of a workgroup (16 waves): shuffles, then the
// 16 wave sums through LDS in a fixed order; every thread returns the total.
__device__ __forceinline__ double block_sum1024(double v, double *sh16)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
    __syncthreads();   // sh16 free (previous readers done)
    if ((threadIdx.x & 63) == 0) sh16[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += sh16[w];
    return t;
}

// Preconditioned CG on (J_b + lam_b I) x = -grad_b, one problem per
// workgroup of 1024 threads: thread (q, i) = (t / 256, t % 256) sums the
// products of quarter q of the columns for component i (n <= 256), so that
// 16 waves stream each product's matrix and its dependent chains are a
// quarter long; every thread then holds component i of the vectors.  J_b and
// P_b symmetric [n][n] (P_b the preconditioner), read by columns so the loads
// of a step are coalesced.  Stops at ||r|| <= eta_b ||grad_b||, at
// non-positive curvature along the search direction, or after max_it steps;
// x_b = 0 and steps_b = 0 for inactive problems (act_b = 0).
__global__ void __launch_bounds__(1024) cg_dense_kernel(const double *__restrict__ J, const double *__restrict__ P,
                                                        const double *__restrict__ grad, Coefs lam,
                                                        const double *__restrict__ diag, Coefs eta,
                                                        Coefs act, int n, int max_it, double *__restrict__ x,
                                                        int *__restrict__ steps)
{
    __shared__ double sv[256];       // the vector of the next product (d, then r)
    __shared__ double part[4][256];  // the quarters' partial products
    __shared__ double sh16[16];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int i = t & 255, q = t >> 8;
    const bool in = i < n;
    const bool own = q == 0 && in;   // the thread that counts component i in the sums
    const double *Jb = J + (int64_t)b * n * n;
    const double *Pb = P + (int64_t)b * n * n;
    double *xb = x + (int64_t)b * n;
    if (!(act.c[b] > 0)) {
        if (own) xb[i] = 0.0;
        if (t == 0) steps[b] = 0;
        return;
    }
    const int qlen = (n + 3) / 4;
    const int j0 = q * qlen, j1 = (j0 + qlen) < n ? (j0 + qlen) : n;
    // the operator's diagonal shift: lam_b, or diag_b[i] (logistic loss)
    const double lb = diag ? (in ? diag[(int64_t)b * n + i] : 0.0) : lam.c[b];
    auto matvec = [&](const double *M, double v) -> double {   // (M v)_i, v_i given per thread
        __syncthreads();   // sv and part free
        if (q == 0) sv[i] = in ? v : 0.0;
        __syncthreads();
        // eight loads in flight per thread, four chains, fixed order
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (in) {
            int j = j0;
            for (; j + 8 <= j1; j += 8) {
                double m[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) m[u] = M[(int64_t)(j + u) * n + i];
                s0 = __builtin_fma(m[0], sv[j], s0);
                s1 = __builtin_fma(m[1], sv[j + 1], s1);
                s2 = __builtin_fma(m[2], sv[j + 2], s2);
                s3 = __builtin_fma(m[3], sv[j + 3], s3);
                s0 = __builtin_fma(m[4], sv[j + 4], s0);
                s1 = __builtin_fma(m[5], sv[j + 5], s1);
                s2 = __builtin_fma(m[6], sv[j + 6], s2);
                s3 = __builtin_fma(m[7], sv[j + 7], s3);
            }
            for (; j < j1; ++j) s0 = __builtin_fma(M[(int64_t)j * n + i], sv[j], s0);
        }
        part[q][i] = (s0 + s1) + (s2 + s3);
        __syncthreads();
        return (part[0][i] + part[1][i]) + (part[2][i] + part[3][i]);
    };
    const double gi = in ? grad[(int64_t)b * n + i] : 0.0;
    const double gn = sqrt(block_sum1024(own ? gi * gi : 0.0, sh16));
    double xi = 0.0, ri = -gi;
    double zi = matvec(Pb, ri);
    double rz = block_sum1024(own ? ri * zi : 0.0, sh16);
    double di = zi;
    int it = 0;
    if (gn > 0 && rz > 0) {
        for (; it < max_it; ++it) {
            const double hi = matvec(Jb, di) + lb * di;
            const double dhd = block_sum1024(own ? di * hi : 0.0, sh16);
            if (!(dhd > 0) || !isfinite(dhd)) break;   // no positive curvature along d
            const double a = rz / dhd;
            xi = __builtin_fma(a, di, xi);
            ri = __builtin_fma(-a, hi, ri);
            const double rr = block_sum1024(own ? ri * ri : 0.0, sh16);
            if (sqrt(rr) <= eta.c[b] * gn) {
                ++it;
                break;
            }
            zi = matvec(Pb, ri);
            const double rzn = block_sum1024(own ? ri * zi : 0.0, sh16);
            const double beta = rzn / rz;
            rz = rzn;
            di = __builtin_fma(beta, di, zi);
        }
    }
    if (own) xb[i] = xi;
    if (t == 0) steps[b] = it;
}

// z_b = g_b + t_b (a_b + t_b (c_b + t_b e_b)), a cubic in the step length.
__global__ void __launch_bounds__(256) poly3_kernel(const double *__restrict__ g, const double *__restrict__ a,
                                                    const double *__restrict__ c, const double *__restrict__ e,
                                                    Coefs t, double *__restrict__ z, int64_t n)
{
    const int b = blockIdx.y;
    const double tb = t.c[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = (int64_t)b * n + i;
        z[j] = g[j] + tb * (a[j] + tb * (c[j] + tb * e[j]));
    }
}

// Streaming read of `words` 16-byte words (instrumentation: the achievable
// HBM read rate of this device, measured beside the kernels that stream the
// packed tensor).  Each thread keeps eight independent non-temporal loads in
// flight; an integer sum of the loaded words per workgroup keeps them live.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---- Newton-Schulz inverse of a dense SPD matrix (preconditioner refresh)
// One workgroup sums n^2 entries in a fixed order: per-thread strided
// partial sums, then a tree over the 256 threads.
__device__ double block_sum_256(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// X = I / ||A||_F in two stages: kInitGroups workgroups each sum the squares
// of a contiguous slice of A = J + diag(d) into part[w]; every thread of the
// fill then adds the partial sums in the same fixed order.
constexpr int kInitGroups = 64;
__global__ void __launch_bounds__(256) ns_init_part_kernel(const double *__restrict__ J, double lam,
                                                           const double *__restrict__ diag, int n,
                                                           double *__restrict__ part)
{
    __shared__ double sh[256];
    const int64_t nn = (int64_t)n * n;
    const int64_t per = (nn + kInitGroups - 1) / kInitGroups;
    const int64_t k0 = blockIdx.x * per, k1 = (k0 + per) < nn ? (k0 + per) : nn;
    double f = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
        const int i = (int)(k / n), j = (int)(k % n);
        const double a = J[k] + (i == j ? (diag ? diag[i] : lam) : 0.0);
        f = __builtin_fma(a, a, f);
    }
    const double fs = block_sum_256(f, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = fs;
}

__global__ void __launch_bounds__(256) ns_init_fill_kernel(const double *__restrict__ part, int n,
                                                           double *__restrict__ X)
{
    double f = 0.0;
    for (int w = 0; w < kInitGroups; ++w) f += part[w];
    const double fro = sqrt(f);
    const double s = fro > 0.0 ? 1.0 / fro : 0.0;
    const int64_t nn = (int64_t)n * n;
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < nn; k += (int64_t)gridDim.x * 256)
        X[k] = (k / n == k % n) ? s : 0.0;
}

// ||I - T||_F^2 and ||J||_F^2 in two stages, each in a fixed order: 64
// workgroups each sum a contiguous slice of the n^2 entries into part[2 w],
// part[2 w + 1]; one workgroup then adds the 64 pairs.
constexpr int kResGroups = 64;
static_assert(kNsResidualDoubles == 2 + 2 * kResGroups, "residual scratch size");
static_assert(kNsResidualDoubles >= kInitGroups, "initial-norm scratch size");
__global__ void __launch_bounds__(256) ns_residual_part_kernel(const double *__restrict__ T,
                                                               const double *__restrict__ J, int n,
                                                               double *__restrict__ part)
{
    __shared__ double sh[256];
    const int64_t nn = (int64_t)n * n;
    const int64_t per = (nn + kResGroups - 1) / kResGroups;
    const int64_t k0 = blockIdx.x * per, k1 = (k0 + per) < nn ? (k0 + per) : nn;
    double r = 0.0, f = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
        const double e = (k / n == k % n ? 1.0 : 0.0) - T[k];
        r = __builtin_fma(e, e, r);
        f = __builtin_fma(J[k], J[k], f);
    }
    const double rs = block_sum_256(r, sh);
    const double fs = block_sum_256(f, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rs;
        part[2 * blockIdx.x + 1] = fs;
    }
}

__global__ void ns_residual_final_kernel(const double *__restrict__ part, double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double r = 0.0, f = 0.0;
    for (int w = 0; w < kResGroups; ++w) {
        r += part[2 * w];
        f += part[2 * w + 1];
    }
    out[0] = sqrt(r);
    out[1] = sqrt(f);
}

__global__ void __launch_bounds__(256) ns_symmetrize_kernel(const double *__restrict__ X, double *__restrict__ Xs,
                                                            int n)
{
    // the thread of entry (i, j), j >= i, averages the pair and writes both
    // (in place when Xs == X: no other thread touches the pair)
    const int64_t nn = (int64_t)n * n;
    for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < nn; k += (int64_t)gridDim.x * 256) {
        const int i = (int)(k / n), j = (int)(k % n);
        if (j < i) continue;
        const double v = 0.5 * (X[k] + X[(int64_t)j * n + i]);
        Xs[k] = v;
        Xs[(int64_t)j * n + i] = v;
    }
}

__global__ void __launch_bounds__(256) stream_read_kernel(const u32x4 *__restrict__ src, int64_t words,
                                                          uint64_t *__restrict__ sink)
{
    __shared__ uint64_t sh[256];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc = 0;
    for (; i + 7 * stride < words; i += 8 * stride) {
        u32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (uint64_t)(v[u].x ^ v[u].y) + (uint64_t)(v[u].z ^ v[u].w);
    }
    for (; i < words; i += stride) {
        const u32x4 a = src[i];
        acc += (uint64_t)(a.x ^ a.y ^ a.z ^ a.w);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = sh[0];
}

}  // namespace

hipError_t probe_stream_read(const void *src, int64_t words, uint64_t *sink, int groups, hipStream_t st)
{
    hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)groups), dim3(256), 0, st,
                       reinterpret_cast<const u32x4 *>(src), words, sink);
    return hipGetLastError();
}

hipError_t vec_grad(const double *g, const double *alpha, const double *y, const Coefs &lam,
                    double *grad, double *stats, int64_t B, int64_t n, hipStream_t st, int64_t y_stride)
{
    hipLaunchKernelGGL(grad_kernel, dim3((unsigned)B), dim3(256), 0, st, g, alpha, y, y_stride, lam, grad, stats, n);
    return hipGetLastError();
}
hipError_t vec_grad_logistic(const double *g, const double *alpha, const double *y, int64_t y_stride,
                             const Coefs &lam, double *grad, double *hdiag, double *stats, int64_t B, int64_t n,
                             hipStream_t st)
{
    hipLaunchKernelGGL(grad_logistic_kernel, dim3((unsigned)B), dim3(256), 0, st, g, alpha, y, y_stride, lam, grad,
                       hdiag, stats, n);
    return hipGetLastError();
}
hipError_t vec_step_cap(const double *alpha, const double *x, const double *y, int64_t y_stride, const Coefs &lam,
                        double *out, int64_t B, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(step_cap_kernel, dim3((unsigned)B), dim3(256), 0, st, alpha, x, y, y_stride, lam, out, n);
    return hipGetLastError();
}
hipError_t vec_logistic_start(const double *y, int64_t y_stride, const Coefs &lam, double *alpha, int64_t B,
                              int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(logistic_start_kernel, dim3(grid_for(n) > 8 ? 8 : grid_for(n), (unsigned)B), dim3(256), 0, st,
                       y, y_stride, lam, alpha, n);
    return hipGetLastError();
}
hipError_t vec_check_labels(const double *y, int64_t len, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(labels_kernel, dim3(grid_for(len)), dim3(256), 0, st, y, len, flag);
    return hipGetLastError();
}
hipError_t vec_mask_diff(const uint8_t *cur, uint8_t *prev, int64_t B, int64_t d, int *count, hipStream_t st)
{
    hipLaunchKernelGGL(mask_diff_kernel, dim3((unsigned)B), dim3(256), 0, st, cur, prev, d, count);
    return hipGetLastError();
}
hipError_t vec_dot(const double *x, const double *y, int64_t y_stride, double *out, int64_t B, int64_t n,
                   hipStream_t st)
{
    hipLaunchKernelGGL(dot_kernel, dim3((unsigned)B), dim3(256), 0, st, x, y, y_stride, out, n);
    return hipGetLastError();
}
hipError_t vec_lin2(const double *x, const double *y, const Coefs &a, const Coefs &c, double *z, int64_t B,
                    int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(lin2_kernel, dim3(grid_for(n) > 8 ? 8 : grid_for(n), (unsigned)B), dim3(256), 0, st, x, y,
                       a, c, z, n);
    return hipGetLastError();
}
hipError_t vec_shift_dot(const double *d, double *hd, const Coefs &lam, double *out, int64_t B, int64_t n,
                         hipStream_t st, const double *diag)
{
    hipLaunchKernelGGL(shift_dot_kernel, dim3((unsigned)B), dim3(256), 0, st, d, hd, lam, diag, out, n);
    return hipGetLastError();
}
hipError_t vec_cg_update(double *x, double *r, const double *d, const double *hd, const Coefs &a, double *out,
                         int64_t B, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(cg_update_kernel, dim3((unsigned)B), dim3(256), 0, st, x, r, d, hd, a, out, n);
    return hipGetLastError();
}
hipError_t vec_pow_mul(const double *u, const double *s, int p, double *out, int64_t len, hipStream_t st)
{
    hipLaunchKernelGGL(pow_mul_kernel, dim3(grid_for(len)), dim3(256), 0, st, u, s, p, out, len);
    return hipGetLastError();
}
hipError_t vec_sub(const double *a, const double *b, double *out, int64_t len, hipStream_t st)
{
    hipLaunchKernelGGL(sub_kernel, dim3(grid_for(len)), dim3(256), 0, st, a, b, out, len);
    return hipGetLastError();
}
hipError_t vec_nonfinite(const double *x, int64_t len, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(len)), dim3(256), 0, st, x, len, flag);
    return hipGetLastError();
}

hipError_t vec_symv(const double *A, const double *x, double *z, int64_t B, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(symv_kernel, dim3((unsigned)((n + 3) / 4), (unsigned)B), dim3(256), 0, st, A, x, z, (int)n);
    return hipGetLastError();
}

hipError_t vec_cg_dense(const double *J, const double *P, const double *grad, const Coefs &lam, const Coefs &eta,
                        const Coefs &act, int64_t B, int64_t n, int max_it, double *x, int *steps, hipStream_t st,
                        const double *diag)
{
    if (n > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cg_dense_kernel, dim3((unsigned)B), dim3(1024), 0, st, J, P, grad, lam, diag, eta, act, (int)n,
                       max_it, x, steps);
    return hipGetLastError();
}

hipError_t vec_poly3(const double *g, const double *a, const double *c, const double *e, const Coefs &t, double *z,
                     int64_t B, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(poly3_kernel, dim3(grid_for(n) > 8 ? 8 : grid_for(n), (unsigned)B), dim3(256), 0, st, g, a, c,
                       e, t, z, n);
    return hipGetLastError();
}

hipError_t ns_init(const double *J, double lam, const double *diag, double *X, int64_t n, double *part,
                   hipStream_t st)
{
    hipLaunchKernelGGL(ns_init_part_kernel, dim3(kInitGroups), dim3(256), 0, st, J, lam, diag, (int)n, part);
    const unsigned g = (unsigned)std::min<int64_t>(256, (n * n + 255) / 256);
    hipLaunchKernelGGL(ns_init_fill_kernel, dim3(g), dim3(256), 0, st, part, (int)n, X);
    return hipGetLastError();
}

hipError_t ns_residual(const double *T, const double *J, int64_t n, double *out, hipStream_t st)
{
    // out[0 .. 2) receives the norms; out[2 .. 2 + 2 kResGroups) holds the partial sums
    hipLaunchKernelGGL(ns_residual_part_kernel, dim3(kResGroups), dim3(256), 0, st, T, J, (int)n, out + 2);
    hipLaunchKernelGGL(ns_residual_final_kernel, dim3(1), dim3(64), 0, st, out + 2, out);
    return hipGetLastError();
}

hipError_t ns_symmetrize(const double *X, double *Xs, int64_t n, hipStream_t st)
{
    const unsigned g = (unsigned)std::min<int64_t>(256, (n * n + 255) / 256);
    hipLaunchKernelGGL(ns_symmetrize_kernel, dim3(g), dim3(256), 0, st, X, Xs, (int)n);
    return hipGetLastError();
}

}  // namespace tk
