// Prediction with a general tensor kernel (Section 4: the model evaluated
// through the kernel when the feature map has no finite form):
//
//   f_b(x) = sum_{sorted (m-1)-tuples T} c(T) alpha_b^T k(x_{T_1}, .., x_{T_{m-1}}, x),
//   c(T) = (m-1)! / prod_v (multiplicity of v in T)!,
//
// the expansion of sum over ordered (m-1)-tuples grouped by their sorted form.
// For the kernels of this library k = kappa(sum_j q_T[j] x[j]) with
// q_T = prod_{t in T} x_t (elementwise) and kappa the identity, a power or exp,
// so a tile of 64 tuples x 64 query points is a product of the (tuples x d)
// matrix Q with X_q^T, formed on FP64 MFMA exactly as in the packed build,
// followed by kappa and the weighted sum over the tile's tuples.  Workgroups
// own a range of tuple tiles and one tile of query points and write one
// partial per (range, vector, point); a second kernel sums the partials in a
// fixed order.
#include "tk_common.hpp"
#include "tk_dense.hpp"

namespace tk {

namespace {

constexpr int PR = 64;    // tuples per tile
constexpr int PC = 64;    // query points per tile
constexpr int PF = 32;    // features per LDS chunk
constexpr int kPredMaxB = 16;

typedef double v4d __attribute__((ext_vector_type(4)));

template <int MP>
__global__ void __launch_bounds__(256) predict_tile_kernel(const double *__restrict__ X, int n, int d,
                                                           const double *__restrict__ Xq, int N, int kernel,
                                                           double kparam, const double *__restrict__ alpha,
                                                           int B, int64_t tuples, int64_t tiles_per_group,
                                                           double *__restrict__ part)
{
    // one buffer holds the staged operands during the products and the kernel
    // values of the tile afterwards (both are PF x 65 + PF x 65 = 64 x 65 doubles)
    __shared__ double buf[PR * (PC + 1)];
    __shared__ double wts[kPredMaxB][PR];
    __shared__ int tup[PR][MP];
    __shared__ int live[PR];
    double(*qs)[PR + 1] = reinterpret_cast<double(*)[PR + 1]>(buf);
    double(*xs)[PC + 1] = reinterpret_cast<double(*)[PC + 1]>(buf + PF * (PR + 1));
    double(*vt)[PC + 1] = reinterpret_cast<double(*)[PC + 1]>(buf);

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
    const int li = lane & 15, lk = lane >> 4;
    const int q0 = blockIdx.y * PC;
    const int64_t ntiles = (tuples + PR - 1) / PR;
    const int64_t tile_lo = (int64_t)blockIdx.x * tiles_per_group;
    const int64_t tile_hi = tile_lo + tiles_per_group < ntiles ? tile_lo + tiles_per_group : ntiles;

    // thread t accumulates the pairs (vector b, point c) = idx / PC, idx % PC
    // for idx = t, t + 256, .. < B * PC
    double acc[kPredMaxB * PC / 256];
#pragma unroll
    for (int i = 0; i < kPredMaxB * PC / 256; ++i) acc[i] = 0.0;

    for (int64_t tile = tile_lo; tile < tile_hi; ++tile) {
        if (t < PR) {
            const int64_t r = tile * PR + t;
            int tt[MP];
            live[t] = r < tuples;
            if (r < tuples) {
                unrank_tuple<MP>(r, n, tt);
                // c(T) = (m-1)! / prod (run lengths)!
                double c = 1.0;
                int run = 1;
                for (int i = 1; i <= MP; ++i) c *= (double)i;
                for (int i = 1; i < MP; ++i) {
                    run = (tt[i] == tt[i - 1]) ? run + 1 : 1;
                    c /= (double)run;
                }
                for (int i = 0; i < MP; ++i) tup[t][i] = tt[i];
                for (int b = 0; b < B; ++b) {
                    double p = c;
                    for (int i = 0; i < MP; ++i) p *= alpha[(int64_t)b * n + tt[i]];
                    wts[b][t] = p;
                }
            } else {
                for (int i = 0; i < MP; ++i) tup[t][i] = 0;
                for (int b = 0; b < B; ++b) wts[b][t] = 0.0;
            }
        }
        __syncthreads();
        v4d c4[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) c4[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int f0 = 0; f0 < d; f0 += PF) {
            for (int i = t; i < PR * PF; i += 256) {
                const int r = i / PF, f = i % PF;
                double q = 0.0;
                if (f0 + f < d && live[r]) {
                    q = 1.0;
                    for (int p = 0; p < MP; ++p) q *= X[(int64_t)tup[r][p] * d + f0 + f];
                }
                qs[f][r] = q;
                const int c = q0 + r;
                xs[f][r] = (f0 + f < d && c < N) ? Xq[(int64_t)c * d + f0 + f] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < PF / 4; ++s) {
                const int f = 4 * s + lk;
                double a[2], bb[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = qs[f][wr + 16 * i + li];
#pragma unroll
                for (int j = 0; j < 2; ++j) bb[j] = xs[f][wc + 16 * j + li];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        c4[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], c4[i][j], 0, 0, 0);
            }
            __syncthreads();
        }
        // kernel values of the tile (lane holds rows wr + 16 i + 4 e + lk,
        // columns wc + 16 j + li)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    double v = c4[i][j][e];
                    if (kernel == TK_POLY) {
                        const int sdeg = (int)kparam;
                        double pw = 1.0;
                        for (int q = 0; q < sdeg; ++q) pw *= v;
                        v = pw;
                    } else if (kernel == TK_EXP) {
                        v = exp(v);
                    }
                    vt[wr + 16 * i + 4 * e + lk][wc + 16 * j + li] = v;
                }
        __syncthreads();
        // weighted sums over the tile's tuples, in tuple order
#pragma unroll
        for (int i = 0; i < kPredMaxB * PC / 256; ++i) {
            const int idx = t + 256 * i;
            if (idx < B * PC) {
                const int b = idx / PC, c = idx % PC;
                double s = acc[i];
                for (int r = 0; r < PR; ++r) s = __builtin_fma(wts[b][r], vt[r][c], s);
                acc[i] = s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kPredMaxB * PC / 256; ++i) {
        const int idx = t + 256 * i;
        if (idx < B * PC) {
            const int b = idx / PC, c = idx % PC;
            if (q0 + c < N) part[((int64_t)blockIdx.x * B + b) * N + q0 + c] = acc[i];
        }
    }
}

// f[b][q] = sum over groups of part[g][b][q], in group order
__global__ void predict_sum_kernel(const double *__restrict__ part, int64_t groups, int B, int N,
                                   double *__restrict__ f, int64_t f_stride)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * N) return;
    const int b = (int)(i / N), q = (int)(i % N);
    double s = 0.0;
    for (int64_t g = 0; g < groups; ++g) s += part[(g * B + b) * N + q];
    f[(int64_t)b * f_stride + q] = s;
}

template <int MP>
hipError_t launch_predict_mp(const double *X, int n, int d, const double *Xq, int N, int kernel, double kparam,
                             const double *alpha, int B, int64_t groups, int64_t tiles_per_group, int64_t tuples,
                             double *part, hipStream_t st)
{
    dim3 grid((unsigned)groups, (unsigned)((N + PC - 1) / PC));
    hipLaunchKernelGGL(predict_tile_kernel<MP>, grid, dim3(256), 0, st, X, n, d, Xq, N, kernel, kparam, alpha, B,
                       tuples, tiles_per_group, part);
    return hipGetLastError();
}

}  // namespace

int64_t predict_groups(int64_t n, int m, int64_t N)
{
    const int64_t tuples = packed_count(n, m - 1);
    const int64_t ntiles = (tuples + PR - 1) / PR;
    const int64_t qtiles = (N + PC - 1) / PC;
    int64_t g = 2048 / (qtiles < 1 ? 1 : qtiles);
    if (g < 1) g = 1;
    if (g > ntiles) g = ntiles;
    return g;
}

int predict_max_batch() { return kPredMaxB; }

hipError_t launch_predict_kernel(const double *X, int64_t n, int64_t d, int m, int kernel, double kparam,
                                 const double *alpha, int64_t B, const double *Xq, int64_t N, double *f,
                                 double *part, hipStream_t st)
{
    const int64_t tuples = packed_count(n, m - 1);
    const int64_t ntiles = (tuples + PR - 1) / PR;
    const int64_t groups = predict_groups(n, m, N);
    const int64_t tpg = (ntiles + groups - 1) / groups;
    for (int64_t b0 = 0; b0 < B; b0 += kPredMaxB) {
        const int nb = (int)((B - b0) < kPredMaxB ? (B - b0) : kPredMaxB);
        const double *a = alpha + b0 * n;
        hipError_t e;
        switch (m - 1) {
        case 1: e = launch_predict_mp<1>(X, (int)n, (int)d, Xq, (int)N, kernel, kparam, a, nb, groups, tpg, tuples, part, st); break;
        case 3: e = launch_predict_mp<3>(X, (int)n, (int)d, Xq, (int)N, kernel, kparam, a, nb, groups, tpg, tuples, part, st); break;
        case 5: e = launch_predict_mp<5>(X, (int)n, (int)d, Xq, (int)N, kernel, kparam, a, nb, groups, tpg, tuples, part, st); break;
        case 7: e = launch_predict_mp<7>(X, (int)n, (int)d, Xq, (int)N, kernel, kparam, a, nb, groups, tpg, tuples, part, st); break;
        default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
        const int64_t outs = (int64_t)nb * N;
        hipLaunchKernelGGL(predict_sum_kernel, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, st, part, groups,
                           nb, (int)N, f + b0 * N, N);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tk
