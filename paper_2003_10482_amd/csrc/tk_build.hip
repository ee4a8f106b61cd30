// Build the packed tensor kernel (Section 4 kernels, Section 5 layout) on gfx950.
//
// Rows are the sorted (m-1)-tuples P in nested-loop order; row P holds the
// entries K[P, l] for l in [P_last, n), contiguous in the packed array.  For the
// linear kernel K[P, l] = sum_j q_P[j] x_l[j] with q_P = prod_{i in P} x_i
// (elementwise), i.e. a product of the (rows x d) matrix Q with X^T restricted
// to l >= P_last.  A workgroup computes a 64-row x 64-column tile: Q and X
// chunks are staged in LDS and each wave accumulates a 32 x 32 quarter with
// FP64 MFMA (v_mfma_f64_16x16x4f64, 2 x 2 tiles: every operand read from LDS
// feeds 16 FMAs), skipping the 16 x 16 blocks that lie wholly left of the
// rows' starts.  The kernel value (linear / polynomial / exponential) is
// formed in FP64 and rounded once to the storage type.
#include "tk_common.hpp"

namespace tk {

namespace {

constexpr int TR = 64;    // rows per tile
constexpr int TC = 64;    // columns per tile
constexpr int FCH = 32;   // features per LDS chunk (8 MFMA k-steps of 4)

template <typename TOut>
__device__ __forceinline__ void store_entry(void *K, int64_t i, double v);
template <>
__device__ __forceinline__ void store_entry<double>(void *K, int64_t i, double v)
{
    reinterpret_cast<double *>(K)[i] = v;
}
template <>
__device__ __forceinline__ void store_entry<float>(void *K, int64_t i, double v)
{
    reinterpret_cast<float *>(K)[i] = (float)v;   // IEEE round-to-nearest-even
}
template <>
__device__ __forceinline__ void store_entry<uint16_t>(void *K, int64_t i, double v)
{
    reinterpret_cast<uint16_t *>(K)[i] = double_to_bf16(v);
}

// BF16 buffers are read a dword at a time: with an odd number of entries the
// 2 bytes after the last one are read with it and must hold a finite value.
__global__ void zero_bf16_tail(uint16_t *K, int64_t count)
{
    if (threadIdx.x == 0) K[count] = 0;
}

typedef double v4d __attribute__((ext_vector_type(4)));

template <int M, typename TOut>
__global__ void __launch_bounds__(256) build_kernel(const double *__restrict__ X, int n, int d,
                                                    int kernel, double kparam, int64_t rows,
                                                    void *K)
{
    constexpr int MP = M - 1;   // prefix length
    __shared__ double qs[FCH][TR + 1];
    __shared__ double xs[FCH][TC + 1];
    __shared__ int pref[TR][MP > 0 ? MP : 1];
    __shared__ int64_t roff[TR];
    __shared__ int rk[TR];
    __shared__ int kmin;
    __shared__ int kmin16[TR / 16];   // smallest row start of each group of 16 rows

    const int t = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int c0 = blockIdx.y * TC;
    if (t == 0) kmin = n;
    __syncthreads();
    if (t < TR) {
        const int64_t r = row0 + t;
        int tup[M];
        if (r < rows) {
            if constexpr (MP > 0) unrank_tuple<MP>(r, n, tup);
            const int k = MP > 0 ? tup[MP - 1] : 0;
            tup[MP] = k;
            roff[t] = rank_tuple<M>(tup, n);   // first entry of the row (l == k)
            rk[t] = k;
            for (int i = 0; i < MP; ++i) pref[t][i] = tup[i];
            atomicMin(&kmin, k);
        } else {
            rk[t] = n;   // empty row
            roff[t] = 0;
            for (int i = 0; i < MP; ++i) pref[t][i] = 0;
        }
    }
    __syncthreads();
    if (kmin > c0 + TC - 1 || c0 >= n) return;   // every row starts right of this tile
    if (t < TR / 16) {
        int m16 = n;
        for (int r = 16 * t; r < 16 * t + 16; ++r) m16 = rk[r] < m16 ? rk[r] : m16;
        kmin16[t] = m16;
    }
    __syncthreads();

    // wave w owns the 32 x 32 quarter (rows 32 (w / 2), columns 32 (w % 2))
    // as 2 x 2 MFMA tiles of 16 x 16; v_mfma_f64_16x16x4f64 takes
    //   A: lane holds A[row0 + lane%16][k0 + lane/16]
    //   B: lane holds B[k0 + lane/16][col0 + lane%16]
    //   C: lane holds C[row0 + 4e + lane/16][col0 + lane%16], e = 0..3
    const int lane = t & 63, w = t >> 6;
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
    const int li = lane & 15, lk = lane >> 4;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    // 16 x 16 blocks whose rows all start right of their columns hold no entry
    // of the tensor: their products are skipped (about half the tile's work
    // near the diagonal; the decision is uniform across the wave)
    bool need[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            need[i][j] = __builtin_amdgcn_readfirstlane(kmin16[(wr >> 4) + i]) <= c0 + wc + 16 * j + 15;

    for (int f0 = 0; f0 < d; f0 += FCH) {
        // stage q_P[f] for the tile rows and x_l[f] for the tile columns
        for (int i = t; i < TR * FCH; i += 256) {
            const int r = i / FCH, f = i % FCH;
            double q = 0.0;
            if (f0 + f < d && rk[r] < n) {
                q = 1.0;
                for (int p = 0; p < MP; ++p) q *= X[(int64_t)pref[r][p] * d + f0 + f];
            }
            qs[f][r] = q;
            const int l = c0 + r;
            xs[f][r] = (f0 + f < d && l < n) ? X[(int64_t)l * d + f0 + f] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < FCH / 4; ++s) {
            const int f = 4 * s + lk;
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = qs[f][wr + 16 * i + li];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = xs[f][wc + 16 * j + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (need[i][j]) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = wr + 16 * i + 4 * e + lk;
            const int k = rk[r];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int l = c0 + wc + 16 * j + li;
                if (l >= k && l < n) {
                    double v = acc[i][j][e];
                    if (kernel == TK_POLY) {
                        const int sdeg = (int)kparam;
                        double pw = 1.0;
                        for (int q = 0; q < sdeg; ++q) pw *= v;
                        v = pw;
                    } else if (kernel == TK_EXP) {
                        v = exp(v);
                    }
                    store_entry<TOut>(K, roff[r] + (l - k), v);
                }
            }
        }
}

template <int M>
hipError_t launch_build_m(const double *X, int n, int d, int kernel, double kparam, int dtype,
                          void *K, hipStream_t st)
{
    const int64_t rows = packed_count(n, M - 1);
    dim3 grid((unsigned)((rows + TR - 1) / TR), (unsigned)((n + TC - 1) / TC));
    if (dtype == TK_F64)
        hipLaunchKernelGGL((build_kernel<M, double>), grid, dim3(256), 0, st, X, n, d, kernel, kparam, rows, K);
    else if (dtype == TK_F32)
        hipLaunchKernelGGL((build_kernel<M, float>), grid, dim3(256), 0, st, X, n, d, kernel, kparam, rows, K);
    else
        hipLaunchKernelGGL((build_kernel<M, uint16_t>), grid, dim3(256), 0, st, X, n, d, kernel, kparam, rows, K);
    if (dtype == TK_BF16 && (packed_count(n, M) & 1))   // the half dword after the last entry is read with it
        hipLaunchKernelGGL(zero_bf16_tail, dim3(1), dim3(64), 0, st, static_cast<uint16_t *>(K), packed_count(n, M));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_build(const double *X, int n, int d, int m, int kernel, double kparam, int dtype,
                        void *K, hipStream_t st)
{
    switch (m) {
    case 2: return launch_build_m<2>(X, n, d, kernel, kparam, dtype, K, st);
    case 4: return launch_build_m<4>(X, n, d, kernel, kparam, dtype, K, st);
    case 6: return launch_build_m<6>(X, n, d, kernel, kparam, dtype, K, st);
    case 8: return launch_build_m<8>(X, n, d, kernel, kparam, dtype, K, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tk
