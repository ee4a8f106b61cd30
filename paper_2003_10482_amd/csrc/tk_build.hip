// Build the packed tensor kernel (Section 4 kernels, Section 5 layout) on gfx950.
//
// Rows are the sorted (m-1)-tuples P in nested-loop order; row P holds the
// entries K[P, l] for l in [P_last, n), contiguous in the packed array.  For the
// linear kernel K[P, l] = sum_j q_P[j] x_l[j] with q_P = prod_{i in P} x_i
// (elementwise), i.e. a product of the (rows x d) matrix Q with X^T restricted
// to l >= P_last.  A workgroup computes 64 rows against up to 256 columns:
// each chunk of features of q_P (gathered and multiplied once for all the
// columns) and of the columns right of the rows' first start is staged in
// LDS, and each wave accumulates its 16 rows against every 16-column block
// with FP64 MFMA (v_mfma_f64_16x16x4f64), skipping the blocks that lie wholly
// left of its rows' starts.  The kernel value (linear / polynomial /
// exponential) is formed in FP64 and rounded once to the storage type.
#include "tk_common.hpp"

namespace tk {

namespace {

constexpr int TR = 64;     // rows per workgroup (16 per pair of waves)
constexpr int TCS = 256;   // columns per workgroup (16 blocks of 16)
constexpr int NCB = TCS / 16;
constexpr int NWB = NCB / 2;   // column blocks per wave: every other one
constexpr int NT = 512;        // threads per workgroup (8 waves)
constexpr int FCH = 16;    // features per LDS chunk (4 MFMA k-steps of 4)

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
__global__ void __launch_bounds__(NT) build_kernel(const double *__restrict__ X, int n, int d,
                                                    int kernel, double kparam, int64_t rows,
                                                    void *K)
{
    constexpr int MP = M - 1;   // prefix length
    __shared__ double qs[FCH][TR + 1];
    __shared__ double xs[FCH][TCS + 1];
    __shared__ int pref[TR][MP > 0 ? MP : 1];
    __shared__ int64_t roff[TR];
    __shared__ int rk[TR];
    __shared__ int kmin;
    __shared__ int kmin16[TR / 16];   // smallest row start of each wave's 16 rows

    const int t = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int cs = blockIdx.y * TCS;   // columns [cs, ce) of this workgroup
    const int ce = cs + TCS < n ? cs + TCS : n;
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
    if (kmin >= ce) return;   // every row starts right of this workgroup's columns
    if (t < TR / 16) {
        int m16 = n;
        for (int r = 16 * t; r < 16 * t + 16; ++r) m16 = rk[r] < m16 ? rk[r] : m16;
        kmin16[t] = m16;
    }
    __syncthreads();
    // staged column blocks: from the one holding the first row start to the
    // last one below n (columns past n within it are zero)
    const int cb0 = ((kmin > cs ? kmin : cs) - cs) >> 4;
    const int cb1 = (ce - cs + 15) >> 4;
    const int c_lo = 16 * cb0, c_cnt = 16 * (cb1 - cb0);

    // wave w owns rows 16 (w % 4) .. + 15 against the column blocks j of
    // parity w / 4 (every other block: rows starting far right still find
    // work for both waves of a row group); the MFMA
    // v_mfma_f64_16x16x4f64 takes
    //   A: lane holds A[row0 + lane%16][k0 + lane/16]
    //   B: lane holds B[k0 + lane/16][col0 + lane%16]
    //   C: lane holds C[row0 + 4e + lane/16][col0 + lane%16], e = 0..3
    const int lane = t & 63, w = t >> 6;
    const int wg = w & 3, wp = w >> 2;
    const int li = lane & 15, lk = lane >> 4;
    const int wk = __builtin_amdgcn_readfirstlane(kmin16[wg]);
    v4d acc[NWB];
    bool need[NWB];   // block 2 i + wp holds an entry of one of the wave's rows (uniform)
#pragma unroll
    for (int i = 0; i < NWB; ++i) {
        const int j = 2 * i + wp;
        acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
        need[i] = j >= cb0 && j < cb1 && wk <= cs + 16 * j + 15;
    }

    for (int f0 = 0; f0 < d; f0 += FCH) {
        // q_P[f] for the 64 rows, x_l[f] for the staged columns
        for (int i = t; i < TR * FCH; i += NT) {
            const int r = i / FCH, f = i % FCH;
            double q = 0.0;
            if (f0 + f < d && rk[r] < n) {
                q = 1.0;
                for (int p = 0; p < MP; ++p) q *= X[(int64_t)pref[r][p] * d + f0 + f];
            }
            qs[f][r] = q;
        }
        for (int i = t; i < c_cnt * FCH; i += NT) {
            const int c = c_lo + i / FCH, f = i % FCH;
            const int l = cs + c;
            xs[f][c] = (f0 + f < d && l < n) ? X[(int64_t)l * d + f0 + f] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < FCH / 4; ++s) {
            const int f = 4 * s + lk;
            const double a = qs[f][16 * wg + li];
#pragma unroll
            for (int i = 0; i < NWB; ++i)
                if (need[i])
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xs[f][16 * (2 * i + wp) + li], acc[i], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NWB; ++i) {
        if (!need[i]) continue;
        const int l = cs + 16 * (2 * i + wp) + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * wg + 4 * e + lk;
            const int k = rk[r];
            if (l >= k && l < n) {
                double v = acc[i][e];
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
    dim3 grid((unsigned)((rows + TR - 1) / TR), (unsigned)((n + TCS - 1) / TCS));
    if (dtype == TK_F64)
        hipLaunchKernelGGL((build_kernel<M, double>), grid, dim3(NT), 0, st, X, n, d, kernel, kparam, rows, K);
    else if (dtype == TK_F32)
        hipLaunchKernelGGL((build_kernel<M, float>), grid, dim3(NT), 0, st, X, n, d, kernel, kparam, rows, K);
    else
        hipLaunchKernelGGL((build_kernel<M, uint16_t>), grid, dim3(NT), 0, st, X, n, d, kernel, kparam, rows, K);
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
