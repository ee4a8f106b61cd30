// Dense shortcut of a finite feature map and the small ops around the solve
// (gfx950): FP64 MFMA products for X^T alpha, X u^{m-1} and X_q w, the 2-std
// support threshold of Section 6.3 and the landmark gather of Section 6.1.
#include "tk_common.hpp"
#include "tk_dense.hpp"

namespace tk {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// C[i][j] = sum_k A[i*lda + k] * B[k*bsk + j*bsj]  (i < M, j < N, k < Kd), then
// one epilogue: epi > 1 raises C to the power epi; epi == kEpiShift adds
// d_i Y[i][j] (d_i = yd[i], or ys without yd); epi == kEpiReflect gives
// 2 Y[i][j] - C (Y has leading dimension ldc).  One workgroup per 16x16
// tile of C (four waves splitting the k-steps); the K loop feeds
// v_mfma_f64_16x16x4f64 four k at a time:
//   A operand: lane holds A[row0 + lane%16][k0 + lane/16]
//   B operand: lane holds B[k0 + lane/16][col0 + lane%16]
//   result:    lane holds C[row0 + 4*j + lane/16][col0 + lane%16], j = 0..3
//              (checked on the device with one-hot operands)
__global__ void __launch_bounds__(256) gemm_f64_mfma(const double *__restrict__ A, int64_t lda,
                                                     const double *__restrict__ Bm, int64_t bsk,
                                                     int64_t bsj, double *__restrict__ C,
                                                     int64_t ldc, int64_t M, int64_t N, int64_t Kd,
                                                     int epi, const double *__restrict__ Y,
                                                     const double *__restrict__ yd, double ys)
{
    // wave w sums the k-steps w, w + 4, ... (K / 16 MFMAs each, eight k-steps
    // of operands loaded ahead); the four partial tiles meet in LDS in a
    // fixed order
    __shared__ double red[4][4][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.y * 16;
    const int64_t col0 = (int64_t)blockIdx.x * 16;
    const int64_t ar = row0 + (lane & 15);
    const int64_t bc = col0 + (lane & 15);
    const int kk = lane >> 4;
    constexpr int U = 8;
    v4d acc = {0.0, 0.0, 0.0, 0.0}, acc2 = acc;
    for (int64_t kb = 4 * wave; kb < Kd; kb += 16 * U) {
        double a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = kb + 16 * u + kk;   // k-steps wave, wave + 4, wave + 8, ... (4 k each)
            a[u] = (ar < M && k < Kd) ? A[ar * lda + k] : 0.0;
            b[u] = (bc < N && k < Kd) ? Bm[k * bsk + bc * bsj] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; u += 2) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 1], b[u + 1], acc2, 0, 0, 0);
        }
    }
    acc += acc2;
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][j][lane] = acc[j];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t r = row0 + 4 * j + (lane >> 4);
        const int64_t c = col0 + (lane & 15);
        if (r < M && c < N) {
            double v = (red[0][j][lane] + red[1][j][lane]) + (red[2][j][lane] + red[3][j][lane]);
            if (epi == kEpiShift) {
                v = __builtin_fma(yd ? yd[r] : ys, Y[r * ldc + c], v);
            } else if (epi == kEpiReflect) {
                v = 2.0 * Y[r * ldc + c] - v;
            } else if (epi > 1) {
                double pw = 1.0;
                for (int e = 0; e < epi; ++e) pw *= v;
                v = pw;
            }
            C[r * ldc + c] = v;
        }
    }
}

// Population standard deviation of each row of W [B][d], tau = 2 std, mask.
__global__ void __launch_bounds__(256) support_kernel(const double *__restrict__ W, int64_t d,
                                                      uint8_t *__restrict__ mask,
                                                      double *__restrict__ tau)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    const double *w = W + (int64_t)b * d;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < d; j += 256) s += w[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double mean = red[0] / (double)d;
    __syncthreads();
    double v = 0.0;
    for (int64_t j = threadIdx.x; j < d; j += 256) {
        const double c = w[j] - mean;
        v += c * c;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double t = 2.0 * sqrt(red[0] / (double)d);
    if (threadIdx.x == 0) tau[b] = t;
    for (int64_t j = threadIdx.x; j < d; j += 256) mask[(int64_t)b * d + j] = fabs(w[j]) > t ? 1 : 0;
}

__global__ void gather_rows_kernel(const double *__restrict__ X, int64_t N, int64_t d,
                                   const int64_t *__restrict__ idx, int64_t l,
                                   double *__restrict__ out, int *__restrict__ bad)
{
    const int64_t i = blockIdx.y;
    const int64_t r = idx[i];
    if (r < 0 || r >= N) {
        if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(bad, 1);
        return;
    }
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < d; j += (int64_t)gridDim.x * blockDim.x)
        out[i * d + j] = X[r * d + j];
}

}  // namespace

hipError_t launch_gemm(const double *A, int64_t lda, const double *B, int64_t bsk, int64_t bsj,
                       double *C, int64_t ldc, int64_t M, int64_t N, int64_t K, int epi,
                       hipStream_t st)
{
    dim3 grid((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16));
    hipLaunchKernelGGL(gemm_f64_mfma, grid, dim3(256), 0, st, A, lda, B, bsk, bsj, C, ldc, M, N, K,
                       epi, (const double *)nullptr, (const double *)nullptr, 0.0);
    return hipGetLastError();
}

hipError_t launch_gemm_square(const double *A, const double *B, double *C, int64_t n, int epi, const double *Y,
                              const double *yd, double ys, hipStream_t st)
{
    if ((epi == kEpiShift || epi == kEpiReflect) && (Y == nullptr || Y == C)) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + 15) / 16), (unsigned)((n + 15) / 16));
    hipLaunchKernelGGL(gemm_f64_mfma, grid, dim3(256), 0, st, A, n, B, n, (int64_t)1, C, n, n, n, n, epi, Y, yd, ys);
    return hipGetLastError();
}

hipError_t launch_support(const double *W, int64_t d, int64_t B, uint8_t *mask, double *tau,
                          hipStream_t st)
{
    hipLaunchKernelGGL(support_kernel, dim3((unsigned)B), dim3(256), 0, st, W, d, mask, tau);
    return hipGetLastError();
}

hipError_t launch_gather(const double *X, int64_t N, int64_t d, const int64_t *idx, int64_t l,
                         double *out, int *bad, hipStream_t st)
{
    const unsigned gx = (unsigned)((d + 255) / 256 < 64 ? (d + 255) / 256 : 64);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(gx, (unsigned)l), dim3(256), 0, st, X, N, d, idx, l,
                       out, bad);
    return hipGetLastError();
}

}  // namespace tk
