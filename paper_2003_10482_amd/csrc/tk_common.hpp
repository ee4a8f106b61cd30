// Shared device/host helpers of the packed tensor-kernel library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>

#include "../../include/tk.h"
#include "tk_limits.hpp"

namespace tk {

// ---------------------------------------------------------------- errors ----
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define TK_HIP_CHECK(call)                                                                 \
    do {                                                                                   \
        hipError_t _e = (call);                                                            \
        if (_e != hipSuccess)                                                              \
            return ::tk::fail(TK_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), \
                              __FILE__, __LINE__);                                         \
    } while (0)


// ------------------------------------------------------------ binomials ----
// C(a, b) for 0 <= b <= 16; exact in int64 for every size this library accepts
// (callers check overflow on the host with checked_binom first).
__host__ __device__ inline int64_t binom(int64_t a, int b)
{
    if (b < 0 || a < b)
        return 0;
    int64_t c = 1;
    for (int i = 1; i <= b; ++i)
        c = c * (a - b + i) / i;   // C(a-b+i, i), exact at every step
    return c;
}

// Host-side C(a, b) with overflow detection (returns -1 on overflow).
inline int64_t checked_binom(int64_t a, int b)
{
    if (b < 0 || a < b)
        return 0;
    __int128 c = 1;
    for (int i = 1; i <= b; ++i) {
        c = c * (a - b + i) / i;
        if (c > (__int128)INT64_MAX)
            return -1;
    }
    return (int64_t)c;
}

// Number of sorted tuples of length q over n points.
__host__ __device__ inline int64_t packed_count(int64_t n, int q)
{
    return binom(n + q - 1, q);
}

// Rank (nested-loop position) of a sorted tuple t[0..q) over n points.  At each
// position p the values lo..t_p-1 are skipped together with their sorted
// completions; the hockey-stick identity sums those block sizes in closed form.
template <int Q>
__host__ __device__ inline int64_t rank_tuple(const int *t, int64_t n)
{
    int64_t r = 0;
    int lo = 0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const int rest = Q - p - 1;
        r += binom(n - lo + rest, rest + 1) - binom(n - t[p] + rest, rest + 1);
        lo = t[p];
    }
    return r;
}

// Inverse of rank_tuple by binary search on the same closed-form counts.
template <int Q>
__host__ __device__ inline void unrank_tuple(int64_t e, int64_t n, int *t)
{
    int lo = 0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const int rest = Q - p - 1;
        const int64_t base = binom(n - lo + rest, rest + 1);
        // largest v in [lo, n-1] with base - C(n-v+rest, rest+1) <= e
        int a = lo, b = (int)n - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (base - binom(n - mid + rest, rest + 1) <= e)
                a = mid;
            else
                b = mid - 1;
        }
        e -= base - binom(n - a + rest, rest + 1);
        t[p] = a;
        lo = a;
    }
}

// -------------------------------------------------- double-double pieces ----
// Error-free transformations (Knuth's TwoSum; TwoProduct through FMA) as used
// by the accurate dot product of Ogita, Rump and Oishi (2005): the pair
// (hi, lo) carries a sum whose error is that of twice the working precision.
struct DD {
    double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// acc += a * b with a, b doubles.
__device__ __forceinline__ void dd_fma(DD &acc, double a, double b)
{
    const double p = a * b;
    const double pe = __builtin_fma(a, b, -p);
    double s, e;
    two_sum(acc.hi, p, s, e);
    acc.hi = s;
    acc.lo += e + pe;
}

// acc += (a.hi + a.lo) * b.
__device__ __forceinline__ void dd_fma(DD &acc, DD a, double b)
{
    const double p = a.hi * b;
    double pe = __builtin_fma(a.hi, b, -p);
    pe = __builtin_fma(a.lo, b, pe);
    double s, e;
    two_sum(acc.hi, p, s, e);
    acc.hi = s;
    acc.lo += e + pe;
}

// acc += a * b with a, b double-doubles (the lo*lo term is dropped).
__device__ __forceinline__ void dd_fma(DD &acc, DD a, DD b)
{
    const double p = a.hi * b.hi;
    double pe = __builtin_fma(a.hi, b.hi, -p);
    pe = __builtin_fma(a.hi, b.lo, pe);
    pe = __builtin_fma(a.lo, b.hi, pe);
    double s, e;
    two_sum(acc.hi, p, s, e);
    acc.hi = s;
    acc.lo += e + pe;
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    return DD{s, e + (a.lo + b.lo)};
}

__device__ __forceinline__ DD dd_mul(DD a, DD b)
{
    DD r{0.0, 0.0};
    dd_fma(r, a, b);
    return r;
}

__device__ __forceinline__ DD dd_mul(DD a, double b)
{
    DD r{0.0, 0.0};
    dd_fma(r, a, b);
    return r;
}

// a / k for a small positive integer k, as a double-double.
__device__ __forceinline__ DD dd_div_int(DD a, double k)
{
    const double q = a.hi / k;
    const double r = __builtin_fma(-q, k, a.hi) + a.lo;   // remainder, exact up to a.lo rounding
    return DD{q, r / k};
}

__device__ __forceinline__ DD dd_norm(DD a)
{
    double s, e;
    two_sum(a.hi, a.lo, s, e);
    return DD{s, e};
}

// ------------------------------------------------------------ storage ----
// BF16 bits -> float (exact).
__device__ __forceinline__ float bf16_to_float(uint16_t b)
{
    return __uint_as_float(((uint32_t)b) << 16);
}

// Round a double to the nearest BF16 (ties to even), directly from the double
// so there is a single rounding.  Overflow goes to +-inf, NaN stays NaN.
__host__ __device__ inline uint16_t double_to_bf16(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof(u));
    const uint64_t sign = u & 0x8000000000000000ull;
    const uint64_t mag = u & 0x7fffffffffffffffull;
    if (mag > 0x7ff0000000000000ull)            // NaN
        return (uint16_t)((sign >> 48) | 0x7fc0u);
    const int e = (int)(mag >> 52);             // biased double exponent
    // BF16 normal range: exponent >= -126 (biased double >= 1023-126 = 897)
    int shift;                                   // number of low double mantissa bits dropped
    uint64_t m = mag & ((1ull << 52) - 1);
    uint64_t full;                               // significand with implicit bit
    int e_out;                                   // biased bf16 exponent of the result
    if (e >= 897) {
        full = m | (1ull << 52);
        shift = 52 - 7;
        e_out = e - 1023 + 127;
    } else {
        // subnormal in bf16 (or zero): quantum 2^-133; value = full * 2^(e-1075)
        if (e == 0)
            return (uint16_t)(sign >> 48);       // double subnormal or zero -> +-0
        full = m | (1ull << 52);
        shift = 52 - 7 + (897 - e);              // bring to multiples of 2^-133
        e_out = 0;
        if (shift > 63)
            return (uint16_t)(sign >> 48);
    }
    uint64_t q = full >> shift;
    const uint64_t rem = full & ((1ull << shift) - 1);
    const uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1)))
        q += 1;
    uint32_t bits;
    if (e_out > 0) {
        // q in [2^7, 2^8]; carry into the exponent when it reaches 2^8
        if (q == (1ull << 8)) {
            q >>= 1;
            e_out += 1;
        }
        if (e_out >= 255)
            return (uint16_t)((sign >> 48) | 0x7f80u);   // inf
        bits = ((uint32_t)e_out << 7) | (uint32_t)(q & 0x7f);
    } else {
        // subnormal result; q may round up to the smallest normal (q == 2^7)
        bits = (uint32_t)q;   // q < 2^7 -> subnormal, q == 2^7 -> exponent 1, mantissa 0
    }
    return (uint16_t)((sign >> 48) | bits);
}

template <typename T>
struct Storage;
template <>
struct Storage<double> {
    __device__ __forceinline__ static double load(const double *p, int64_t i) { return p[i]; }
};
template <>
struct Storage<float> {
    __device__ __forceinline__ static float load(const float *p, int64_t i) { return p[i]; }
};
template <>
struct Storage<uint16_t> {
    __device__ __forceinline__ static float load(const uint16_t *p, int64_t i)
    {
        return bf16_to_float(p[i]);
    }
};

inline size_t dtype_size(int dtype)
{
    return dtype == TK_F64 ? 8 : dtype == TK_F32 ? 4 : 2;
}

// Instrumentation of the passes that stream the packed tensor (tk_timing_*):
// kinds 0 compensated contraction, 1 directional derivative, 2 plain
// contraction, 3 and 4 the two streaming kernels of the Hessian.
constexpr int kTimingKinds = 5;
struct TimedLaunch {
    hipEvent_t a, b;
    int kind;
    double bytes;
    bool on;
};
TimedLaunch timing_begin(int kind, double bytes, hipStream_t st);
void timing_end(TimedLaunch &t, hipStream_t st);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace tk
