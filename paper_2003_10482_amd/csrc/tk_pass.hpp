// Packed symmetric-tensor contraction g = K . alpha^{m-1} and its directional
// derivative, for gfx950.
//
// Decomposition (exact; follows from grouping the terms of the contraction of
// Section 4 by the sorted tuple's prefix).  For an order-q packed array A over
// n points, write a sorted tuple as (P, l) with P its first q-1 indices ("row"
// P, entries l in [P_last, n)).  With r_p(t) the length of the run of equal
// values ending at position p of a sorted tuple t,
//
//   contract_q(A)_a = colsum_q(A)_a + (q-1) contract_{q-1}(S)_a
//   colsum_q(A)_l   = sum_P [(q-1)!/prod_{p<q} r_p(P)] alpha^P A_{P,l} / r_q(P,l)
//   S_P             = sum_l A_{P,l} alpha_l / r_q(P,l)          (an order q-1 array)
//
// and contract_1(S) = S.  One pass of `pair_kernel` applies two levels (q and
// q-1) to one array: waves own whole "units" (the q-2 leading indices P'),
// whose rows k in [P'_last, n) are contiguous in memory.  Lanes own fixed
// columns l = 64 b + lane, so every column sum stays in registers; row sums
// (S_{P',k}) are produced by a transposed reduction through LDS, and the unit
// sums S_{P'} form the order q-2 array of the next pass.  A last pass reduces
// the per-workgroup column sums in a fixed order, so results are bitwise
// reproducible.
//
// Accumulation modes: compensated FP64 (error-free products and sums, so the
// heavy cancellation of the contraction near the dual optimum does not eat the
// FP64 result), plain FP64, plain FP32.  The directional derivative runs the
// same recursion on dual numbers alpha + eps v.
#pragma once

#include "tk_common.hpp"
#include "tk_contract.hpp"

namespace tk {


template <int MODE>
struct ModeT;
template <>
struct ModeT<ACC_DD> {
    using V = double;   // arithmetic type of values and coefficients
    using P = DD;       // accumulator / partial type
    using S = DD;       // type of the intermediate arrays
};
template <>
struct ModeT<ACC_PLAIN64> {
    using V = double;
    using P = double;
    using S = double;
};
template <>
struct ModeT<ACC_PLAIN32> {
    using V = float;
    using P = float;
    using S = float;
};

// ----------------------------------------------------- accumulator ops ----
__device__ __forceinline__ void acc_fma(DD &a, DD c, double v) { dd_fma(a, c, v); }
__device__ __forceinline__ void acc_fma(DD &a, DD c, DD v) { dd_fma(a, c, v); }
__device__ __forceinline__ void acc_fma(DD &a, double c, double v) { dd_fma(a, c, v); }
__device__ __forceinline__ void acc_fma(DD &a, double c, DD v) { dd_fma(a, v, c); }
__device__ __forceinline__ void acc_fma(double &a, double c, double v) { a = __builtin_fma(c, v, a); }
__device__ __forceinline__ void acc_fma(float &a, float c, float v) { a = __builtin_fmaf(c, v, a); }

__device__ __forceinline__ DD p_add(DD a, DD b) { return dd_add(a, b); }
__device__ __forceinline__ double p_add(double a, double b) { return a + b; }
__device__ __forceinline__ float p_add(float a, float b) { return a + b; }

template <typename T>
__device__ __forceinline__ T p_zero() { return T(0); }
template <>
__device__ __forceinline__ DD p_zero<DD>() { return DD{0.0, 0.0}; }

// Cross-lane moves within rows of 16 lanes (DPP): xor 1, xor 2, the mirror
// inside 8 lanes and the mirror inside 16 lanes.  Successive additions with
// these four patterns sum groups of 2, 4, 8 and 16 lanes.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int CTRL>
__device__ __forceinline__ float p_dpp(float a)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double p_dpp(double a)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(a), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(a), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ DD p_dpp(DD a)
{
    return DD{p_dpp<CTRL>(a.hi), p_dpp<CTRL>(a.lo)};
}

__device__ __forceinline__ DD p_shfl_xor(DD a, int m)
{
    return DD{__shfl_xor(a.hi, m), __shfl_xor(a.lo, m)};
}
__device__ __forceinline__ double p_shfl_xor(double a, int m) { return __shfl_xor(a, m); }
__device__ __forceinline__ float p_shfl_xor(float a, int m) { return __shfl_xor(a, m); }

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of a
// group receives the group's sum (fixed order, so results are reproducible).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T s)
{
    if constexpr (G >= 2) s = p_add(s, p_dpp<kDppXor1>(s));
    if constexpr (G >= 4) s = p_add(s, p_dpp<kDppXor2>(s));
    if constexpr (G >= 8) s = p_add(s, p_dpp<kDppHalfMirror>(s));
    if constexpr (G >= 16) s = p_add(s, p_dpp<kDppMirror>(s));
    if constexpr (G >= 32) s = p_add(s, p_shfl_xor(s, 16));
    if constexpr (G >= 64) s = p_add(s, p_shfl_xor(s, 32));
    return s;
}

// Pairwise sum of N consecutive values v[0..N).
template <int N, typename T, typename F>
__device__ __forceinline__ T tree_sum(F v)
{
    if constexpr (N == 1) return v(0);
    else {
        constexpr int H = N / 2;
        const T a = tree_sum<H, T>(v);
        const T b = tree_sum<N - H, T>([&](int i) { return v(H + i); });
        return p_add(a, b);
    }
}

// Coefficient types: DD carries a low part (exact quotients alpha/r), plain
// modes use the value type.
template <int MODE>
struct Coef {
    using T = typename ModeT<MODE>::V;
    __device__ __forceinline__ static T make(double x) { return (T)x; }
    __device__ __forceinline__ static T div(T a, int r)
    {
        if (r == 1) return a;
        if (r == 2) return a * (T)0.5;
        return a / (T)r;
    }
    __device__ __forceinline__ static T mul(T a, T b) { return a * b; }
};
template <>
struct Coef<ACC_DD> {
    using T = DD;
    __device__ __forceinline__ static DD make(double x) { return DD{x, 0.0}; }
    __device__ __forceinline__ static DD div(DD a, int r)
    {
        if (r == 1) return a;
        if (r == 2) return DD{a.hi * 0.5, a.lo * 0.5};   // exact
        return dd_div_int(a, (double)r);
    }
    __device__ __forceinline__ static DD mul(DD a, DD b) { return dd_mul(a, b); }
};

// DD accumulator as a value: hi + lo (for conversions at the end).
__device__ __forceinline__ double p_value(DD a) { return a.hi + a.lo; }
__device__ __forceinline__ double p_value(double a) { return a; }
__device__ __forceinline__ double p_value(float a) { return (double)a; }

// Load one entry of an input array as the value type (+ low part for DD arrays).
template <typename TIn, int MODE>
struct In;
// Buffer-resource loads: a byte offset past the descriptor's range (or a
// negative one, which wraps) reads 0 instead of faulting, so rows past a batch
// and lanes left of the diagonal need no address clamping or branches.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc make_rsrc(const void *base, int64_t bytes)
{
    const int64_t cap = 0xffffffffLL;
    const uint32_t nr = (uint32_t)(bytes < 0 ? 0 : (bytes > cap ? cap : bytes));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nr, 0x00020000);
}

template <int MODE>
struct In<double, MODE> {
    using R = typename ModeT<MODE>::V;
    static constexpr int kSize = 8;
    __device__ __forceinline__ static R load(const double *p, uint32_t i) { return (R)p[i]; }
    __device__ __forceinline__ static R load_buf(Rsrc rs, uint32_t byte_off)
    {
        return (R)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, byte_off, 0, 0));
    }
};
template <int MODE>
struct In<float, MODE> {
    using R = typename ModeT<MODE>::V;
    static constexpr int kSize = 4;
    __device__ __forceinline__ static R load(const float *p, uint32_t i) { return (R)p[i]; }
    __device__ __forceinline__ static R load_buf(Rsrc rs, uint32_t byte_off)
    {
        return (R)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, byte_off, 0, 0));
    }
};
template <int MODE>
struct In<uint16_t, MODE> {
    using R = typename ModeT<MODE>::V;
    static constexpr int kSize = 2;
    __device__ __forceinline__ static R load_buf(Rsrc rs, uint32_t byte_off)
    {
        const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, byte_off & ~3u, 0, 0);
        const uint32_t bits = (byte_off & 2u) ? (w & 0xffff0000u) : (w << 16);
        return (R)__uint_as_float(bits);
    }
    // 16-bit loads are slow in the memory pipeline: load the aligned dword that
    // holds the value (the packed BF16 buffer is padded to whole dwords) and
    // take its upper or lower half
    __device__ __forceinline__ static R load(const uint16_t *p, uint32_t i)
    {
        const uintptr_t a = reinterpret_cast<uintptr_t>(p + i);
        const uint32_t w = *reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
        const uint32_t bits = (a & 2) ? (w & 0xffff0000u) : (w << 16);
        return (R)__uint_as_float(bits);
    }
};
template <>
struct In<DD, ACC_DD> {
    using R = DD;
    static constexpr int kSize = 16;
    __device__ __forceinline__ static DD load(const DD *p, uint32_t i) { return p[i]; }
    __device__ __forceinline__ static DD load_buf(Rsrc rs, uint32_t byte_off)
    {
        return __builtin_bit_cast(DD, __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off, 0, 0));
    }
};

// acc += c * v where v may be a DD (intermediate arrays in DD mode).
template <typename PT, typename CT, typename VT>
__device__ __forceinline__ void acc_cv(PT &acc, CT c, VT v) { acc_fma(acc, c, v); }

// Entry weight on the block of the diagonal: d = column - row.  Left of the
// diagonal (d < 0) the lane holds another row's entry; on it (a tie between
// the last two indices) every coefficient of the entry is halved, exactly.
__device__ __forceinline__ double tie_scale(int d, double x) { return d < 0 ? 0.0 : (d == 0 ? 0.5 * x : x); }
__device__ __forceinline__ float tie_scale(int d, float x) { return d < 0 ? 0.0f : (d == 0 ? 0.5f * x : x); }
// The same with the tie weight w (1/2, or 1/(r+1) on a unit's first row).
__device__ __forceinline__ double tie_scale_w(int d, double x, double w) { return d < 0 ? 0.0 : (d == 0 ? w * x : x); }
__device__ __forceinline__ float tie_scale_w(int d, float x, float w) { return d < 0 ? 0.0f : (d == 0 ? w * x : x); }
__device__ __forceinline__ DD tie_scale(int d, DD x)
{
    const double f = d < 0 ? 0.0 : (d == 0 ? 0.5 : 1.0);
    return DD{f * x.hi, f * x.lo};
}

__device__ __forceinline__ DD zero_like(DD) { return DD{0.0, 0.0}; }
__device__ __forceinline__ double zero_like(double) { return 0.0; }
__device__ __forceinline__ float zero_like(float) { return 0.0f; }

template <typename T>
__device__ __forceinline__ void store_s(void *p, int64_t i, T v)
{
    reinterpret_cast<T *>(p)[i] = v;
}
template <>
__device__ __forceinline__ void store_s<DD>(void *p, int64_t i, DD v)
{
    double *q = reinterpret_cast<double *>(p) + 2 * i;
    q[0] = v.hi;
    q[1] = v.lo;
}

// DD x coefficient for the unit multiplier (plain modes: ordinary products).
__device__ __forceinline__ void acc_unit(DD &acc, DD c, DD z) { dd_fma(acc, c, z); }
__device__ __forceinline__ void acc_unit(double &acc, double c, double z) { acc = __builtin_fma(c, z, acc); }
__device__ __forceinline__ void acc_unit(float &acc, float c, float z) { acc = __builtin_fmaf(c, z, acc); }

// --------------------------------------------------------------- kernel ----
// Rows are processed in batches that never straddle a 64-column block, so the
// first block touched (KB) is a compile-time constant inside a batch: the
// diagonal tie and the lower mask sit in block KB, blocks KB+1.. are full, and
// the level q-1 update touches block KB only.  Loads address the row through a
// uniform pointer plus the lane's constant offset.

// Rows loaded per batch: about 16 loads per batch, 32 for BF16 storage (its
// loads and conversions, not HBM, bound the pass: more rows in flight
// measured 14 % faster there and slower for FP64).  With units of two
// leading indices (order 4: triangles of up to n rows) the rows of the last
// column block (at most 64 entries, about half of each load left of the
// diagonal) come 16 at a time (2-4 % faster passes at n = 256); the shorter
// units of higher orders keep 8 (16 measured 8-12 % slower at order 6).
// The row partials go through LDS RBMAX rows at a time.
template <int NB, int KB, bool WIDE = false, bool LONG = false>
constexpr int batch_rows_kb()
{
    constexpr int segs = NB - KB;
    constexpr int r0 = (WIDE ? 32 : 16) / segs;
    return (LONG && segs == 1 && r0 >= 16) ? 16 : r0 >= 8 ? 8 : r0 >= 4 ? 4 : 2;
}

template <int Q, int NB, typename TIn, int MODE, int HV, int BT, int RBMAX>
struct Pass {
    static constexpr bool HVP = HV > 0;
    static constexpr bool ATAN = HV > 1;   // the input array carries a tangent
    using V = typename ModeT<MODE>::V;
    using PT = typename ModeT<MODE>::P;
    using CT = typename Coef<MODE>::T;
    using InL = In<TIn, MODE>;
    using VIn = typename InL::R;
    static constexpr int NC = BT * (HVP ? 2 : 1);   // reduced components per row
    static constexpr int QP = Q - 2;                // unit prefix length

    // per-lane registers: column l = 64 b + lane
    V a_l[BT][NB], v_l[BT][NB];
    PT U[BT][NB], Ud[BT][NB];        // column sums within the current unit
    PT unitS[BT], unitSd[BT];        // lane partials of S_{P'}
    // unit constants (uniform)
    CT ak0_rr[BT], vk0_rr[BT], cu_tie0[BT], ck_tie0[BT], cud_tie0[BT], vk_tie0[BT];
    CT inv_rr;
    // plain modes take a unit's first row (run rr > 1) through batch_fast:
    // row factor inv_rr on alpha_k and tie weight tie0 = 1 / (rr + 1) there,
    // against 1 and 1/2 on every other row (one batch less per unit: -10 %
    // for the directional derivatives of FP32 storage and of order 6, -1 to
    // -4 % elsewhere; the contraction of FP32 storage measured 4 % slower
    // that way and keeps the general path, as the compensated mode does)
    static constexpr bool FOLD = MODE != ACC_DD && !(MODE == ACC_PLAIN32 && !HVP && sizeof(TIn) == 4);
    V tie0;
    int k0, rr;
    // pointers
    const TIn *A;
    const TIn *Ad;
    Rsrc rs, rsd;      // descriptors of A and Ad from the wave's first entry e_base on
    int64_t e_base;
    const V *alpha_s;
    const V *vdir_s;
    PT *buf;      // [RBMAX][NC][64] row partials
    PT *sbatch;   // [RBMAX][NC] row sums
    int n, lane;

    // Descriptors for the wave's entries, based 64 entries before its first
    // entry e0 (clamped to the array start, 16-byte aligned so BF16 dword
    // loads stay aligned); count entries per input array.  An out-of-range
    // lane of a buffer load zeroes the other lanes of its quad as well, so no
    // live row may reach below the base: the lanes left of the first row's
    // diagonal (at most 63 entries back) must stay in range.
    int32_t dshift;   // byte shift of the tangent array's descriptor
    __device__ __forceinline__ void set_base(int64_t e0, int64_t count)
    {
        constexpr int64_t ES = InL::kSize;
        const int64_t end_bytes = (count * ES + 3) & ~(int64_t)3;
        const int64_t e1 = e0 >= kWave ? e0 - kWave : 0;
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(A + e1) & ~(uintptr_t)15;
        e_base = e1 - (int64_t)(reinterpret_cast<uintptr_t>(A + e1) - a0) / ES;
        rs = make_rsrc(reinterpret_cast<const void *>(a0), end_bytes - e_base * ES);
        dshift = 0;
        if constexpr (ATAN) {
            const uintptr_t d0 = reinterpret_cast<uintptr_t>(Ad + e1) & ~(uintptr_t)15;
            const int64_t eb_d = e1 - (int64_t)(reinterpret_cast<uintptr_t>(Ad + e1) - d0) / ES;
            rsd = make_rsrc(reinterpret_cast<const void *>(d0), end_bytes - eb_d * ES);
            dshift = (int32_t)((e_base - eb_d) * ES);
        }
    }

    __device__ __forceinline__ void begin_unit()
    {
#pragma unroll
        for (int bt = 0; bt < BT; ++bt) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                U[bt][b] = p_zero<PT>();
                Ud[bt][b] = p_zero<PT>();
            }
            unitS[bt] = p_zero<PT>();
            unitSd[bt] = p_zero<PT>();
            const V ak = alpha_s[bt * n + k0];
            ak0_rr[bt] = Coef<MODE>::div(Coef<MODE>::make((double)ak), rr);
            cu_tie0[bt] = Coef<MODE>::div(ak0_rr[bt], rr + 1);
            ck_tie0[bt] = Coef<MODE>::div(Coef<MODE>::make((double)ak), rr + 1);
            if constexpr (HVP) {
                const V vk = vdir_s[bt * n + k0];
                vk0_rr[bt] = Coef<MODE>::div(Coef<MODE>::make((double)vk), rr);
                cud_tie0[bt] = Coef<MODE>::div(vk0_rr[bt], rr + 1);
                vk_tie0[bt] = Coef<MODE>::div(Coef<MODE>::make((double)vk), rr + 1);
            }
        }
        inv_rr = Coef<MODE>::div(Coef<MODE>::make(1.0), rr);
        if constexpr (FOLD) tie0 = Coef<MODE>::div(Coef<MODE>::make(1.0), rr + 1);
    }

    // Rows [k, k + nrows) with k >> 6 == KB; `off` is the packed offset of row k.
    template <int KB>
    __device__ __forceinline__ void batch(int &k, int k_hi, int64_t &off)
    {
        constexpr int RB0 = batch_rows_kb<NB, KB, sizeof(TIn) == 2, Q == 4>();
        constexpr int RB = RB0 < RBMAX ? RB0 : RBMAX;
        constexpr int SEG = NB - KB;
        constexpr int LPR = kWave / RB;
        const int blk_end = (KB + 1) * kWave;
        const int lim = blk_end < k_hi ? blk_end : k_hi;
        const int nrows = (lim - k) < RB ? (lim - k) : RB;
        const int lane_lo = k - KB * kWave;   // lanes >= lane_lo + r are on or right of the diagonal of row r

        // ---- phase 1: loads of the batch (row r at offset off + r(n-k) - r(r-1)/2)
        VIn val[RB][SEG];
        VIn vald[RB][ATAN ? SEG : 1];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int64_t roff = off + (int64_t)r * (n - k) - (int64_t)(r * (r - 1) / 2);
            const TIn *rowp = A + (roff - (k + r));        // rowp[l] is entry (row, l)
            const TIn *rowd = ATAN ? Ad + (roff - (k + r)) : nullptr;
#pragma unroll
            for (int j = 0; j < SEG; ++j) {
                const int b = KB + j;
                val[r][j] = zero_like(VIn());
                if constexpr (ATAN) vald[r][j] = zero_like(VIn());
                bool ok = r < nrows;
                if (j == 0) ok = ok && (lane >= lane_lo + r);
                ok = ok && b * kWave + lane < n;   // columns past n (any block: NB may exceed the blocks of n)
                if (ok) {
                    val[r][j] = InL::load(rowp, b * kWave + lane);
                    if constexpr (ATAN) vald[r][j] = InL::load(rowd, b * kWave + lane);
                }
            }
        }
        // ---- phase 2: in-unit column sums and row partials
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (r >= nrows) break;
            const int kr = k + r;
            const bool first = (kr == k0);                 // r_{Q-1} = rr only there
            const bool tie_lane = (lane == lane_lo + r);   // entry l == kr (block KB)
#pragma unroll
            for (int bt = 0; bt < BT; ++bt) {
                const V ak = alpha_s[bt * n + kr];
                const CT akc = Coef<MODE>::make((double)ak);
                const CT half_ak = Coef<MODE>::div(akc, 2);
                const CT cu = first ? ak0_rr[bt] : akc;
                const CT cu_tie = first ? cu_tie0[bt] : half_ak;
                const CT ck_tie = first ? ck_tie0[bt] : half_ak;
                CT cud{}, cud_tie{}, vk_tie{};
                if constexpr (HVP) {
                    const V vk = vdir_s[bt * n + kr];
                    const CT vkc = Coef<MODE>::make((double)vk);
                    const CT half_vk = Coef<MODE>::div(vkc, 2);
                    cud = first ? vk0_rr[bt] : vkc;
                    cud_tie = first ? cud_tie0[bt] : half_vk;
                    vk_tie = first ? vk_tie0[bt] : half_vk;
                }
                PT part = p_zero<PT>(), partd = p_zero<PT>();
#pragma unroll
                for (int j = 0; j < SEG; ++j) {
                    const int b = KB + j;
                    const VIn x = val[r][j];
                    if (j == 0) {
                        const CT cU = tie_lane ? cu_tie : cu;
                        const CT cP = tie_lane ? ck_tie : Coef<MODE>::make((double)a_l[bt][b]);
                        acc_cv(U[bt][b], cU, x);
                        acc_cv(part, cP, x);
                        if constexpr (HVP) {
                            const CT cUd = tie_lane ? cud_tie : cud;
                            const CT cPd = tie_lane ? vk_tie : Coef<MODE>::make((double)v_l[bt][b]);
                            acc_cv(Ud[bt][b], cUd, x);
                            acc_cv(partd, cPd, x);
                            if constexpr (ATAN) {
                                acc_cv(Ud[bt][b], cU, vald[r][j]);
                                acc_cv(partd, cP, vald[r][j]);
                            }
                        }
                    } else {
                        acc_cv(U[bt][b], cu, x);
                        acc_cv(part, a_l[bt][b], x);
                        if constexpr (HVP) {
                            acc_cv(Ud[bt][b], cud, x);
                            acc_cv(partd, v_l[bt][b], x);
                            if constexpr (ATAN) {
                                acc_cv(Ud[bt][b], cu, vald[r][j]);
                                acc_cv(partd, a_l[bt][b], vald[r][j]);
                            }
                        }
                    }
                }
                buf[(r * NC + bt) * kWave + lane] = part;
                if constexpr (HVP) buf[(r * NC + BT + bt) * kWave + lane] = partd;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // ---- transposed reduction: lanes [r LPR, (r+1) LPR) sum row r
        {
            const int r = lane / LPR, seg = lane % LPR;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                PT s = p_zero<PT>();
#pragma unroll
                for (int j = 0; j < RB; ++j) s = p_add(s, buf[(r * NC + c) * kWave + seg * RB + j]);
#pragma unroll
                for (int m = 1; m < LPR; m <<= 1) s = p_add(s, p_shfl_xor(s, m));
                if (seg == 0) sbatch[r * NC + c] = s;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // ---- level Q-1: S_{P',k}/r_k joins the column sums at index k (block KB),
        // and S_{P'} += S_k alpha_k / r_k
        {
            const int r = lane - lane_lo;
            if (r >= 0 && r < nrows) {
                const bool first = (k + r == k0);
#pragma unroll
                for (int bt = 0; bt < BT; ++bt) {
                    const PT s = sbatch[r * NC + bt];
                    const CT inv = first ? inv_rr : Coef<MODE>::make(1.0);
                    acc_cv(U[bt][KB], inv, s);
                    const CT ak = first ? ak0_rr[bt] : Coef<MODE>::make((double)a_l[bt][KB]);
                    acc_cv(unitS[bt], ak, s);
                    if constexpr (HVP) {
                        const PT sd = sbatch[r * NC + BT + bt];
                        acc_cv(Ud[bt][KB], inv, sd);
                        const CT vk = first ? vk0_rr[bt] : Coef<MODE>::make((double)v_l[bt][KB]);
                        acc_cv(unitSd[bt], ak, sd);
                        acc_cv(unitSd[bt], vk, s);
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        off += (int64_t)nrows * (n - k) - (int64_t)(nrows * (nrows - 1) / 2);
        k += nrows;
    }

    // Rows [k, k + nrows) with k >> 6 == KB, none of them the first row of a
    // unit with a run multiplicity (their coefficients are the plain alpha_k,
    // halved on the diagonal).  No divergent branches around the loads.
    template <int KB>
    __device__ __forceinline__ void batch_fast(int &k, int k_hi, int64_t &off)
    {
        constexpr int RB = batch_rows_kb<NB, KB, sizeof(TIn) == 2, Q == 4>();   // rows loaded together
        constexpr int RBR = RB < RBMAX ? RB : RBMAX;                      // rows per pass through buf
        static_assert(RB % RBR == 0, "row groups");
        constexpr int SEG = NB - KB;
        constexpr int LPR = kWave / RBR;
        const int blk_end = (KB + 1) * kWave;
        const int lim = blk_end < k_hi ? blk_end : k_hi;
        const int nrows = (lim - k) < RB ? (lim - k) : RB;
        const int lane_lo = k - KB * kWave;

        // ---- phase 1: every lane loads every segment of every row through the
        // buffer descriptor.  Left of the diagonal the lane reads another row's
        // entry (zeroed in phase 2); columns past n re-read column n-1
        // (their alpha and v are 0).
        VIn val[RB][SEG];
        VIn vald[RB][ATAN ? SEG : 1];
        constexpr uint32_t ES = (uint32_t)InL::kSize;
        // byte offset (from the descriptor base) of entry (row, column KB*64) of
        // row r; rows past the batch follow the same recurrence and read either
        // real entries or zeros (their row coefficients are zero below).
        // Columns past n re-read column n-1 of the same row, so the live rows
        // never reach past the array (whose padding may hold anything).
        uint32_t so = (uint32_t)((off - k - e_base + KB * kWave) * (int64_t)ES);
        const uint32_t vlane = (uint32_t)lane * ES;
        // lanes past column n-1 (in whichever block: NB may exceed the blocks
        // that n fills) re-read column n-1 of the same row: 0 but for tail lanes
        uint32_t vtail[SEG];
#pragma unroll
        for (int j = 0; j < SEG; ++j) {
            const int l = (KB + j) * kWave + lane;
            vtail[j] = l < n ? 0u : (uint32_t)(n - 1 - l) * ES;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const uint32_t vo = so + vlane;
#pragma unroll
            for (int j = 0; j < SEG; ++j) {
                const uint32_t o = vo + (uint32_t)(j * kWave) * ES + vtail[j];
                val[r][j] = InL::load_buf(rs, o);
                if constexpr (ATAN) vald[r][j] = InL::load_buf(rsd, o + (uint32_t)dshift);
            }
            so += (uint32_t)(n - k - 1 - r) * ES;
        }
        // ---- phase 2: in-unit column sums and row partials, RBR rows at a
        // time.  Rows past the batch run with zero row coefficients (their row
        // partials are never read), so the loads above are not tied to per-row
        // branches.  Plain modes accumulate odd rows into a second set of
        // column sums, halving the dependent chains.
        constexpr bool SPLIT = MODE != ACC_DD;
#pragma unroll
        for (int h = 0; h < RB / RBR; ++h) {
            const int rb0 = h * RBR;
            if (rb0 >= nrows) break;
            PT Uo[BT][SPLIT ? SEG : 1], Udo[BT][SPLIT ? SEG : 1];
#pragma unroll
            for (int bt = 0; bt < BT; ++bt)
#pragma unroll
                for (int j = 0; j < (SPLIT ? SEG : 1); ++j) {
                    Uo[bt][j] = p_zero<PT>();
                    Udo[bt][j] = p_zero<PT>();
                }
#pragma unroll
            for (int rl = 0; rl < RBR; ++rl) {
                const int r = rb0 + rl;
                const bool live = r < nrows;
                const int kr = live ? k + r : k;
                const int d = lane - (lane_lo + r);
                // a unit's first row with a repeated last index (plain modes)
                V fr = V(1), tw = V(0.5);
                if constexpr (FOLD) {
                    const bool first = live && rr > 1 && kr == k0;
                    fr = first ? inv_rr : V(1);
                    tw = first ? tie0 : V(0.5);
                }
#pragma unroll
                for (int bt = 0; bt < BT; ++bt) {
                    const V ak_r = alpha_s[bt * n + kr];
                    V ak = live ? ak_r : V(0);
                    if constexpr (FOLD) ak = ak * fr;
                    V vk{};
                    if constexpr (HVP) {
                        const V vk_r = vdir_s[bt * n + kr];
                        vk = live ? vk_r : V(0);
                        if constexpr (FOLD) vk = vk * fr;
                    }
                    PT part = p_zero<PT>(), partd = p_zero<PT>();
#pragma unroll
                    for (int j = 0; j < SEG; ++j) {
                        const int b = KB + j;
                        VIn x = val[r][j];
                        if (j == 0) {
                            if constexpr (FOLD) x = tie_scale_w(d, x, tw);
                            else x = tie_scale(d, x);
                        }
                        PT &u = (SPLIT && (rl & 1)) ? Uo[bt][SPLIT ? j : 0] : U[bt][b];
                        PT &ud = (SPLIT && (rl & 1)) ? Udo[bt][SPLIT ? j : 0] : Ud[bt][b];
                        acc_cv(u, ak, x);
                        acc_cv(part, a_l[bt][b], x);
                        if constexpr (HVP) {
                            acc_cv(ud, vk, x);
                            acc_cv(partd, v_l[bt][b], x);
                            if constexpr (ATAN) {
                                VIn xd = vald[r][j];
                                if (j == 0) {
                                    if constexpr (FOLD) xd = tie_scale_w(d, xd, tw);
                                    else xd = tie_scale(d, xd);
                                }
                                acc_cv(ud, ak, xd);
                                acc_cv(partd, a_l[bt][b], xd);
                            }
                        }
                    }
                    buf[(rl * NC + bt) * kWave + lane] = part;
                    if constexpr (HVP) buf[(rl * NC + BT + bt) * kWave + lane] = partd;
                }
            }
            if constexpr (SPLIT) {
#pragma unroll
                for (int bt = 0; bt < BT; ++bt)
#pragma unroll
                    for (int j = 0; j < SEG; ++j) {
                        U[bt][KB + j] = p_add(U[bt][KB + j], Uo[bt][j]);
                        if constexpr (HVP) Ud[bt][KB + j] = p_add(Ud[bt][KB + j], Udo[bt][j]);
                    }
            }
            __builtin_amdgcn_wave_barrier();
            // ---- transposed reduction: lanes [r LPR, (r+1) LPR) sum row rb0 + r
            {
                const int r = lane / LPR, seg = lane % LPR;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const PT *src = buf + (r * NC + c) * kWave + seg * RBR;
                    PT s = tree_sum<RBR, PT>([&](int j) { return src[j]; });
                    s = group_sum<LPR>(s);
                    if (seg == 0) sbatch[r * NC + c] = s;
                }
            }
            __builtin_amdgcn_wave_barrier();
            // ---- level Q-1: S_{P',k} joins the column sums at index k (block KB),
            // and S_{P'} += S_k alpha_k
            {
                const int r = lane - lane_lo - rb0;
                if (r >= 0 && r < RBR && rb0 + r < nrows) {
                    const bool first = FOLD && rr > 1 && k + rb0 + r == k0;
#pragma unroll
                    for (int bt = 0; bt < BT; ++bt) {
                        PT s = sbatch[r * NC + bt];
                        if constexpr (FOLD) s = first ? s * inv_rr : s;
                        U[bt][KB] = p_add(U[bt][KB], s);
                        acc_cv(unitS[bt], a_l[bt][KB], s);
                        if constexpr (HVP) {
                            PT sd = sbatch[r * NC + BT + bt];
                            if constexpr (FOLD) sd = first ? sd * inv_rr : sd;
                            Ud[bt][KB] = p_add(Ud[bt][KB], sd);
                            acc_cv(unitSd[bt], a_l[bt][KB], sd);
                            acc_cv(unitSd[bt], v_l[bt][KB], s);
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        off += (int64_t)nrows * (n - k) - (int64_t)(nrows * (nrows - 1) / 2);
        k += nrows;
    }

    __device__ __forceinline__ void rows(int k_lo, int k_hi, int64_t off)
    {
        int k = k_lo;
        // the first row of a unit repeats the prefix's last index (run rr):
        // in the compensated mode general coefficients, one row (the plain
        // modes fold its two weights into batch_fast)
        if (!FOLD && rr > 1 && k == k0 && k < k_hi) {
            const int kb = k >> 6;
            if (kb == 0) batch<0>(k, k + 1, off);
            else if constexpr (NB > 1) {
                if (kb == 1) batch<(NB > 1 ? 1 : 0)>(k, k + 1, off);
                else if constexpr (NB > 2) {
                    if (kb == 2) batch<(NB > 2 ? 2 : 0)>(k, k + 1, off);
                    else if constexpr (NB > 3) batch<(NB > 3 ? 3 : 0)>(k, k + 1, off);
                }
            }
        }
        while (k < k_hi) {
            const int kb = k >> 6;
            if (kb == 0) batch_fast<0>(k, k_hi, off);
            else if constexpr (NB > 1) {
                if (kb == 1) batch_fast<(NB > 1 ? 1 : 0)>(k, k_hi, off);
                else if constexpr (NB > 2) {
                    if (kb == 2) batch_fast<(NB > 2 ? 2 : 0)>(k, k_hi, off);
                    else if constexpr (NB > 3) batch_fast<(NB > 3 ? 3 : 0)>(k, k_hi, off);
                }
            }
        }
    }
};

template <int Q, int NB, typename TIn, int MODE, int HV, int BT, int RBMAX>
__global__ void __launch_bounds__(256) pair_kernel(PairParams p)
{
    using Ps = Pass<Q, NB, TIn, MODE, HV, BT, RBMAX>;
    using V = typename Ps::V;
    using PT = typename Ps::PT;
    using CT = typename Ps::CT;
    constexpr bool HVP = Ps::HVP;
    constexpr int NC = Ps::NC;
    constexpr int QP = Ps::QP;

    extern __shared__ __align__(16) unsigned char smem[];
    V *alpha_s = reinterpret_cast<V *>(smem);                 // [BT][n]
    V *vdir_s = alpha_s + BT * p.n;                           // [BT][n] (HVP)
    const int n = p.n;
    const int lane = threadIdx.x & (kWave - 1);
    // the wave index is uniform across the wave: keep it (and all the unit and
    // row bookkeeping derived from it) in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    size_t stage_bytes = (size_t)BT * n * sizeof(V) * (HVP ? 2 : 1);
    stage_bytes = (stage_bytes + 15) & ~(size_t)15;
    PT *wave_base = reinterpret_cast<PT *>(smem + stage_bytes);
    PT *buf = wave_base + (size_t)wid * (RBMAX * NC * kWave + RBMAX * NC);
    PT *sbatch = buf + RBMAX * NC * kWave;
    // column sums across units (times the unit multipliers), one slot per lane
    PT *colw = wave_base + (size_t)nw * (RBMAX * NC * kWave + RBMAX * NC) +
               (size_t)wid * (BT * NB * kWave * (HVP ? 2 : 1));
    PT *coldw = colw + BT * NB * kWave;

    const int b0 = blockIdx.y * BT;      // first alpha vector of this tile
    Ps ps;
    ps.n = n;
    ps.lane = lane;
    ps.alpha_s = alpha_s;
    ps.vdir_s = vdir_s;
    ps.buf = buf;
    ps.sbatch = sbatch;
    // per-vector arrays (lower passes, BT == 1) sit a_stride entries apart
    ps.A = reinterpret_cast<const TIn *>(p.A) + (size_t)b0 * p.a_stride;
    ps.Ad = Ps::ATAN ? reinterpret_cast<const TIn *>(p.Ad) + (size_t)b0 * p.a_stride : nullptr;

    for (int i = threadIdx.x; i < BT * n; i += blockDim.x) {
        const int bt = i / n, j = i - bt * n;
        const bool ok = b0 + bt < p.B;
        alpha_s[i] = ok ? (V)p.alpha[(int64_t)(b0 + bt) * n + j] : V(0);
        if constexpr (HVP) vdir_s[i] = ok ? (V)p.vdir[(int64_t)(b0 + bt) * n + j] : V(0);
    }
    __syncthreads();
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int l = b * kWave + lane;
            ps.a_l[bt][b] = l < n ? alpha_s[bt * n + l] : V(0);
            ps.v_l[bt][b] = (HVP && l < n) ? vdir_s[bt * n + l] : V(0);
            colw[(bt * NB + b) * kWave + lane] = p_zero<PT>();
            if constexpr (HVP) coldw[(bt * NB + b) * kWave + lane] = p_zero<PT>();
        }

    const int64_t wave = (int64_t)blockIdx.x * nw + wid;
    // work plan: wave w owns units (Q >= 4) or rows (Q == 2) [plan[w], plan[w+1]),
    // cut on the host so that every wave gets the same modelled cost
    const int64_t u_lo = p.plan[wave];
    const int64_t u_hi = p.plan[wave + 1];

    if constexpr (QP > 0) {
        int P[QP];
        int64_t uidx = u_lo, ustart = 0;
        if (u_lo < u_hi) {
            unrank_tuple<QP>(u_lo, n, P);
            int tt[Q];
#pragma unroll
            for (int i = 0; i < QP; ++i) tt[i] = P[i];
            tt[QP] = tt[QP + 1] = P[QP - 1];
            ustart = rank_tuple<Q>(tt, n);
            ps.set_base(ustart, p.count);
        }
        double fq1 = 1.0;
        for (int i = 2; i <= Q - 1; ++i) fq1 *= (double)i;
        for (; uidx < u_hi; ++uidx) {
            // unit multiplier (q-1)!/prod r_p(P') alpha^{P'} and its tangent
            const int k0 = P[QP - 1];
            int run = 1;
            int wden = 1;
            for (int i = 1; i < QP; ++i) {
                run = (P[i] == P[i - 1]) ? run + 1 : 1;
                wden *= run;
            }
            CT Cu[BT], Cud[BT];
#pragma unroll
            for (int bt = 0; bt < BT; ++bt) {
                CT c = Coef<MODE>::make(fq1);
                CT cd = Coef<MODE>::make(0.0);
                for (int i = 0; i < QP; ++i) {
                    const CT ai = Coef<MODE>::make((double)alpha_s[bt * n + P[i]]);
                    if constexpr (HVP) {
                        const CT vi = Coef<MODE>::make((double)vdir_s[bt * n + P[i]]);
                        CT t2 = Coef<MODE>::mul(c, vi);
                        cd = Coef<MODE>::mul(cd, ai);
                        if constexpr (MODE == ACC_DD) cd = dd_add(cd, t2); else cd = cd + t2;
                    }
                    c = Coef<MODE>::mul(c, ai);
                }
                Cu[bt] = Coef<MODE>::div(c, wden);
                Cud[bt] = Coef<MODE>::div(cd, wden);
            }
            ps.k0 = k0;
            ps.rr = run + 1;
            ps.begin_unit();
            ps.rows(k0, n, ustart);
            // fold the unit into the running column sums
#pragma unroll
            for (int bt = 0; bt < BT; ++bt)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    PT c = colw[(bt * NB + b) * kWave + lane];
                    acc_unit(c, Cu[bt], ps.U[bt][b]);
                    colw[(bt * NB + b) * kWave + lane] = c;
                    if constexpr (HVP) {
                        PT cd = coldw[(bt * NB + b) * kWave + lane];
                        acc_unit(cd, Cud[bt], ps.U[bt][b]);
                        acc_unit(cd, Cu[bt], ps.Ud[bt][b]);
                        coldw[(bt * NB + b) * kWave + lane] = cd;
                    }
                }
            // S_{P'}: wave reduction, written by lane 0
#pragma unroll
            for (int bt = 0; bt < BT; ++bt) {
                const PT s = group_sum<kWave>(ps.unitS[bt]);
                PT sd = ps.unitSd[bt];
                if constexpr (HVP) sd = group_sum<kWave>(sd);
                if (lane == 0 && b0 + bt < p.B) {
                    store_s(p.S_out, (int64_t)(b0 + bt) * p.units + uidx, s);
                    if constexpr (HVP) store_s(p.Sd_out, (int64_t)(b0 + bt) * p.units + uidx, sd);
                }
            }
            // next unit in nested-loop order
            ustart += (int64_t)(n - k0) * (n - k0 + 1) / 2;
            int pos = QP - 1;
            while (pos >= 0 && P[pos] == n - 1) --pos;
            if (pos < 0) break;
            P[pos] += 1;
            for (int i = pos + 1; i < QP; ++i) P[i] = P[pos];
        }
    } else {
        // Q == 2: the single unit (empty prefix, multiplier 1); the wave owns rows [u_lo, u_hi)
        if (u_lo < u_hi) {
            ps.k0 = 0;
            ps.rr = 1;
            ps.begin_unit();
            const int k_first = (int)u_lo;
            const int64_t off0 = (int64_t)k_first * n - (int64_t)k_first * (k_first - 1) / 2;
            ps.set_base(off0, p.count);
            ps.rows(k_first, (int)u_hi, off0);
#pragma unroll
            for (int bt = 0; bt < BT; ++bt)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    PT c = colw[(bt * NB + b) * kWave + lane];
                    c = p_add(c, ps.U[bt][b]);
                    colw[(bt * NB + b) * kWave + lane] = c;
                    if constexpr (HVP) coldw[(bt * NB + b) * kWave + lane] = p_add(coldw[(bt * NB + b) * kWave + lane], ps.Ud[bt][b]);
                }
        }
    }

    // ---- workgroup reduction of the column sums, scaled by mu, to partials
    __syncthreads();
    // gather the per-wave column sums into the (now free) batch-buffer region
    // as [waves][NC][NB*64] and reduce
    PT *red = wave_base;
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            red[((size_t)wid * NC + bt) * (NB * kWave) + b * kWave + lane] = colw[(bt * NB + b) * kWave + lane];
            if constexpr (HVP)
                red[((size_t)wid * NC + BT + bt) * (NB * kWave) + b * kWave + lane] = coldw[(bt * NB + b) * kWave + lane];
        }
    __syncthreads();
    for (int i = threadIdx.x; i < NC * n; i += blockDim.x) {
        const int c = i / n, l = i - c * n;
        PT s = p_zero<PT>();
        for (int w = 0; w < nw; ++w) s = p_add(s, red[((size_t)w * NC + c) * (NB * kWave) + l]);
        const int bt = c % BT;
        const bool tan = c >= BT;
        if (b0 + bt >= p.B) continue;
        // partial layout: [vector][workgroup][n] as (hi, lo) pairs
        double *dst = (tan ? p.part_d : p.part) + 2 * (((int64_t)(b0 + bt) * gridDim.x + blockIdx.x) * n + l);
        double hi, lo;
        if constexpr (MODE == ACC_DD) {
            // exact scaling by the integer mu: (s.hi + s.lo) * mu as a pair
            hi = s.hi * p.mu;
            lo = __builtin_fma(s.hi, p.mu, -hi) + s.lo * p.mu;
        } else {
            hi = (double)s * p.mu;
            lo = 0.0;
        }
        dst[0] = hi;
        dst[1] = lo;
    }
}

// ------------------------------------------------------------- launchers ----
namespace {

template <int Q, int NB, typename TIn, int MODE, int HV, int BT>
constexpr int batch_rows()
{
    constexpr bool HVP = HV > 0;
    using PT = typename ModeT<MODE>::P;
    constexpr int NC = BT * (HVP ? 2 : 1);
    constexpr int bytes = NC * kWave * (int)sizeof(PT);
    constexpr int rb0 = 8192 / bytes;
    return rb0 >= 8 ? 8 : rb0 >= 4 ? 4 : 2;   // rows per batch at most (LDS budget)
}

template <int Q, int NB, typename TIn, int MODE, int HV, int BT>
hipError_t launch_pair(const PairParams &pp, int groups, int btiles, hipStream_t st)
{
    constexpr bool HVP = HV > 0;
    constexpr int RB = batch_rows<Q, NB, TIn, MODE, HV, BT>();
    using V = typename ModeT<MODE>::V;
    using PT = typename ModeT<MODE>::P;
    constexpr int NC = BT * (HVP ? 2 : 1);
    size_t stage = (size_t)BT * pp.n * sizeof(V) * (HVP ? 2 : 1);
    stage = (stage + 15) & ~(size_t)15;
    const size_t per_wave = (size_t)(RB * NC * kWave + RB * NC) * sizeof(PT);
    const size_t cols = (size_t)4 * BT * NB * kWave * (HVP ? 2 : 1) * sizeof(PT);
    const size_t red = (size_t)4 * NC * NB * kWave * sizeof(PT);
    if (red > per_wave * 4 + cols) return hipErrorInvalidValue;
    const size_t lds = stage + per_wave * 4 + cols;
    auto kern = pair_kernel<Q, NB, TIn, MODE, HV, BT, RB>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (pp.occ_query) {
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, lds);
        *pp.occ_query = nb;
        return e;
    }
    hipLaunchKernelGGL(kern, dim3(groups, btiles), dim3(256), lds, st, pp);
    return hipGetLastError();
}

template <int Q, int NB, typename TIn, int MODE, int HV>
hipError_t dispatch_bt(const PairParams &pp, int groups, int bt, hipStream_t st)
{
    // vector tiles (several vectors per read of a shared input array): FP32
    // and plain FP64 accumulation, first pass (a shared tensor) only
    if constexpr (MODE == ACC_PLAIN32 || (MODE == ACC_PLAIN64 && HV < 2)) {
        if (bt >= 4 && pp.a_stride == 0)
            return launch_pair<Q, NB, TIn, MODE, HV, 4>(pp, groups, (int)((pp.B + 3) / 4), st);
        if (bt >= 2 && pp.a_stride == 0)
            return launch_pair<Q, NB, TIn, MODE, HV, 2>(pp, groups, (int)((pp.B + 1) / 2), st);
    }
    (void)bt;
    return launch_pair<Q, NB, TIn, MODE, HV, 1>(pp, groups, (int)pp.B, st);
}

template <int Q, typename TIn, int MODE, int HV>
hipError_t dispatch_nb(const PairParams &pp, int groups, int bt, hipStream_t st)
{
    const int nb = (pp.n + kWave - 1) / kWave;
    if (nb <= 1) return dispatch_bt<Q, 1, TIn, MODE, HV>(pp, groups, bt, st);
    if (nb <= 2) return dispatch_bt<Q, 2, TIn, MODE, HV>(pp, groups, bt, st);
    return dispatch_bt<Q, 4, TIn, MODE, HV>(pp, groups, bt, st);
}

template <typename TIn, int MODE, int HV>
hipError_t dispatch_q(int q, const PairParams &pp, int groups, int bt, hipStream_t st)
{
    switch (q) {
    case 2: return dispatch_nb<2, TIn, MODE, HV>(pp, groups, bt, st);
    case 4: return dispatch_nb<4, TIn, MODE, HV>(pp, groups, bt, st);
    case 6: return dispatch_nb<6, TIn, MODE, HV>(pp, groups, bt, st);
    case 8: return dispatch_nb<8, TIn, MODE, HV>(pp, groups, bt, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace tk
