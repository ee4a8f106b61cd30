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
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

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

__device__ __forceinline__ DD p_shfl_xor(DD a, int m)
{
    return DD{__shfl_xor(a.hi, m), __shfl_xor(a.lo, m)};
}
__device__ __forceinline__ double p_shfl_xor(double a, int m) { return __shfl_xor(a, m); }
__device__ __forceinline__ float p_shfl_xor(float a, int m) { return __shfl_xor(a, m); }

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
template <int MODE>
struct In<double, MODE> {
    using R = typename ModeT<MODE>::V;
    __device__ __forceinline__ static R load(const void *p, int64_t i)
    {
        return (R) reinterpret_cast<const double *>(p)[i];
    }
};
template <int MODE>
struct In<float, MODE> {
    using R = typename ModeT<MODE>::V;
    __device__ __forceinline__ static R load(const void *p, int64_t i)
    {
        return (R) reinterpret_cast<const float *>(p)[i];
    }
};
template <int MODE>
struct In<uint16_t, MODE> {
    using R = typename ModeT<MODE>::V;
    __device__ __forceinline__ static R load(const void *p, int64_t i)
    {
        return (R)bf16_to_float(reinterpret_cast<const uint16_t *>(p)[i]);
    }
};
template <>
struct In<DD, ACC_DD> {
    using R = DD;
    __device__ __forceinline__ static DD load(const void *p, int64_t i)
    {
        const double *q = reinterpret_cast<const double *>(p) + 2 * i;
        return DD{q[0], q[1]};
    }
};

// acc += c * v where v may be a DD (intermediate arrays in DD mode).
template <typename PT, typename CT, typename VT>
__device__ __forceinline__ void acc_cv(PT &acc, CT c, VT v) { acc_fma(acc, c, v); }

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
// Template parameters:
//   Q     order of the input array (even, >= 2)
//   NB    column blocks per lane (n <= 64 NB)
//   TIn   element type of the input array (double, float, uint16_t = BF16, DD)
//   MODE  accumulation mode
//   HV    0: values only; 1: tangents of alpha (directional derivative along v);
//         2: tangents of alpha and of the input array (lower passes of a derivative)
//   BT    number of alpha vectors handled together (blockIdx.y selects the tile)
//   RB    rows per transposed-reduction batch
template <int Q, int NB, typename TIn, int MODE, int HV, int BT, int RB>
__global__ void __launch_bounds__(256) pair_kernel(PairParams p)
{
    constexpr bool HVP = HV > 0;
    constexpr bool ATAN = HV > 1;   // the input array carries a tangent
    using V = typename ModeT<MODE>::V;
    using PT = typename ModeT<MODE>::P;
    using CT = typename Coef<MODE>::T;
    using InL = In<TIn, MODE>;
    using VIn = typename InL::R;               // value type read from the array
    constexpr int NC = BT * (HVP ? 2 : 1);     // reduced components per row
    constexpr int LPR = kWave / RB;            // lanes per row in the batch reduction
    constexpr int QP = Q - 2;                  // unit prefix length

    extern __shared__ __align__(16) unsigned char smem[];
    V *alpha_s = reinterpret_cast<V *>(smem);                 // [BT][n]
    V *vdir_s = alpha_s + BT * p.n;                           // [BT][n] (HVP)
    const int n = p.n;
    const int lane = threadIdx.x & (kWave - 1);
    // the wave index is uniform across the wave: keep it (and all the unit and
    // row bookkeeping derived from it) in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    size_t stage_bytes = (size_t)BT * n * sizeof(V) * (HVP ? 2 : 1);
    stage_bytes = (stage_bytes + 15) & ~(size_t)15;
    PT *buf = reinterpret_cast<PT *>(smem + stage_bytes) + (size_t)wid * (RB * NC * kWave + RB * NC);
    PT *sbatch = buf + RB * NC * kWave;                      // [RB][NC] row sums of a batch
    // column sums across units (times the unit multipliers), one slot per lane
    PT *colw = reinterpret_cast<PT *>(smem + stage_bytes) + (size_t)(blockDim.x / kWave) * (RB * NC * kWave + RB * NC) +
               (size_t)wid * (BT * NB * kWave * (HVP ? 2 : 1));
    PT *coldw = colw + BT * NB * kWave;

    const int b0 = blockIdx.y * BT;      // first alpha vector of this tile
    // per-vector arrays (lower passes, BT == 1) sit a_stride entries apart
    const void *A = p.A;
    const void *Ad = p.Ad;
    if (p.a_stride) {
        const size_t esz = sizeof(TIn);
        A = reinterpret_cast<const unsigned char *>(p.A) + (size_t)b0 * p.a_stride * esz;
        if (ATAN) Ad = reinterpret_cast<const unsigned char *>(p.Ad) + (size_t)b0 * p.a_stride * esz;
    }
    for (int i = threadIdx.x; i < BT * n; i += blockDim.x) {
        const int bt = i / n, j = i - bt * n;
        const bool ok = b0 + bt < p.B;
        alpha_s[i] = ok ? (V)p.alpha[(int64_t)(b0 + bt) * n + j] : V(0);
        if constexpr (HVP)
            vdir_s[i] = ok ? (V)p.vdir[(int64_t)(b0 + bt) * n + j] : V(0);
    }
    __syncthreads();

    // per-lane column state: l = 64 b + lane
    V a_l[BT][NB], v_l[BT][NB];
    PT U[BT][NB], Ud[BT][NB];         // column sums within the current unit
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int l = b * kWave + lane;
            a_l[bt][b] = l < n ? alpha_s[bt * n + l] : V(0);
            v_l[bt][b] = (HVP && l < n) ? vdir_s[bt * n + l] : V(0);
            colw[(bt * NB + b) * kWave + lane] = p_zero<PT>();
            if constexpr (HVP) coldw[(bt * NB + b) * kWave + lane] = p_zero<PT>();
        }

    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wid;
    // work plan: wave w owns units (Q >= 4) or rows (Q == 2) [plan[w], plan[w+1]),
    // cut on the host so that every wave gets the same modelled cost
    const int64_t u_lo = p.plan[wave];
    const int64_t u_hi = p.plan[wave + 1];
    bool active = u_lo < u_hi;

    int P[QP > 0 ? QP : 1];
    int64_t uidx = u_lo, ustart = 0;
    int k_first = 0, k_end = n;
    if constexpr (QP > 0) {
        if (active) {
            unrank_tuple<QP>(u_lo, n, P);
            int tt[Q];
#pragma unroll
            for (int i = 0; i < QP; ++i) tt[i] = P[i];
            tt[QP] = tt[QP + 1] = P[QP - 1];
            ustart = rank_tuple<Q>(tt, n);
        }
    } else {
        // Q == 2: one unit, the wave owns rows [u_lo, u_hi); row k starts at k n - k(k-1)/2
        k_first = (int)u_lo;
        k_end = (int)u_hi;
        ustart = (int64_t)k_first * n - (int64_t)k_first * (k_first - 1) / 2;
    }

    // ---- loop over units
    while (active) {
        int k0, rr;
        CT Cu[BT], Cud[BT];        // unit multiplier (q-1)!/prod r_p(P') alpha^{P'} and its tangent
        if constexpr (QP > 0) {
            if (uidx >= u_hi) break;
            k0 = P[QP - 1];
            int run = 1;
            double wden = 1.0;
            for (int i = 1; i < QP; ++i) {
                run = (P[i] == P[i - 1]) ? run + 1 : 1;
                wden *= (double)run;
            }
            rr = run + 1;   // r_{Q-1} of the first row (k == k0)
            double fq1 = 1.0;
            for (int i = 2; i <= Q - 1; ++i) fq1 *= (double)i;
#pragma unroll
            for (int bt = 0; bt < BT; ++bt) {
                CT c = Coef<MODE>::div(Coef<MODE>::make(fq1), 1);
                CT cd = Coef<MODE>::make(0.0);
                for (int i = 0; i < QP; ++i) {
                    const V ai = alpha_s[bt * n + P[i]];
                    if constexpr (HVP) {
                        const V vi = vdir_s[bt * n + P[i]];
                        // (c + eps cd)(ai + eps vi)
                        cd = Coef<MODE>::mul(cd, Coef<MODE>::make((double)ai));
                        CT t2 = Coef<MODE>::mul(c, Coef<MODE>::make((double)vi));
                        if constexpr (MODE == ACC_DD)
                            cd = dd_add(cd, t2);
                        else
                            cd = cd + t2;
                    }
                    c = Coef<MODE>::mul(c, Coef<MODE>::make((double)ai));
                }
                // divide by the product of run-length factorials (exact integer)
                Cu[bt] = Coef<MODE>::div(c, (int)wden);
                Cud[bt] = Coef<MODE>::div(cd, (int)wden);
            }
        } else {
            k0 = 0;
            rr = 1;
#pragma unroll
            for (int bt = 0; bt < BT; ++bt) {
                Cu[bt] = Coef<MODE>::make(1.0);
                Cud[bt] = Coef<MODE>::make(0.0);
            }
        }
        const int k_lo = (QP > 0) ? k0 : k_first;
        const int k_hi = (QP > 0) ? n : k_end;
        // 1/r, alpha_k0/r and v_k0/r for the unit's first row (r = rr)
        const CT inv_rr = Coef<MODE>::div(Coef<MODE>::make(1.0), rr);
        CT ak0_rr[BT], vk0_rr[BT];
#pragma unroll
        for (int bt = 0; bt < BT; ++bt) {
            ak0_rr[bt] = Coef<MODE>::div(Coef<MODE>::make((double)alpha_s[bt * n + k0]), rr);
            vk0_rr[bt] = HVP ? Coef<MODE>::div(Coef<MODE>::make((double)vdir_s[bt * n + k0]), rr)
                             : Coef<MODE>::make(0.0);
        }

#pragma unroll
        for (int bt = 0; bt < BT; ++bt)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                U[bt][b] = p_zero<PT>();
                Ud[bt][b] = p_zero<PT>();
            }
        PT unitS[BT], unitSd[BT];   // lane partial of S_{P'}
#pragma unroll
        for (int bt = 0; bt < BT; ++bt) {
            unitS[bt] = p_zero<PT>();
            unitSd[bt] = p_zero<PT>();
        }

        int64_t off = ustart;   // offset of row k_lo
        for (int kb0 = k_lo; kb0 < k_hi; kb0 += RB) {
            const int nrows = min(RB, k_hi - kb0);
            // ---- phase 1: issue the loads of the batch
            VIn val[RB][NB];
            VIn vald[RB][NB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int k = kb0 + r;
                const int64_t roff = off + (int64_t)r * (n - kb0) - (int64_t)r * (r - 1) / 2;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int l = b * kWave + lane;
                    val[r][b] = zero_like(VIn());
                    vald[r][b] = zero_like(VIn());
                    if (r < nrows && b >= (k >> 6)) {
                        if (l >= k && l < n) {
                            val[r][b] = InL::load(A, roff + (l - k));
                            if constexpr (ATAN)
                                vald[r][b] = InL::load(Ad, roff + (l - k));
                        }
                    }
                }
            }
            // ---- phase 2: row partials and in-unit column sums.  Only the block
            // holding the diagonal entry l == k carries the tie factor 1/(r_k+1).
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (r >= nrows) break;
                const int k = kb0 + r;
                const int kb = k >> 6;
                const int rk = (QP > 0 && k == k0) ? rr : 1;          // r_{Q-1}(P', k)
#pragma unroll
                for (int bt = 0; bt < BT; ++bt) {
                    const V ak = alpha_s[bt * n + k];
                    const CT cu = Coef<MODE>::div(Coef<MODE>::make((double)ak), rk);
                    const CT cu_tie = Coef<MODE>::div(cu, rk + 1);
                    const CT ck_tie = Coef<MODE>::div(Coef<MODE>::make((double)ak), rk + 1);
                    CT cud = Coef<MODE>::make(0.0), cud_tie = cud, vk_tie = cud;
                    if constexpr (HVP) {
                        const V vk = vdir_s[bt * n + k];
                        cud = Coef<MODE>::div(Coef<MODE>::make((double)vk), rk);
                        cud_tie = Coef<MODE>::div(cud, rk + 1);
                        vk_tie = Coef<MODE>::div(Coef<MODE>::make((double)vk), rk + 1);
                    }
                    PT part = p_zero<PT>(), partd = p_zero<PT>();
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (b < kb) continue;
                        const int l = b * kWave + lane;
                        const VIn x = val[r][b];
                        if (b == kb) {
                            const bool tie = (l == k);
                            const CT cU = tie ? cu_tie : cu;
                            const CT cP = tie ? ck_tie : Coef<MODE>::make((double)a_l[bt][b]);
                            acc_cv(U[bt][b], cU, x);
                            acc_cv(part, cP, x);
                            if constexpr (HVP) {
                                const VIn xd = vald[r][b];
                                const CT cUd = tie ? cud_tie : cud;
                                const CT cPd = tie ? vk_tie : Coef<MODE>::make((double)v_l[bt][b]);
                                acc_cv(Ud[bt][b], cUd, x);
                                acc_cv(partd, cPd, x);
                                if constexpr (ATAN) {
                                    acc_cv(Ud[bt][b], cU, xd);
                                    acc_cv(partd, cP, xd);
                                }
                            }
                        } else {
                            acc_cv(U[bt][b], cu, x);
                            acc_cv(part, a_l[bt][b], x);
                            if constexpr (HVP) {
                                const VIn xd = vald[r][b];
                                acc_cv(Ud[bt][b], cud, x);
                                acc_cv(partd, v_l[bt][b], x);
                                if constexpr (ATAN) {
                                    acc_cv(Ud[bt][b], cu, xd);
                                    acc_cv(partd, a_l[bt][b], xd);
                                }
                            }
                        }
                    }
                    buf[(r * NC + bt) * kWave + lane] = part;
                    if constexpr (HVP)
                        buf[(r * NC + BT + bt) * kWave + lane] = partd;
                }
            }
            __builtin_amdgcn_wave_barrier();
            // ---- transposed reduction: lanes [r*LPR, (r+1)*LPR) sum row r
            {
                const int r = lane / LPR, seg = lane % LPR;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    PT s = p_zero<PT>();
#pragma unroll
                    for (int j = 0; j < RB; ++j)
                        s = p_add(s, buf[(r * NC + c) * kWave + seg * RB + j]);
#pragma unroll
                    for (int m = 1; m < LPR; m <<= 1)
                        s = p_add(s, p_shfl_xor(s, m));
                    if (seg == 0)
                        sbatch[r * NC + c] = s;
                }
            }
            __builtin_amdgcn_wave_barrier();
            // ---- level Q-1: S_{P',k}/r_k joins the column sums at index k; S_{P'} partial.
            // r_k = rr only for the unit's first row (k == k0), 1 otherwise.
            const int bfirst = kb0 >> 6, blast = (kb0 + nrows - 1) >> 6;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b < bfirst || b > blast) continue;   // blocks holding no row of the batch
                const int k = b * kWave + lane;
                if (k >= kb0 && k < kb0 + nrows) {
                    const int r = k - kb0;
                    const bool first = (QP > 0) && (k == k0);
#pragma unroll
                    for (int bt = 0; bt < BT; ++bt) {
                        const PT s = sbatch[r * NC + bt];
                        const CT one = Coef<MODE>::make(1.0);
                        const CT inv = first ? inv_rr : one;
                        acc_cv(U[bt][b], inv, s);
                        // S_{P'} += S_k alpha_k / r_k
                        const CT ak = first ? ak0_rr[bt] : Coef<MODE>::make((double)a_l[bt][b]);
                        acc_cv(unitS[bt], ak, s);
                        if constexpr (HVP) {
                            const PT sd = sbatch[r * NC + BT + bt];
                            acc_cv(Ud[bt][b], inv, sd);
                            const CT vk = first ? vk0_rr[bt] : Coef<MODE>::make((double)v_l[bt][b]);
                            acc_cv(unitSd[bt], ak, sd);
                            acc_cv(unitSd[bt], vk, s);
                        }
                    }
                }
            }
            off += (int64_t)nrows * (n - kb0) - (int64_t)nrows * (nrows - 1) / 2;
            __builtin_amdgcn_wave_barrier();
        }

        // ---- unit end: fold the unit into the running column sums
#pragma unroll
        for (int bt = 0; bt < BT; ++bt)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                PT c = colw[(bt * NB + b) * kWave + lane];
                acc_unit(c, Cu[bt], U[bt][b]);
                colw[(bt * NB + b) * kWave + lane] = c;
                if constexpr (HVP) {
                    PT cd = coldw[(bt * NB + b) * kWave + lane];
                    acc_unit(cd, Cud[bt], U[bt][b]);
                    acc_unit(cd, Cu[bt], Ud[bt][b]);
                    coldw[(bt * NB + b) * kWave + lane] = cd;
                }
            }
        if constexpr (QP > 0) {
            // S_{P'}: wave reduction, written by lane 0
#pragma unroll
            for (int bt = 0; bt < BT; ++bt) {
                PT s = unitS[bt];
                for (int m = 1; m < kWave; m <<= 1) s = p_add(s, p_shfl_xor(s, m));
                PT sd = unitSd[bt];
                if constexpr (HVP)
                    for (int m = 1; m < kWave; m <<= 1) sd = p_add(sd, p_shfl_xor(sd, m));
                if (lane == 0 && b0 + bt < p.B) {
                    store_s(p.S_out, (int64_t)(b0 + bt) * p.units + uidx, s);
                    if constexpr (HVP)
                        store_s(p.Sd_out, (int64_t)(b0 + bt) * p.units + uidx, sd);
                }
            }
            // next unit
            ustart += (int64_t)(n - k0) * (n - k0 + 1) / 2;
            int pos = QP - 1;
            while (pos >= 0 && P[pos] == n - 1) --pos;
            if (pos < 0) break;
            P[pos] += 1;
            for (int i = pos + 1; i < QP; ++i) P[i] = P[pos];
            uidx += 1;
        } else {
            break;   // Q == 2: the wave's rows are done
        }
    }

    // ---- workgroup reduction of the column sums, scaled by mu, to partials
    __syncthreads();
    // the per-wave column sums sit after the batch buffers; gather them into the
    // (now free) batch-buffer region as [waves][NC][NB*64] and reduce
    PT *red = reinterpret_cast<PT *>(smem + stage_bytes);
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int bt = 0; bt < BT; ++bt)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            red[((size_t)wid * NC + bt) * (NB * kWave) + b * kWave + lane] = colw[(bt * NB + b) * kWave + lane];
            if constexpr (HVP)
                red[((size_t)wid * NC + BT + bt) * (NB * kWave) + b * kWave + lane] =
                    coldw[(bt * NB + b) * kWave + lane];
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
        double *dst = (tan ? p.part_d : p.part) +
                      2 * (((int64_t)(b0 + bt) * gridDim.x + blockIdx.x) * n + l);
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

// Final pass: g[b][l] = sum over passes and workgroups of the partials, in a
// fixed order (compensated).
__global__ void __launch_bounds__(256) reduce_partials_kernel(ReduceParams p)
{
    __shared__ double sh_hi[256], sh_lo[256];
    const int cols = 8;                       // columns per block
    const int lane_col = threadIdx.x % cols;
    const int slot = threadIdx.x / cols;      // 32 slots
    const int b = blockIdx.y;
    const int l = blockIdx.x * cols + lane_col;
    DD s{0.0, 0.0};
    if (l < p.n) {
        for (int ps = 0; ps < p.npass; ++ps) {
            const double *src = p.part[ps] + 2 * ((int64_t)b * p.groups[ps]) * p.n;
            for (int w = slot; w < p.groups[ps]; w += 32) {
                const double *q = src + 2 * ((int64_t)w * p.n + l);
                double t, e;
                two_sum(s.hi, q[0], t, e);
                s.hi = t;
                s.lo += e + q[1];
            }
        }
    }
    sh_hi[threadIdx.x] = s.hi;
    sh_lo[threadIdx.x] = s.lo;
    __syncthreads();
    for (int stride = 16; stride >= 1; stride >>= 1) {
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
    constexpr int rb = rb0 >= 8 ? 8 : rb0 >= 4 ? 4 : 2;
    // the load buffer holds RB x NB values per lane: keep it at <= 16 entries
    return (rb * NB > 16) ? (16 / NB >= 2 ? 16 / NB : 2) : rb;
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
    hipLaunchKernelGGL(kern, dim3(groups, btiles), dim3(256), lds, st, pp);
    return hipGetLastError();
}

template <int Q, int NB, typename TIn, int MODE, int HV>
hipError_t dispatch_bt(const PairParams &pp, int groups, int bt, hipStream_t st)
{
    if constexpr (MODE == ACC_PLAIN32) {
        if (bt >= 4 && pp.a_stride == 0)
            return launch_pair<Q, NB, TIn, MODE, HV, 4>(pp, groups, (int)((pp.B + 3) / 4), st);
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


// ------------------------------------------------------------ work plans ----
// Modelled cost of one row (fixed part plus one term per 64-column block it
// touches) and of one unit (fixed part).  The weights approximate the
// instruction counts of the kernel; only their ratios matter.
namespace {
constexpr double kCostRow = 6.0, kCostBlock = 8.0, kCostBatch = 4.0, kCostUnit = 60.0;

std::vector<int64_t> make_plan_host(int q, int64_t n, int64_t waves)
{
    const int nb = (int)((n + kWave - 1) / kWave);
    // cost of the rows k in [k0, n) of a unit whose leading indices end at k0
    std::vector<double> tail(n + 1, 0.0);
    for (int64_t k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + kCostRow + kCostBlock * (nb - (k >> 6));
    std::vector<int64_t> plan(waves + 1, 0);
    if (q == 2) {
        double total = tail[0];
        int64_t w = 1;
        double acc = 0.0;
        for (int64_t k = 0; k < n && w < waves; ++k) {
            acc += kCostRow + kCostBlock * (nb - (k >> 6));
            while (w < waves && acc >= total * (double)w / (double)waves) plan[w++] = k + 1;
        }
        while (w <= waves) plan[w++] = n;
        plan[waves] = n;
        return plan;
    }
    const int qp = q - 2;
    auto unit_cost = [&](int k0) {
        const double rows = (double)(n - k0);
        return tail[k0] + kCostBatch * std::ceil(rows / 4.0) + kCostUnit;
    };
    // units in nested-loop order; only the last index matters for the cost
    std::vector<int> t(qp, 0);
    double total = 0.0;
    int64_t units = 0;
    while (true) {
        total += unit_cost(t[qp - 1]);
        ++units;
        int pos = qp - 1;
        while (pos >= 0 && t[pos] == n - 1) --pos;
        if (pos < 0) break;
        t[pos] += 1;
        for (int i = pos + 1; i < qp; ++i) t[i] = t[pos];
    }
    std::fill(t.begin(), t.end(), 0);
    int64_t w = 1, u = 0;
    double acc = 0.0;
    while (u < units && w < waves) {
        acc += unit_cost(t[qp - 1]);
        ++u;
        while (w < waves && acc >= total * (double)w / (double)waves) plan[w++] = u;
        int pos = qp - 1;
        while (pos >= 0 && t[pos] == n - 1) --pos;
        if (pos < 0) break;
        t[pos] += 1;
        for (int i = pos + 1; i < qp; ++i) t[i] = t[pos];
    }
    while (w <= waves) plan[w++] = units;
    plan[waves] = units;
    return plan;
}

std::mutex g_plan_mu;
std::map<std::tuple<int, int, int64_t, int>, int64_t *> g_plans;
}  // namespace

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
    const std::vector<int64_t> h = make_plan_host(q, n, (int64_t)groups * 4);
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
int pass_groups(int q, int64_t n, int64_t count)
{
    if (q == 2) {   // waves split the rows of the single unit: a few rows per wave
        int64_t g = (n + 15) / 16;
        return (int)(g < 1 ? 1 : g);
    }
    // about 4K entries per wave, at most 3 resident workgroups per CU on 256 CUs
    int64_t g = (count + 4 * 4096 - 1) / (4 * 4096);
    if (g < 1) g = 1;
    if (g > 768) g = 768;
    return (int)g;
}

hipError_t launch_pass(int q, int in_kind, int mode, int hv, int bt, const PairParams &pp,
                       int groups, hipStream_t st)
{
    // in_kind: 0 double, 1 float, 2 bf16, 3 DD intermediate;
    // hv: 0 value only, 1 tangent of alpha, 2 tangent of alpha and of the array
    if (mode == ACC_DD) {
        if (hv) return hipErrorInvalidValue;
        if (in_kind == 0) return dispatch_q<double, ACC_DD, 0>(q, pp, groups, bt, st);
        if (in_kind == 3) return dispatch_q<DD, ACC_DD, 0>(q, pp, groups, bt, st);
        return hipErrorInvalidValue;
    }
    if (mode == ACC_PLAIN64) {
        if (in_kind != 0) return hipErrorInvalidValue;
        if (hv == 0) return dispatch_q<double, ACC_PLAIN64, 0>(q, pp, groups, bt, st);
        if (hv == 1) return dispatch_q<double, ACC_PLAIN64, 1>(q, pp, groups, bt, st);
        return dispatch_q<double, ACC_PLAIN64, 2>(q, pp, groups, bt, st);
    }
    if (mode == ACC_PLAIN32) {
        if (in_kind == 1) {
            if (hv == 0) return dispatch_q<float, ACC_PLAIN32, 0>(q, pp, groups, bt, st);
            if (hv == 1) return dispatch_q<float, ACC_PLAIN32, 1>(q, pp, groups, bt, st);
            return dispatch_q<float, ACC_PLAIN32, 2>(q, pp, groups, bt, st);
        }
        if (in_kind == 2) {
            if (hv == 0) return dispatch_q<uint16_t, ACC_PLAIN32, 0>(q, pp, groups, bt, st);
            if (hv == 1) return dispatch_q<uint16_t, ACC_PLAIN32, 1>(q, pp, groups, bt, st);
            return hipErrorInvalidValue;   // BF16 is a storage type of the top array only
        }
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceParams &rp, int64_t B, hipStream_t st)
{
    dim3 grid((rp.n + 7) / 8, (unsigned)B);
    hipLaunchKernelGGL(reduce_partials_kernel, grid, dim3(256), 0, st, rp);
    return hipGetLastError();
}

}  // namespace tk
