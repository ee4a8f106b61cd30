// First pass of the contraction for a batch of vectors on FP64 MFMA.
//
// For one unit P' (the q-2 leading indices of a packed tuple, k0 = P'_last),
// the rows k in [k0, n) and their entries l >= k form a triangle.  With the
// entries weighted by their multiplicities (off the diagonal 1, on it 1/2;
// in the unit's first row, whose index repeats the prefix's run of length
// rr - 1, 1/rr off and 1/(rr (rr+1)) on the diagonal) into the upper
// triangular T^, and M = T^ + T^T the symmetric matrix of the unit, the first
// two levels of the contraction (see tk_pass.hpp) are, for every vector v,
//
//   U_v = M alpha_v              (column sums plus row sums of the unit),
//   S_v = alpha_v^T M alpha_v / 2 (the unit's entry of the next pass's array),
//
// and the unit adds Cu_v U_v to the column sums, Cu_v = (q-1)!/prod r_p(P')
// alpha_v^{P'}.  For a tile of 16 vectors, U restricted to the 16 rows of one
// row tile t is a dense product M[tile t, :] A, run on v_mfma_f64_16x16x4f64.
//
// Each wave owns a range of units and sweeps the row tiles t = 0, 1, ...: for
// each t it walks its units (those with rows in tile t), stages M[tile t, :]
// from the packed array into its own LDS buffer in chunks of 16 x 64 (each
// entry read from its place in the upper triangle, weighted, zero outside the
// unit: such loads are sent past the unit's buffer range), with the loads of
// the next chunk in flight while the current chunk is multiplied, and adds
// Cu U to one accumulator for tile t.  Row offsets come from a table of row
// starts and are set up once per (unit, row tile), so a chunk costs little
// more than its loads, LDS traffic and MFMAs.  So every entry of
// the triangle is read twice (once for its row tile, once for its column
// tile), and a wave holds a single accumulator, with no data-dependent
// register indexing.  S is built up over the sweeps in the output array.  The
// wave writes its column sums as one partial per wave (the vector kernels'
// partial layout, with lo = 0), so the lower passes and the final reduction
// are shared; the reduction order is fixed by the launch shape.  The vector
// tiles of one range of units run on the same XCD (workgroup ids that differ
// by a multiple of 8), so that the range is read from HBM about once per batch.
#include "tk_common.hpp"
#include "tk_contract.hpp"

namespace tk {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kVB = 16;       // vectors per tile (MFMA columns)
constexpr int kXcds = 8;      // XCDs of the device: workgroup ids are dealt to them in turn
constexpr int kXW = 70;       // row stride (doubles) of a staged chunk (16 rows x 64 columns)
constexpr int kAS = kVB + 1;  // row stride of the alpha tile [k][v]

struct BatchArgs {
    const double *K;
    int n;
    const double *alpha;   // [B][n]
    int64_t B;
    int groups, tiles;
    const int64_t *plan;   // [groups * 4 + 1]: wave w takes units [plan[w], plan[w + 1])
    int64_t units;
    double *S_out;         // [B][units]
    double *part;          // [B][groups * 4][n] (hi, lo) pairs: one partial per wave
};

// Buffer-resource loads: an offset past the descriptor's range (or a negative
// one, which wraps) reads 0 instead of faulting.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc unit_rsrc(const double *base, int64_t entries)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base), (short)0, (int)(entries * 8), 0x00020000);
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A unit of a wave's range: its prefix, k0, run multiplicity and offset.
// Every field is uniform across the wave.
template <int QP>
struct Unit {
    int P[QP];
    int k0, rr;
    int64_t uidx, uoff;   // unit index; packed offset of entry (P', k0, k0)

    __device__ void set()
    {
        k0 = P[QP - 1];
        int run = 1;
#pragma unroll
        for (int i = 1; i < QP; ++i) run = (P[i] == P[i - 1]) ? run + 1 : 1;
        rr = run + 1;
    }
    __device__ void start(int64_t u, int n)
    {
        uidx = u;
        unrank_tuple<QP>(u, n, P);
        int tt[QP + 2];
#pragma unroll
        for (int i = 0; i < QP; ++i) tt[i] = P[i];
        tt[QP] = tt[QP + 1] = P[QP - 1];
        uoff = uni64(rank_tuple<QP + 2>(tt, n));
#pragma unroll
        for (int i = 0; i < QP; ++i) P[i] = uni(P[i]);
        set();
    }
    // the next unit in nested-loop order (fixed register indexing only)
    __device__ void next(int n)
    {
        ++uidx;
        uoff += (int64_t)(n - k0) * (n - k0 + 1) / 2;   // the units follow each other in the array
        int pos = 0;
#pragma unroll
        for (int i = 1; i < QP; ++i)
            if (P[i] != n - 1) pos = i;
        int v = 0;
#pragma unroll
        for (int i = 0; i < QP; ++i)
            if (i == pos) v = P[i] + 1;
#pragma unroll
        for (int i = 0; i < QP; ++i)
            if (i >= pos) P[i] = v;
        set();
    }
    // offset, from entry (P', k0, k0), of entry (r, l), k0 <= r <= l < n
    __device__ int entry(int r, int l, int n) const { return (r - k0) * (2 * n - k0 - r + 1) / 2 - r + l; }
};

// A step of a wave's walk: chunk c (columns [64 c, 64 c + 64)) of row tile t
// of one unit; tiles left of the unit's first row tile are skipped.
template <int QP>
struct Walk {
    Unit<QP> u, first;
    int t, c;
    int64_t u_hi;
    bool valid;

    // the first unit at or after u (within the range) with rows in tile t
    __device__ bool seek(int n)
    {
        while (u.uidx < u_hi && (u.k0 >> 4) > t) {
            if (u.uidx + 1 >= u_hi) return false;
            u.next(n);
        }
        return u.uidx < u_hi;
    }
    __device__ void start(int64_t u_lo, int64_t hi, int n)
    {
        u_hi = hi;
        valid = u_lo < u_hi;
        if (!valid) return;
        first.start(u_lo, n);
        u = first;
        const int ntile = (n + 15) >> 4;
        for (t = 0; t < ntile; ++t) {
            u = first;
            if (seek(n)) break;
        }
        valid = t < ntile;
        c = (u.k0 >> 4) >> 2;
    }
    __device__ void advance(int n)
    {
        const int ntile = (n + 15) >> 4;
        if (c + 1 <= (ntile - 1) >> 2) {   // next chunk of the row tile
            ++c;
            return;
        }
        if (u.uidx + 1 < u_hi) {           // next unit with rows in tile t
            u.next(n);
            if (seek(n)) {
                c = (u.k0 >> 4) >> 2;
                return;
            }
        }
        for (++t; t < ntile; ++t) {        // next row tile: the range again from its first unit
            u = first;
            if (seek(n)) {
                c = (u.k0 >> 4) >> 2;
                return;
            }
        }
        valid = false;
    }
};

// Offset (in entries) that puts a load past any unit's range: it reads 0.
// Sums of up to two of them stay below 2^32 bytes.
constexpr int kFar = 1 << 27;

template <int QP>
__global__ void __launch_bounds__(256) batch_mfma_kernel(BatchArgs p)
{
    __shared__ double as[256 * kAS];        // alpha of the tile's vectors, [k][v]
    __shared__ double xwall[4 * 16 * kXW];  // each wave's staged chunk of M: 16 rows x 64 columns
    __shared__ int fl[256];                 // F(l) - l, F(l) = entries of rows 0 .. l-1 of an n-wide triangle
    const int n = p.n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int ntile = (n + 15) >> 4;
    // workgroup -> (range of units, vector tile): the tiles of one range share an XCD
    const int L = blockIdx.x;
    const int xcd = L % kXcds, qq = L / kXcds;
    const int tile = qq % p.tiles;
    const int group = (qq / p.tiles) * kXcds + xcd;   // < groups: the grid is groups * tiles
    const int64_t b0 = (int64_t)tile * kVB;
    double *xw = xwall + wid * 16 * kXW;

    for (int i = tid; i < 256 * kVB; i += 256) {
        const int k = i / kVB, v = i % kVB;
        as[k * kAS + v] = (k < n && b0 + v < p.B) ? p.alpha[(b0 + v) * n + k] : 0.0;
    }
    fl[tid] = tid * n - tid * (tid - 1) / 2 - tid;
    __syncthreads();   // the only workgroup barrier: alpha and the row table are read-only from here on

    double fq1 = 1.0;
    for (int i = 2; i <= QP + 1; ++i) fq1 *= (double)i;   // (q-1)!
    const int64_t wave = (int64_t)group * 4 + wid;
    const int64_t pw = (int64_t)p.groups * 4;
    Walk<QP> cur;
    cur.start(uni64(p.plan[wave]), uni64(p.plan[wave + 1]), n);

    // Slot 4j + q of a lane holds, for the chunk's tile u = 4c + j, entry
    // (16 t + a, 16 u + b') of M, read from its place (min, max) in the upper
    // triangle; entry (r, l) of a unit is at fl[r] - F(k0) + l.  Rows of M
    // (tiles u >= t): (a, b') = (4q + lk, li); columns of M (tiles u < t,
    // where M = T^T and the triangle is read along its rows): (a, b') =
    // (li, 4q + lk).  The 16 lanes of one lk read 16 consecutive entries.
    // Entries outside the unit get an offset past its range and read 0.
    int Rq[4], Dq[4], Tq[4], Cq = 0;   // offsets of the segment being loaded
    auto seg_offsets = [&](const Walk<QP> &w) {
        const int t = w.t, k0 = w.u.k0, ulo = k0 >> 4;
        const int Fk0 = k0 * n - k0 * (k0 - 1) / 2;
        const int l = 16 * t + li;
        const int fll = fl[l] - Fk0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * t + 4 * q + lk;
            const int flr = fl[r] - Fk0;
            Rq[q] = (r >= k0 && r < n) ? flr : kFar;                             // entry (r, x) = Rq + x
            const int lo = r < l ? r : l;
            Dq[q] = (lo >= k0 && r < n && l < n) ? (l >= r ? flr + l : fll + r) : kFar;   // diagonal tile
            Tq[q] = (16 * ulo + 4 * q + lk < k0) ? kFar : 0;                      // rows above k0 in tile ulo
        }
        Cq = l < n ? l - Fk0 : kFar;   // columns of M: entry (lm, l) = fl[lm] + Cq
    };
    double stg[16];
    auto issue = [&](const Walk<QP> &w) {
        const Rsrc rs = unit_rsrc(p.K + w.u.uoff, (int64_t)(n - w.u.k0) * (n - w.u.k0 + 1) / 2);
        const int t = w.t, ulo = w.u.k0 >> 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 4 * w.c + j;
            if (u < ulo || u >= ntile) continue;
            if (u > t) {
                const int cj = 16 * u + li + ((16 * u + li < n) ? 0 : kFar);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    stg[4 * j + q] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (uint32_t)(Rq[q] + cj) * 8u, 0, 0));
            } else if (u == t) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    stg[4 * j + q] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (uint32_t)Dq[q] * 8u, 0, 0));
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int o = fl[16 * u + 4 * q + lk] + Cq + (u == ulo ? Tq[q] : 0);
                    stg[4 * j + q] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (uint32_t)o * 8u, 0, 0));
                }
            }
        }
    };

    v4d colt = v4d{0.0, 0.0, 0.0, 0.0};
    double cu = 0.0, sacc = 0.0, sold = 0.0;
    double wr[4], dw[4], tw[4];   // multiplicity weights of the segment being staged
    uint32_t written = 0;         // row tiles whose column sums this wave has written
    if (cur.valid) {
        seg_offsets(cur);
        issue(cur);
    }
    bool seg_start = true;   // first chunk of (unit, row tile)
    while (cur.valid) {
        const int t = cur.t, k0 = cur.u.k0, ulo = k0 >> 4;
        if (seg_start) {
            const double wf = 1.0 / cur.u.rr, wd0 = 2.0 / ((double)cur.u.rr * (cur.u.rr + 1));
            const int l = 16 * t + li;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * t + 4 * q + lk;
                wr[q] = r == k0 ? wf : 1.0;
                const int lo = r < l ? r : l;
                dw[q] = r == l ? (r == k0 ? wd0 : 1.0) : (lo == k0 ? wf : 1.0);
                tw[q] = 16 * ulo + 4 * q + lk == k0 ? wf : 1.0;
            }
        }
        // the staged entries, weighted, into the wave's chunk buffer (tiles the
        // unit does not reach are neither loaded nor multiplied)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 4 * cur.c + j;
            if (u < ulo || u >= ntile) continue;
            // weights differ from 1 only on the diagonal tile and on row or column k0 (tile ulo)
            if (u > t) {
                if (t == ulo) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) xw[(4 * q + lk) * kXW + 16 * j + li] = stg[4 * j + q] * wr[q];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) xw[(4 * q + lk) * kXW + 16 * j + li] = stg[4 * j + q];
                }
            } else if (u == t) {
#pragma unroll
                for (int q = 0; q < 4; ++q) xw[(4 * q + lk) * kXW + 16 * j + li] = stg[4 * j + q] * dw[q];
            } else if (u == ulo) {
#pragma unroll
                for (int q = 0; q < 4; ++q) xw[li * kXW + 16 * j + 4 * q + lk] = stg[4 * j + q] * tw[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) xw[li * kXW + 16 * j + 4 * q + lk] = stg[4 * j + q];
            }
        }
        double *sd = p.S_out + (b0 + li) * p.units + cur.u.uidx;
        const bool s_lane = lk == 0 && b0 + li < p.B;
        if (seg_start) {
            // Cu for vector li; S so far (earlier row tiles of the unit), read
            // before the next chunk's loads so that waiting for it leaves them in flight
            int run = 1, wden = 1;
#pragma unroll
            for (int i = 1; i < QP; ++i) {
                run = (cur.u.P[i] == cur.u.P[i - 1]) ? run + 1 : 1;
                wden *= run;
            }
            cu = fq1 / (double)wden;
#pragma unroll
            for (int i = 0; i < QP; ++i) cu *= as[cur.u.P[i] * kAS + li];
            sacc = 0.0;
            sold = (t != ulo && s_lane) ? *sd : 0.0;
        }
        Walk<QP> nxt = cur;
        nxt.advance(n);
        if (nxt.valid) {   // in flight while this chunk is multiplied
            if (nxt.t != t || nxt.u.uidx != cur.u.uidx) seg_offsets(nxt);
            issue(nxt);
        }
        // U[tile t rows, vectors] += M[tile t, chunk columns] A[chunk columns, :], four chains
        v4d U[4] = {v4d{0.0, 0.0, 0.0, 0.0}, v4d{0.0, 0.0, 0.0, 0.0}, v4d{0.0, 0.0, 0.0, 0.0},
                    v4d{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 4 * cur.c + j;
            if (u >= ulo && u < ntile) {
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    U[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(xw[li * kXW + 16 * j + 4 * s + lk],
                                                                as[(16 * u + 4 * s + lk) * kAS + li], U[s], 0, 0, 0);
            }
        }
        const v4d Us = (U[0] + U[1]) + (U[2] + U[3]);
        // Cu U joins the column sums of tile t (rows 16 t + 4e + lk, vector li)
#pragma unroll
        for (int e = 0; e < 4; ++e) colt[e] = __builtin_fma(cu, Us[e], colt[e]);
        // S += alpha_t . U / 2 over the unit's row tiles
#pragma unroll
        for (int e = 0; e < 4; ++e) sacc = __builtin_fma(as[(16 * t + 4 * e + lk) * kAS + li], Us[e], sacc);
        const bool tile_end = !nxt.valid || nxt.t != t;
        const bool seg_end = tile_end || nxt.u.uidx != cur.u.uidx;
        if (seg_end) {
            double sp = sacc;
            sp += __shfl_xor(sp, 16);
            sp += __shfl_xor(sp, 32);
            if (s_lane) *sd = sold + 0.5 * sp;
        }
        if (tile_end) {   // this wave's column sums of tile t
            if (b0 + li < p.B) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int l = 16 * t + 4 * e + lk;
                    if (l < n) {
                        double *dst = p.part + 2 * (((b0 + li) * pw + wave) * n + l);
                        dst[0] = colt[e];
                        dst[1] = 0.0;
                    }
                }
            }
            written |= 1u << t;
            colt = v4d{0.0, 0.0, 0.0, 0.0};
        }
        seg_start = seg_end;
        cur = nxt;
    }
    // row tiles no unit of the range reaches: zero column sums
    if (b0 + li < p.B) {
        for (int t = 0; t < ntile; ++t) {
            if (written & (1u << t)) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = 16 * t + 4 * e + lk;
                if (l < n) {
                    double *dst = p.part + 2 * (((b0 + li) * pw + wave) * n + l);
                    dst[0] = 0.0;
                    dst[1] = 0.0;
                }
            }
        }
    }
}

}  // namespace

// Workgroups per vector tile: about 1024 workgroups in all (two rounds of the
// two resident per CU, so the dispatcher can even out ranges that run slower
// than their modelled share), at most 512 and at most one per 16 units, a
// multiple of 8 so that every XCD gets the same share of ranges.
int batch_groups(int64_t units, int64_t B)
{
    const int64_t tiles = (B + kVB - 1) / kVB;
    int64_t g = 1024 / (tiles < 1 ? 1 : tiles);
    const int64_t cap = (units + 15) / 16;
    if (g > cap) g = cap;
    if (g > 512) g = 512;
    g = (g + kXcds - 1) / kXcds * kXcds;
    if (g < kXcds) g = kXcds;
    return (int)g;
}

hipError_t launch_batch_mfma(const void *K, int64_t count, int n, int q, const double *alpha, int64_t B,
                             const int64_t *plan, int groups, int64_t units, double *S_out, double *part,
                             hipStream_t st)
{
    (void)count;
    if (n < 1 || n > 256 || groups < kXcds || groups % kXcds || B < 1) return hipErrorInvalidValue;
    BatchArgs a{};
    a.K = reinterpret_cast<const double *>(K);
    a.n = n;
    a.alpha = alpha;
    a.B = B;
    a.groups = groups;
    a.tiles = (int)((B + kVB - 1) / kVB);
    a.plan = plan;
    a.units = units;
    a.S_out = S_out;
    a.part = part;
    const unsigned grid = (unsigned)groups * (unsigned)a.tiles;
    switch (q) {
    case 4: hipLaunchKernelGGL(batch_mfma_kernel<2>, dim3(grid), dim3(256), 0, st, a); break;
    case 6: hipLaunchKernelGGL(batch_mfma_kernel<4>, dim3(grid), dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL(batch_mfma_kernel<6>, dim3(grid), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tk
