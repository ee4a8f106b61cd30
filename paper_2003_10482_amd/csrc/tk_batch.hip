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
typedef double d2 __attribute__((ext_vector_type(2)));
constexpr int kVB = 16;       // vectors per tile (MFMA columns)
constexpr int kXcds = 8;      // XCDs of the device: workgroup ids are dealt to them in turn
constexpr int kXW = 70;       // row stride (doubles) of a staged chunk (16 rows x 64 columns)
// row stride of the alpha tile [k][v] with VT tiles of 16 vectors: the B
// operand reads (16 rows x 4 k-steps per MFMA) spread over the banks
template <int VT>
constexpr int alpha_stride() { return VT == 1 ? kVB + 1 : 40; }

struct BatchArgs {
    const double *K;
    int n;
    const double *alpha;   // [B][n]
    int64_t B;
    int groups, tiles;     // workgroup ranges per vector tile, vector tiles (of 16 VT)
    int64_t pw;            // plan waves = column-sum partials per vector
    const int64_t *plan;   // [groups * 4 + 1]: wave w takes units [plan[w], plan[w + 1])
    int64_t units;
    double *S_t;           // [units][B]: S unit by unit (a vector tile's 16 values share a cache line)
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

// VT tiles of 16 vectors share every staged chunk; 4 VT waves per workgroup.
template <int QP, int VT>
__global__ void __launch_bounds__(256 * VT) batch_mfma_kernel(BatchArgs p)
{
    constexpr int NW = 4 * VT;                 // waves per workgroup
    constexpr int kAS = alpha_stride<VT>();
    constexpr int NV = kVB * VT;               // vectors per workgroup
    __shared__ double as[256 * kAS];           // alpha of the workgroup's vectors, [k][v]
    __shared__ double xwall[NW * 16 * kXW];    // each wave's staged chunk of M: 16 rows x 64 columns
    __shared__ int fl[256];                    // F(l) - l, F(l) = entries of rows 0 .. l-1 of an n-wide triangle
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
    const int64_t b0 = (int64_t)tile * NV;
    double *xw = xwall + wid * 16 * kXW;

    for (int i = tid; i < 256 * NV; i += 256 * VT) {
        const int k = i / NV, v = i % NV;
        as[k * kAS + v] = (k < n && b0 + v < p.B) ? p.alpha[(b0 + v) * n + k] : 0.0;
    }
    if (tid < 256) fl[tid] = tid * n - tid * (tid - 1) / 2 - tid;
    __syncthreads();   // the only workgroup barrier: alpha and the row table are read-only from here on

    double fq1 = 1.0;
    for (int i = 2; i <= QP + 1; ++i) fq1 *= (double)i;   // (q-1)!
    const int64_t wave = (int64_t)group * NW + wid;
    const int64_t pw = p.pw;
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

    v4d colt[VT];
    double cu[VT], sacc[VT], sold[VT];
#pragma unroll
    for (int v2 = 0; v2 < VT; ++v2) {
        colt[v2] = v4d{0.0, 0.0, 0.0, 0.0};
        cu[v2] = sacc[v2] = sold[v2] = 0.0;
    }
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
        double *sd = p.S_t + cur.u.uidx * p.B + b0 + li;   // + 16 v2 for vector tile v2
        if (seg_start) {
            // Cu for vector 16 v2 + li; S so far (earlier row tiles of the
            // unit), read before the next chunk's loads so that waiting for it
            // leaves them in flight
            int run = 1, wden = 1;
#pragma unroll
            for (int i = 1; i < QP; ++i) {
                run = (cur.u.P[i] == cur.u.P[i - 1]) ? run + 1 : 1;
                wden *= run;
            }
#pragma unroll
            for (int v2 = 0; v2 < VT; ++v2) {
                double c = fq1 / (double)wden;
#pragma unroll
                for (int i = 0; i < QP; ++i) c *= as[cur.u.P[i] * kAS + kVB * v2 + li];
                cu[v2] = c;
                sacc[v2] = 0.0;
                const bool s_lane = lk == 0 && b0 + kVB * v2 + li < p.B;
                sold[v2] = (t != ulo && s_lane) ? sd[kVB * v2] : 0.0;
            }
        }
        Walk<QP> nxt = cur;
        nxt.advance(n);
        if (nxt.valid) {   // in flight while this chunk is multiplied
            if (nxt.t != t || nxt.u.uidx != cur.u.uidx) seg_offsets(nxt);
            issue(nxt);
        }
        // U[tile t rows, vectors] += M[tile t, chunk columns] A[chunk columns, :]:
        // every A operand read from LDS serves the VT vector tiles, two chains each
        v4d U[VT][2];
#pragma unroll
        for (int v2 = 0; v2 < VT; ++v2) U[v2][0] = U[v2][1] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 4 * cur.c + j;
            if (u >= ulo && u < ntile) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double xa = xw[li * kXW + 16 * j + 4 * s + lk];
#pragma unroll
                    for (int v2 = 0; v2 < VT; ++v2)
                        U[v2][s & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            xa, as[(16 * u + 4 * s + lk) * kAS + kVB * v2 + li], U[v2][s & 1], 0, 0, 0);
                }
            }
        }
        const bool tile_end = !nxt.valid || nxt.t != t;
        const bool seg_end = tile_end || nxt.u.uidx != cur.u.uidx;
#pragma unroll
        for (int v2 = 0; v2 < VT; ++v2) {
            const v4d Us = U[v2][0] + U[v2][1];
            // Cu U joins the column sums of tile t (rows 16 t + 4e + lk, vector 16 v2 + li)
#pragma unroll
            for (int e = 0; e < 4; ++e) colt[v2][e] = __builtin_fma(cu[v2], Us[e], colt[v2][e]);
            // S += alpha_t . U / 2 over the unit's row tiles
#pragma unroll
            for (int e = 0; e < 4; ++e)
                sacc[v2] = __builtin_fma(as[(16 * t + 4 * e + lk) * kAS + kVB * v2 + li], Us[e], sacc[v2]);
            if (seg_end) {
                double sp = sacc[v2];
                sp += __shfl_xor(sp, 16);
                sp += __shfl_xor(sp, 32);
                if (lk == 0 && b0 + kVB * v2 + li < p.B) sd[kVB * v2] = sold[v2] + 0.5 * sp;
            }
            if (tile_end) {   // this wave's column sums of tile t
                const int64_t b = b0 + kVB * v2 + li;
                if (b < p.B) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int l = 16 * t + 4 * e + lk;
                        if (l < n) {
                            double *dst = p.part + 2 * ((b * pw + wave) * n + l);
                            *reinterpret_cast<d2 *>(dst) = d2{colt[v2][e], 0.0};
                        }
                    }
                }
                colt[v2] = v4d{0.0, 0.0, 0.0, 0.0};
            }
        }
        if (tile_end) written |= 1u << t;
        seg_start = seg_end;
        cur = nxt;
    }
    // row tiles no unit of the range reaches: zero column sums
#pragma unroll
    for (int v2 = 0; v2 < VT; ++v2) {
        const int64_t b = b0 + kVB * v2 + li;
        if (b >= p.B) continue;
        for (int t = 0; t < ntile; ++t) {
            if (written & (1u << t)) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = 16 * t + 4 * e + lk;
                if (l < n) {
                    double *dst = p.part + 2 * ((b * pw + wave) * n + l);
                    *reinterpret_cast<d2 *>(dst) = d2{0.0, 0.0};
                }
            }
        }
    }
}

// S [B][units] (the next pass's per-vector arrays) from S_t [units][B]
__global__ void __launch_bounds__(256) transpose_s_kernel(const double *S_t, double *S, int64_t units, int64_t B)
{
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t u0 = (int64_t)blockIdx.x * 32, b0 = (int64_t)blockIdx.y * 32;
    for (int r = ty; r < 32; r += 8) {
        const int64_t u = u0 + r, b = b0 + tx;
        tile[r][tx] = (u < units && b < B) ? S_t[u * B + b] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t b = b0 + r, u = u0 + tx;
        if (b < B && u < units) S[b * units + u] = tile[tx][r];
    }
}

}  // namespace

// Vector tiles per workgroup: two from 17 vectors on (every staged chunk then
// feeds twice the MFMAs), one below.
int batch_vt(int64_t B) { return B > kVB ? 2 : 1; }

// Plan groups (of four waves) of the batch pass: about two rounds of
// workgroups (two resident per CU with one vector tile, one with two), at
// most one group per 16 units, a multiple of 8 VT so that every XCD gets the
// same share of ranges.
int batch_groups(int64_t units, int64_t B)
{
    const int vt = batch_vt(B);
    const int64_t tiles = (B + kVB * vt - 1) / (kVB * vt);
    int64_t wg = (vt == 1 ? 1024 : 512) / (tiles < 1 ? 1 : tiles);   // workgroups per tile
    int64_t g = wg * vt;
    const int64_t cap = (units + 15) / 16;
    if (g > cap) g = cap;
    if (g > 512 * vt) g = 512 * vt;
    const int64_t step = (int64_t)kXcds * vt;
    g = (g + step - 1) / step * step;
    if (g < step) g = step;
    return (int)g;
}

hipError_t launch_batch_mfma(const void *K, int64_t count, int n, int q, const double *alpha, int64_t B,
                             const int64_t *plan, int groups, int64_t units, double *S_t, double *S_out,
                             double *part, hipStream_t st)
{
    (void)count;
    const int vt = batch_vt(B);
    if (n < 1 || n > 256 || groups < kXcds * vt || groups % (kXcds * vt) || B < 1) return hipErrorInvalidValue;
    BatchArgs a{};
    a.K = reinterpret_cast<const double *>(K);
    a.n = n;
    a.alpha = alpha;
    a.B = B;
    a.groups = groups;
    a.tiles = (int)((B + kVB * vt - 1) / (kVB * vt));
    a.plan = plan;
    a.units = units;
    a.S_t = S_t;
    a.part = part;
    // workgroups: groups / vt ranges (of 4 vt waves each) times the vector tiles
    const unsigned grid = (unsigned)(groups / vt) * (unsigned)a.tiles;
    const dim3 blk(256 * vt);
    // kernel argument `groups` is the plan's group count: the workgroup's
    // range index runs to groups / vt
    BatchArgs ak = a;
    ak.groups = groups / vt;
    ak.pw = (int64_t)groups * 4;
    switch (q * 4 + vt) {
    case 17: hipLaunchKernelGGL((batch_mfma_kernel<2, 1>), dim3(grid), blk, 0, st, ak); break;
    case 18: hipLaunchKernelGGL((batch_mfma_kernel<2, 2>), dim3(grid), blk, 0, st, ak); break;
    case 25: hipLaunchKernelGGL((batch_mfma_kernel<4, 1>), dim3(grid), blk, 0, st, ak); break;
    case 26: hipLaunchKernelGGL((batch_mfma_kernel<4, 2>), dim3(grid), blk, 0, st, ak); break;
    case 33: hipLaunchKernelGGL((batch_mfma_kernel<6, 1>), dim3(grid), blk, 0, st, ak); break;
    case 34: hipLaunchKernelGGL((batch_mfma_kernel<6, 2>), dim3(grid), blk, 0, st, ak); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(transpose_s_kernel, dim3((unsigned)((units + 31) / 32), (unsigned)((B + 31) / 32)), dim3(256), 0,
                       st, S_t, S_out, units, B);
    return hipGetLastError();
}

}  // namespace tk
