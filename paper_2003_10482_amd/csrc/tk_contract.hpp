// Host-visible pieces of the contraction kernels (parameters and launchers).
#pragma once

#include <vector>

#include "tk_common.hpp"

namespace tk {

enum AccMode { ACC_DD = 0, ACC_PLAIN64 = 1, ACC_PLAIN32 = 2 };

// One pass over an order-q packed array (levels q and q-1).
struct PairParams {
    const void *A;        // input array (storage type or intermediate type)
    const void *Ad;       // tangent of the input array (lower passes of a derivative) or null
    int64_t a_stride;     // entries between the per-vector input arrays (0: shared array)
    int64_t count;        // entries of one input array: C(n+q-1, q)
    int64_t units;        // C(n+q-3, q-2): leading (q-2)-tuples (1 when q == 2)
    int64_t B;            // number of alpha vectors
    int n;
    double mu;            // integer multiplier of this pass (product of (q'-1) over earlier levels)
    const double *alpha; // [B][n]
    const double *vdir;  // [B][n] direction of the derivative (HV > 0)
    void *S_out;         // [B][units] order q-2 array for the next pass (q >= 4)
    void *Sd_out;        // its tangent
    double *part;        // [B][groups][n] (hi, lo) column-sum partials, already scaled by mu
    double *part_d;      // tangent partials
    const int64_t *plan; // [waves + 1] first unit (q >= 4) or row (q == 2) of every wave
    int *occ_query;      // host only: when set, the launcher stores the resident workgroups per CU
                         // of the selected kernel here instead of launching it
};

constexpr int kMaxPasses = kMaxOrder / 2;

struct ReduceParams {
    const double *part[kMaxPasses];
    int groups[kMaxPasses];
    int npass;
    int n;
    double *out;          // [B][n]
};

// Resident workgroups per CU of the kernel that launch_pass selects (cached).
int pass_resident(int q, int in_kind, int mode, int hv, int bt, int64_t n);
// Workgroups of one pass per tile of vectors: together the tiles fill every
// CU to the kernel's occupancy once, fewer for small arrays.
int pass_groups(int q, int64_t n, int64_t count, int resident, int64_t tiles);
// Device copy of the balanced work plan of one pass (cached per (n, q, groups)).
const int64_t *pass_plan(int q, int64_t n, int groups, int *err);
// Host copy of the same plan (groups * 4 + 1 entries; cached, never freed).
const std::vector<int64_t> &pass_plan_host(int q, int64_t n, int groups);
hipError_t launch_pass(int q, int in_kind, int mode, int hv, int bt, const PairParams &pp,
                       int groups, hipStream_t st);
// per accumulation mode (separate translation units)
hipError_t launch_pass_dd(int q, int in_kind, int hv, int bt, const PairParams &pp, int groups, hipStream_t st);
hipError_t launch_pass_f64(int q, int in_kind, int hv, int bt, const PairParams &pp, int groups, hipStream_t st);
hipError_t launch_pass_f32(int q, int in_kind, int hv, int bt, const PairParams &pp, int groups, hipStream_t st);
hipError_t launch_reduce(const ReduceParams &rp, int64_t B, hipStream_t st);

// First pass of a plain-FP64 contraction of a batch of vectors on FP64 MFMA
// (tk_batch.hip): the outputs of the vector kernel's first pass, with one
// partial per wave (partials [B][4 groups][n] as (hi, lo) pairs, and the
// order q-2 array [B][units], built in S_t [units][B] and transposed).
// groups: a multiple of 8 (batch_groups(units, B)); plan: pass_plan(q, n, groups).
constexpr int kBatchTile = 16;   // vectors per MFMA tile; batches from this size use it
int batch_groups(int64_t units, int64_t B);
hipError_t launch_batch_mfma(const void *K, int64_t count, int n, int q, const double *alpha, int64_t B,
                             const int64_t *plan, int groups, int64_t units, double *S_t, double *S_out,
                             double *part, hipStream_t st);

}  // namespace tk
