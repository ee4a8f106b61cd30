// C ABI of the packed tensor-kernel library: argument checks, workspace
// planning, the pass sequence of the contraction, and the host-driven loops of
// the dual solve and of the model-selection derivative.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tk_common.hpp"
#include "tk_contract.hpp"
#include "tk_host.hpp"
#include "tk_dense.hpp"
#include "tk_hess.hpp"
#include "tk_vec.hpp"

namespace tk {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_nm(int64_t n, int m)
{
    if (n < 1) return fail(TK_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (m < 2 || (m & 1)) return fail(TK_EINVAL, "tensor order m must be even and >= 2 (got %d)", m);
    if (m > kMaxOrder) return fail(TK_EUNSUPPORTED, "tensor order m = %d above the compiled maximum %d", m, kMaxOrder);
    if (n > kMaxPoints) return fail(TK_EUNSUPPORTED, "n = %lld above the compiled maximum %d", (long long)n, kMaxPoints);
    if (checked_binom(n + m - 1, m) < 0) return fail(TK_EOVERFLOW, "C(n+m-1, m) overflows int64");
    return TK_OK;
}

int check_dtype(int dtype)
{
    if (dtype != TK_F64 && dtype != TK_F32 && dtype != TK_BF16) return fail(TK_EINVAL, "unknown dtype %d", dtype);
    return TK_OK;
}

// Layout of the contraction workspace for (n, m, B, mode, tangents).
struct PassPlan {
    int q;
    int64_t count, units;
    int groups;
    int parts;                 // column-sum partials per vector: one per workgroup (per wave on MFMA)
    int bt;                    // vectors per tile
    size_t s_off, s_bytes;     // order q-2 output (and its tangent right after when hv)
    size_t p_off, p_bytes;     // partials (and tangent partials right after)
    size_t t_off;              // MFMA batch pass: the order q-2 array unit by unit, before its transpose
};

struct ContractPlan {
    int npass = 0;
    PassPlan pass[kMaxPasses];
    size_t bytes = 0;
};

size_t inter_size(int mode) { return mode == ACC_DD ? 16 : mode == ACC_PLAIN64 ? 8 : 4; }

// Kernel selection of pass i (first pass reads the stored tensor, later ones
// the intermediate arrays): input kind, tangent kind and vector tile.
int pass_in_kind(int i, int dtype, int mode)
{
    if (i == 0) return dtype == TK_F64 ? 0 : dtype == TK_F32 ? 1 : 2;
    return mode == ACC_DD ? 3 : mode == ACC_PLAIN64 ? 0 : 1;
}
int pass_hv(int i, bool hv) { return hv ? (i == 0 ? 1 : 2) : 0; }

// Vector tile of the first pass: the autotuner's choice for this device and
// shape when it has run, else 4 vectors per tile with FP32 arithmetic and 1
// otherwise.  Later passes read per-vector arrays: always 1.
struct TileKey {
    int dev, dtype, mode, hv, m;
    int64_t n, B;
    bool operator<(const TileKey &o) const
    {
        return std::tie(dev, dtype, mode, hv, m, n, B) < std::tie(o.dev, o.dtype, o.mode, o.hv, o.m, o.n, o.B);
    }
};
std::mutex g_tile_mu;
std::map<TileKey, int> g_tiles;

int tile_limit(int mode, bool hv)
{
    if (mode == ACC_PLAIN32) return 4;
    if (mode == ACC_PLAIN64) return hv ? 2 : 4;
    return 1;
}

// The first pass of a plain-FP64 contraction (no tangent) can run on FP64
// MFMA, kBatchTile vectors per tile (tile id kBatchTile): by default from
// kBatchTile vectors on, unless the autotuner chose otherwise for the shape.
// force = kBatchTile selects it for any batch, another force a vector tile.
bool mfma_ok(int mode, int dtype, bool hv, int64_t n, int m)
{
    return mode == ACC_PLAIN64 && dtype == TK_F64 && !hv && n <= 256 && m >= 4;
}

int pass_bt(int i, int mode, int64_t B, int64_t n, int m, int dtype, bool hv, int force)
{
    if (i != 0) return 1;
    const bool mf = mfma_ok(mode, dtype, hv, n, m);
    if (force == kBatchTile) return mf ? kBatchTile : 1;
    if (B < 2) return 1;
    if (force > 0) return force < tile_limit(mode, hv) ? force : tile_limit(mode, hv);
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(g_tile_mu);
        auto it = g_tiles.find(TileKey{dev, dtype, mode, hv ? 1 : 0, m, n, B});
        if (it != g_tiles.end()) return it->second;
    }
    if (mf && B >= kBatchTile) return kBatchTile;
    return (mode == ACC_PLAIN32 && B >= 4) ? 4 : 1;
}

ContractPlan make_plan(int64_t n, int m, int64_t B, int mode, bool hv, int dtype, int force_bt = 0)
{
    ContractPlan pl;
    size_t off = 0;
    for (int q = m; q >= 2; q -= 2) {
        const int i = pl.npass;
        PassPlan &p = pl.pass[pl.npass++];
        p.q = q;
        p.count = packed_count(n, q);
        p.units = q >= 4 ? packed_count(n, q - 2) : 1;
        const int bt = pass_bt(i, mode, B, n, m, dtype, hv, force_bt);
        p.bt = bt;
        if (bt == kBatchTile)
            p.groups = batch_groups(p.units, B);
        else
            p.groups = pass_groups(q, n, p.count,
                                   q >= 4 ? pass_resident(q, pass_in_kind(i, dtype, mode), mode, pass_hv(i, hv), bt, n)
                                          : 1,
                                   (B + bt - 1) / bt);
        p.s_bytes = q >= 4 ? align256((size_t)B * p.units * inter_size(mode)) : 0;
        p.s_off = off;
        off += p.s_bytes * (hv ? 2 : 1);
        p.t_off = off;
        if (bt == kBatchTile) off += p.s_bytes;
        p.parts = bt == kBatchTile ? 4 * p.groups : p.groups;
        p.p_bytes = align256((size_t)B * p.parts * n * 2 * sizeof(double));
        p.p_off = off;
        off += p.p_bytes * (hv ? 2 : 1);
    }
    pl.bytes = off;
    return pl;
}

int mode_for(int dtype, int acc, bool hv, int *mode)
{
    if (dtype == TK_F64) {
        if (hv && acc == TK_ACC_COMPENSATED) { *mode = ACC_DD; return TK_OK; }
        if (hv && (acc == TK_ACC_AUTO || acc == TK_ACC_F64)) { *mode = ACC_PLAIN64; return TK_OK; }
        if (acc == TK_ACC_AUTO || acc == TK_ACC_COMPENSATED) { *mode = ACC_DD; return TK_OK; }
        if (acc == TK_ACC_F64) { *mode = ACC_PLAIN64; return TK_OK; }
        if (acc == TK_ACC_F32) { *mode = ACC_PLAIN32; return TK_OK; }
        return fail(TK_EINVAL, "accumulation %d not available for FP64 storage", acc);
    }
    if (acc == TK_ACC_AUTO || acc == TK_ACC_F32) { *mode = ACC_PLAIN32; return TK_OK; }
    return fail(TK_EINVAL, "accumulation %d not available for FP32/BF16 storage", acc);
}

// ------------------------------------------------------- instrumentation ----
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<TimedLaunch> g_timing;

}  // namespace

TimedLaunch timing_begin(int kind, double bytes, hipStream_t st)
{
    TimedLaunch tl{};
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (g_timing_on && hipEventCreate(&tl.a) == hipSuccess && hipEventCreate(&tl.b) == hipSuccess) {
        tl.on = true;
        tl.kind = kind;
        tl.bytes = bytes;
        hipEventRecord(tl.a, st);
    }
    return tl;
}

void timing_end(TimedLaunch &tl, hipStream_t st)
{
    if (!tl.on) return;
    hipEventRecord(tl.b, st);
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing.push_back(tl);
    tl.on = false;
}

namespace {

// Device memory that receives the work plans of the passes (instead of the
// library's cached device plans, which are allocated on first use of a
// shape), for callers that cannot allocate.  Timing instrumentation is off
// on that route (it creates events).
struct PlanArea {
    unsigned char *dev;
    size_t bytes;
};

size_t plan_area_bytes(const ContractPlan &pl)
{
    size_t b = 0;
    for (int i = 0; i < pl.npass; ++i) b += align256(((size_t)pl.pass[i].groups * 4 + 1) * sizeof(int64_t));
    return b;
}

// Run every pass of the contraction (and its tangent when vdir != null).
int run_contract(const void *K, int dtype, int64_t n, int m, const double *alpha, const double *vdir,
                 int64_t B, double *g, double *h, int mode, void *work, size_t work_bytes, hipStream_t st,
                 int force_bt = 0, const PlanArea *area = nullptr, int64_t k_stride = 0)
{
    const bool hv = vdir != nullptr;
    // several tensors (vector b contracts tensor b, k_stride entries apart):
    // one vector per tile
    if (k_stride > 0) force_bt = 1;
    const ContractPlan pl = make_plan(n, m, B, mode, hv, dtype, force_bt);
    if (work_bytes < pl.bytes || (pl.bytes && !work))
        return fail(TK_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", work_bytes, pl.bytes);
    if (area && plan_area_bytes(pl) > area->bytes)
        return fail(TK_ENOMEM, "work plans need %zu bytes of the %zu reserved", plan_area_bytes(pl), area->bytes);
    size_t area_off = 0;
    unsigned char *w = reinterpret_cast<unsigned char *>(work);
    const void *A = K;
    const void *Ad = nullptr;
    int in_kind = pass_in_kind(0, dtype, mode);
    int64_t a_stride = k_stride;
    double mu = 1.0;
    ReduceParams rv{}, rt{};
    for (int i = 0; i < pl.npass; ++i) {
        const PassPlan &pp = pl.pass[i];
        PairParams prm{};
        prm.A = A;
        prm.Ad = Ad;
        prm.a_stride = a_stride;
        prm.count = pp.count;
        prm.units = pp.units;
        prm.B = B;
        prm.n = (int)n;
        prm.mu = mu;
        prm.alpha = alpha;
        prm.vdir = vdir;
        prm.S_out = pp.s_bytes ? w + pp.s_off : nullptr;
        prm.Sd_out = (pp.s_bytes && hv) ? w + pp.s_off + pp.s_bytes : nullptr;
        prm.part = reinterpret_cast<double *>(w + pp.p_off);
        prm.part_d = hv ? reinterpret_cast<double *>(w + pp.p_off + pp.p_bytes) : nullptr;
        int perr = 0;
        if (area) {
            // the host plan lives for the process, so the copy may complete later
            const std::vector<int64_t> &hp = pass_plan_host(pp.q, n, pp.groups);
            int64_t *dp = reinterpret_cast<int64_t *>(area->dev + area_off);
            area_off += align256(hp.size() * sizeof(int64_t));
            TK_HIP_CHECK(hipMemcpyAsync(dp, hp.data(), hp.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
            prm.plan = dp;
        } else {
            prm.plan = pass_plan(pp.q, n, pp.groups, &perr);
        }
        if (perr || !prm.plan) return fail(TK_EHIP, "could not place the work plan of pass q=%d", pp.q);
        const int hvl = pass_hv(i, hv);
        const int bt = pp.bt;
        TimedLaunch tl{};
        if (i == 0 && !area)   // one read of the stored tensor(s) per tile of bt vectors (per batch on MFMA)
            tl = timing_begin(hv ? 1 : (mode == ACC_DD ? 0 : 2),
                              (double)pp.count * (double)dtype_size(dtype) *
                                  (double)(bt == kBatchTile ? 1 : (B + bt - 1) / bt),
                              st);
        hipError_t e;
        if (bt == kBatchTile)   // a batch on FP64 MFMA: one read of K for all the vectors
            e = launch_batch_mfma(A, pp.count, (int)n, pp.q, alpha, B, prm.plan, pp.groups, pp.units,
                                  reinterpret_cast<double *>(w + pp.t_off), reinterpret_cast<double *>(prm.S_out),
                                  prm.part, st);
        else
            e = launch_pass(pp.q, in_kind, mode, hvl, bt, prm, pp.groups, st);
        if (e != hipSuccess) return fail(TK_EHIP, "contraction pass q=%d failed: %s", pp.q, hipGetErrorString(e));
        timing_end(tl, st);
        rv.part[i] = prm.part;
        rv.groups[i] = pp.parts;
        rt.part[i] = prm.part_d;
        rt.groups[i] = pp.parts;
        A = prm.S_out;
        Ad = prm.Sd_out;
        a_stride = pp.units;
        in_kind = pass_in_kind(i + 1, dtype, mode);
        mu *= (double)(pp.q - 1) * (double)(pp.q - 2);
    }
    rv.npass = rt.npass = pl.npass;
    rv.n = rt.n = (int)n;
    if (g) {
        rv.out = g;
        hipError_t e = launch_reduce(rv, B, st);
        if (e != hipSuccess) return fail(TK_EHIP, "reduction failed: %s", hipGetErrorString(e));
    }
    if (hv && h) {
        rt.out = h;
        hipError_t e = launch_reduce(rt, B, st);
        if (e != hipSuccess) return fail(TK_EHIP, "reduction failed: %s", hipGetErrorString(e));
    }
    return TK_OK;
}

size_t contract_ws(int64_t n, int m, int64_t B, int dtype)
{
    // every accumulation mode and both the value and the derivative pass can
    // run in one workspace; grids follow each kernel's occupancy
    size_t w = 0;
    const int modes[3] = {dtype == TK_F64 ? ACC_DD : ACC_PLAIN32, dtype == TK_F64 ? ACC_PLAIN64 : ACC_PLAIN32,
                          ACC_PLAIN32};
    for (int mode : modes)
        for (int hv = 0; hv < 2; ++hv) {
            for (int t = 1; t <= tile_limit(mode, hv != 0); t *= 2) {
                const size_t b = make_plan(n, m, B, mode, hv != 0, dtype, t).bytes;
                if (b > w) w = b;
            }
            if (mfma_ok(mode, dtype, hv != 0, n, m)) {
                const size_t b = make_plan(n, m, B, mode, hv != 0, dtype, kBatchTile).bytes;
                if (b > w) w = b;
            }
        }
    return w;
}

// Time each vector tile (1, 2, 4 where the mode has it) for B vectors on this
// tensor and keep the fastest for the device and shape.  alpha/vdir [B][n]
// are timing inputs, out [B][n] receives results.  ms[t] = time of tile 2^t.
int autotune_tile(const void *K, int dtype, int64_t n, int m, const double *alpha, const double *vdir, int64_t B,
                  int mode, double *out, void *work, size_t work_bytes, hipStream_t st, int *tile, double ms[4])
{
    const bool hv = vdir != nullptr;
    for (int t = 0; t < 4; ++t) ms[t] = -1.0;
    *tile = 1;
    if (B < 2) return TK_OK;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(TK_EHIP, "event create failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(TK_EHIP, "event create failed");
    }
    int rc = TK_OK;
    double best = INFINITY;
    // vector tiles 1, 2, 4 (as the mode allows), then the MFMA tile where it applies
    int cand[4], nc = 0;
    for (int t = 1; t <= tile_limit(mode, hv); t *= 2) cand[nc++] = t;
    if (mfma_ok(mode, dtype, hv, n, m)) cand[nc++] = kBatchTile;
    for (int ci = 0; ci < nc && !rc; ++ci) {
        const int t = cand[ci], ti = t == kBatchTile ? 3 : ci;
        for (int rep = 0; rep < 3 && !rc; ++rep) {   // one untimed launch, then two timed
            if (rep == 1) hipEventRecord(e0, st);
            rc = run_contract(K, dtype, n, m, alpha, vdir, B, hv ? nullptr : out, hv ? out : nullptr, mode, work,
                              work_bytes, st, t);
        }
        if (rc) break;
        hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(TK_EHIP, "event synchronize failed");
            break;
        }
        float f = 0.f;
        hipEventElapsedTime(&f, e0, e1);
        ms[ti] = 0.5 * (double)f;
        if (ms[ti] < best) {
            best = ms[ti];
            *tile = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tiles[TileKey{dev, dtype, mode, hv ? 1 : 0, m, n, B}] = *tile;
    return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

const char *tk_last_error(void) { return tk::g_err; }

int64_t tk_max_points(void) { return kMaxPoints; }

int tk_packed_count(int64_t n, int m, int64_t *h_count)
{
    if (!h_count) return fail(TK_EINVAL, "null output pointer");
    if (n < 1 || m < 1) return fail(TK_EINVAL, "n and m must be >= 1");
    const int64_t c = checked_binom(n + m - 1, m);
    if (c < 0) return fail(TK_EOVERFLOW, "C(n+m-1, m) overflows int64");
    *h_count = c;
    return TK_OK;
}

int tk_packed_bytes(int64_t n, int m, int dtype, int64_t *h_bytes)
{
    int64_t c;
    int rc = tk_packed_count(n, m, &c);
    if (rc) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    const int64_t s = (int64_t)dtype_size(dtype);
    if (c > INT64_MAX / s - 4) return fail(TK_EOVERFLOW, "packed byte count overflows int64");
    if (!h_bytes) return fail(TK_EINVAL, "null output pointer");
    // BF16 tensors are read a dword at a time: round the buffer up to whole dwords
    *h_bytes = dtype == TK_BF16 ? ((c * s + 3) & ~(int64_t)3) : c * s;
    return TK_OK;
}

int tk_build_packed_tensor(const double *d_X, int64_t n, int64_t d, int m, int kernel, double kparam,
                           int dtype, void *d_K, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (d < 1 || d > INT32_MAX) return fail(TK_EINVAL, "d must be in [1, 2^31) (got %lld)", (long long)d);
    if (!d_X || !d_K) return fail(TK_EINVAL, "null device pointer");
    if (kernel == TK_POLY) {
        if (!(kparam >= 1.0) || kparam != std::floor(kparam) || kparam > 64)
            return fail(TK_EINVAL, "polynomial degree must be an integer in [1, 64]");
    } else if (kernel != TK_LINEAR && kernel != TK_EXP) {
        return fail(TK_EINVAL, "unknown kernel %d", kernel);
    }
    hipError_t e = launch_build(d_X, (int)n, (int)d, m, kernel, kparam, dtype, d_K, as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "build launch failed: %s", hipGetErrorString(e));
    return TK_OK;
}

}  // extern "C"

// ------------------------------------------- allocation-free contraction ----
// Device scratch of tk_contract_noalloc: the work plans of the passes (first
// kScratchPlanBytes) and the contraction workspace (the rest).  Every device
// the library runs on holds its own copy until the process ends.  In host
// code `scratch` only names the symbol: its address on the current device
// comes from hipGetSymbolAddress (scratch_address) and is the only form
// passed to copies and kernels.
namespace tk {
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kScratchPlanBytes = (size_t)1 << 20;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;

// Address of `scratch` on the current device, looked up once per device.
int scratch_address(unsigned char **out)
{
    int dev = 0;
    TK_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TK_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        it = g_scratch_addr.emplace(dev, reinterpret_cast<unsigned char *>(p)).first;
    }
    *out = it->second;
    return TK_OK;
}
}  // namespace
}  // namespace tk

extern "C" {

size_t tk_contract_noalloc_max_bytes(void) { return kScratchBytes - kScratchPlanBytes; }

int tk_contract_noalloc(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha, int64_t B,
                        double *d_g, int acc, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1 || B > 65535) return fail(TK_EINVAL, "B must be in [1, 65535]");
    if (!d_K || !d_alpha || !d_g) return fail(TK_EINVAL, "null device pointer");
    int mode;
    if ((rc = mode_for(dtype, acc, false, &mode))) return rc;
    const ContractPlan pl = make_plan(n, m, B, mode, false, dtype);
    const size_t cap = kScratchBytes - kScratchPlanBytes;
    if (pl.bytes > cap)
        return fail(TK_ENOMEM,
                    "n = %lld, m = %d, B = %lld needs %zu bytes of scratch; the allocation-free entry point holds "
                    "%zu (use tk_contract with a caller workspace)",
                    (long long)n, m, (long long)B, pl.bytes, cap);
    if (plan_area_bytes(pl) > kScratchPlanBytes)
        return fail(TK_ENOMEM, "work plans need %zu bytes, above the %zu reserved", plan_area_bytes(pl),
                    kScratchPlanBytes);
    unsigned char *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    const PlanArea area{base, kScratchPlanBytes};
    return run_contract(d_K, dtype, n, m, d_alpha, nullptr, B, d_g, nullptr, mode, base + kScratchPlanBytes, cap,
                        as_stream(stream), 0, &area);
}

int tk_contract_workspace(int64_t n, int m, int64_t B, int dtype, size_t *h_bytes)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1) return fail(TK_EINVAL, "B must be >= 1");
    if (!h_bytes) return fail(TK_EINVAL, "null output pointer");
    *h_bytes = contract_ws(n, m, B, dtype);
    return TK_OK;
}

int tk_contract(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha, int64_t B, double *d_g,
                int acc, void *d_work, size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1 || B > 65535) return fail(TK_EINVAL, "B must be in [1, 65535]");
    if (!d_K || !d_alpha || !d_g) return fail(TK_EINVAL, "null device pointer");
    int mode;
    if ((rc = mode_for(dtype, acc, false, &mode))) return rc;
    return run_contract(d_K, dtype, n, m, d_alpha, nullptr, B, d_g, nullptr, mode, d_work, work_bytes,
                        as_stream(stream));
}

int tk_hvp(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha, const double *d_v, int64_t B,
           double *d_h, double *d_g, int acc, void *d_work, size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1 || B > 65535) return fail(TK_EINVAL, "B must be in [1, 65535]");
    if (!d_K || !d_alpha || !d_v || !d_h) return fail(TK_EINVAL, "null device pointer");
    int mode;
    if ((rc = mode_for(dtype, acc, true, &mode))) return rc;
    return run_contract(d_K, dtype, n, m, d_alpha, d_v, B, d_g, d_h, mode, d_work, work_bytes, as_stream(stream));
}

int tk_hessian_workspace(int64_t n, int m, size_t *h_bytes)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if (!h_bytes) return fail(TK_EINVAL, "null output pointer");
    *h_bytes = hessian_ws(n, m);
    return TK_OK;
}

int tk_hessian(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha, double *d_J, void *d_work,
               size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (!d_K || !d_alpha || !d_J || !d_work) return fail(TK_EINVAL, "null device pointer");
    return run_hessian(d_K, dtype, n, m, d_alpha, d_J, d_work, work_bytes, as_stream(stream), nullptr);
}

int tk_autotune(const void *d_K, int dtype, int64_t n, int m, const double *d_alpha, const double *d_v, int64_t B,
                int acc, double *d_out, void *d_work, size_t work_bytes, void *stream, int *h_tile, double *h_ms)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1) return fail(TK_EINVAL, "B must be >= 1");
    if (!d_K || !d_alpha || !d_out || !h_tile) return fail(TK_EINVAL, "null pointer");
    int mode;
    if ((rc = mode_for(dtype, acc, d_v != nullptr, &mode))) return rc;
    const size_t need = contract_ws(n, m, B, dtype);
    if (work_bytes < need || (need && !d_work))
        return fail(TK_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", work_bytes, need);
    double ms[4];
    rc = autotune_tile(d_K, dtype, n, m, d_alpha, d_v, B, mode, d_out, d_work, work_bytes, as_stream(stream), h_tile,
                       ms);
    if (h_ms)
        for (int t = 0; t < 4; ++t) h_ms[t] = ms[t];
    return rc;
}

int tk_probe_stream_read(const void *d_src, int64_t bytes, uint64_t *d_sink, int groups, void *stream)
{
    if (!d_src || !d_sink) return fail(TK_EINVAL, "null device pointer");
    if (bytes < 16 || (bytes & 15)) return fail(TK_EINVAL, "bytes must be a positive multiple of 16");
    if (reinterpret_cast<uintptr_t>(d_src) & 15) return fail(TK_EINVAL, "d_src must be 16-byte aligned");
    if (groups < 1 || groups > 65536) return fail(TK_EINVAL, "groups must be in [1, 65536]");
    hipError_t e = probe_stream_read(d_src, bytes / 16, d_sink, groups, as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "stream read failed: %s", hipGetErrorString(e));
    return TK_OK;
}

int tk_timing_start(void)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    for (auto &t : g_timing) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_timing.clear();
    g_timing_on = true;
    return TK_OK;
}

int tk_timing_stop(int64_t *h_launches, double *h_ms, double *h_bytes)
{
    if (!h_launches || !h_ms || !h_bytes) return fail(TK_EINVAL, "null output pointer");
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_on = false;
    for (int k = 0; k < kTimingKinds; ++k) {
        h_launches[k] = 0;
        h_ms[k] = 0.0;
        h_bytes[k] = 0.0;
    }
    int rc = TK_OK;
    for (auto &t : g_timing) {
        float ms = 0.f;
        if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess)
            rc = fail(TK_EHIP, "timing events failed");
        h_launches[t.kind] += 1;
        h_ms[t.kind] += ms;
        h_bytes[t.kind] += t.bytes;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_timing.clear();
    return rc;
}

void tk_solve_opts_default(tk_solve_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_newton = 100;
    o->max_cg = 2000;
    o->tol = 1e-11;
    o->polish_dtype = TK_F64;
    o->precond = 1;
    o->precond_refresh = 25;
    o->continuation = 1;
}

}  // extern "C"

// ------------------------------------------------------------ dual solve ----
namespace tk {
namespace {

struct SolveBuffers {
    double *g, *grad, *x, *r, *dv, *hd, *at, *gt, *z, *best, *hdiag, *stats, *stats2;
    double *P;             // [B][n][n] preconditioners (inverse Hessians)
    double *Jd;            // [B][n][n] Hessians J at the current iterates
    unsigned char *hw;     // Hessian kernel workspace
    size_t hw_bytes;
    double *supW;          // [B][d] primal weights for the support test (early stopping)
    uint8_t *mask_cur, *mask_prev;   // [B][d] current and previous supports
    double *sup_tau;       // [B] thresholds
    int *sup_cnt;          // [B] changed entries since the last Newton step
    unsigned char *cw;
    size_t cw_bytes;
};

// Extensions of one batch of dual solves beyond the square loss on a shared
// tensor: several tensors (problem b on the tensor k_stride entries after
// problem b-1's) with their own responses, the logistic loss, and the
// stable-support stopping rule.
struct SolveCtx {
    int64_t k_stride = 0;   // entries between the problems' tensors (0: one tensor)
    int64_t y_stride = 0;   // entries between the problems' responses (0: one response)
    int loss = TK_LOSS_SQUARE;
    int support_stop = 0;   // Newton steps in a row with an unchanged support that end a solve
    const double *sX = nullptr;   // points of the linear tensor kernel [n][d] (support test)
    int64_t sd = 0;
};

size_t support_ws(int64_t B, int64_t d)
{
    if (d <= 0) return 0;
    return align256((size_t)B * d * sizeof(double)) + 2 * align256((size_t)B * d) + align256((size_t)B * 8) +
           align256((size_t)B * sizeof(int));
}

size_t solve_ws(int64_t n, int m, int64_t B, int dtype, int64_t support_d = 0)
{
    const size_t vec = align256((size_t)B * n * sizeof(double));
    // passes for the whole batch (lock step) or one problem at a time
    // (continuation): a single vector's launch has more workgroups, so its
    // partials can outgrow a batch's
    size_t cw = 0;
    for (int64_t bb : {B, (int64_t)1})
        for (int dt : {dtype, (int)TK_F64}) {   // polish passes run on an FP64 tensor
            const size_t c = contract_ws(n, m, bb, dt);
            if (c > cw) cw = c;
        }
    return 11 * vec + 2 * align256((size_t)B * 8 * sizeof(double)) + align256((size_t)B * n * n * sizeof(double)) +
           align256((size_t)B * n * n * sizeof(double)) + align256(hessian_ws(n, m)) + support_ws(B, support_d) + cw;
}

SolveBuffers carve(void *work, int64_t n, int m, int64_t B, size_t total, int64_t support_d = 0)
{
    SolveBuffers s{};
    const size_t vec = align256((size_t)B * n * sizeof(double));
    unsigned char *w = reinterpret_cast<unsigned char *>(work);
    double **v[11] = {&s.g, &s.grad, &s.x, &s.r, &s.dv, &s.hd, &s.at, &s.gt, &s.z, &s.best, &s.hdiag};
    for (int i = 0; i < 11; ++i) *v[i] = reinterpret_cast<double *>(w + i * vec);
    size_t used = 11 * vec;
    s.stats = reinterpret_cast<double *>(w + used);
    used += align256((size_t)B * 8 * sizeof(double));
    s.stats2 = reinterpret_cast<double *>(w + used);
    used += align256((size_t)B * 8 * sizeof(double));
    s.P = reinterpret_cast<double *>(w + used);
    used += align256((size_t)B * n * n * sizeof(double));
    s.Jd = reinterpret_cast<double *>(w + used);
    used += align256((size_t)B * n * n * sizeof(double));
    s.hw = w + used;
    s.hw_bytes = align256(hessian_ws(n, m));
    used += s.hw_bytes;
    if (support_d > 0) {
        const int64_t d = support_d;
        s.supW = reinterpret_cast<double *>(w + used);
        used += align256((size_t)B * d * sizeof(double));
        s.mask_cur = w + used;
        used += align256((size_t)B * d);
        s.mask_prev = w + used;
        used += align256((size_t)B * d);
        s.sup_tau = reinterpret_cast<double *>(w + used);
        used += align256((size_t)B * 8);
        s.sup_cnt = reinterpret_cast<int *>(w + used);
        used += align256((size_t)B * sizeof(int));
    }
    s.cw = w + used;
    s.cw_bytes = total - used;
    return s;
}

// (dot4 and spd_inverse are in tk_host.cpp.)

// Step length along a Newton direction p for an order-4 (or 2) dual: with
// s1 = grad . p < 0, s2 = p . (J + lambda I) p, f3 = K . alpha p^3 and
// f4 = K . p^4, D(alpha + t p) - D(alpha) = s1 t + s2 t^2/2 + f3 t^3 + f4 t^4/4
// exactly.  Returns the first t > 0 where the derivative turns non-negative
// (the minimiser when D is convex along p), bracketed on a logarithmic grid
// and refined by bisection, at most tmax; 1 when p is not a descent direction.
double quartic_step(double s1, double s2, double f3, double f4)
{
    constexpr double tmax = 8.0;
    if (!(s1 < 0) || !std::isfinite(s1) || !std::isfinite(s2) || !std::isfinite(f3) || !std::isfinite(f4))
        return 1.0;
    auto dpsi = [&](double t) { return s1 + t * (s2 + t * (3.0 * f3 + t * f4)); };
    double lo = 0.0, hi = -1.0;
    for (int i = 0; i <= 320; ++i) {
        const double t = std::min(tmax, std::pow(10.0, -14.0 + 0.05 * i));
        if (dpsi(t) >= 0) {
            hi = t;
            break;
        }
        lo = t;
        if (t == tmax) break;
    }
    if (hi < 0) return tmax;
    for (int i = 0; i < 200 && hi - lo > 1e-15 * hi; ++i) {
        const double mid = 0.5 * (lo + hi);
        (dpsi(mid) >= 0 ? hi : lo) = mid;
    }
    return hi;
}

// Device slot b of the preconditioner holds an inverse (J' + lambda' I)^{-1}
// from an earlier iterate (and, along a lambda path, an earlier lambda): a
// stale inverse still preconditions the current system well.
// Pinned host staging for the solver's small readbacks (per host thread,
// grown as needed and kept until the process ends): copies into it need no
// pageable bounce.  Every readback is synchronised before the next use.
void *pinned_stage(size_t bytes)
{
    thread_local void *p = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        void *q = nullptr;
        if (hipHostMalloc(&q, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        if (p) (void)hipHostFree(p);
        p = q;
        cap = bytes;
    }
    return p;
}

// Wait for the work enqueued on `st` so far by polling an event: the solver
// waits on a small readback after every few kernels, and a polling wait
// resumes within microseconds where a blocking one can take tens.
hipError_t spin_sync(hipStream_t st)
{
    thread_local hipEvent_t ev = nullptr;
    if (!ev) {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            ev = nullptr;
            return e;
        }
    }
    hipError_t e = hipEventRecord(ev, st);
    if (e != hipSuccess) return e;
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
    return e;
}

struct Precond {
    bool dev = false;
    bool ident = false;   // ... and that inverse is I / lambda' (from J = 0 at alpha = 0)
    // the device Hessian slot b holds J at an iterate this far (sum of the
    // accepted steps' lengths) from the current one; J does not depend on
    // lambda, so it carries along a path
    bool have_J = false;
    double moved = 0.0;
    double jnorm = 0.0;   // Frobenius norm of the last J inverted (>= ||J||_2)
    // the last refresh was a warm Newton-Schulz update (a few steps from the
    // inverse before it) that held: refreshing is then cheap
    bool warm_ok = false;
    // the held inverse came from Newton-Schulz on the device (not the host
    // factorisation, which takes milliseconds and retries on a J that
    // rounding left indefinite)
    bool ns_ok = false;
    // since the held inverse was made: the iterate moved this far, from an
    // iterate of norm an_inv, and lambda was lam_inv
    double moved_inv = 0.0, an_inv = 0.0, lam_inv = 0.0;
};

struct ProblemState {
    double lam;
    double D, gn, an, ag, aa, ya;
    int newton, cg, status;
    int last_cg;       // CG steps of the last Newton step
    bool done;
};

// One batch (B <= kMaxCoefs) of dual solves.  Each Newton step: the Hessian
// J assembled at alpha (two reads of the tensor; reused while its change stays
// below lambda / 10), CG on the dense system (J + lambda I) p = -grad on the
// device (preconditioned with a host-factored inverse from an earlier
// Hessian, truncated with an Eisenstat-Walker forcing term), the exact step
// length along p for m = 2, 4 (D is a polynomial in the step), Armijo
// backtracking as the safeguard.  Gradients: plain FP64 far from the optimum
// on a cold start and compensated FP64 near it on FP64 storage, FP32
// accumulation on reduced storage; the optional polish continues on an FP64
// tensor.  precond = 0 runs unpreconditioned CG whose products are
// directional-derivative passes over the tensor instead.
int solve_batch(const void *K, int dtype, int64_t n, int m, const double *y, const double *lams, int64_t B,
                const tk_solve_opts &o, double *alpha, tk_solve_info *info, SolveBuffers &sb, hipStream_t st,
                std::vector<Precond> &pc, const SolveCtx &cx)
{
    const bool logistic = cx.loss == TK_LOSS_LOGISTIC;
    // D from the statistics [a.g, a.a, y.a or S, grad.grad] of one problem
    auto dual_of = [&](const double *st4, double lam_b) {
        return logistic ? st4[0] / m + st4[2] / lam_b : st4[0] / m + 0.5 * lam_b * st4[1] - st4[2];
    };
    // tensor of problem b (and of its polish)
    auto kptr = [&](const void *Kb, int dt, int64_t b) -> const void * {
        return reinterpret_cast<const unsigned char *>(Kb) + (size_t)b * (size_t)cx.k_stride * dtype_size(dt);
    };
    std::vector<int> stable(B, 0);
    // why a problem stopped: TK_STOP_TOL, TK_STOP_SUPPORT, TK_STOP_FLOOR
    std::vector<int> reason(B, TK_STOP_TOL);
    std::vector<ProblemState> ps(B);
    for (int64_t b = 0; b < B; ++b) {
        ps[b] = ProblemState{};
        ps[b].lam = lams[b];
    }
    Coefs lam{}, zero{}, one{}, minus1{};
    for (int64_t b = 0; b < B; ++b) {
        lam.c[b] = lams[b];
        one.c[b] = 1.0;
        minus1.c[b] = -1.0;
    }
    int passes = 0, hess_passes = 0;
    std::vector<int> pc_updates(B, 0);
    std::vector<double> hst(B * 4), hd(B), hr(B);
    const bool use_pc = o.precond != 0 && n <= 256;
    const int refresh = o.precond_refresh > 0 ? o.precond_refresh : 8;

    auto sync_copy = [&](double *dst, const double *src, size_t cnt) -> int {
        void *pin = pinned_stage(cnt * sizeof(double));
        if (!pin) return fail(TK_EHIP, "pinned host buffer allocation failed");
        TK_HIP_CHECK(hipMemcpyAsync(pin, src, cnt * sizeof(double), hipMemcpyDeviceToHost, st));
        TK_HIP_CHECK(spin_sync(st));
        std::memcpy(dst, pin, cnt * sizeof(double));
        return TK_OK;
    };
    // On FP64 storage, from a cold start (alpha = 0), the gradient passes use
    // plain FP64 accumulation while ||grad|| is far above their rounding
    // error, and compensated accumulation from the first of: ||grad|| <=
    // 1e-5 ||y||; two Newton steps in a row that neither cut ||grad|| by 10 %
    // nor decrease D by more than 1e-9 of it (the error of a plain pass grows
    // like |K| |alpha|^{m-1}, which at small lambda reaches ||grad||); a line
    // search at its rounding floor.  Convergence is only decided on a
    // compensated gradient.
    bool accurate = true;
    double ynorm = 0.0;
    {
        const int64_t rows = cx.y_stride > 0 ? B : 1;   // per-problem responses (y_stride = n) or one
        std::vector<double> yy(rows);
        TK_HIP_CHECK(vec_dot(y, y, cx.y_stride, sb.stats, rows, n, st));
        TK_HIP_CHECK(hipMemcpyAsync(yy.data(), sb.stats, rows * sizeof(double), hipMemcpyDeviceToHost, st));
        TK_HIP_CHECK(spin_sync(st));
        for (double v : yy) ynorm = std::max(ynorm, std::sqrt(v));
    }
    // gradient pass at `a` into (gdst, graddst), statistics to the host
    auto gradient = [&](const void *Kp, int dt, const double *a, double *gdst, double *graddst,
                        std::vector<double> &out) -> int {
        int mode = dt == TK_F64 ? (accurate ? ACC_DD : ACC_PLAIN64) : ACC_PLAIN32;
        int rc = run_contract(Kp, dt, n, m, a, nullptr, B, gdst, nullptr, mode, sb.cw, sb.cw_bytes, st, 0, nullptr,
                              cx.k_stride);
        if (rc) return rc;
        passes++;
        if (logistic)
            TK_HIP_CHECK(vec_grad_logistic(gdst, a, y, cx.y_stride, lam, graddst, sb.hdiag, sb.stats, B, n, st));
        else
            TK_HIP_CHECK(vec_grad(gdst, a, y, lam, graddst, sb.stats, B, n, st, cx.y_stride));
        return sync_copy(out.data(), sb.stats, B * 4);
    };

    // Hessian J_b = (m-1) K . alpha_b^{m-2} of problem b at its current alpha
    // into its device slot (two reads of the tensor); at alpha = 0 it is zero
    // for m >= 4.  At the dual optimum the products behind J cancel by orders
    // of magnitude (alpha is large where X^T alpha is not), so they run in
    // FP64 on an FP64 tensor: the polish tensor when the solve runs on reduced
    // storage, else the reduced tensor itself.
    auto assemble = [&](const void *Kp, int dt, int64_t b, bool zero) -> int {
        double *Jb = sb.Jd + b * n * n;
        if (zero) {
            TK_HIP_CHECK(hipMemsetAsync(Jb, 0, (size_t)n * n * sizeof(double), st));
            return TK_OK;
        }
        const void *Kh = (dt != TK_F64 && o.polish_K) ? o.polish_K : Kp;
        const int dth = (dt != TK_F64 && o.polish_K) ? TK_F64 : dt;
        int hp = 0;
        int rc = run_hessian(kptr(Kh, dth, b), dth, n, m, alpha + b * n, Jb, sb.hw, sb.hw_bytes, st, &hp);
        if (rc) return rc;
        hess_passes += hp;
        return TK_OK;
    };
    // (J_b + lambda I)^{-1} (J_b + diag(h_b) for the logistic loss) by
    // Newton-Schulz on the device, X <- 2 X - X A X with the dense MFMA
    // products: four steps from the previous inverse (J has moved little),
    // else from I / ||A||_F, where ||I - A X_0||_2 <= 1 - lambda / ||A||_F
    // (J is positive semidefinite) squares at every step: about
    // log2(||A||_F / lambda) + 4 steps, ||A||_F taken from the last inverse
    // (at most 45); kept when ||I - A X||_F < 1/4 (one synchronisation).
    // ok = 0 leaves it to the host factorisation.
    auto refresh_inverse_device = [&](int64_t b, int &ok) -> int {
        ok = 0;
        pc[b].warm_ok = false;
        if (n < 2 || sb.cw_bytes < (2 * (size_t)n * n + kNsResidualDoubles) * sizeof(double)) return TK_OK;
        double *X = sb.P + b * n * n;
        const double *J = sb.Jd + b * n * n;
        double *T = reinterpret_cast<double *>(sb.cw);
        double *XT = T + n * n;
        const double *dg = logistic ? sb.hdiag + b * n : nullptr;
        const double lb = ps[b].lam;
        // ||I - A X_old|| <= (||J - J_old|| + |lambda - lambda_old|) / lambda with
        // ||J - J_old|| about (m-2) ||J||_F moved / ||alpha|| (J homogeneous of
        // degree m-2): four steps from X_old square that bound four times, so
        // they are tried only when it is below 1/2
        const double rho = pc[b].an_inv > 0 ? ((double)(m - 2) * pc[b].jnorm * pc[b].moved_inv / pc[b].an_inv +
                                               std::fabs(lb - pc[b].lam_inv)) / lb
                                            : 1e300;
        for (int attempt = 0; attempt < 2; ++attempt) {
            const bool warm = attempt == 0;
            if (warm && !(pc[b].dev && !pc[b].ident && rho < 0.5)) continue;   // no usable previous inverse
            if (!warm) TK_HIP_CHECK(ns_init(J, lb, dg, X, n, XT, st));   // XT: scratch until the first step
            int iters = warm ? 4 : 45;
            if (!warm && pc[b].jnorm > 0) {
                const double afro = pc[b].jnorm + lb * std::sqrt((double)n);
                iters = std::min(45, std::max(8, (int)std::ceil(std::log2(afro / lb)) + 5));
            }
            // the iterates alternate between X and XT; the symmetrised last one lands in X
            double *xs[2] = {X, XT};
            int cur = 0;
            for (int k = 0; k < iters; ++k, cur ^= 1) {
                TK_HIP_CHECK(launch_gemm_square(J, xs[cur], T, n, kEpiShift, xs[cur], dg, lb, st));   // T = A X
                TK_HIP_CHECK(launch_gemm_square(xs[cur], T, xs[cur ^ 1], n, kEpiReflect, xs[cur], nullptr, 0.0,
                                                st));   // 2 X - X A X
            }
            TK_HIP_CHECK(ns_symmetrize(xs[cur], X, n, st));
            TK_HIP_CHECK(launch_gemm_square(J, X, T, n, kEpiShift, X, dg, lb, st));
            TK_HIP_CHECK(ns_residual(T, J, n, XT, st));
            double out[2];
            TK_HIP_CHECK(hipMemcpyAsync(out, XT, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            TK_HIP_CHECK(spin_sync(st));
            if (o.verbose)
                fprintf(stderr, "[tk_solve] inverse %lld: %s Newton-Schulz, %d steps, ||I - A X||_F %.3e\n",
                        (long long)b, warm ? "warm" : "cold", iters, out[0]);
            if (std::isfinite(out[0]) && out[0] < 0.25) {
                pc[b].jnorm = out[1];
                pc[b].warm_ok = warm;
                pc[b].ns_ok = true;
                pc[b].moved_inv = 0.0;
                pc[b].an_inv = ps[b].an;
                pc[b].lam_inv = lb;
                ok = 1;
                return TK_OK;
            }
        }
        return TK_OK;
    };
    // The same on the host (Cholesky), when Newton-Schulz does not settle: a
    // rounded J may miss positive definiteness by its rounding: shift more.
    // J = 0 gives I / lambda directly.
    auto refresh_inverse = [&](int64_t b, bool zero) -> int {
        if (!zero) {
            int ok = 0;
            if (int rc2 = refresh_inverse_device(b, ok)) return rc2;
            if (ok) {
                pc_updates[b]++;
                pc[b].dev = true;
                pc[b].ident = false;
                return TK_OK;
            }
        }
        std::vector<double> A((size_t)n * n, 0.0);
        std::vector<double> hdg;
        if (zero) {
            for (int64_t i = 0; i < n; ++i) A[i * n + i] = 1.0 / ps[b].lam;
        } else {
            TK_HIP_CHECK(hipMemcpyAsync(A.data(), sb.Jd + b * n * n, (size_t)n * n * sizeof(double),
                                        hipMemcpyDeviceToHost, st));
            if (logistic) {
                hdg.resize(n);
                TK_HIP_CHECK(hipMemcpyAsync(hdg.data(), sb.hdiag + b * n, n * sizeof(double), hipMemcpyDeviceToHost,
                                            st));
            }
            TK_HIP_CHECK(spin_sync(st));
            double tr = 0.0, fro = 0.0;
            for (int64_t i = 0; i < n; ++i) tr += std::fabs(A[i * n + i]);
            for (int64_t i = 0; i < n * n; ++i) fro += A[i] * A[i];
            pc[b].jnorm = std::sqrt(fro);
            double shift = ps[b].lam;
            bool ok = false;
            for (int attempt = 0; attempt < 40 && !ok; ++attempt) {
                std::vector<double> T = A;
                for (int64_t i = 0; i < n; ++i) T[i * n + i] += shift + (logistic ? hdg[i] - ps[b].lam : 0.0);
                if (spd_inverse(T, (int)n)) {
                    A.swap(T);
                    ok = true;
                } else {
                    shift = ps[b].lam + (attempt == 0 ? 1e-7 : shift * 10.0) * (tr / (double)n + 1e-300);
                }
            }
            if (!ok) return fail(TK_EHIP, "could not factor the preconditioner");
        }
        TK_HIP_CHECK(hipMemcpyAsync(sb.P + b * n * n, A.data(), (size_t)n * n * sizeof(double), hipMemcpyHostToDevice,
                                    st));
        TK_HIP_CHECK(spin_sync(st));
        pc_updates[b]++;
        pc[b].dev = true;
        pc[b].ident = zero;
        pc[b].warm_ok = false;
        pc[b].ns_ok = zero;   // I / lambda: free to remake
        pc[b].moved_inv = 0.0;
        pc[b].an_inv = zero ? 0.0 : ps[b].an;
        pc[b].lam_inv = ps[b].lam;
        return TK_OK;
    };

    const int phases = (dtype != TK_F64 && o.polish_K) ? 2 : 1;
    int rc = TK_OK;
    for (int phase = 0; phase < phases; ++phase) {
        if (phase == 1)   // the polish may restart from another iterate
            for (int64_t b = 0; b < B; ++b) pc[b].have_J = false;
        const void *Kp = phase == 0 ? K : o.polish_K;
        const int dt = phase == 0 ? dtype : TK_F64;
        // a phase on reduced storage: its gradients carry the storage rounding,
        // so it keeps its iterate of smallest gradient and ends at the noise
        // floor that rounding sets (handing over to the polish when there is one)
        const bool reduced = dt != TK_F64;
        const int hv_mode = dt == TK_F64 ? ACC_PLAIN64 : ACC_PLAIN32;
        // reduced-precision phase followed by a polish: stop the first phase at a looser tolerance
        const double tol = (phases == 2 && phase == 0) ? std::max(o.tol, 1e-6) : o.tol;
        for (int64_t b = 0; b < B; ++b) {
            ps[b].done = false;
            ps[b].status = TK_OK;
        }
        accurate = true;   // plain passes only from a cold start (a warm start sits near the optimum)
        auto take_stats = [&]() {
            for (int64_t b = 0; b < B; ++b) {
                ProblemState &s = ps[b];
                s.ag = hst[4 * b];
                s.aa = hst[4 * b + 1];
                s.ya = hst[4 * b + 2];
                s.gn = std::sqrt(hst[4 * b + 3]);
                s.an = std::sqrt(s.aa);
                s.D = dual_of(&hst[4 * b], s.lam);
            }
        };
        if ((rc = gradient(Kp, dt, alpha, sb.g, sb.grad, hst))) return rc;
        take_stats();
        if (dt == TK_F64) {
            bool cold = true;
            for (int64_t b = 0; b < B; ++b) cold = cold && !(ps[b].an > 0);
            accurate = !cold;
        }
        const int max_newton = o.fixed_iters > 0 ? o.fixed_iters : (o.max_newton > 0 ? o.max_newton : 100);
        double gn0[kMaxCoefs];
        for (int64_t b = 0; b < B; ++b) gn0[b] = ps[b].gn > 0 ? ps[b].gn : 1.0;
        // reduced-precision phase before a polish: hand over once the gradient
        // stops shrinking (the rounded tensor's noise floor)
        std::vector<double> best_gn(B, INFINITY), prev_Dr(B, INFINITY);
        std::vector<int> stalled(B, 0), loose(B, 0);
        // ... and keep its iterate of smallest gradient: at small lambda the
        // rounded tensor's quartic form is not convex (its rounding reaches the
        // null space of X^T), Newton steps can run off along it, and the polish
        // then starts from the kept iterate
        std::vector<double> kept_gn(B, INFINITY);
        // accepted step length of the last Newton step (1 in the quadratic regime)
        std::vector<double> last_t(B, 0.0);
        std::vector<double> prev_gn(B, INFINITY), prev_D(B, INFINITY);
        std::vector<int> flat(B, 0);   // Newton steps in a row without progress (see below)
        for (int it = 0; it < max_newton; ++it) {
            if (!accurate) {   // near the optimum, stagnating, or a plain gradient claims convergence
                bool sw = false;
                for (int64_t b = 0; b < B; ++b) {
                    if (ps[b].done || !std::isfinite(ps[b].gn)) continue;
                    // no 10 % cut of ||grad|| and (next to) no decrease of D: the
                    // plain passes' rounding, not the damped phase of Newton
                    const bool no_gain = !(prev_D[b] - ps[b].D > 1e-9 * std::fabs(ps[b].D));
                    flat[b] = (ps[b].gn > 0.9 * prev_gn[b] && no_gain) ? flat[b] + 1 : 0;
                    prev_gn[b] = ps[b].gn;
                    prev_D[b] = ps[b].D;
                    // plain FP64 gradients still steer Newton well down to
                    // ||grad|| ~ 1e-7 ||y|| (switching there rather than at 1e-5
                    // saved a compensated step at n = 256 and left the lambda
                    // path unchanged); convergence is only decided on compensated
                    // ones.  Reduced storage keeps 1e-5: its solves meet the
                    // storage floor, and a later switch measured 35 % slower there.
                    const double sw_at = dt == TK_F64 ? 1e-7 : 1e-5;
                    if (ps[b].gn <= sw_at * ynorm || ps[b].gn <= tol * ps[b].lam * ps[b].an || flat[b] >= 2) sw = true;
                }
                if (sw) {
                    accurate = true;
                    if ((rc = gradient(Kp, dt, alpha, sb.g, sb.grad, hst))) return rc;
                    take_stats();
                }
            }
            // stable-support stopping (Section 6.3 threshold): the support of
            // w = (X^T alpha)^{m-1} compared with the last Newton step's
            if (cx.support_stop > 0 && phase == phases - 1) {
                TK_HIP_CHECK(launch_gemm(alpha, n, cx.sX, cx.sd, 1, sb.supW, cx.sd, B, cx.sd, n, m - 1, st));
                TK_HIP_CHECK(launch_support(sb.supW, cx.sd, B, sb.mask_cur, sb.sup_tau, st));
                TK_HIP_CHECK(vec_mask_diff(sb.mask_cur, sb.mask_prev, B, cx.sd, sb.sup_cnt, st));
                std::vector<int> cnt(B);
                TK_HIP_CHECK(hipMemcpyAsync(cnt.data(), sb.sup_cnt, B * sizeof(int), hipMemcpyDeviceToHost, st));
                TK_HIP_CHECK(spin_sync(st));
                for (int64_t b = 0; b < B; ++b) {
                    if (ps[b].done) continue;
                    stable[b] = (it > 0 && cnt[b] == 0) ? stable[b] + 1 : 0;
                    if (stable[b] >= cx.support_stop) {
                        ps[b].done = true;
                        reason[b] = TK_STOP_SUPPORT;
                    }
                }
            }
            bool any = false;
            for (int64_t b = 0; b < B; ++b) {
                ProblemState &s = ps[b];
                if (!std::isfinite(s.gn) || !std::isfinite(s.D)) {
                    s.done = true;
                    s.status = TK_ENAN;
                    reason[b] = TK_STOP_TOL;
                }
                if (!s.done && reduced) {
                    if (s.gn < kept_gn[b]) {
                        kept_gn[b] = s.gn;
                        TK_HIP_CHECK(hipMemcpyAsync(sb.best + b * n, alpha + b * n, n * sizeof(double),
                                                    hipMemcpyDeviceToDevice, st));
                    } else if (!(s.gn <= 1e3 * kept_gn[b])) {
                        s.done = true;   // running off on the rounded tensor
                        reason[b] = TK_STOP_FLOOR;
                    }
                }
                // an exactly zero gradient is the optimum (y = 0 gives alpha = 0)
                if (!s.done && o.fixed_iters <= 0 && (s.gn == 0 || (s.gn <= tol * s.lam * s.an && s.an > 0)))
                    s.done = true;
                // the floor: Newton steps that no longer halve the gradient,
                // three in a row, counted where the step was a full one (the
                // local regime, where the exact problem's gradient would fall
                // quadratically) or left D flat (below 1e-8 of it); damped
                // steps that still decrease D (after a cold or warm start) do
                // not count.  Twelve non-halving steps in a row end it anyway
                // (at small lambda the rounded tensor's Hessian can be
                // indefinite, and steepest-descent steps then crawl).  The
                // iterate of smallest gradient is the one returned.
                if (!s.done && reduced) {
                    const bool flat = !(prev_Dr[b] - s.D > 1e-8 * std::fabs(s.D));
                    if (s.gn < 0.5 * best_gn[b]) {
                        best_gn[b] = s.gn;
                        stalled[b] = 0;
                        loose[b] = 0;
                    } else {
                        // a step without positive curvature (CG took no step: the
                        // rounded tensor's Hessian is indefinite there) counts too
                        // (with a polish tensor to hand over to, any non-halving
                        // step counts: a late hand-over costs more than an early one)
                        if (phases == 2 || std::fabs(last_t[b] - 1.0) <= 0.1 || flat ||
                            (it > 0 && ps[b].last_cg == 0))
                            ++stalled[b];
                        if (stalled[b] >= 3 || ++loose[b] >= 12) {
                            s.done = true;
                            reason[b] = TK_STOP_FLOOR;
                        }
                    }
                    prev_Dr[b] = s.D;
                }
                any |= !s.done;
            }
            if (!any) break;
            // ---- Hessians at the current iterates (the CG operator), and the
            // inverse preconditioner where none is held or the last Newton
            // step needed many CG steps
            std::vector<bool> jfresh(B, false);   // J assembled at the current iterate
            if (use_pc) {
                for (int64_t b = 0; b < B; ++b) {
                    if (ps[b].done) continue;
                    // at alpha = 0 the Hessian of an order m >= 4 dual term is zero
                    const bool zero = !(ps[b].an > 0) && m >= 4;
                    // J from a nearby iterate still serves as the Newton operator
                    // (convergence is decided on exact gradients) while its change,
                    // about (m-2) ||J|| moved / ||alpha|| for a J homogeneous of
                    // degree m-2, stays below lambda / 10
                    const bool reuse = pc[b].have_J && !zero && pc[b].jnorm > 0 &&
                                       (double)(m - 2) * pc[b].jnorm * pc[b].moved <= 0.1 * ps[b].lam * ps[b].an;
                    if (!reuse) {
                        if ((rc = assemble(Kp, dt, b, zero))) return rc;
                        pc[b].have_J = !zero;
                        pc[b].moved = 0.0;
                        jfresh[b] = true;
                    }
                    // the logistic loss's separable Hessian lambda / (p (1-p)) changes
                    // fast as iterates near the domain's boundary: a stale inverse
                    // then steers CG into the step cap, so it is refreshed every step
                    // after a warm update held, refresh whenever CG needed more than
                    // one step (along a path J moves little from lambda to lambda);
                    // an inverse made (on the device) at a lambda more than twice
                    // the current one misses the small eigenvalues that now bound CG;
                    // not on a J from reduced storage, whose rounding leaves it
                    // indefinite at small lambda
                    const int rlim = pc[b].warm_ok ? 1 : refresh;
                    const bool j_exact = dt == TK_F64 || o.polish_K;
                    const bool lam_fell = j_exact && pc[b].ns_ok && pc[b].lam_inv > 2.0 * ps[b].lam;
                    if (!pc[b].dev || (pc[b].ident && !zero) || ps[b].last_cg > rlim || lam_fell || logistic)
                        if ((rc = refresh_inverse(b, zero))) return rc;
                }
            }
            // ---- CG on (J + lam I) x = -grad for the active problems, truncated at
            // ||r|| <= eta ||grad|| (Eisenstat-Walker forcing)
            Coefs act{};
            for (int64_t b = 0; b < B; ++b) act.c[b] = ps[b].done ? 0.0 : 1.0;
            const int max_cg = o.max_cg > 0 ? o.max_cg : 2000;
            std::vector<int> cg_steps(B, 0);
            bool cg_pending = false;
            std::vector<double> eta(B);
            for (int64_t b = 0; b < B; ++b) eta[b] = std::min(0.5, std::max(std::sqrt(ps[b].gn / gn0[b]), 1e-12));
            if (use_pc) {
                // on the dense system, preconditioned, entirely on the device:
                // one launch and one synchronisation per Newton step
                Coefs etac{};
                for (int64_t b = 0; b < B; ++b) etac.c[b] = eta[b];
                int *dsteps = reinterpret_cast<int *>(sb.stats2);
                TK_HIP_CHECK(vec_cg_dense(sb.Jd, sb.P, sb.grad, lam, etac, act, B, n, max_cg, sb.x, dsteps, st,
                                          logistic ? sb.hdiag : nullptr));
                cg_pending = true;   // the step counts come back with the line statistics below
            } else {
                // unpreconditioned, every product one directional-derivative pass over the tensor
                std::vector<double> rz(B);
                std::vector<bool> cg_on(B);
                TK_HIP_CHECK(vec_lin2(sb.grad, sb.grad, zero, zero, sb.x, B, n, st));     // x = 0
                TK_HIP_CHECK(vec_lin2(sb.grad, sb.grad, minus1, zero, sb.r, B, n, st));   // r = -grad
                TK_HIP_CHECK(vec_lin2(sb.r, sb.r, one, zero, sb.dv, B, n, st));           // d = r
                for (int64_t b = 0; b < B; ++b) {
                    rz[b] = ps[b].gn * ps[b].gn;
                    cg_on[b] = !ps[b].done && ps[b].gn > 0;
                }
                for (int j = 0; j < max_cg; ++j) {
                    bool anycg = false;
                    for (int64_t b = 0; b < B; ++b) anycg |= cg_on[b];
                    if (!anycg) break;
                    if ((rc = run_contract(Kp, dt, n, m, alpha, sb.dv, B, nullptr, sb.hd, hv_mode, sb.cw, sb.cw_bytes,
                                           st, 0, nullptr, cx.k_stride)))
                        return rc;
                    passes++;
                    TK_HIP_CHECK(vec_shift_dot(sb.dv, sb.hd, lam, sb.stats, B, n, st, logistic ? sb.hdiag : nullptr));
                    if ((rc = sync_copy(hd.data(), sb.stats, B))) return rc;
                    Coefs a{};
                    for (int64_t b = 0; b < B; ++b) {
                        if (!cg_on[b]) continue;
                        if (!(hd[b] > 0) || !std::isfinite(hd[b])) {   // no positive curvature along d
                            cg_on[b] = false;
                            continue;
                        }
                        a.c[b] = rz[b] / hd[b];
                        ps[b].cg++;
                        cg_steps[b]++;
                    }
                    TK_HIP_CHECK(vec_cg_update(sb.x, sb.r, sb.dv, sb.hd, a, sb.stats, B, n, st));   // stats = r.r
                    if ((rc = sync_copy(hr.data(), sb.stats, B))) return rc;
                    Coefs beta{}, keep{};
                    for (int64_t b = 0; b < B; ++b) {
                        keep.c[b] = 1.0;
                        if (!cg_on[b]) continue;
                        if (std::sqrt(hr[b]) <= eta[b] * ps[b].gn) {
                            cg_on[b] = false;
                            continue;
                        }
                        beta.c[b] = hr[b] / rz[b];
                        rz[b] = hr[b];
                    }
                    TK_HIP_CHECK(vec_lin2(sb.r, sb.dv, keep, beta, sb.dv, B, n, st));   // d = r + beta d
                }
            }
            // ---- the line along x: ||x||^2, the slope grad . x and, for the
            // exact step, the model of D along x, all read back in one copy
            // with the CG step counts (statistics slices: model [0, 3B),
            // x.x [3B, 4B), grad.x [4B, 5B))
            bool need_model = false;   // the model pass is skipped once every problem takes unit steps
            for (int64_t b = 0; b < B; ++b)
                if (!ps[b].done && !(std::fabs(last_t[b] - 1.0) <= 0.05)) need_model = true;
            const bool model = !logistic && use_pc && (m == 2 || m == 4) && need_model;
            // m = 4 on FP64 storage with plain gradients and J fresh at alpha:
            // the contraction along the line is the cubic
            //   K (alpha + t x)^3 = g + t J x + t^2 (3 K x^2 alpha) + t^3 K x^3,
            // so one directional-derivative pass at x along alpha (which also
            // returns K x^3) replaces the gradient passes of the line search
            bool algebraic = false;
            std::vector<double> mod(3 * B, 0.0);
            // s2 from the assembled Hessian, and for m = 4 the cubic and quartic
            // terms from one pass giving dv = K . x^3 (D is a quartic in the step)
            auto enqueue_model = [&]() -> int {
                algebraic = m == 4 && dt == TK_F64 && !accurate && !o.polish_K;
                for (int64_t b = 0; b < B; ++b)
                    if (!ps[b].done && !jfresh[b]) algebraic = false;
                TK_HIP_CHECK(vec_symv(sb.Jd, sb.x, sb.z, B, n, st));                 // z = J x
                TK_HIP_CHECK(vec_lin2(sb.z, sb.z, one, zero, sb.hd, B, n, st));
                TK_HIP_CHECK(vec_shift_dot(sb.x, sb.hd, lam, sb.stats, B, n, st));
                if (m == 4) {
                    int rc2;
                    if (algebraic) {   // r = 3 K x^2 alpha, dv = K x^3
                        if ((rc2 = run_contract(Kp, dt, n, m, sb.x, alpha, B, sb.dv, sb.r, ACC_PLAIN64, sb.cw,
                                                sb.cw_bytes, st, 0, nullptr, cx.k_stride)))
                            return rc2;
                    } else {
                        const int pm = dt == TK_F64 ? ACC_PLAIN64 : ACC_PLAIN32;
                        if ((rc2 = run_contract(Kp, dt, n, m, sb.x, nullptr, B, sb.dv, nullptr, pm, sb.cw,
                                                sb.cw_bytes, st, 0, nullptr, cx.k_stride)))
                            return rc2;
                    }
                    passes++;
                    TK_HIP_CHECK(vec_dot(alpha, sb.dv, n, sb.stats + B, B, n, st));
                    TK_HIP_CHECK(vec_dot(sb.x, sb.dv, n, sb.stats + 2 * B, B, n, st));
                }
                return TK_OK;
            };
            std::vector<double> hr0(B), slope(B), t(B, 1.0);
            {
                TK_HIP_CHECK(vec_dot(sb.x, sb.x, n, sb.stats + 3 * B, B, n, st));
                TK_HIP_CHECK(vec_dot(sb.grad, sb.x, n, sb.stats + 4 * B, B, n, st));
                if (model && (rc = enqueue_model())) return rc;
                unsigned char *pin = reinterpret_cast<unsigned char *>(pinned_stage(5 * B * sizeof(double) + B * sizeof(int)));
                if (!pin) return fail(TK_EHIP, "pinned host buffer allocation failed");
                TK_HIP_CHECK(hipMemcpyAsync(pin, sb.stats, 5 * B * sizeof(double), hipMemcpyDeviceToHost, st));
                if (cg_pending)
                    TK_HIP_CHECK(hipMemcpyAsync(pin + 5 * B * sizeof(double), sb.stats2, B * sizeof(int),
                                                hipMemcpyDeviceToHost, st));
                TK_HIP_CHECK(spin_sync(st));
                const double *pd = reinterpret_cast<const double *>(pin);
                for (int64_t b = 0; b < B; ++b) {
                    mod[b] = pd[b];
                    mod[B + b] = pd[B + b];
                    mod[2 * B + b] = pd[2 * B + b];
                    hr0[b] = pd[3 * B + b];
                    slope[b] = pd[4 * B + b];
                }
                if (cg_pending) {
                    std::memcpy(cg_steps.data(), pin + 5 * B * sizeof(double), B * sizeof(int));
                    for (int64_t b = 0; b < B; ++b)
                        if (!ps[b].done) ps[b].cg += cg_steps[b];
                }
            }
            for (int64_t b = 0; b < B; ++b)
                if (!ps[b].done) ps[b].last_cg = cg_steps[b];
            // if CG produced nothing (zero curvature at the first step), fall back
            // to steepest descent; the slope and model are then taken again
            bool fallback = false;
            {
                Coefs c1{}, c2{};
                for (int64_t b = 0; b < B; ++b) {
                    c1.c[b] = 1.0;
                    if (!ps[b].done && !(hr0[b] > 0)) {
                        c1.c[b] = 0.0;
                        c2.c[b] = -1.0 / std::max(ps[b].lam, 1e-300);
                        fallback = true;
                    }
                }
                if (fallback) {
                    TK_HIP_CHECK(vec_lin2(sb.x, sb.grad, c1, c2, sb.x, B, n, st));
                    TK_HIP_CHECK(vec_dot(sb.grad, sb.x, n, sb.stats + 4 * B, B, n, st));
                    if (model && (rc = enqueue_model())) return rc;
                    std::vector<double> all(5 * B);
                    if ((rc = sync_copy(all.data(), sb.stats, 5 * B))) return rc;
                    for (int64_t b = 0; b < B; ++b) {
                        if (model) {
                            mod[b] = all[b];
                            mod[B + b] = all[B + b];
                            mod[2 * B + b] = all[2 * B + b];
                        }
                        slope[b] = all[4 * B + b];
                    }
                }
            }
            std::vector<double> xnorm(B);
            for (int64_t b = 0; b < B; ++b) xnorm[b] = hr0[b] > 0 ? std::sqrt(hr0[b]) : INFINITY;
            if (logistic) {
                // the separable term is not a polynomial: start the backtracking
                // at the full step, shortened to stay inside the domain
                std::vector<double> cap(B);
                TK_HIP_CHECK(vec_step_cap(alpha, sb.x, y, cx.y_stride, lam, sb.stats, B, n, st));
                if ((rc = sync_copy(cap.data(), sb.stats, B))) return rc;
                for (int64_t b = 0; b < B; ++b)
                    if (!ps[b].done) t[b] = std::min(1.0, 0.99 * cap[b]);
            } else if (model) {
                for (int64_t b = 0; b < B; ++b)
                    if (!ps[b].done) t[b] = quartic_step(slope[b], mod[b], mod[B + b], mod[2 * B + b]);
            }
            std::vector<bool> ls(B);
            for (int64_t b = 0; b < B; ++b) ls[b] = !ps[b].done;
            bool floor_plain = false;
            for (int trial = 0; trial < 60; ++trial) {
                bool anyls = false;
                Coefs tc{};
                for (int64_t b = 0; b < B; ++b) {
                    anyls |= ls[b];
                    tc.c[b] = ls[b] ? t[b] : 0.0;
                }
                if (!anyls) break;
                TK_HIP_CHECK(vec_lin2(alpha, sb.x, one, tc, sb.at, B, n, st));   // at = alpha + t x
                if (algebraic) {   // gt = g + t J x + t^2 r + t^3 dv
                    TK_HIP_CHECK(vec_poly3(sb.g, sb.z, sb.r, sb.dv, tc, sb.gt, B, n, st));
                    TK_HIP_CHECK(vec_grad(sb.gt, sb.at, y, lam, sb.hd, sb.stats, B, n, st, cx.y_stride));
                    if ((rc = sync_copy(hst.data(), sb.stats, B * 4))) return rc;
                } else if ((rc = gradient(Kp, dt, sb.at, sb.gt, sb.hd, hst))) {
                    return rc;
                }
                Coefs acc_c{}, keep_c{};
                bool anyacc = false;
                for (int64_t b = 0; b < B; ++b) {
                    keep_c.c[b] = 1.0;
                    if (!ls[b]) continue;
                    const double Dn = dual_of(&hst[4 * b], ps[b].lam);
                    const bool ok = std::isfinite(Dn) &&
                                    (Dn <= ps[b].D + 1e-4 * t[b] * slope[b] ||
                                     // below rounding of D: accept if the gradient norm decreased
                                     (std::fabs(Dn - ps[b].D) <= 1e-14 * (std::fabs(ps[b].D) + 1) &&
                                      std::sqrt(hst[4 * b + 3]) < ps[b].gn));
                    if (ok) {
                        ls[b] = false;
                        acc_c.c[b] = 1.0;
                        keep_c.c[b] = 0.0;
                        anyacc = true;
                        ProblemState &s = ps[b];
                        s.ag = hst[4 * b];
                        s.aa = hst[4 * b + 1];
                        s.ya = hst[4 * b + 2];
                        s.gn = std::sqrt(hst[4 * b + 3]);
                        s.an = std::sqrt(s.aa);
                        s.D = Dn;
                        s.newton++;
                        last_t[b] = t[b];
                        pc[b].moved += t[b] * xnorm[b];
                        pc[b].moved_inv += t[b] * xnorm[b];
                    } else {
                        t[b] *= 0.5;
                        // reduced storage: D comes from FP32-accumulated passes, so a
                        // first-order decrease below about 1e-6 |D| is noise: that is
                        // the floor too (halving on to 1e-14 cost ~40 passes per lambda)
                        const bool noise = reduced && t[b] * std::fabs(slope[b]) < 1e-6 * (std::fabs(ps[b].D) + 1.0);
                        if (t[b] < 1e-14 || noise) {   // no decrease visible: rounding floor of D
                            ls[b] = false;
                            if (accurate) {
                                ps[b].done = true;
                                if (reduced) reason[b] = TK_STOP_FLOOR;   // ... of the rounded tensor
                            } else {
                                floor_plain = true;   // ... of the plain passes: go on compensated
                            }
                        }
                    }
                }
                if (anyacc) {
                    // accepted problems: alpha <- at, g <- gt, grad <- (hd holds grad of at)
                    TK_HIP_CHECK(vec_lin2(alpha, sb.at, keep_c, acc_c, alpha, B, n, st));
                    TK_HIP_CHECK(vec_lin2(sb.g, sb.gt, keep_c, acc_c, sb.g, B, n, st));
                    TK_HIP_CHECK(vec_lin2(sb.grad, sb.hd, keep_c, acc_c, sb.grad, B, n, st));
                }
            }
            if (floor_plain) {
                accurate = true;
                if ((rc = gradient(Kp, dt, alpha, sb.g, sb.grad, hst))) return rc;
                take_stats();
            }
            if (o.verbose) {
                for (int64_t b = 0; b < B; ++b)
                    fprintf(stderr, "[tk_solve] phase %d it %d lam %.3e |grad| %.3e D %.15e |a| %.3e cg %d\n", phase, it,
                            ps[b].lam, ps[b].gn, ps[b].D, ps[b].an, ps[b].cg);
            }
        }
        if (!accurate) {   // Newton limit reached on plain gradients: report a compensated one
            accurate = true;
            if ((rc = gradient(Kp, dt, alpha, sb.g, sb.grad, hst))) return rc;
            take_stats();
        }
        bool restored = false;
        for (int64_t b = 0; b < B; ++b) {
            ProblemState &s = ps[b];
            if (reduced) {
                if (std::isfinite(kept_gn[b]) && kept_gn[b] < s.gn) {   // back to the kept iterate
                    if (s.status == TK_ENAN) s.status = TK_OK;
                    TK_HIP_CHECK(hipMemcpyAsync(alpha + b * n, sb.best + b * n, n * sizeof(double),
                                                hipMemcpyDeviceToDevice, st));
                    restored = true;
                } else if (phases == 2 && s.status == TK_ENAN) {   // restart the polish from zero
                    s.status = TK_OK;
                    TK_HIP_CHECK(hipMemsetAsync(alpha + b * n, 0, n * sizeof(double), st));
                }
            }
        }
        if (phases == 2 && phase == 0) {
            for (int64_t b = 0; b < B; ++b) reason[b] = TK_STOP_TOL;
            continue;   // the polish follows
        }
        if (restored) {   // statistics of the returned iterates
            if ((rc = gradient(Kp, dt, alpha, sb.g, sb.grad, hst))) return rc;
            take_stats();
        }
        for (int64_t b = 0; b < B; ++b) {
            ProblemState &s = ps[b];
            if (s.status == TK_OK && (s.gn == 0 || s.gn <= tol * s.lam * s.an)) reason[b] = TK_STOP_TOL;
            if (s.status == TK_OK && o.fixed_iters <= 0 && reason[b] == TK_STOP_TOL && s.gn != 0 &&
                !(s.gn <= tol * s.lam * s.an))
                s.status = TK_ENOCONV;
        }
    }
    int overall = TK_OK;
    for (int64_t b = 0; b < B; ++b) {
        tk_solve_info &inf = info[b];
        inf.newton_iters = ps[b].newton;
        inf.cg_iters = ps[b].cg;
        inf.passes = passes;
        inf.grad_norm = ps[b].gn;
        inf.objective = ps[b].D;
        inf.alpha_norm = ps[b].an;
        inf.status = ps[b].status;
        inf.hess_passes = hess_passes;
        inf.precond_updates = pc_updates[b];
        inf.stop_reason = ps[b].status == TK_OK ? reason[b] : TK_STOP_TOL;
        if (ps[b].status != TK_OK) overall = ps[b].status;
    }
    return overall;
}

}  // namespace
}  // namespace tk

extern "C" {

int tk_solve_workspace_ex(int64_t n, int m, int64_t B, int dtype, int64_t support_d, size_t *h_bytes)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1) return fail(TK_EINVAL, "B must be >= 1");
    if (support_d < 0) return fail(TK_EINVAL, "support_d must be >= 0");
    if (!h_bytes) return fail(TK_EINVAL, "null output pointer");
    const int64_t bb = B < kMaxCoefs ? B : kMaxCoefs;
    *h_bytes = solve_ws(n, m, bb, dtype, support_d);
    return TK_OK;
}

int tk_solve_workspace(int64_t n, int m, int64_t B, int dtype, size_t *h_bytes)
{
    return tk_solve_workspace_ex(n, m, B, dtype, 0, h_bytes);
}

}  // extern "C"

namespace tk {
namespace {

// Options shared by the single-tensor and the multi-tensor solves: defaults,
// validation, and the solve context they imply.
int prepare_solve(const tk_solve_opts *h_opts, tk_solve_opts &o, SolveCtx &cx)
{
    tk_solve_opts_default(&o);
    if (h_opts) o = *h_opts;
    if (o.polish_K && o.polish_dtype != TK_F64) return fail(TK_EINVAL, "the polish tensor must be FP64");
    if (o.loss != TK_LOSS_SQUARE && o.loss != TK_LOSS_LOGISTIC) return fail(TK_EINVAL, "unknown loss %d", o.loss);
    if (o.support_stop < 0) return fail(TK_EINVAL, "support_stop must be >= 0");
    if (o.support_stop > 0 && (!o.support_X || o.support_d < 1))
        return fail(TK_EINVAL, "support_stop needs the points (support_X) and their dimension (support_d)");
    cx.loss = o.loss;
    cx.support_stop = o.support_stop;
    cx.sX = o.support_stop > 0 ? o.support_X : nullptr;
    cx.sd = o.support_stop > 0 ? o.support_d : 0;
    return TK_OK;
}

// Checks of the responses and of the warm start before any pass: finite
// values; for the logistic loss labels in {-1, +1} and a warm start inside the
// dual's domain.
int check_solve_inputs(const tk_solve_opts &o, const double *d_y, int64_t ylen, const double *d_alpha,
                       int64_t alen, const double *h_lams, int64_t nlam, void *d_work, hipStream_t st)
{
    int *flag = reinterpret_cast<int *>(d_work);
    int bad[2] = {0, 0};
    TK_HIP_CHECK(hipMemsetAsync(flag, 0, 2 * sizeof(int), st));
    TK_HIP_CHECK(vec_nonfinite(d_y, ylen, flag, st));
    if (o.warm_start) TK_HIP_CHECK(vec_nonfinite(d_alpha, alen, flag, st));
    if (o.loss == TK_LOSS_LOGISTIC) TK_HIP_CHECK(vec_check_labels(d_y, ylen, flag + 1, st));
    TK_HIP_CHECK(hipMemcpyAsync(bad, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    TK_HIP_CHECK(hipStreamSynchronize(st));
    if (bad[0]) return fail(TK_ENAN, "non-finite value in y%s", o.warm_start ? " or in the warm start" : "");
    if (bad[1]) return fail(TK_EINVAL, "the logistic loss needs labels y in {-1, +1}");
    (void)h_lams;
    (void)nlam;
    return TK_OK;
}

}  // namespace
}  // namespace tk

extern "C" {

int tk_solve_dual(const void *d_K, int dtype, int64_t n, int m, const double *d_y, const double *h_lambdas,
                  int64_t B, const tk_solve_opts *h_opts, double *d_alpha, tk_solve_info *h_info, void *d_work,
                  size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (B < 1) return fail(TK_EINVAL, "B must be >= 1");
    if (!d_K || !d_y || !h_lambdas || !d_alpha || !h_info) return fail(TK_EINVAL, "null pointer");
    tk_solve_opts o;
    SolveCtx cx;
    if ((rc = prepare_solve(h_opts, o, cx))) return rc;
    for (int64_t b = 0; b < B; ++b)
        if (!(h_lambdas[b] > 0) || !std::isfinite(h_lambdas[b]))
            return fail(TK_EINVAL, "lambda[%lld] must be positive and finite", (long long)b);
    const int64_t bb = B < kMaxCoefs ? B : kMaxCoefs;
    const size_t need = solve_ws(n, m, bb, dtype, cx.sd);
    if (work_bytes < need || !d_work) return fail(TK_ENOMEM, "solve workspace of %zu bytes < %zu", work_bytes, need);
    hipStream_t st = as_stream(stream);
    if ((rc = check_solve_inputs(o, d_y, n, d_alpha, B * n, h_lambdas, B, d_work, st))) return rc;
    // cold starts: alpha = 0 (square loss), the centre of the domain (logistic)
    auto cold = [&](double *a, const double *lams, int64_t nb) -> int {
        if (o.loss == TK_LOSS_LOGISTIC) {
            Coefs lc{};
            for (int64_t b = 0; b < nb; ++b) lc.c[b] = lams[b];
            TK_HIP_CHECK(vec_logistic_start(d_y, 0, lc, a, nb, n, st));
        } else {
            TK_HIP_CHECK(hipMemsetAsync(a, 0, (size_t)nb * n * sizeof(double), st));
        }
        return TK_OK;
    };
    int overall = TK_OK;
    if (B > 1 && o.continuation) {
        // lambda path: from the largest lambda down, each solve starts from the
        // previous solution and keeps its Hessian for the preconditioner
        std::vector<int64_t> order(B);
        for (int64_t b = 0; b < B; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t u, int64_t v) { return h_lambdas[u] > h_lambdas[v]; });
        std::vector<Precond> pc(1);
        SolveBuffers sb = carve(d_work, n, m, 1, work_bytes, cx.sd);
        int64_t prev = -1;
        for (int64_t idx = 0; idx < B; ++idx) {
            const int64_t b = order[idx];
            double *a = d_alpha + b * n;
            if (prev >= 0 && !o.warm_start)
                TK_HIP_CHECK(hipMemcpyAsync(a, d_alpha + prev * n, n * sizeof(double), hipMemcpyDeviceToDevice, st));
            else if (prev < 0 && !o.warm_start && (rc = cold(a, h_lambdas + b, 1)))
                return rc;
            rc = solve_batch(d_K, dtype, n, m, d_y, h_lambdas + b, 1, o, a, h_info + b, sb, st, pc, cx);
            if (rc != TK_OK && rc != TK_ENOCONV && rc != TK_ENAN) return rc;
            if (rc != TK_OK) overall = rc;
            prev = b;
        }
    } else {
        for (int64_t b0 = 0; b0 < B; b0 += kMaxCoefs) {
            const int64_t nb = (B - b0) < kMaxCoefs ? (B - b0) : kMaxCoefs;
            double *a = d_alpha + b0 * n;
            if (!o.warm_start && (rc = cold(a, h_lambdas + b0, nb))) return rc;
            SolveBuffers sb = carve(d_work, n, m, nb, work_bytes, cx.sd);
            std::vector<Precond> pc(nb);
            rc = solve_batch(d_K, dtype, n, m, d_y, h_lambdas + b0, nb, o, a, h_info + b0, sb, st, pc, cx);
            if (rc != TK_OK && rc != TK_ENOCONV && rc != TK_ENAN) return rc;
            if (rc != TK_OK) overall = rc;
        }
    }
    if (overall == TK_ENOCONV) fail(TK_ENOCONV, "at least one lambda did not reach the tolerance");
    if (overall == TK_ENAN) fail(TK_ENAN, "non-finite values met during the solve");
    return overall;
}

int tk_packed_stride(int64_t n, int m, int dtype, int64_t *h_stride)
{
    int rc;
    int64_t c;
    if ((rc = tk_packed_count(n, m, &c))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (!h_stride) return fail(TK_EINVAL, "null output pointer");
    const int64_t per = 256 / (int64_t)dtype_size(dtype);   // entries per 256 bytes
    if (c > INT64_MAX - per) return fail(TK_EOVERFLOW, "stride overflows int64");
    *h_stride = (c + per - 1) / per * per;
    return TK_OK;
}

int tk_build_packed_multi(const double *d_X, int64_t T, int64_t n, int64_t d, int m, int kernel, double kparam,
                          int dtype, void *d_K, int64_t k_stride, void *stream)
{
    int rc;
    if (T < 1 || T > 65535) return fail(TK_EINVAL, "T must be in [1, 65535]");
    int64_t need;
    if ((rc = tk_packed_stride(n, m, dtype, &need))) return rc;
    if (k_stride < need) return fail(TK_EINVAL, "k_stride %lld is below tk_packed_stride (%lld)", (long long)k_stride,
                                     (long long)need);
    if (((size_t)k_stride * dtype_size(dtype)) % 16) return fail(TK_EINVAL, "k_stride must keep 16-byte alignment");
    if (!d_X || !d_K) return fail(TK_EINVAL, "null device pointer");
    for (int64_t t = 0; t < T; ++t) {
        rc = tk_build_packed_tensor(d_X + t * n * d, n, d, m, kernel, kparam, dtype,
                                    reinterpret_cast<unsigned char *>(d_K) + (size_t)t * k_stride * dtype_size(dtype),
                                    stream);
        if (rc) return rc;
    }
    return TK_OK;
}

int tk_contract_multi(const void *d_K, int dtype, int64_t n, int m, int64_t T, int64_t k_stride,
                      const double *d_alpha, double *d_g, int acc, void *d_work, size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (T < 1 || T > 65535) return fail(TK_EINVAL, "T must be in [1, 65535]");
    int64_t need;
    if ((rc = tk_packed_stride(n, m, dtype, &need))) return rc;
    if (k_stride < need) return fail(TK_EINVAL, "k_stride below tk_packed_stride");
    if (((size_t)k_stride * dtype_size(dtype)) % 16) return fail(TK_EINVAL, "k_stride must keep 16-byte alignment");
    if (!d_K || !d_alpha || !d_g) return fail(TK_EINVAL, "null device pointer");
    int mode;
    if ((rc = mode_for(dtype, acc, false, &mode))) return rc;
    return run_contract(d_K, dtype, n, m, d_alpha, nullptr, T, d_g, nullptr, mode, d_work, work_bytes,
                        as_stream(stream), 1, nullptr, k_stride);
}

int tk_solve_dual_multi(const void *d_K, int dtype, int64_t n, int m, int64_t T, int64_t k_stride,
                        const double *d_y, const double *h_lambdas, int64_t L, const tk_solve_opts *h_opts,
                        double *d_alpha, tk_solve_info *h_info, void *d_work, size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (T < 1 || T > 65535 || L < 1) return fail(TK_EINVAL, "T must be in [1, 65535] and L >= 1");
    int64_t need_stride;
    if ((rc = tk_packed_stride(n, m, dtype, &need_stride))) return rc;
    if (k_stride < need_stride) return fail(TK_EINVAL, "k_stride below tk_packed_stride");
    if (((size_t)k_stride * dtype_size(dtype)) % 16) return fail(TK_EINVAL, "k_stride must keep 16-byte alignment");
    if (!d_K || !d_y || !h_lambdas || !d_alpha || !h_info) return fail(TK_EINVAL, "null pointer");
    tk_solve_opts o;
    SolveCtx cx;
    if ((rc = prepare_solve(h_opts, o, cx))) return rc;
    if (o.polish_K) return fail(TK_EINVAL, "the multi-tensor solve takes no polish tensor");
    if (o.support_stop > 0) return fail(TK_EINVAL, "the multi-tensor solve has no stable-support stop");
    for (int64_t l = 0; l < L; ++l)
        if (!(h_lambdas[l] > 0) || !std::isfinite(h_lambdas[l]))
            return fail(TK_EINVAL, "lambda[%lld] must be positive and finite", (long long)l);
    cx.k_stride = k_stride;
    cx.y_stride = n;
    const int64_t bb = T < kMaxCoefs ? T : kMaxCoefs;
    const size_t need = solve_ws(n, m, bb, dtype);
    if (work_bytes < need || !d_work) return fail(TK_ENOMEM, "solve workspace of %zu bytes < %zu", work_bytes, need);
    hipStream_t st = as_stream(stream);
    if ((rc = check_solve_inputs(o, d_y, T * n, d_alpha, L * T * n, h_lambdas, L, d_work, st))) return rc;
    std::vector<int64_t> order(L);
    for (int64_t l = 0; l < L; ++l) order[l] = l;
    std::stable_sort(order.begin(), order.end(), [&](int64_t u, int64_t v) { return h_lambdas[u] > h_lambdas[v]; });
    int overall = TK_OK;
    // draws in lock step (up to 64 per batch, every pass shared), lambdas by
    // continuation from the largest down; each draw keeps its Hessian and
    // preconditioner from lambda to lambda
    for (int64_t t0 = 0; t0 < T; t0 += kMaxCoefs) {
        const int64_t nb = (T - t0) < kMaxCoefs ? (T - t0) : kMaxCoefs;
        SolveBuffers sb = carve(d_work, n, m, nb, work_bytes);
        std::vector<Precond> pc(nb);
        const void *Kb = reinterpret_cast<const unsigned char *>(d_K) + (size_t)t0 * k_stride * dtype_size(dtype);
        const double *yb = d_y + t0 * n;
        int64_t prev = -1;
        for (int64_t idx = 0; idx < L; ++idx) {
            const int64_t l = order[idx];
            double *a = d_alpha + (l * T + t0) * n;
            std::vector<double> lams(nb, h_lambdas[l]);
            if (!o.warm_start) {
                if (prev >= 0) {
                    TK_HIP_CHECK(hipMemcpyAsync(a, d_alpha + (prev * T + t0) * n, (size_t)nb * n * sizeof(double),
                                                hipMemcpyDeviceToDevice, st));
                } else if (o.loss == TK_LOSS_LOGISTIC) {
                    Coefs lc{};
                    for (int64_t b = 0; b < nb; ++b) lc.c[b] = h_lambdas[l];
                    TK_HIP_CHECK(vec_logistic_start(yb, n, lc, a, nb, n, st));
                } else {
                    TK_HIP_CHECK(hipMemsetAsync(a, 0, (size_t)nb * n * sizeof(double), st));
                }
            }
            rc = solve_batch(Kb, dtype, n, m, yb, lams.data(), nb, o, a, h_info + l * T + t0, sb, st, pc, cx);
            if (rc != TK_OK && rc != TK_ENOCONV && rc != TK_ENAN) return rc;
            if (rc != TK_OK) overall = rc;
            prev = l;
        }
    }
    if (overall == TK_ENOCONV) fail(TK_ENOCONV, "at least one problem did not reach the tolerance");
    if (overall == TK_ENAN) fail(TK_ENAN, "non-finite values met during the solve");
    return overall;
}

int tk_primal_weights(const double *d_X, int64_t n, int64_t d, int m, const double *d_alpha, int64_t B,
                      double *d_W, void *stream)
{
    if (n < 1 || d < 1 || B < 1) return fail(TK_EINVAL, "sizes must be >= 1");
    if (m < 2 || (m & 1)) return fail(TK_EINVAL, "m must be even and >= 2");
    if (!d_X || !d_alpha || !d_W) return fail(TK_EINVAL, "null device pointer");
    // W[b][j] = (sum_i alpha[b][i] X[i][j])^{m-1}
    hipError_t e = launch_gemm(d_alpha, n, d_X, d, 1, d_W, d, B, d, n, m - 1, as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "gemm failed: %s", hipGetErrorString(e));
    return TK_OK;
}

int tk_predict(const double *d_W, int64_t d, int64_t B, const double *d_Xq, int64_t N, double *d_f, void *stream)
{
    if (d < 1 || B < 1 || N < 1) return fail(TK_EINVAL, "sizes must be >= 1");
    if (!d_W || !d_Xq || !d_f) return fail(TK_EINVAL, "null device pointer");
    // f[b][q] = sum_j W[b][j] Xq[q][j]
    hipError_t e = launch_gemm(d_W, d, d_Xq, 1, d, d_f, N, B, N, d, 1, as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "gemm failed: %s", hipGetErrorString(e));
    return TK_OK;
}

int tk_predict_kernel_workspace(int64_t n, int m, int64_t B, int64_t N, size_t *h_bytes)
{
    if (n < 1 || B < 1 || N < 1) return fail(TK_EINVAL, "sizes must be >= 1");
    if (m < 2 || (m & 1) || m > kMaxOrder) return fail(TK_EINVAL, "m must be even and in [2, %d]", kMaxOrder);
    if (!h_bytes) return fail(TK_EINVAL, "null output pointer");
    const int64_t tuples = checked_binom(n + m - 2, m - 1);
    if (tuples < 0 || tuples > ((int64_t)1 << 40)) return fail(TK_EOVERFLOW, "too many (m-1)-tuples");
    const int64_t bb = B < predict_max_batch() ? B : predict_max_batch();
    *h_bytes = (size_t)predict_groups(n, m, N) * (size_t)bb * (size_t)N * sizeof(double);
    return TK_OK;
}

int tk_predict_kernel(const double *d_X, int64_t n, int64_t d, int m, int kernel, double kparam,
                      const double *d_alpha, int64_t B, const double *d_Xq, int64_t N, double *d_f, void *d_work,
                      size_t work_bytes, void *stream)
{
    int rc;
    size_t need;
    if ((rc = tk_predict_kernel_workspace(n, m, B, N, &need))) return rc;
    if (d < 1 || d > INT32_MAX || n > INT32_MAX) return fail(TK_EINVAL, "n and d must be in [1, 2^31)");
    if (N > (int64_t)65535 * 64) return fail(TK_EINVAL, "N must be at most %d", 65535 * 64);
    if (kernel == TK_POLY) {
        if (!(kparam >= 1.0) || kparam != std::floor(kparam) || kparam > 64)
            return fail(TK_EINVAL, "polynomial degree must be an integer in [1, 64]");
    } else if (kernel != TK_LINEAR && kernel != TK_EXP) {
        return fail(TK_EINVAL, "unknown kernel %d", kernel);
    }
    if (!d_X || !d_alpha || !d_Xq || !d_f) return fail(TK_EINVAL, "null device pointer");
    if (work_bytes < need || !d_work) return fail(TK_ENOMEM, "workspace of %zu bytes < %zu", work_bytes, need);
    hipError_t e = launch_predict_kernel(d_X, n, d, m, kernel, kparam, d_alpha, B, d_Xq, N, d_f,
                                         reinterpret_cast<double *>(d_work), as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "prediction failed: %s", hipGetErrorString(e));
    return TK_OK;
}

int tk_contract_dense(const double *d_X, int64_t n, int64_t d, int m, const double *d_alpha, int64_t B,
                      double *d_g, double *d_work, void *stream)
{
    int rc = tk_primal_weights(d_X, n, d, m, d_alpha, B, d_work, stream);
    if (rc) return rc;
    if (!d_g) return fail(TK_EINVAL, "null device pointer");
    // g[b][i] = sum_j W[b][j] X[i][j]
    hipError_t e = launch_gemm(d_work, d, d_X, 1, d, d_g, n, B, n, d, 1, as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "gemm failed: %s", hipGetErrorString(e));
    return TK_OK;
}

int tk_support(const double *d_W, int64_t d, int64_t B, uint8_t *d_mask, double *d_tau, void *stream)
{
    if (d < 1 || B < 1) return fail(TK_EINVAL, "sizes must be >= 1");
    if (!d_W || !d_mask || !d_tau) return fail(TK_EINVAL, "null device pointer");
    hipError_t e = launch_support(d_W, d, B, d_mask, d_tau, as_stream(stream));
    if (e != hipSuccess) return fail(TK_EHIP, "support failed: %s", hipGetErrorString(e));
    return TK_OK;
}

int tk_gather_rows(const double *d_X, int64_t N, int64_t d, const int64_t *d_idx, int64_t l, double *d_out,
                   void *stream)
{
    if (N < 1 || d < 1 || l < 1 || l > 65535) return fail(TK_EINVAL, "sizes out of range");
    if (!d_X || !d_idx || !d_out) return fail(TK_EINVAL, "null device pointer");
    hipStream_t st = as_stream(stream);
    int *flag = nullptr;
    TK_HIP_CHECK(hipMallocAsync((void **)&flag, sizeof(int), st));
    TK_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), st));
    hipError_t e = launch_gather(d_X, N, d, d_idx, l, d_out, flag, st);
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFreeAsync(flag, st);
    if (e != hipSuccess) return fail(TK_EHIP, "gather failed: %s", hipGetErrorString(e));
    if (bad) return fail(TK_EINVAL, "an index is outside [0, N)");
    return TK_OK;
}

int tk_dmse_workspace(int64_t n, int m, int64_t d, int64_t nval, int dtype, size_t *h_bytes)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (!h_bytes) return fail(TK_EINVAL, "null output pointer");
    const size_t vn = align256(n * sizeof(double)), vd = align256(d * sizeof(double));
    const size_t vv = align256(nval * sizeof(double));
    *h_bytes = 6 * vn + 4 * vd + vv + align256(64 * sizeof(double)) + contract_ws(n, m, 1, dtype);
    return TK_OK;
}

int tk_dmse_dlambda(const void *d_K, int dtype, int64_t n, int m, const double *d_X, int64_t d,
                    const double *d_alpha, double lambda, const double *d_Xval, const double *d_yval, int64_t nval,
                    double cg_tol, int max_cg, double *h_mse, double *h_dmse, double *d_z, void *d_work,
                    size_t work_bytes, void *stream)
{
    int rc;
    if ((rc = check_nm(n, m))) return rc;
    if ((rc = check_dtype(dtype))) return rc;
    if (!(lambda > 0)) return fail(TK_EINVAL, "lambda must be positive");
    if (d < 1 || nval < 1) return fail(TK_EINVAL, "sizes must be >= 1");
    if (!d_K || !d_X || !d_alpha || !d_Xval || !d_yval || !h_mse || !h_dmse) return fail(TK_EINVAL, "null pointer");
    size_t need;
    if ((rc = tk_dmse_workspace(n, m, d, nval, dtype, &need))) return rc;
    if (work_bytes < need || !d_work) return fail(TK_ENOMEM, "workspace of %zu bytes < %zu", work_bytes, need);
    hipStream_t st = as_stream(stream);
    const size_t vn = align256(n * sizeof(double)), vd = align256(d * sizeof(double));
    const size_t vv = align256(nval * sizeof(double));
    unsigned char *w = reinterpret_cast<unsigned char *>(d_work);
    double *u = (double *)w;            w += vd;   // X^T alpha
    double *wv = (double *)w;           w += vd;   // w = u^{m-1}
    double *sv = (double *)w;           w += vd;   // X_val^T r
    double *tv = (double *)w;           w += vd;   // u^{m-2} * s
    double *res = (double *)w;          w += vv;   // residual on the validation set
    double *rhs = (double *)w;          w += vn;
    double *x = (double *)w;            w += vn;
    double *r = (double *)w;            w += vn;
    double *dv = (double *)w;           w += vn;
    double *hd = (double *)w;           w += vn;
    double *tmp = (double *)w;          w += vn;
    double *sc = (double *)w;           w += align256(64 * sizeof(double));
    unsigned char *cw = w;
    const size_t cw_bytes = work_bytes - (size_t)(w - reinterpret_cast<unsigned char *>(d_work));
    (void)tmp;
    hipError_t e;
#define TK_CHK(x)                                                                   \
    do {                                                                            \
        e = (x);                                                                    \
        if (e != hipSuccess) return fail(TK_EHIP, "%s: %s", #x, hipGetErrorString(e)); \
    } while (0)
    {
        // non-finite inputs end the call before any pass
        int *flag = reinterpret_cast<int *>(sc);
        int bad = 0;
        TK_CHK(hipMemsetAsync(flag, 0, sizeof(int), st));
        TK_CHK(vec_nonfinite(d_alpha, n, flag, st));
        TK_CHK(vec_nonfinite(d_X, n * d, flag, st));
        TK_CHK(vec_nonfinite(d_Xval, nval * d, flag, st));
        TK_CHK(vec_nonfinite(d_yval, nval, flag, st));
        TK_CHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        TK_CHK(hipStreamSynchronize(st));
        if (bad) return fail(TK_ENAN, "non-finite value in alpha, X, X_val or y_val");
        if (!std::isfinite(lambda)) return fail(TK_EINVAL, "lambda must be finite");
    }
    // u = X^T alpha, w = u^{m-1}
    TK_CHK(launch_gemm(d_alpha, n, d_X, d, 1, u, d, 1, d, n, 1, st));
    TK_CHK(launch_gemm(d_alpha, n, d_X, d, 1, wv, d, 1, d, n, m - 1, st));
    // res = X_val w - y_val
    TK_CHK(launch_gemm(wv, d, d_Xval, 1, d, res, nval, 1, nval, d, 1, st));
    TK_CHK(vec_sub(res, d_yval, res, nval, st));
    double hs[2];
    TK_CHK(vec_dot(res, res, 0, sc, 1, nval, st));
    TK_CHK(hipMemcpyAsync(hs, sc, sizeof(double), hipMemcpyDeviceToHost, st));
    TK_CHK(hipStreamSynchronize(st));
    *h_mse = hs[0] / (double)nval;
    // s = X_val^T res ; t = u^{m-2} s ; rhs = (2/N)(m-1) X t
    TK_CHK(launch_gemm(res, nval, d_Xval, d, 1, sv, d, 1, d, nval, 1, st));
    TK_CHK(vec_pow_mul(u, sv, m - 2, tv, d, st));
    TK_CHK(launch_gemm(tv, d, d_X, 1, d, rhs, n, 1, n, d, 1, st));
    Coefs sc2{}, zc{}, onec{}, lamc{};
    sc2.c[0] = 2.0 * (m - 1) / (double)nval;
    onec.c[0] = 1.0;
    lamc.c[0] = lambda;
    TK_CHK(vec_lin2(rhs, rhs, sc2, zc, rhs, 1, n, st));
    // CG on (J + lambda I) z = rhs
    TK_CHK(vec_lin2(rhs, rhs, zc, zc, x, 1, n, st));
    TK_CHK(vec_lin2(rhs, rhs, onec, zc, r, 1, n, st));
    TK_CHK(vec_lin2(rhs, rhs, onec, zc, dv, 1, n, st));
    TK_CHK(vec_dot(r, r, 0, sc, 1, n, st));
    double rr;
    TK_CHK(hipMemcpyAsync(&rr, sc, sizeof(double), hipMemcpyDeviceToHost, st));
    TK_CHK(hipStreamSynchronize(st));
    const double r0 = std::sqrt(rr);
    const int maxit = max_cg > 0 ? max_cg : 5000;
    const double tol = cg_tol > 0 ? cg_tol : 1e-12;
    bool curvature_lost = false;
    for (int j = 0; j < maxit && std::sqrt(rr) > tol * r0 && rr > 0; ++j) {
        // compensated directional derivatives on FP64 storage: at the dual
        // optimum the products cancel heavily and CG amplifies their error
        if ((rc = run_contract(d_K, dtype, n, m, d_alpha, dv, 1, nullptr, hd,
                               dtype == TK_F64 ? ACC_DD : ACC_PLAIN32, cw, cw_bytes, st)))
            return rc;
        TK_CHK(vec_shift_dot(dv, hd, lamc, sc, 1, n, st));
        double dhd;
        TK_CHK(hipMemcpyAsync(&dhd, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        TK_CHK(hipStreamSynchronize(st));
        if (!(dhd > 0)) {
            curvature_lost = true;
            break;
        }
        Coefs a{};
        a.c[0] = rr / dhd;
        TK_CHK(vec_cg_update(x, r, dv, hd, a, sc, 1, n, st));
        double rn;
        TK_CHK(hipMemcpyAsync(&rn, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        TK_CHK(hipStreamSynchronize(st));
        Coefs bc{};
        bc.c[0] = rn / rr;
        rr = rn;
        TK_CHK(vec_lin2(r, dv, onec, bc, dv, 1, n, st));
    }
    // dMSE/dlambda = -z . alpha
    TK_CHK(vec_dot(x, d_alpha, 0, sc, 1, n, st));
    TK_CHK(hipMemcpyAsync(hs, sc, sizeof(double), hipMemcpyDeviceToHost, st));
    TK_CHK(hipStreamSynchronize(st));
    *h_dmse = -hs[0];
    if (d_z) TK_CHK(hipMemcpyAsync(d_z, x, n * sizeof(double), hipMemcpyDeviceToDevice, st));
#undef TK_CHK
    if (!std::isfinite(*h_dmse) || !std::isfinite(*h_mse)) return fail(TK_ENAN, "non-finite dMSE/dlambda");
    // the outputs hold the last CG iterate either way; the status says whether
    // CG reached its tolerance
    if (curvature_lost || (rr > 0 && std::sqrt(rr) > tol * r0))
        return fail(TK_ENOCONV, "CG stopped at relative residual %.3e (tolerance %.3e)%s", std::sqrt(rr) / r0, tol,
                    curvature_lost ? " after losing positive curvature" : "");
    return TK_OK;
}

}  // extern "C"
