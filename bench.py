"""Benchmark of the packed tensor-kernel hot path on one MI355X.

One step = one pass of the whole hot path on the workload n=256, d=200, m=4,
lambda=1e-2 (synthetic, Section 5.4 data model, seed 1002), inputs resident in
HBM: build the packed FP64 tensor (C(259,4) = 183,181,376 entries, 1.47 GB),
contract it with one vector (g = K . alpha^3, plain FP64 accumulation: the
metric's operation), solve the dual to ||grad D|| <= 1e-11 lambda ||alpha||
(Newton on the Hessian assembled in two passes, CG on the dense system, the
step length and the line search's gradients from one directional-derivative
pass, compensated gradient passes for the last steps), recover
w = (X^T alpha)^3, take the 2-std support and predict on X.

value    = K . alpha^{m-1} contractions per second of that one-vector FP64
           contraction (whole call: every pass and the final reduction), from
           HIP events around it inside the timed steps.
ms_per_step = wall time of one step; "solve" holds the dual solve's own time.
roofline = the contraction's pass over the tensor (the metric's kernel):
           algorithmic bytes C x 8 B per launch / its average launch duration
           (HIP events on its launch stream); "kernels" lists every kernel that
           streams the tensor inside the timed steps the same way, and names
           the one with the most time ("dominant").
After the timed steps: the contraction alone per storage type and
accumulation ("contraction"), a plain streaming read of the same 1.47 GB
("stream_read", the device's achievable read rate), the 64-value lambda path
("lambda_path", also on FP32/BF16 storage alone), the time to the support
with the stable-support stop ("support_stop"), the subsample x lambda grid
of Section 6.1 ("subsample_grid"), the logistic-loss dual ("logistic"), and
the CPU oracle ("cpu_baseline": the packed FP64 contraction at 1 thread and
at all cores, plus oracle solve times).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64, vector and matrix
CSRC = os.path.join(ROOT, "paper_2003_10482_amd", "csrc")
# timing kind -> (kernel, its source file, committed counter summary)
KERNELS = {
    "contract": ("pair_kernel<4,4,double,0,0,1,8>: contraction pass, compensated FP64",
                 "tk_pass.hpp", "traffic_contract_dd_n256_m4_f64.json"),
    "hvp": ("pair_kernel<4,4,double,1,1,1,8>: directional-derivative pass, plain FP64",
            "tk_pass.hpp", "traffic_hvp_n256_m4_f64.json"),
    "contract_plain": ("pair_kernel<4,4,double,1,0,1,8>: contraction pass, plain FP64",
                       "tk_pass.hpp", "traffic_contract_plain_n256_m4_f64.json"),
    "hessian_tiles": ("hess_tri_kernel<2,double>: Hessian tile sums", "tk_hess.hip",
                      "traffic_hess_tri_n256_m4_f64.json"),
    "hessian_units": ("hess_unit_kernel<2,double>: Hessian unit vectors", "tk_hess.hip",
                      "traffic_hess_unit_n256_m4_f64.json"),
    # not a timing kind of its own (its launches time as contract_plain): the
    # batch of 64 vectors in contraction_rates and counter runs
    "contract_batch64": ("batch_mfma_kernel<2,2>: first pass on FP64 MFMA, two tiles of 16 vectors", "tk_batch.hip",
                         "traffic_batch_mfma_n256_m4_b64_f64.json"),
}


def digest_sources(src: str) -> list:
    """Files whose bytes the counter summaries of a kernel depend on: the
    kernel's source, plus the host code that sizes its grids and plans."""
    extra = {"tk_pass.hpp": ["tk_contract.hip", "tk_host.cpp"], "tk_hess.hip": ["tk_host.cpp"],
             "tk_batch.hip": ["tk_host.cpp"]}
    return [src] + extra.get(src, [])


def source_digest(src: str) -> str:
    """sha256 (first 16 hex digits) of digest_sources(src)."""
    import hashlib
    h = hashlib.sha256()
    for name in digest_sources(src):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kind: str):
    """HBM bytes per read of the tensor by kernel `kind` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or None when there are none or the
    kernel source has changed since they were taken."""
    _, src, fname = KERNELS[kind]
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != source_digest(src):
        return None
    return float(t["fetch_bytes_per_launch"]) + float(t["write_bytes_per_launch"])


def pass_only(count: int, kind: str) -> int:
    """One kernel alone, for counter runs: `count` launches of kernel `kind`
    over the FP64 tensor of the benchmark workload (same launch shape as in
    the solve), then one 1 GiB device-to-device copy whose counters give the
    scale of FETCH_SIZE and WRITE_SIZE."""
    import torch

    import paper_2003_10482_amd as tk
    from synth import make_workload

    dev = torch.device("cuda:0")
    wl = make_workload("c2_n256_m4")
    X = torch.as_tensor(wl.X, device=dev)
    K = tk.build_packed_tensor(X, wl.m, dtype="f64")
    g = torch.Generator(device="cpu").manual_seed(5)
    a = torch.randn(1, wl.n, generator=g, dtype=torch.float64).to(dev)
    v = torch.randn(1, wl.n, generator=g, dtype=torch.float64).to(dev)
    a64 = torch.randn(64, wl.n, generator=g, dtype=torch.float64).to(dev)
    for _ in range(count):
        if kind == "hvp":
            tk.hvp(K, a, v)
        elif kind == "contract":
            tk.contract(K, a, acc=tk.ACC_COMPENSATED)
        elif kind == "contract_plain":
            tk.contract(K, a, acc=tk.ACC_F64)
        elif kind == "contract_batch64":
            tk.contract(K, a64, acc=tk.ACC_F64)
        else:   # both Hessian kernels run in one call
            tk.hessian(K, a[0])
    src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pass_only": count, "kind": kind, "packed_bytes": K.count * 8, "copy_bytes": 2 ** 30}))
    return 0


def host_threads() -> int:
    """CPU threads this process may use (its affinity set; at most 16, the
    CPU share of one GPU on the benchmark hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_info() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline() -> dict:
    """The oracle as it stands, on this host: its packed FP64 contraction at
    n=256, m=4 (a seeded random symmetric tensor of C(259,4) entries; the work
    does not depend on the values) on one thread, then on every thread at once
    (independent contractions of the same tensor, one per thread: the C oracle
    releases the interpreter lock), and the oracle's dual solves of the n=64
    and n=256 workloads (closed-form damped Newton, the reference the GPU
    solves are compared with)."""
    import numpy as np

    from oracle import dual as D
    from oracle import tensor as T
    from oracle.layout import packed_count
    from synth import make_workload, random_alpha, random_symmetric_packed_values

    n, m = 256, 4
    K = random_symmetric_packed_values(packed_count(n, m), seed=77)
    a = random_alpha(n, seed=78)
    t0 = time.perf_counter()
    passes1 = 2
    for _ in range(passes1):
        T.contract_packed(K, n, m, a)
    dt1 = time.perf_counter() - t0
    threads = host_threads()
    per_thread = 1
    errs = []

    def work():
        try:
            for _ in range(per_thread):
                T.contract_packed(K, n, m, a)
        except Exception as e:   # pragma: no cover - reported below
            errs.append(repr(e))

    ths = [threading.Thread(target=work) for _ in range(threads)]
    t0 = time.perf_counter()
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    dtn = time.perf_counter() - t0
    rate1 = passes1 / dt1
    raten = threads * per_thread / dtn if not errs else None
    solves = {}
    for name in ("c1_n64_m4", "c2_n256_m4"):
        wl = make_workload(name)
        t0 = time.perf_counter()
        _, info = D.solve_linear(wl.X, wl.y, wl.lam, wl.m)
        solves[name] = {"seconds": time.perf_counter() - t0, "newton_iters": info.iterations,
                        "method": "damped Newton, closed-form contraction and Hessian, Cholesky (numpy/LAPACK)"}
    nbytes = packed_count(n, m) * 8
    return {"value": raten if raten is not None else rate1, "unit": "contractions/s",
            "cores": threads if raten is not None else 1, "kind": "oracle",
            "sample": (f"packed FP64 contraction at n=256, m=4 ({packed_count(n, m)} entries) on a seeded random "
                       f"symmetric tensor: {threads} concurrent single-threaded C oracle calls, {dtn:.1f} s; "
                       f"one thread: {passes1} calls, {dt1:.1f} s"),
            "single_thread": {"value": rate1, "GBs": rate1 * nbytes / 1e9, "seconds": dt1},
            "all_threads": {"value": raten, "threads": threads, "GBs": (raten or 0) * nbytes / 1e9,
                            "seconds": dtn, "errors": errs},
            "host": {"nproc": os.cpu_count(), "affinity": host_threads(), "cpu": cpu_info()},
            "oracle_solves": solves}


def lambda_path(tk, torch, dev) -> dict:
    """Solve time of the 64-value lambda path of the same data (1e-4 .. 1), FP64
    tensor, from the largest lambda down; support recovery per lambda against
    the planted support.  Runs after the timed steps."""
    import numpy as np

    from synth import make_workload

    wl = make_workload("c4_lampath")
    X = torch.as_tensor(wl.X, device=dev)
    y = torch.as_tensor(wl.y, device=dev)
    K = tk.build_packed_tensor(X, wl.m, dtype="f64")
    out = {"lambdas": len(wl.lambdas), "range": [float(wl.lambdas.min()), float(wl.lambdas.max())]}
    true = set(wl.support.tolist())

    def f1_of(alpha):
        W = tk.primal_weights(X, alpha, wl.m)
        mask, _ = tk.support(W)
        m = mask.cpu().numpy().astype(bool)
        f1 = []
        for b in range(m.shape[0]):
            sel = set(np.flatnonzero(m[b]).tolist())
            tp = len(sel & true)
            f1.append(0.0 if tp == 0 else 2 * tp / (len(sel) + len(true)))
        return f1

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    for tol in (1e-10, 1e-4):
        tk.solve_dual(K, y, wl.lambdas[-2:], tol=tol)   # warm the plan caches
        (alpha, infos), dt = timed(lambda: tk.solve_dual(K, y, wl.lambdas, tol=tol))
        f1 = f1_of(alpha)
        rec = {"seconds": dt, "passes": sum(i["passes"] + i["hess_passes"] for i in infos),
               "newton_iters": sum(i["newton_iters"] for i in infos),
               "all_converged": all(i["status"] == 0 for i in infos),
               "support_f1_min": min(f1), "support_f1_mean": float(np.mean(f1))}
        if tol == 1e-4:
            # the same lambdas in lock step (every pass one launch for all 64
            # vectors, the plain passes on the FP64-MFMA batch kernel; one
            # Hessian per lambda and Newton step)
            tk.solve_dual(K, y, wl.lambdas[-2:], tol=tol, continuation=False)
            (al, il), dl = timed(lambda: tk.solve_dual(K, y, wl.lambdas, tol=tol, continuation=False))
            fl = f1_of(al)
            rec["lock_step"] = {"seconds": dl, "newton_iters_max": max(i["newton_iters"] for i in il),
                                "all_converged": all(i["status"] == 0 for i in il),
                                "support_f1_min": min(fl), "speed_vs_continuation": dt / dl}
        # the same 64 lambdas as independent cold FP64 solves: the speedup of
        # the batched form at equal support accuracy
        A, di = timed(lambda: torch.cat([tk.solve_dual(K, y, [lam], tol=tol)[0] for lam in wl.lambdas]))
        fi = f1_of(A)
        rec["independent_fp64"] = {"seconds": di, "support_f1_min": min(fi), "speedup_of_path": di / dt}
        out[f"tol_{tol:g}"] = rec
    # reduced-precision storage alone (FP32 accumulation, no FP64 tensor):
    # each lambda ends at the tolerance or at its storage-rounding floor
    for dtype in ("f32", "bf16"):
        Kr = tk.build_packed_tensor(X, wl.m, dtype=dtype)
        tk.solve_dual(Kr, y, wl.lambdas[-2:], tol=1e-4)
        (alpha, infos), dr = timed(lambda: tk.solve_dual(Kr, y, wl.lambdas, tol=1e-4))
        fr = f1_of(alpha)
        out["tol_0.0001"][f"{dtype}_storage_alone"] = {
            "seconds": dr, "status_ok": sum(i["status"] == 0 for i in infos),
            "floor_stops": sum(i["stop_reason"] == 2 for i in infos if i["status"] == 0),
            "support_f1_min": min(fr), "support_f1_mean": float(np.mean(fr)),
            "lambdas_with_f1_below_1": int(sum(f < 1 for f in fr)),
            "speedup_vs_fp64_path": out["tol_0.0001"]["seconds"] / dr}
        del Kr
    # reduced-precision storage along the path, finished on the FP64 tensor
    for dtype in ("f32", "bf16"):
        Kr = tk.build_packed_tensor(X, wl.m, dtype=dtype)
        (alpha, infos), dr = timed(lambda: tk.solve_dual(Kr, y, wl.lambdas, tol=1e-4, polish=K))
        fr = f1_of(alpha)
        out["tol_0.0001"][f"{dtype}_storage_fp64_polish"] = {
            "seconds": dr, "all_converged": all(i["status"] == 0 for i in infos), "support_f1_min": min(fr),
            "speedup_vs_fp64_path": out["tol_0.0001"]["seconds"] / dr}
        del Kr
    del K
    return out


def support_stop_timing(tk, torch, dev) -> dict:
    """Time to the support (Section 6.3 threshold) with the stable-support
    stop (3 Newton steps without a change) against the full solves, on the
    benchmark workload and along the 64-lambda path; F1 against the planted
    support."""
    import numpy as np

    from synth import make_workload

    out = {}
    for name in ("c2_n256_m4", "c4_lampath"):
        wl = make_workload(name)
        X = torch.as_tensor(wl.X, device=dev)
        y = torch.as_tensor(wl.y, device=dev)
        K = tk.build_packed_tensor(X, wl.m)
        lams = [wl.lam] if wl.lambdas is None else list(wl.lambdas)
        tk.solve_dual(K, y, lams[:1], tol=1e-4)
        rec = {"lambdas": len(lams)}
        for label, kw in (("tol_1e-10", {"tol": 1e-10}), ("tol_1e-4", {"tol": 1e-4}),
                          ("support_stop_3", {"tol": 1e-10, "support_stop": 3, "support_X": X})):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            alpha, infos = tk.solve_dual(K, y, lams, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            W = tk.primal_weights(X, alpha, wl.m)
            mask, _ = tk.support(W)
            m = mask.cpu().numpy().astype(bool)
            true = set(wl.support.tolist())
            f1 = []
            for b in range(m.shape[0]):
                sel = set(np.flatnonzero(m[b]).tolist())
                tp = len(sel & true)
                f1.append(0.0 if tp == 0 else 2 * tp / (len(sel) + len(true)))
            rec[label] = {"seconds": dt, "newton_iters": sum(i["newton_iters"] for i in infos),
                          "support_f1_min": min(f1), "masks": m}
        for label in ("tol_1e-4", "support_stop_3"):
            rec[label]["same_supports_as_tol_1e-10"] = bool(np.array_equal(rec[label]["masks"],
                                                                           rec["tol_1e-10"]["masks"]))
            rec[label]["speedup_vs_tol_1e-10"] = rec["tol_1e-10"]["seconds"] / rec[label]["seconds"]
        for label in ("tol_1e-10", "tol_1e-4", "support_stop_3"):
            del rec[label]["masks"]
        out[name] = rec
        del K
    return out


def subsample_grid(tk, torch, dev) -> dict:
    """Section 6.1 grid on the Nystrom workload (20000 points, d = 1000): 10
    uniform draws of 200 landmarks (C(203,4) entries each, 0.55 GB FP64), 8
    lambdas in [1e-3, 1]; draws solved in lock step (one launch per pass for
    all ten tensors), lambdas by continuation; test MSE of every (draw,
    lambda) model on the other points, F1 of its support."""
    import numpy as np

    from synth import landmark_draws, make_workload

    wl = make_workload("c3_nystrom")
    draws = landmark_draws(wl.X.shape[0], 200, 10, seed=2003)
    lams = list(10.0 ** np.linspace(0, -3, 8))
    Xs = torch.as_tensor(np.stack([wl.X[i] for i in draws]), device=dev)
    Ys = torch.as_tensor(np.stack([wl.y[i] for i in draws]), device=dev)
    Xtest = torch.as_tensor(wl.X[:2000], device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Km = tk.build_packed_multi(Xs, 4)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    alpha, infos = tk.solve_dual_multi(Km, Ys, lams, tol=1e-8)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    mse = np.zeros((len(lams), len(draws)))
    f1 = np.zeros_like(mse)
    true = set(wl.support.tolist())
    ytest = wl.y[:2000]
    for l in range(len(lams)):
        for t in range(len(draws)):
            W = tk.primal_weights(Xs[t], alpha[l, t], 4)
            f = tk.predict(W, Xtest).cpu().numpy()
            mse[l, t] = float(np.mean((f - ytest) ** 2))
            mask, _ = tk.support(W)
            sel = set(np.flatnonzero(mask.cpu().numpy()).tolist())
            tp = len(sel & true)
            f1[l, t] = 0.0 if tp == 0 else 2 * tp / (len(sel) + len(true))
    conv = sum(infos[l][t]["status"] == 0 for l in range(len(lams)) for t in range(len(draws)))
    passes = sum(infos[l][0]["passes"] + infos[l][0]["hess_passes"] for l in range(len(lams)))
    del Km
    return {"draws": len(draws), "landmarks": 200, "lambdas": lams, "tensor_bytes_each": tk.packed_count(200, 4) * 8,
            "build_seconds": t_build, "solve_seconds": t_solve, "converged": int(conv),
            "problems": len(lams) * len(draws), "launch_passes": int(passes),
            "test_mse_mean_by_lambda": mse.mean(axis=1).tolist(), "support_f1_mean_by_lambda": f1.mean(axis=1).tolist()}


def logistic_timing(tk, torch, dev) -> dict:
    """The logistic-loss dual (Fenchel conjugate of the loss) on the
    benchmark's shape: n = 256, d = 200, m = 4, labels sign(X w*) with 5 %
    flipped, lambda = 1e-2 from the centre of the domain."""
    import numpy as np

    from synth import planted_classification

    rng = np.random.default_rng(1077)
    Xh, yh, w, sup = planted_classification(rng, 256, 200, 10, flip=0.05)
    X = torch.as_tensor(Xh, device=dev)
    y = torch.as_tensor(yh, device=dev)
    K = tk.build_packed_tensor(X, 4)
    tk.solve_dual(K, y, [1e-1], tol=1e-6, loss="logistic")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alpha, infos = tk.solve_dual(K, y, [1e-2], tol=1e-10, loss="logistic")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mask, _ = tk.support(tk.primal_weights(X, alpha, 4))
    sel = set(np.flatnonzero(mask.cpu().numpy()[0]).tolist())
    tp = len(sel & set(sup.tolist()))
    del K
    return {"seconds": dt, "status": infos[0]["status"], "newton_iters": infos[0]["newton_iters"],
            "passes": infos[0]["passes"] + infos[0]["hess_passes"],
            "support_f1": 0.0 if tp == 0 else 2 * tp / (len(sel) + len(sup))}


def time_calls(torch, fn, reps: int) -> float:
    """Average milliseconds of fn() over reps calls, from events on the current
    stream (every call enqueues its kernels on it)."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def contraction_rates(tk, torch, dev, X, wl, K64) -> dict:
    """The contraction K . alpha^{m-1} alone on the benchmark points, outside
    the timed steps: one vector for every storage type and accumulation (the
    pass over the tensor from the library's own HIP events, and the whole call
    from events around it), the directional derivative, and a batch of 64
    vectors with the vector tile the autotuner picks.  GB/s counts the tensor
    bytes per read."""
    n = wl.n
    g = torch.Generator(device="cpu").manual_seed(11)
    a1 = (0.1 * torch.randn(1, n, generator=g, dtype=torch.float64)).to(dev)
    v1 = (0.1 * torch.randn(1, n, generator=g, dtype=torch.float64)).to(dev)
    a64 = (0.1 * torch.randn(64, n, generator=g, dtype=torch.float64)).to(dev)
    out = {}
    tensors = {"f64": K64}
    for dt in ("f32", "bf16"):
        tensors[dt] = tk.build_packed_tensor(X, wl.m, dtype=dt)
    cases = (("one_vector_plain_fp64", "f64", tk.ACC_F64, "contract_plain", 1, None),
             ("one_vector_compensated_fp64", "f64", tk.ACC_COMPENSATED, "contract", 1, None),
             ("one_vector_fp32_storage", "f32", tk.ACC_F32, "contract_plain", 1, None),
             ("one_vector_bf16_storage", "bf16", tk.ACC_F32, "contract_plain", 1, None),
             ("directional_derivative_plain_fp64", "f64", tk.ACC_F64, "hvp", 1, v1),
             ("directional_derivative_fp32_storage", "f32", tk.ACC_F32, "hvp", 1, v1),
             ("directional_derivative_bf16_storage", "bf16", tk.ACC_F32, "hvp", 1, v1),
             ("batch_64_plain_fp64", "f64", tk.ACC_F64, "contract_plain", 64, None))
    for name, dt, acc, kind, vectors, vdir in cases:
        K = tensors[dt]
        alpha = a1 if vectors == 1 else a64
        if vectors > 1:
            tile, _, _ = tk.autotune(K, alpha, acc=acc)
        if vdir is None:
            call = lambda: tk.contract(K, alpha, acc=acc)   # noqa: E731
        else:
            call = lambda: tk.hvp(K, alpha, vdir, acc=acc)   # noqa: E731
        reps = 20 if vectors == 1 else 4
        call_ms = time_calls(torch, call, reps)
        torch.cuda.synchronize()
        tk.timing_start()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        launches, ms, nbytes = tk.timing_stop()[kind]
        avg = ms / launches
        gbs = (nbytes / launches) / (avg * 1e-3) / 1e9
        rec = {"pass_ms": avg, "call_ms": call_ms, "contractions_per_s": vectors / (call_ms * 1e-3),
               "pass_GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
               "tensor_bytes": K.nbytes}
        if vectors > 1:
            rec["vector_tile"] = tile
            rec["effective_GBs"] = vectors * K.nbytes / (avg * 1e-3) / 1e9
            if tile == 16:   # the FP64-MFMA batch pass: 2 FMAs per entry and vector (row and column sums)
                flops = 4.0 * K.count * vectors
                rec["kernel"] = KERNELS["contract_batch64"][0]
                rec["TFLOPs"] = flops / (avg * 1e-3) / 1e12
                rec["frac_of_fp64_peak"] = rec["TFLOPs"] / FP64_PEAK_TFLOPS
                t = measured_traffic("contract_batch64") if vectors == 64 else None
                rec["traffic"] = t
                rec["traffic_per_tensor_read"] = None if t is None else t / K.nbytes
        out[name] = rec
    return out


def stream_read(tk, torch, buf) -> dict:
    """Achievable read rate: a plain streaming-read kernel over the same
    buffer, several grid sizes, best average of 20 launches each."""
    best = None
    res = {}
    for groups in (1024, 2048, 4096, 8192, 16384):
        sink = torch.empty(groups, dtype=torch.int64, device=buf.device)
        ms = time_calls(torch, lambda: tk.probe_stream_read(buf, groups, sink), 20)
        gbs = (buf.numel() * buf.element_size() // 16 * 16) / (ms * 1e-3) / 1e9
        res[str(groups)] = gbs
        best = gbs if best is None or gbs > best else best
    return {"GBs": best, "frac_of_peak": best / HBM_PEAK_GBS, "by_groups": res,
            "bytes": buf.numel() * buf.element_size()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-path", action="store_true", help="skip the 64-lambda path (outside the timed steps)")
    ap.add_argument("--no-contraction", action="store_true",
                    help="skip the standalone contraction timings (outside the timed steps)")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the stable-support, subsample-grid and logistic timings (outside the timed steps)")
    ap.add_argument("--pass-only", type=int, default=0,
                    help="run only this many launches of one kernel (for counter runs)")
    ap.add_argument("--pass-kind", default="hvp", choices=sorted(KERNELS))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library runs on one GPU (no multi-GPU path is built)",
              file=sys.stderr)
        return 2

    if args.pass_only:
        return pass_only(args.pass_only, args.pass_kind)

    import numpy as np
    import torch

    import paper_2003_10482_amd as tk
    from synth import make_workload

    dev = torch.device("cuda:0")
    wl = make_workload("c2_n256_m4")
    X = torch.as_tensor(wl.X, device=dev)
    y = torch.as_tensor(wl.y, device=dev)
    count = tk.packed_count(wl.n, wl.m)
    g = torch.Generator(device="cpu").manual_seed(3)
    a_c = (0.1 * torch.randn(1, wl.n, generator=g, dtype=torch.float64)).to(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    contract_ms, solve_ms = [], []

    def step():
        K = tk.build_packed_tensor(X, wl.m, dtype="f64")
        ev[0].record()
        gout = tk.contract(K, a_c, acc=tk.ACC_F64)
        ev[1].record()
        ev[2].record()
        alpha, infos = tk.solve_dual(K, y, [wl.lam], tol=1e-11)
        ev[3].record()
        W = tk.primal_weights(X, alpha, wl.m)
        mask, tau = tk.support(W)
        f = tk.predict(W, X)
        ev[3].synchronize()
        contract_ms.append(ev[0].elapsed_time(ev[1]))
        solve_ms.append(ev[2].elapsed_time(ev[3]))
        del K
        return gout, alpha, infos, W, mask, f

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    contract_ms.clear()
    solve_ms.clear()
    tk.timing_start()
    passes = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gout, alpha, infos, W, mask, f = step()
        passes += infos[0]["passes"] + infos[0]["hess_passes"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = tk.timing_stop()
    ms_step = 1e3 * elapsed / args.steps

    ran = {k: v for k, v in timing.items() if v[0]}
    dominant = max(ran, key=lambda k: ran[k][1])   # the kernel with the most time in the timed steps
    kind = "contract_plain"                         # the metric's pass over the tensor
    launches, kms, kbytes = ran[kind]
    avg_ms = kms / launches
    achieved = (kbytes / launches) / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(kind)
    mask_np = mask.cpu().numpy()[0].astype(bool)
    sel = set(np.flatnonzero(mask_np).tolist())
    true = set(wl.support.tolist())
    tp = len(sel & true)
    f1 = 0.0 if tp == 0 else 2 * tp / (len(sel) + len(true))
    c_ms = float(np.mean(contract_ms))

    out = {
        "metric": "K·α^{m-1} contractions/s + HBM GB/s (m=4,n=256); solve time at fixed support accuracy",
        "value": 1e3 / c_ms,
        "unit": "contractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "n=256 d=200 m=4 lambda=1e-2 FP64: build, one-vector contraction, dual solve, "
                               "support, prediction",
                   "n": wl.n, "d": wl.d, "m": wl.m, "lambda": wl.lam, "packed_entries": count,
                   "packed_bytes": count * 8},
        "contraction_in_step": {"ms_per_call": c_ms, "contractions_per_s": 1e3 / c_ms,
                                "tensor_GBs_per_call": count * 8 / (c_ms * 1e-3) / 1e9},
        "solve": {"ms": float(np.mean(solve_ms)), "passes_per_step": passes / args.steps,
                  "newton_iters": infos[0]["newton_iters"], "cg_iters": infos[0]["cg_iters"],
                  "hessian_passes": infos[0]["hess_passes"], "grad_norm": infos[0]["grad_norm"],
                  "status": infos[0]["status"], "support_f1": f1, "support_size": len(sel)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # counters are per read of the tensor; a launch reads it
                     # kbytes / launches / (C * 8) times
                     "traffic": (traffic * (kbytes / launches) / (count * 8.0) if traffic is not None else None),
                     "kernel": KERNELS[kind][0], "avg_launch_ms": avg_ms, "launches": launches,
                     "dominant": dominant,
                     "kernels": {k: {"kernel": KERNELS[k][0], "launches": l, "total_ms": ms, "avg_launch_ms": ms / l,
                                     "achieved_GBs": (b / l) / (ms / l * 1e-3) / 1e9,
                                     "frac": (b / l) / (ms / l * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "traffic": (measured_traffic(k) * (b / l) / (count * 8.0)
                                                 if measured_traffic(k) is not None else None)}
                                 for k, (l, ms, b) in ran.items()}},
    }
    if not args.no_contraction:
        K = tk.build_packed_tensor(X, wl.m, dtype="f64")
        out["stream_read"] = stream_read(tk, torch, K.data)
        out["contraction"] = contraction_rates(tk, torch, dev, X, wl, K)
        sr = out["stream_read"]["GBs"]
        for rec in out["contraction"].values():
            rec["frac_of_stream_read"] = rec["pass_GBs"] / sr
        del K
    if not args.no_path:
        out["lambda_path"] = lambda_path(tk, torch, dev)
    if not args.no_extensions:
        out["support_stop"] = support_stop_timing(tk, torch, dev)
        out["subsample_grid"] = subsample_grid(tk, torch, dev)
        out["logistic"] = logistic_timing(tk, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
