"""Benchmark of the packed tensor-kernel hot path on one MI355X.

One step = one pass of the whole hot path on the workload n=256, d=200, m=4,
lambda=1e-2 (synthetic, Section 5.4 data model, seed 1002), inputs resident in
HBM: build the packed FP64 tensor (C(259,4) = 183,181,376 entries, 1.47 GB),
solve the dual to ||grad D|| <= 1e-11 lambda ||alpha|| with the Newton solver
(the Hessian assembled in two passes at every Newton step, CG on the dense
system, the step length and the line search's gradients from one
directional-derivative pass, compensated gradient passes for the last
steps), recover w = (X^T alpha)^3, take the 2-std support and predict on X.
After the timed steps, the contraction alone is timed ("contraction": one
vector, plain and compensated, and a batch of 64 with the autotuned tile),
and the 64-value lambda path of the same data is solved
and timed separately ("lambda_path"): by continuation, as 64 independent
cold solves (the batched form's speedup at equal support accuracy), and
with FP32/BF16 storage finished on the FP64 tensor.

value = passes over the packed tensor per second across the timed steps
        (contractions, and the two streaming passes of each Hessian).
roofline = the kernel with the most time in the timed steps, timed with HIP
        events on its launch stream: algorithmic bytes = C x 8 B per read of
        the tensor; "kernels" lists every streaming kernel the same way.
cpu_baseline = the CPU oracle's packed FP64 contraction (single thread) on a
        seeded random symmetric tensor of the same size.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2003_10482_amd", "csrc")
# timing kind -> (kernel, its source file, committed counter summary)
KERNELS = {
    "contract": ("pair_kernel<4,4,double,0,0,1,8>: contraction pass, compensated FP64",
                 "tk_pass.hpp", "traffic_contract_dd_n256_m4_f64.json"),
    "hvp": ("pair_kernel<4,4,double,1,1,1,8>: directional-derivative pass, plain FP64",
            "tk_pass.hpp", "traffic_hvp_n256_m4_f64.json"),
    "contract_plain": ("pair_kernel<4,4,double,1,0,*,8>: contraction pass, plain FP64",
                       "tk_pass.hpp", "traffic_contract_plain_n256_m4_f64.json"),
    "hessian_tiles": ("hess_tri_kernel<2,double>: Hessian tile sums", "tk_hess.hip",
                      "traffic_hess_tri_n256_m4_f64.json"),
    "hessian_units": ("hess_unit_kernel<2,double>: Hessian unit vectors", "tk_hess.hip",
                      "traffic_hess_unit_n256_m4_f64.json"),
}


def source_digest(src: str) -> str:
    """sha256 (first 16 hex digits) of the kernel's source and, for the
    contraction passes, of the host code that sizes their grids."""
    import hashlib
    h = hashlib.sha256()
    for name in (src, "tk_contract.hip") if src == "tk_pass.hpp" else (src,):
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
    for _ in range(count):
        if kind == "hvp":
            tk.hvp(K, a, v)
        elif kind == "contract":
            tk.contract(K, a, acc=tk.ACC_COMPENSATED)
        elif kind == "contract_plain":
            tk.contract(K, a, acc=tk.ACC_F64)
        else:   # both Hessian kernels run in one call
            tk.hessian(K, a[0])
    src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pass_only": count, "kind": kind, "packed_bytes": K.count * 8, "copy_bytes": 2 ** 30}))
    return 0


def cpu_baseline(passes: int = 2) -> dict:
    import numpy as np

    from oracle import tensor as T
    from oracle.layout import packed_count
    from synth import random_alpha, random_symmetric_packed_values

    n, m = 256, 4
    K = random_symmetric_packed_values(packed_count(n, m), seed=77)
    a = random_alpha(n, seed=78)
    t0 = time.perf_counter()
    for _ in range(passes):
        T.contract_packed(K, n, m, a)
    dt = time.perf_counter() - t0
    return {"value": passes / dt, "unit": "contractions/s", "cores": 1, "kind": "oracle",
            "sample": f"{passes} passes of the packed FP64 contraction at n=256, m=4 "
                      f"(C(259,4) entries) on a seeded random symmetric tensor, "
                      f"single-threaded C oracle, {dt:.1f} s"}


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
        # the same 64 lambdas as independent cold FP64 solves: the speedup of
        # the batched form at equal support accuracy
        A, di = timed(lambda: torch.cat([tk.solve_dual(K, y, [lam], tol=tol)[0] for lam in wl.lambdas]))
        fi = f1_of(A)
        rec["independent_fp64"] = {"seconds": di, "support_f1_min": min(fi), "speedup_of_path": di / dt}
        out[f"tol_{tol:g}"] = rec
    # reduced-precision storage along the path, finished on the FP64 tensor
    # (without the FP64 finish these solves do not converge at small lambda)
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


def contraction_rates(tk, torch, dev, K, n: int) -> dict:
    """The contraction K . alpha^{m-1} alone on the benchmark tensor, outside
    the timed steps: one vector with plain and with compensated FP64
    accumulation, and a batch of 64 vectors (the lambda-path shape) with the
    vector tile the autotuner picks.  HIP events per launch; GB/s counts the
    tensor bytes per read (a tile of t vectors shares one read)."""
    g = torch.Generator(device="cpu").manual_seed(11)
    a1 = (0.1 * torch.randn(1, n, generator=g, dtype=torch.float64)).to(dev)
    a64 = (0.1 * torch.randn(64, n, generator=g, dtype=torch.float64)).to(dev)
    tile, _, _ = tk.autotune(K, a64, acc=tk.ACC_F64)
    out = {}
    for name, alpha, acc, kind, vectors in (("one_vector_plain_fp64", a1, tk.ACC_F64, "contract_plain", 1),
                                             ("one_vector_compensated_fp64", a1, tk.ACC_COMPENSATED, "contract", 1),
                                             ("batch_64_plain_fp64", a64, tk.ACC_F64, "contract_plain", 64)):
        for _ in range(3):
            tk.contract(K, alpha, acc=acc)
        torch.cuda.synchronize()
        tk.timing_start()
        reps = 20 if vectors == 1 else 4
        for _ in range(reps):
            tk.contract(K, alpha, acc=acc)
        torch.cuda.synchronize()
        launches, ms, nbytes = tk.timing_stop()[kind]
        avg = ms / launches
        rec = {"ms_per_launch": avg, "contractions_per_s": vectors / (avg * 1e-3),
               "hbm_GBs": (nbytes / launches) / (avg * 1e-3) / 1e9,
               "frac_of_peak": (nbytes / launches) / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if vectors > 1:
            rec["vector_tile"] = tile
            rec["effective_GBs"] = vectors * K.count * 8 / (avg * 1e-3) / 1e9
        out[name] = rec
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-path", action="store_true", help="skip the 64-lambda path (outside the timed steps)")
    ap.add_argument("--no-contraction", action="store_true",
                    help="skip the standalone contraction timings (outside the timed steps)")
    ap.add_argument("--pass-only", type=int, default=0,
                    help="run only this many launches of one kernel (for counter runs)")
    ap.add_argument("--pass-kind", default="hvp", choices=sorted(KERNELS))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path", file=sys.stderr)
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

    def step():
        K = tk.build_packed_tensor(X, wl.m, dtype="f64")
        alpha, infos = tk.solve_dual(K, y, [wl.lam], tol=1e-11)
        W = tk.primal_weights(X, alpha, wl.m)
        mask, tau = tk.support(W)
        f = tk.predict(W, X)
        del K
        return alpha, infos, W, mask, f

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tk.timing_start()
    passes = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        alpha, infos, W, mask, f = step()
        passes += infos[0]["passes"] + infos[0]["hess_passes"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = tk.timing_stop()
    ms_step = 1e3 * elapsed / args.steps

    ran = {k: v for k, v in timing.items() if v[0]}
    kind = max(ran, key=lambda k: ran[k][1])   # the kernel with the most time in the timed steps
    launches, kms, kbytes = ran[kind]
    avg_ms = kms / launches
    achieved = (kbytes / launches) / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(kind)
    mask_np = mask.cpu().numpy()[0].astype(bool)
    sel = set(np.flatnonzero(mask_np).tolist())
    true = set(wl.support.tolist())
    tp = len(sel & true)
    f1 = 0.0 if tp == 0 else 2 * tp / (len(sel) + len(true))

    out = {
        "metric": "K·α^{m-1} contractions/s + HBM GB/s (m=4,n=256); solve time at fixed support accuracy",
        "value": passes / elapsed,
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
        "config": {"workload": "n=256 d=200 m=4 lambda=1e-2 FP64 build + dual solve + support",
                   "n": wl.n, "d": wl.d, "m": wl.m, "lambda": wl.lam, "packed_entries": count,
                   "packed_bytes": count * 8},
        "solve": {"passes_per_step": passes / args.steps, "newton_iters": infos[0]["newton_iters"],
                  "cg_iters": infos[0]["cg_iters"], "hessian_passes": infos[0]["hess_passes"],
                  "grad_norm": infos[0]["grad_norm"],
                  "status": infos[0]["status"], "support_f1": f1, "support_size": len(sel)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # counters are per read of the tensor; a launch reads it
                     # kbytes / launches / (C * 8) times
                     "traffic": (traffic * (kbytes / launches) / (count * 8.0) if traffic is not None else None),
                     "kernel": KERNELS[kind][0], "avg_launch_ms": avg_ms, "launches": launches,
                     "kernels": {k: {"launches": l, "total_ms": ms, "avg_launch_ms": ms / l,
                                     "achieved_GBs": (b / l) / (ms / l * 1e-3) / 1e9}
                                 for k, (l, ms, b) in ran.items()}},
    }
    if not args.no_contraction:
        K = tk.build_packed_tensor(X, wl.m, dtype="f64")
        out["contraction"] = contraction_rates(tk, torch, dev, K, wl.n)
        del K
    if not args.no_path:
        out["lambda_path"] = lambda_path(tk, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
