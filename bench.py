"""Benchmark of the CCMF ADMM solver on one MI355X.

A step is one full solve (all loads of the workload, batched in one launch
sequence, every problem to its tolerance) with the crack-resistance field
already resident in HBM.  The metric is voxel-iterations per second:
N * (sum over problems of ADMM iterations) / wall time of the timed steps.

Default workload: 256^3 FP32 aligned fibres along e3 (r = 5, 20 %, kappa 10/1),
loads e1, e2, e3, tol 1e-5.  The FP32 results are checked (untimed) against
FP64 references: the fibres are extruded along e3, so the e1 and e2 problems
equal the FP64 solve of a single e1-e2 slice, and e3 gives the mean kappa.

Prints one JSON line.  Extra objects:
  roofline     -- the fused update kernel (the dominant kernel): algorithmic
                  bytes per launch / average launch duration from HIP events on
                  the solver's stream, against the 8 TB/s HBM peak;
  cpu_baseline -- the FP64 NumPy reference implementation timed on this host on
                  a bounded sample (a few ADMM iterations of the same workload).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# Fabric traffic of the fused update kernel per launch and active problem on the 256^3 FP32
# workload: rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by what they read for the 2 GiB copy
# kernel, see profiles/k_update_ud_fibres256_f32_traffic.md.  None once the kernel changes.
K_UPDATE_TRAFFIC_C2 = 1.233e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import numpy as np
    from paper_2103_05968_amd import microstructures as M
    cfg = dict(M.CONFIGS[name])
    if name == "c1":
        kap = M.config_c1()[None]
        dtype = "f64"
    elif name == "c2":
        kap = M.config_c2()[None]
        dtype = "f32"
    elif name == "c3":
        kap = np.stack([M.config_c3(r) for r in range(int(os.environ.get("CCMF_C3_FIELDS", "64")))])
        dtype = "f32"
    elif name == "c4":
        kap = M.config_c4()[None]
        dtype = "f32"
    elif name == "c5":
        kap = M.config_c5()[None]
        dtype = "f32"
    else:
        raise SystemExit(f"unknown workload {name}")
    return cfg, kap, dtype


def stream_ceiling(torch, nbytes=1 << 31, reps=10):
    """Device copy bandwidth (read + write bytes / time) with the library's copy kernel."""
    from paper_2103_05968_amd.ccmf import stream_copy
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    stream_copy(dst, src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        stream_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(kap, loads, budget_s=20.0):
    """FP64 oracle on this host: ADMM iterations of the first problem of the
    workload, as many as fit the time budget (at least 2 after 1 warm-up)."""
    import numpy as np
    from oracle import ccmf_oracle as O
    gamma = np.asarray(kap[0], dtype=np.float64)
    xb = np.asarray(loads[0], dtype=np.float64)
    xb = xb / np.linalg.norm(xb)
    e = O.A_xibar(xb, gamma.shape)
    v = gamma[None] * e
    rho = O.rho_initial(gamma)
    O.admm_step(e, v, rho, xb, gamma, 0.25)          # warm-up
    t0 = time.perf_counter()
    n = 0
    while True:
        _, _, e, v = O.admm_step(e, v, rho, xb, gamma, 0.25)
        n += 1
        el = time.perf_counter() - t0
        if n >= 2 and el >= budget_s:
            break
        if el + el / n > 3 * budget_s:
            break
    rate = gamma.size * n / el
    return dict(value=rate, unit="voxel-iters/s", cores=1, kind="oracle",
                sample=f"{n} ADMM iterations of problem 0 ({'x'.join(map(str, gamma.shape))}, "
                       f"load {tuple(float(x) for x in loads[0])}) in FP64 NumPy after 1 warm-up; "
                       f"NumPy FFT and element-wise kernels are single-threaded",
                seconds=el)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--max-iter", type=int, default=60000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; "
              "multi-GPU runs (--gpus > 1) are not supported.", file=sys.stderr)
        raise SystemExit(2)

    import numpy as np
    import torch
    from paper_2103_05968_amd.ccmf import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg, kap_np, dtype = workload(args.workload)
    loads = cfg["loads"]
    tol = cfg["tol"]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    N = int(np.prod(kap_np.shape[1:]))
    F = kap_np.shape[0]
    log(f"workload {cfg['name']} fields={F} dims={kap_np.shape[1:]} loads={len(loads)} tol={tol} dtype={dtype}")

    kap = torch.as_tensor(kap_np, dtype=tdt, device="cuda:0")
    plan = Plan(kap)

    # FP64 reference (untimed) for the accuracy check of the FP32 path
    ref = None
    if not args.no_reference:
        t = time.perf_counter()
        if args.workload == "c2":
            # the fibres are extruded along e3, so the e1 and e2 problems equal the
            # FP64 solve of one e1-e2 slice (N3 = 1) and e3 gives the mean exactly
            sl = Plan(torch.as_tensor(np.ascontiguousarray(kap_np[:, :, :, :1]), dtype=torch.float64,
                                      device="cuda:0"))
            r2 = sl.solve(loads[:2], tol=1e-6, max_iter=400000)
            sl.close()
            ref_geff = np.array([[r2.geff[0, 0], r2.geff[0, 1], kap_np[0].mean()]])
            ref_iters = [int(r2.iterations[0, 0]), int(r2.iterations[0, 1]), 1]
        elif dtype == "f64":
            rr = plan.solve(loads, tol=tol * 0.1, max_iter=4 * args.max_iter)
            ref_geff, ref_iters = rr.geff, rr.iterations.ravel().tolist()
        else:
            p64 = Plan(kap.double())
            rr = p64.solve(loads, tol=1e-6, max_iter=args.max_iter)
            p64.close()
            del p64
            ref_geff, ref_iters = rr.geff, rr.iterations.ravel().tolist()
        torch.cuda.synchronize()
        ref = dict(geff=np.asarray(ref_geff), iterations=ref_iters)
        log(f"fp64 reference: geff={np.asarray(ref_geff).ravel().tolist()} iters={ref_iters} "
            f"({time.perf_counter() - t:.1f}s)")

    plan.solve(loads, tol=tol, max_iter=2)   # allocates the solver state (untimed)
    for w in range(args.warmup):
        r = plan.solve(loads, tol=tol, max_iter=args.max_iter)
        log(f"warmup {w}: iters={r.iterations.ravel().tolist()}")
    plan.kernel_times()  # reset

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_iters = 0
    results = []
    for s in range(args.steps):
        r = plan.solve(loads, tol=tol, max_iter=args.max_iter, time_kernels=True)
        tot_iters += int(r.iterations.sum())
        results.append(r)
        log(f"step {s}: iters={r.iterations.ravel().tolist()} geff={r.geff.ravel().tolist()}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = N * tot_iters / elapsed
    avg_ms, launches, bytes_per_problem = plan.kernel_times()
    # every problem is active in exactly `iterations` update launches
    alg_bytes = bytes_per_problem * tot_iters
    achieved = alg_bytes / (avg_ms * 1e-3 * launches) / 1e9 if launches else float("nan")
    last = results[-1]

    esz = 8 if dtype == "f64" else 4
    # algorithmic bytes per voxel and iteration over all kernels of one iteration
    # (power-of-two n3: divergence fused with the forward k pass):
    # div+k 7s+s, j fwd 2s, i s+8, j inv 16, k inv 16, update 15s+8
    iter_bytes = {8: 256.0, 4: 152.0}[esz]
    iter_frac = value * iter_bytes / 1e9 / HBM_PEAK_GBPS

    accuracy = {}
    if ref is not None:
        rel = np.abs(last.geff - ref["geff"]) / np.abs(ref["geff"])
        accuracy["geff_rel_err_vs_fp64"] = float(rel.max())
        accuracy["fp64_ref_geff"] = ref["geff"].ravel().tolist()
        accuracy["fp64_ref_iterations"] = ref["iterations"]
    if args.workload == "c2":
        accuracy["e3_closed_form_rel_err"] = float(abs(last.geff[0, 2] - kap_np[0].mean()) / kap_np[0].mean())

    try:
        ceiling = stream_ceiling(torch)
    except Exception as exc:  # measurement aid only
        log(f"stream ceiling failed: {exc}")
        ceiling = None

    out = {
        "metric": "ADMM voxel-iters/s at geff rel.err 1e-4 (FP32 vs FP64); % HBM roofline",
        "value": value,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": cfg["name"],
            "grid": list(kap_np.shape[1:]),
            "fields": F,
            "loads": [list(l) for l in loads],
            "tol": tol,
            "iterations": last.iterations.ravel().tolist(),
            "geff": last.geff.ravel().tolist(),
            **accuracy,
            "iteration_bytes_per_voxel": iter_bytes,
            "iteration_hbm_frac": iter_frac,
            "stream_copy_GBps": ceiling,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_update (fused xi-step assembly, relaxation, ball projection, multiplier update, FP64 partials)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            # per launch like `achieved`: the per-problem figure times the mean number of
            # active problems per launch of the timed region
            "traffic": (K_UPDATE_TRAFFIC_C2 * tot_iters / launches
                        if args.workload == "c2" and K_UPDATE_TRAFFIC_C2 and launches else None),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_ms": avg_ms,
            "launches": launches,
            "bytes_per_launch_per_problem": bytes_per_problem,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(kap_np, loads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
