#!/usr/bin/env python3
"""Benchmark of the Wilson-Dirac hot path on one MI355X.

A step is one batched solve of M^dag M x = phi (even-odd, Mhat^dag Mhat) for
all right-hand sides of the workload to a true FP64 relative residual of
1e-10: the stencil sweeps, fused CG vector updates, device reductions and
FP64 reliable updates, i.e. every stage of the path.  Inputs (gauge field,
sources) are resident in HBM before the timed region starts.

Default workload: 32^3 x 64 lattice, one random SU(3) field (eps = 0.5),
12 Gaussian right-hand sides solved together, kappa = 0.156, FP16 spinors
with per-site norms, FP32 12-real links, FP32 arithmetic, FP64 reliable
updates.  Printed: one JSON line with solves/s (value), the FP64 solve rate
on the same inputs, the dominant kernel's roofline entry (live HIP-event
timing) and the CPU oracle baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    # name: dims, eps, kappa, nrhs, seed index
    "c3_32c64_12rhs": dict(dims=(32, 32, 32, 64), eps=0.5, kappa=0.156, nrhs=12, cfg=2),
    "c2_16c32": dict(dims=(16, 16, 16, 32), eps=0.5, kappa=0.155, nrhs=8, cfg=1),
    "c1_4c4": dict(dims=(4, 4, 4, 4), eps=0.3, kappa=0.15, nrhs=1, cfg=0),
}
PRECS = {"f64": 0, "f32": 1, "f16": 2, "f16l16": 2 | 0x10, "f32l16": 1 | 0x10,
         "f16r18": 2 | 0x20, "f32r18": 1 | 0x20}
DTYPE = {"f64": "f64", "f32": "f32", "f16": "f16+norm/f32", "f16l16": "f16+norm/f32",
         "f32l16": "f32", "f16r18": "f16+norm/f32", "f32r18": "f32"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_32c64_12rhs", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="f16", choices=sorted(PRECS))
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tuned", type=int, default=1, help="autotune launch shapes before timing")
    ap.add_argument("--tune-only", action="store_true",
                    help="autotune (filling WD_TUNE_CACHE when set) and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def make_inputs(w):
    import lattice_inputs as li
    dims = w["dims"]
    t = time.time()
    U = li.random_su3_field(dims, w["eps"], seed=li.config_seed(w["cfg"]))
    B = li.gaussian_spinor(li.volume(dims) // 2, seed=li.config_seed(w["cfg"]) + 1000, nrhs=w["nrhs"])
    log(f"[bench] inputs {dims} nrhs {w['nrhs']} generated in {time.time() - t:.1f}s")
    return U, B


def cpu_baseline(U, dims, kappa, iters_per_solve, budget_s):
    """Oracle (plain C, OpenMP) applications of Mhat^dag Mhat on one RHS,
    scaled to solves/s with the FP64 iteration count of the GPU solve."""
    from oracle import wdref
    import lattice_inputs as li
    wdref.lib()
    b = li.gaussian_spinor(li.volume(dims) // 2, seed=77)
    t0 = time.time()
    n = 0
    while True:
        wdref.mhatdag_mhat(dims, U, kappa, b)
        n += 1
        if time.time() - t0 > budget_s or n >= 50:
            break
    t_apply = (time.time() - t0) / n
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": 1.0 / (t_apply * iters_per_solve),
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{n} oracle applications of Mhat^dag Mhat on one {dims} right-hand side "
                   f"({t_apply:.3f} s each), times {iters_per_solve} CG iterations per solve"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1207_2223_amd import wd

    w = WORKLOADS[args.workload]
    dims, kappa, nrhs = w["dims"], w["kappa"], w["nrhs"]
    U, B = make_inputs(w)
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    Xd = torch.empty_like(Bd)
    lat = wd.Lattice(dims)
    lat.gauge_load(Ud, recon=12)
    params = wd.solver_params(prec=PRECS[args.prec], eo=1, tuned=args.tuned)
    if args.tuned:
        t = time.time()
        for code in {PRECS[args.prec], 0}:
            for row in wd.wd_tune(lat.ctx, nrhs, code):
                log(f"[bench] tuned {code:#x} {row['sweep']}: block {row['block']} nr {row['nr']} "
                    f"rl {row['rl']} remap {row['remap']} {row['us']:.1f} us")
        log(f"[bench] autotune {time.time() - t:.1f}s")
    if args.tune_only:
        lat.close()
        return
    torch.cuda.synchronize()

    def solve(p):
        st, stats = lat.cg_solve(Xd, Bd, [kappa] * nrhs, p)
        return st, stats

    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy probe: 1 GiB read + 1 GiB written by one copy kernel")
        del a, b
    for k in range(args.warmup):
        st, stats = solve(params)
        log(f"[bench] warmup {k}: status {st} iters {[s['iters'] for s in stats][:4]}...")
    wd.wd_timing_enable(lat.ctx, True)
    step_ms = []
    iters, resid, ok = [], [], True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st, stats = solve(params)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        ok &= st == wd.WD_OK and all(s["true_resid"] <= 1e-10 for s in stats)
        iters.append(max(s["iters"] for s in stats))
        resid.append(max(s["true_resid"] for s in stats))
        log(f"[bench] step {k}: {step_ms[-1]:.1f} ms, status {st}, iters {iters[-1]}, "
            f"max true resid {resid[-1]:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    report = wd.wd_timing_report(lat.ctx)
    wd.wd_timing_read(lat.ctx)
    wd.wd_timing_enable(lat.ctx, False)
    value = args.steps * nrhs / elapsed

    # dominant stencil kernel by total time
    name, (n, ms, by, units) = max(report.items(), key=lambda kv: kv[1][1])
    avg_ms = ms / n
    achieved = (by / n) / (avg_ms * 1e-3) / 1e9
    flops_site = 1320.0
    log(f"[bench] kernels: " + "; ".join(f"{k}: {v[0]} x {v[1] / v[0] * 1e3:.1f} us" for k, v in report.items()))
    all_ms = sum(v[1] for v in report.values())
    all_by = sum(v[2] for v in report.values())

    fp64 = None
    if not args.no_fp64 and args.prec != "f64":
        p64 = wd.solver_params(prec=0, eo=1, tuned=args.tuned)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st64, s64 = solve(p64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - ts
        fp64 = {"solves_per_s": nrhs / t64, "iters": max(s["iters"] for s in s64),
                "status": st64, "max_true_resid": max(s["true_resid"] for s in s64)}
        log(f"[bench] fp64 solve: {t64 * 1e3:.1f} ms, iters {fp64['iters']}")
    iters64 = fp64["iters"] if fp64 else iters[-1]

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(U, dims, kappa, iters64, args.cpu_seconds)
        log(f"[bench] cpu oracle: {cpu['value']:.4g} solves/s ({cpu['sample']})")

    out = {
        "metric": "Dslash HBM GB/s + GFLOP/s; M†M solves/s mixed vs FP64 at 1e-10, p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic (seeded random SU(3) field and Gaussian sources)",
        "config": {"workload": f"{args.workload}: {'x'.join(map(str, dims))} lattice, {nrhs} RHS, "
                               f"kappa {kappa}, eps {w['eps']}, even-odd CG to 1e-10",
                   "prec_sloppy": args.prec, "nrhs": nrhs, "lattice": list(dims)},
        "converged": bool(ok),
        "iters": iters[-1],
        "max_true_resid": max(resid),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "stencil": {"GB_s_all_launches": all_by / (all_ms * 1e-3) / 1e9,
                    "share_of_step": all_ms / (elapsed * 1e3)},
        "dominant_kernel": {"name": name, "launches": n, "avg_us": avg_ms * 1e3,
                            "bytes_per_launch": by / n, "site_rhs_per_launch": units / n,
                            "GFLOP_s": flops_site * (units / n) / (avg_ms * 1e-3) / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "fp64": fp64,
        "mixed_vs_fp64": (value / fp64["solves_per_s"]) if fp64 else None,
        "cpu_baseline": cpu,
    }
    lat.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
