"""Benchmark of the Toom-Cook hot path on one MI355X.

A step is one whole product w = u v through every phase of the path:
evaluation, schoolbook leaves, interpolation (even-odd combine, Newton
loops), recomposition.  The default workload is two 2^19-limb (2^24-bit)
uniform operands with a 16-way top level and 3-way levels below, schoolbook
leaves of 137 limbs; inputs are resident in HBM before the timed region.

Prints one JSON line: throughput in n^2-equivalent limb-mults/s (nu*nv per
second), ns per product limb, p50/p99 of the per-step times, the roofline of
the dominant kernel class, and the CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "limb-mults/s (n^2-equiv) + ns/limb at 2^20 limbs; batched vs single; p50/p99"

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz; the 32x32->64 multiply-add
# v_mad_u64_u32 issues at a quarter of the full VALU rate.
CU, SIMD, LANES, CLOCK = 256, 4, 16, 2.4e9
PEAK_LIMB_MAC = CU * SIMD * LANES * CLOCK / 4  # limb products per second
PEAK_HBM = 8.0e12  # bytes/s

CONFIGS = {
    "c2": dict(workload="2^19 x 2^19 limbs, 16-way top, 3-way below, schoolbook leaves",
               n=1 << 19, plan=[16, 3, 3, 3, 3, 3]),
    "c1": dict(workload="1024 x 1024 limbs, one 3-way level (0,1,-1,2,inf), schoolbook leaves",
               n=1024, plan=[3], variants=[1]),
    "c5": dict(workload="2^25 x 2^25 limbs, 32-way top, 16-way, 3-way below",
               n=1 << 25, plan=[32, 16, 16, 16, 3]),
}


def plan_stats(n, plan, variants=None):
    """Nominal leaf products and the node counts of a plan (sizes only)."""
    variants = variants or [0] * len(plan)
    nodes, width = 1, n
    levels = []
    for B, var in zip(plan, variants):
        bl = -(-width // B)
        g = 1 if (var == 1 or B == 2) else ((B - 1) * (B - 2) + 1 + 31) // 32
        levels.append(dict(B=B, nodes=nodes, n=width, bl=bl, nc=bl + g))
        nodes *= 2 * B - 1
        width = bl + g
    return dict(levels=levels, leaves=nodes, leaf_n=width, leaf_mults=nodes * width * width)


def leaf_bytes(st):
    # operands read once, products written once
    return st["leaves"] * st["leaf_n"] * 4 * 4


def cpu_baseline(u, v, plan, variants, budget_s=10.0):
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.mul_toom(u, v, plan, variants, threads=threads)
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= 100:
            break
    dt = (time.perf_counter() - t0) / reps
    return dict(value=len(u) * len(v) / dt, unit="limb-mults/s", cores=threads, kind="oracle",
                sample=f"{reps} full product(s) of the same workload, top-level products on "
                       f"{threads} threads (section 2), {dt:.3f} s each")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--plan", default=None,
                    help="comma-separated B per level, overriding the workload's plan")
    ap.add_argument("--no-fusion", action="store_true",
                    help="launch every recursion level separately (no fused bottom nodes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs one product on one GPU; --gpus {args.gpus} is not "
              "supported (the path would shard its 2B-1 top-level products across GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1602_02740_amd import inputs as I
    from paper_1602_02740_amd import toom

    cfg = CONFIGS[args.config]
    n = cfg["n"]
    plan_list, variants = cfg["plan"], cfg.get("variants")
    if args.plan:
        plan_list = [int(x) for x in args.plan.split(",")]
        variants = None
    if args.config == "c1":
        u, v = I.config1_uniform(n)
    elif args.config == "c5":
        u, v = I.config5(n)
    else:
        u, v = I.config2(n)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    toom.set_fusion(not args.no_fusion)
    du, dv = toom.to_device(u), toom.to_device(v)
    dw = toom.empty(2 * n)
    plan = toom.Plan.make(plan_list, variants)
    for _ in range(args.warmup):
        toom.mul(du, dv, plan=plan, out=dw)
    toom.sync()

    # timed region: K whole products, per-step events for p50/p99 and the
    # library's per-launch events for the kernel classes
    toom.timing_enable(True)
    toom.timing_read()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(args.steps):
        toom.mul(du, dv, plan=plan, out=dw)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    toom.sync()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    total_ms = ev[0].elapsed_time(ev[-1])
    kt = toom.timing_read()
    toom.timing_enable(False)
    ms = total_ms / args.steps

    st = plan_stats(n, plan_list, variants)
    # dominant kernel class by summed time
    dom = max(kt, key=lambda k: kt[k][1])
    launches, dom_ms = kt[dom]
    per_launch_ms = dom_ms / max(launches, 1)
    if dom == "leaf":
        # one leaf launch per product: algorithmic limb products of the plan
        work = st["leaf_mults"] * args.steps / max(launches, 1)
        achieved = work / (per_launch_ms * 1e-3)
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_LIMB_MAC / 1e12,
                    unit="T limb-products/s", frac=achieved / PEAK_LIMB_MAC, traffic=None,
                    kernel="k_leaf")
    else:
        roof = dict(bound="hbm", achieved=None, peak=PEAK_HBM / 1e9, unit="GB/s", frac=None,
                    traffic=None, kernel=dom)
    out = {
        "metric": METRIC,
        "value": n * n / (ms * 1e-3),
        "unit": "limb-mults/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": cfg["workload"], "nu": n, "nv": n,
                   "plan": [[b, (variants or [0] * len(plan_list))[i]]
                            for i, b in enumerate(plan_list)],
                   "leaf_limbs": st["leaf_n"], "leaves": st["leaves"]},
        "ns_per_limb": ms * 1e6 / (2 * n),
        "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)),
        "kernel_ms_per_step": {k: kt[k][1] / args.steps for k in kt},
        "kernel_launches_per_step": {k: kt[k][0] / args.steps for k in kt},
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(u, v, plan_list, variants)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
