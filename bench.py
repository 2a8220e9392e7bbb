"""Benchmark of the Toom-Cook hot path on one MI355X.

A step is one whole product w = u v through every phase of the path:
evaluation, leaf products, interpolation (even-odd combine, Newton loops),
recomposition.  The default workload is two 2^19-limb (2^24-bit) uniform
operands, 16-way at the top and 3-way below; inputs are resident in HBM
before the timed region.

The timed region launches each product as the library's captured HIP graph.
A second, separately timed pass turns on the library's per-launch HIP events
(direct launches on the same stream) to get the average duration of each
kernel class; the roofline of the dominant class divides its algorithmic
work (tc_plan_cost_get) by that duration.

Prints one JSON line: throughput in n^2-equivalent limb-mults/s (nu*nv per
second), ns per product limb, p50/p99 of the per-step times, the roofline of
the dominant kernel class (and of the matrix-core leaf), the batched-vs-single
comparison on a batch of 4096 independent products, the serving loop under
Poisson arrivals (saturation, then p50/p99 at three offered loads of 20000
requests each), sub-records for the 1024-limb Toom-3 product and the 2^25-limb
product, and the CPU oracle timed on this host for each of them.  Every
timed GPU result is checked: the products against the oracle's, batched items
and served requests against their products alone.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "limb-mults/s (n^2-equiv) + ns/limb at 2^20 limbs; batched vs single; p50/p99"

# MI355X published peaks.
PEAK_HBM = 8.0e12        # bytes/s
PEAK_INT8_MFMA = 5.0e15  # dense int8 ops/s (multiply and add counted separately)
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz; one 32x32+32->64
# multiply-add (v_mad_u64_u32) issues at half the full rate (tc_measure_mad_rate
# measures it: 1.98e13/s on MI355X)
PEAK_MAD = 256 * 4 * 16 * 2.4e9 / 2

CONFIGS = {
    "c2": dict(workload="2^19 x 2^19 limbs (2^20-limb product), 16-way top level, 3-way below",
               n=1 << 19, plan=[16, 3, 3, 3]),
    "c1": dict(workload="1024 x 1024 limbs, one 3-way level (0,1,-1,2,inf), schoolbook leaves",
               n=1024, plan=[3], variants=[1]),
    "c5": dict(workload="2^25 x 2^25 limbs (2^30-bit operands), 32-way top level, "
                         "16-way and 3-way below",
               n=1 << 25, plan=[32, 16, 16, 3]),
    # unbalanced: tc_mul's own cut into 4096-limb pieces (plan None), beside
    # the zero-padded balanced plan for 2^20 limbs
    # squaring: u and v the same operand (one evaluation per node), beside the
    # same operand in a second buffer (general path)
    "sq": dict(workload="2^19-limb square (u = v), 16-way top level, 3-way below",
               n=1 << 19, plan=[16, 3, 3, 3], square=True),
    "unb": dict(workload="2^20 x 2^12 limbs (unbalanced 256:1), cut into 2^12-limb pieces",
                n=1 << 20, nv=1 << 12, plan=None),
}

PROFILE_DIR = os.path.join(ROOT, "profiles")
SRC_DIR = os.path.join(ROOT, "paper_1602_02740_amd", "csrc")


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


DEVICE_SOURCES = ("tc_kernels.hip", "tc_engine.hpp", "tc_types.hpp", "tc_internal.hpp")


def kernel_source_hash() -> str:
    """sha256 over the device-code sources; a stored HBM traffic figure is
    used only while the kernels it was measured on are unchanged."""
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(SRC_DIR, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def stored_traffic(kernel_class: str, workload_key: str):
    """HBM bytes per launch of a kernel class from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy-kernel calibration), or None
    when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel_class}_{workload_key}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"^source_sha256:\s*([0-9a-f]{64})", text, re.M)
    m_val = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def host_threads() -> int:
    """Host threads for the oracle: the CPU share this process may use."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(u, v, plan, variants, budget_s=10.0, max_reps=100, keep=None):
    """The oracle (plain recursive Toom-Cook, top-level products on
    P = min(host threads, 2B-1) threads, section 2's scheme) on the same
    operands and plan, repeated for about budget_s seconds; keep (a list)
    receives the oracle's product."""
    import oracle
    nthr = host_threads()
    threads = min(nthr, 2 * plan[0] - 1) if plan else 1
    t0 = time.perf_counter()
    reps = 0
    while True:
        w = oracle.mul_toom(u, v, plan, variants, threads=threads)
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= max_reps:
            break
    dt = (time.perf_counter() - t0) / reps
    if keep is not None:
        keep.append(w)
    what = "schoolbook product(s)" if not plan else "Toom-Cook product(s) of the same plan"
    return dict(value=len(u) * len(v) / dt, unit="limb-mults/s", cores=threads, kind="oracle",
                sample=f"{reps} full {what} of the same operands, top-level products on "
                       f"{threads} of {nthr} host threads, {dt:.4f} s each",
                seconds_per_product=dt)


def time_steps(fn, steps, stream, torch, np):
    """Per-step and total milliseconds of `steps` calls of fn, HIP events on stream."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return per, ev[0].elapsed_time(ev[-1])


def roofline(kt, cost, steps):
    """Roofline of the kernel class with the largest summed time."""
    dom = max(kt, key=lambda k: kt[k][1])
    launches, ms = kt[dom]
    avg_s = ms * 1e-3 / max(launches, 1)
    per_step_launches = launches / steps
    if dom == "leaf" and cost["launches"]["leaf"] > 0:
        # leaves of a plan are either all vector-ALU or all matrix-core ones
        ops = cost["leaf_limb_products"] / per_step_launches
        return dom, dict(bound="mfma", achieved=ops * 32 / avg_s / 1e12,
                         peak=PEAK_INT8_MFMA / 1e12, unit="TOP/s",
                         frac=ops * 32 / avg_s / PEAK_INT8_MFMA, traffic=None,
                         kernel="k_mleaf/k_leaf",
                         note="32 int8 ops (16 byte products, multiply+add) per limb product")
    per_launch_bytes = cost["bytes"][dom] / max(per_step_launches, 1e-30)
    achieved = per_launch_bytes / avg_s
    return dom, dict(bound="hbm", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                     frac=achieved / PEAK_HBM, traffic=None, kernel=f"k_{dom}",
                     algorithmic_bytes_per_launch=per_launch_bytes,
                     avg_launch_us=avg_s * 1e6)


TUNING_TABLE = os.path.join(ROOT, "paper_1602_02740_amd", "tuning.json")


def leaf_roofline(kt, cost, steps):
    """The matrix-core leaf class against the int8 MFMA peak (32 int8 ops,
    16 byte products with their additions, per limb product)."""
    launches, ms = kt.get("leaf", (0, 0.0))
    if not launches or not cost["leaf_limb_products"]:
        return None
    per_step_s = ms * 1e-3 / steps
    ops = cost["leaf_limb_products"] * 32
    return dict(bound="mfma", kernel="k_mleaf", achieved=ops / per_step_s / 1e12,
                peak=PEAK_INT8_MFMA / 1e12, unit="TOP/s", frac=ops / per_step_s / PEAK_INT8_MFMA,
                ms_per_product=ms / steps)


RETUNE = False  # --retune: measure every class now, ignoring the committed table
TUNED_HERE = set()  # classes measured by this process


def autotune_classes(toom, sizes, save_to=None):
    """Makes a tuned plan the default for every quarter-octave size class the
    sizes touch: the committed tuning table of this kind of device where it
    has the class, else measured now (tc_autotune).  Returns (classes,
    measured now); save_to receives the table when anything was measured."""
    import math
    have = set()
    if not RETUNE and os.path.exists(TUNING_TABLE) and toom.autotune_load(TUNING_TABLE):
        with open(TUNING_TABLE) as f:
            have = {int(c["class"]) for c in json.load(f)["classes"]}
    done, tuned = set(), 0
    for n in sorted(set(int(x) for x in sizes)):
        c = math.floor(4 * math.log2(n))
        if c in done:
            continue
        done.add(c)
        if c not in have and c not in TUNED_HERE:
            toom.autotune(n)
            TUNED_HERE.add(c)
            tuned += 1
    if tuned and save_to:
        toom.autotune_save(save_to)
    return len(done), tuned


TABLE_OUT = None  # --table-out: where a newly measured tuning table is written


def table_out():
    """Where a newly measured tuning table goes (None: not saved)."""
    return TABLE_OUT


def batch_leg(torch, np, toom, I, stream, steps=3, warmup=1, count=4096):
    """Batch of independent products: one tc_mul_batch vs a loop of tc_mul,
    every batched output checked against the single product of its item."""
    classes, tuned = autotune_classes(toom, I.config3_sizes(count), table_out())
    log(f"batch leg: {classes} size classes ({tuned} measured now)")
    pairs = I.config3(count)
    us, vs = [], []
    for a, b in pairs:
        us.append(toom.to_device(a))
        vs.append(toom.to_device(b))
    outs = [toom.empty(u.numel() + v.numel()) for u, v in zip(us, vs)]
    ref = [toom.empty(u.numel() + v.numel()) for u, v in zip(us, vs)]
    work = float(sum(int(u.numel()) * int(v.numel()) for u, v in zip(us, vs)))
    status = torch.zeros(count, dtype=torch.int32, device="cuda")

    descs = toom.batch_descs(us, vs, outs)
    import ctypes
    f = toom.lib().tc_mul
    sp = ctypes.c_void_p(stream.cuda_stream)
    args = [(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(u.data_ptr()), u.numel(),
             ctypes.c_void_p(v.data_ptr()), v.numel(), sp) for u, v, w in zip(us, vs, ref)]

    def batched():
        toom.mul_batch(us, vs, outs=outs, descs=descs, stream=stream, status=status)

    def single():
        # tc_mul per item, arguments marshalled beforehand
        for a in args:
            rc = f(*a)
            if rc != 0:
                raise toom.ToomError(rc, "tc_mul")

    log(f"batch leg: {count} products resident")
    t0 = time.perf_counter()
    batched()
    toom.sync()
    first_s = time.perf_counter() - t0
    for _ in range(warmup):
        batched()
        single()
    toom.sync()
    log("batch leg: timing")
    pb, tb = time_steps(batched, steps, stream, torch, np)
    ps, ts = time_steps(single, steps, stream, torch, np)
    toom.sync()
    # every batched item equals its single product, and no item reported an error
    bad = [i for i in range(count) if not torch.equal(outs[i], ref[i])]
    if bad or int(status.abs().sum()):
        raise RuntimeError(f"batch leg: items {bad[:10]} differ from their single products")
    # launches of one batched call
    toom.timing_enable(True)
    toom.timing_read()
    batched()
    kt = toom.timing_read()
    toom.timing_enable(False)
    toom.sync()
    # the oracle on the same items, spread over the host threads
    import concurrent.futures as cf
    import oracle
    nthr = host_threads()

    def oracle_item(p):
        a, b = p
        return oracle.mul_school(a, b) if len(a) * len(b) <= 1 << 20 else \
            oracle.mul_toom(a, b, [3] * max(1, int(math.log(max(len(a), 1) / 256) / math.log(3))))

    import math
    log(f"batch leg: oracle on {nthr} threads")
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nthr) as ex:
        list(ex.map(oracle_item, pairs))
    oracle_s = time.perf_counter() - t0
    return dict(workload=f"{count} balanced products, n log-uniform in [64, 16384] limbs, "
                         "90% uniform / 5% all-ones / 5% sparse operands",
                batched_value=work * steps / (tb * 1e-3), single_value=work * steps / (ts * 1e-3),
                unit="limb-mults/s", batched_ms=tb / steps, single_ms=ts / steps,
                ratio=ts / tb, batched_p50_ms=float(np.percentile(pb, 50)),
                batched_p99_ms=float(np.percentile(pb, 99)),
                launches_per_batch={k: kt[k][0] for k in kt if kt[k][0]},
                # the launches' own durations (HIP events around each, in a
                # separate pass): their sum against batched_ms bounds what
                # launch gaps cost the graph replay
                kernel_ms_per_batch={k: kt[k][1] for k in kt if kt[k][0]},
                kernel_ms_sum=sum(kt[k][1] for k in kt if kt[k][0]),
                first_call_s=first_s, sum_n2=work, size_classes=classes,
                classes_tuned_now=tuned, verified="every item equals its tc_mul product",
                cpu_baseline=dict(value=work / oracle_s, unit="limb-mults/s", cores=nthr,
                                  kind="oracle", seconds=oracle_s,
                                  sample=f"all {count} products once, items spread over "
                                         f"{nthr} host threads"))


def serving_leg(torch, np, toom, I, count=20000, sat_count=2000, loads=(0.5, 0.8, 0.95)):
    """Poisson arrivals of products with Zipf(1.2) sizes over 2^5..2^20 limbs
    through the serving loop: saturation throughput in a closed loop, then
    latency percentiles at three offered loads; every served result is
    compared with tc_mul of the same operands alone."""
    classes = [1 << k for k in range(5, 21)]
    ops = {n: (toom.to_device(I.random_limbs(4, 2 * i, n)),
               toom.to_device(I.random_limbs(4, 2 * i + 1, n))) for i, n in enumerate(classes)}
    alone = {n: toom.mul(u, v) for n, (u, v) in ops.items()}
    toom.sync()
    checked = [0]

    lag = [0.0]  # latest submit behind its scheduled arrival (s)

    def run(srv, sizes, arrivals):
        t0 = time.perf_counter()
        i = 0
        pending = {}
        done = []
        lag[0] = 0.0
        while i < len(sizes) or pending:
            now = time.perf_counter() - t0
            while i < len(sizes) and (arrivals is None or arrivals[i] <= now):
                if arrivals is not None:
                    lag[0] = max(lag[0], now - float(arrivals[i]))
                n = int(sizes[i])
                u, v = ops[n]
                w = toom.empty(2 * n)
                pending[srv.submit(u, v, w)] = (n, w)
                i += 1
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    if r["status"] != 0:
                        raise toom.ToomError(r["status"], "served request")
                    done.append(pending.pop(t))
            if pending or i < len(sizes):
                time.sleep(0.0001)
        el = time.perf_counter() - t0
        for n, w in done:
            if not torch.equal(w, alone[n]):
                raise RuntimeError(f"serving: a {n}-limb result differs from its product alone")
        checked[0] += len(done)
        return el

    out = {"workload": "Poisson arrivals, sizes 2^5..2^20 limbs with Zipf(1.2) over the 16 "
                       "powers of two, uniform operands resident in HBM",
           "unit": "limb-mults/s"}
    out["size_classes"], out["classes_tuned_now"] = autotune_classes(toom, classes, table_out())
    with toom.Server(streams=4, max_batch=64) as srv:
        # warm-up: every size class once, bursts of 1, 2, 4, .., 64 requests of
        # each size the server merges (below 2^16 limbs; a batch takes a power
        # of two of them, and every new shape compiles on first use), and the
        # saturation stream itself
        run(srv, classes, None)
        for n in classes:
            if n < 1 << 16:
                for k in (1, 2, 4, 8, 16, 32, 64):
                    run(srv, [n] * k, None)
        sizes = I.zipf_sizes(sat_count, seed=4)
        run(srv, sizes, None)
        srv.reset_stats()
        el = run(srv, sizes, None)
        lam = sat_count / el
        st = srv.stats()
        out["saturation"] = {"requests": sat_count, "requests_per_s": lam,
                             "value": st["limb_mults_per_s"], "p50_us": st["p50_us"],
                             "p99_us": st["p99_us"], "batches": st["batches"]}
        log(f"serving: saturation {lam:.0f} requests/s")
        out["loads"] = []
        # the arrival loop runs without Python's cyclic collector: a full
        # collection over this process's objects pauses it for tens of
        # milliseconds and then submits the arrivals it held back as one burst
        gc.collect()
        gc.freeze()
        gc.disable()
        try:
            for k, f in enumerate(loads):
                srv.reset_stats()
                sizes = I.zipf_sizes(count, seed=40 + k)
                arr = I.poisson_arrivals(count, f * lam, seed=40 + k)
                el = run(srv, sizes, arr)
                st = srv.stats()
                out["loads"].append({"offered_fraction": f, "offered_requests_per_s": f * lam,
                                     "requests": count, "value": st["limb_mults_per_s"],
                                     "p50_us": st["p50_us"], "p99_us": st["p99_us"],
                                     "batches": st["batches"], "elapsed_s": el,
                                     "max_submit_lag_us": lag[0] * 1e6})
                log(f"serving: load {f}: p50 {st['p50_us']:.0f} us, p99 {st['p99_us']:.0f} us, "
                    f"latest submit {lag[0] * 1e6:.0f} us behind its arrival")
        finally:
            gc.enable()
            gc.unfreeze()
    out["verified"] = f"all {checked[0]} served results equal their products alone"
    return out


# Section 5's Toom-Cook over an FFT product: Toom levels over transform leaves
# (an exact NTT), timed on the same operands as the workload's own plan.
NTT_PLANS = {"c2": [[], [3], [16]], "c5": [[8], [16], [32]]}


def ntt_leg(torch, np, toom, du, dv, stream, steps, plans):
    """Records of the same product through Toom levels over transform
    leaves, and host copies of their products (for the oracle comparison)."""
    recs, prods = [], []
    nu, nv = du.numel(), dv.numel()
    for Bs in plans:
        plan = toom.Plan.make(Bs, leaf=toom.LEAF_NTT)
        dw = toom.empty(nu + nv)
        step = lambda: toom.mul(du, dv, plan=plan, out=dw)
        for _ in range(2):
            step()
        toom.sync()
        per, total = time_steps(step, steps, stream, torch, np)
        toom.sync()
        ms = total / steps
        toom.timing_enable(True)
        toom.timing_read()
        step()
        kt = toom.timing_read()
        toom.timing_enable(False)
        toom.sync()
        # leaf width: blocks of ceil(n / B) limbs plus the evaluation growth
        # ceil(((B-1)(B-2)+1) / 32) limbs per level
        lw = [nu, nv]
        if Bs:
            n = max(nu, nv)
            for B in Bs:
                n = -(-n // B) + ((B - 1) * (B - 2) + 32) // 32
            lw = [n, n]
        bits, N, _ = toom.ntt_params(*lw)
        # the transform kernels against the multiplier: per leaf three
        # N-point transforms of (N/2) log2 N butterflies, one field product
        # (four 32x32+32->64 multiply-adds) each
        leaves = 1
        for B in Bs:
            leaves *= 2 * B - 1
        mads = leaves * 3 * (N // 2) * (N.bit_length() - 1) * 4
        leaf_s = kt["leaf"][1] * 1e-3
        recs.append({"plan": list(Bs), "leaf": "ntt", "piece_bits": bits, "transform_length": N,
                     "ms_per_product": ms, "p50_ms": float(np.percentile(per, 50)),
                     "p99_ms": float(np.percentile(per, 99)), "value": nu * nv / (ms * 1e-3),
                     "unit": "limb-mults/s",
                     "kernel_ms": {k: kt[k][1] for k in kt if kt[k][0]},
                     "leaf_roofline": {"bound": "alu", "kernel": "k_ntt_*",
                                       "achieved": mads / leaf_s / 1e12, "peak": PEAK_MAD / 1e12,
                                       "unit": "T multiply-adds/s",
                                       "frac": mads / leaf_s / PEAK_MAD,
                                       "butterflies": mads // 4}})
        prods.append(toom.to_host(dw))
        del dw
    return recs, prods


def single_config_leg(torch, np, toom, I, stream, key, steps, warmup, oracle_budget_s):
    """One product of a named workload: GPU p50/p99 of the captured-graph
    replays, n^2-equivalent rate, ns per product limb, and the oracle on the
    same operands and plan; the GPU product is compared with the oracle's."""
    cfg = CONFIGS[key]
    n = cfg["n"]
    u, v = (I.config1_uniform(n) if key == "c1" else I.config5(n))
    plan = toom.Plan.make(cfg["plan"], cfg.get("variants"))
    du, dv = toom.to_device(u), toom.to_device(v)
    dw = toom.empty(2 * n)
    step = lambda: toom.mul(du, dv, plan=plan, out=dw)
    for _ in range(warmup):
        step()
    toom.sync()
    per, total = time_steps(step, steps, stream, torch, np)
    toom.sync()
    ms = total / steps
    got = toom.to_host(dw)
    del dw
    ntt_recs, ntt_prods = [], []
    if key in NTT_PLANS:
        log(f"{key}: Toom-Cook over transform leaves")
        ntt_recs, ntt_prods = ntt_leg(torch, np, toom, du, dv, stream, steps, NTT_PLANS[key])
    del du, dv
    torch.cuda.empty_cache()
    log(f"{key}: {ms:.4f} ms per product; oracle")
    kept = []
    cb = cpu_baseline(u, v, cfg["plan"], cfg.get("variants"), budget_s=oracle_budget_s,
                      max_reps=1000, keep=kept)
    if not np.array_equal(got, kept[0]):
        raise RuntimeError(f"{key}: the GPU product differs from the oracle's")
    for r, w in zip(ntt_recs, ntt_prods):
        if not np.array_equal(w, kept[0]):
            raise RuntimeError(f"{key}: the product over transform leaves differs from the oracle's")
        r["verified"] = "GPU product equals the oracle's"
    extra = {"toom_over_ntt": ntt_recs} if ntt_recs else {}
    return {**extra, "workload": cfg["workload"], "nu": n, "nv": n,
            "plan": [[b, (cfg.get("variants") or [0] * len(cfg["plan"]))[i]]
                     for i, b in enumerate(cfg["plan"])],
            "value": n * n / (ms * 1e-3), "unit": "limb-mults/s", "steps": steps,
            "ms_per_product": ms, "p50_ms": float(np.percentile(per, 50)),
            "p99_ms": float(np.percentile(per, 99)), "ns_per_limb": ms * 1e6 / (2 * n),
            "verified": "GPU product equals the oracle's", "cpu_baseline": cb}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-single leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1024-limb and 2^25-limb sub-records")
    ap.add_argument("--no-compare", action="store_true",
                    help="unb/sq: skip the padded-plan / general-path comparison")
    ap.add_argument("--plan", default=None,
                    help="comma-separated B per level (or none), overriding the workload's plan")
    ap.add_argument("--retune", action="store_true",
                    help="tune every size class the legs touch now instead of loading the "
                         "committed table")
    ap.add_argument("--table-out", default=None, metavar="PATH",
                    help="write the tuning table measured in this run to PATH")
    ap.add_argument("--leaf", default="school", choices=["school", "ntt"],
                    help="leaves of the main product: schoolbook (the workloads' own) or "
                         "transform leaves (section 5's Toom-Cook over an FFT product)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB, the known-size "
                         "reference that scales hardware byte counters")
    args = ap.parse_args()
    global RETUNE, TABLE_OUT
    RETUNE = args.retune
    TABLE_OUT = args.table_out
    if args.gpus != 1:
        print(f"bench.py: one product runs on one GPU here; --gpus {args.gpus} is not "
              "supported (across GPUs the path would shard its 2B-1 top-level products)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1602_02740_amd import inputs as I
    from paper_1602_02740_amd import toom

    cfg = CONFIGS[args.config]
    n = cfg["n"]
    nv = cfg.get("nv", n)
    plan_list, variants = cfg["plan"], cfg.get("variants")
    if args.plan:
        plan_list = [] if args.plan == "none" else [int(x) for x in args.plan.split(",")]
        variants = None
    if args.config == "c1":
        u, v = I.config1_uniform(n)
    elif args.config == "c5":
        u, v = I.config5(n)
    elif args.config == "unb":
        u, v = I.unbalanced(n, nv)
    elif args.config == "sq":
        u = I.config2(n)[0]
        v = u
    else:
        u, v = I.config2(n)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    du = toom.to_device(u)
    dv = du if cfg.get("square") else toom.to_device(v)
    dw = toom.empty(n + nv)
    ntt = args.leaf == "ntt"
    plan = (toom.Plan.make(plan_list or [], variants, leaf=toom.LEAF_NTT) if ntt
            else toom.Plan.make(plan_list, variants) if plan_list else None)
    cost = toom.plan_cost(n, nv, plan)

    def step():
        toom.mul(du, dv, plan=plan, out=dw)

    log(f"{args.config}: plan {plan_list}, warmup")
    for _ in range(args.warmup):
        step()
    toom.sync()
    log("timed region")

    # timed region: K whole products as graph launches, no per-kernel events
    per, total_ms = time_steps(step, args.steps, stream, torch, np)
    toom.sync()
    ms = total_ms / args.steps

    # kernel-class durations: the library's HIP events around each launch
    ksteps = max(1, min(args.steps, 5))
    toom.timing_enable(True)
    toom.timing_read()
    for _ in range(ksteps):
        step()
    kt = toom.timing_read()
    toom.timing_enable(False)
    toom.sync()
    dom, roof = roofline(kt, cost, ksteps)
    roof["traffic"] = stored_traffic(dom, args.config)
    if ntt and dom == "leaf":
        # transform leaves: the multiplier roofline of the transform kernels
        lw = [n, nv]
        if plan_list:
            m = max(n, nv)
            for B in plan_list:
                m = -(-m // B) + ((B - 1) * (B - 2) + 32) // 32
            lw = [m, m]
        _, N, _ = toom.ntt_params(*lw)
        leaves = 1
        for B in plan_list or []:
            leaves *= 2 * B - 1
        mads = leaves * 3 * (N // 2) * (N.bit_length() - 1) * 4
        leaf_s = kt["leaf"][1] * 1e-3 / ksteps
        roof = dict(bound="alu", kernel="k_ntt_*", achieved=mads / leaf_s / 1e12,
                    peak=PEAK_MAD / 1e12, unit="T multiply-adds/s", frac=mads / leaf_s / PEAK_MAD,
                    traffic=None, transform_length=N)

    out = {
        "metric": METRIC,
        "value": n * nv / (ms * 1e-3),
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
        "config": {"workload": cfg["workload"], "nu": n, "nv": nv,
                   "plan": [[b, (variants or [0] * len(plan_list))[i]]
                            for i, b in enumerate(plan_list)] if plan_list else "cut",
                   **({"leaf": "ntt"} if ntt else {})},
        "ns_per_limb": ms * 1e6 / (n + nv),
        "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)),
        "kernel_ms_per_step": {k: kt[k][1] / ksteps for k in kt if kt[k][0]},
        "kernel_launches_per_step": {k: kt[k][0] / ksteps for k in kt if kt[k][0]},
        "leaf_limb_products": cost["leaf_limb_products"],
        "roofline": roof,
        "leaf_roofline": leaf_roofline(kt, cost, ksteps),
        "host": {"nproc": host_threads(), "cpu_model": cpu_model()},
        "alu": {"mad_per_s_measured": toom.measure_mad_rate(), "mad_per_s_peak": PEAK_MAD,
                "note": "v_mad_u64_u32 issue rate: probe vs 256 CUs x 64 lanes x 2.4 GHz / 2"},
    }
    ntt_prods = []
    if args.config == "c2" and not args.no_configs:
        log("c2: Toom-Cook over transform leaves")
        out["toom_over_ntt"], ntt_prods = ntt_leg(torch, np, toom, du, dv, stream,
                                                  args.steps, NTT_PLANS["c2"])
    if not args.no_batch and args.config == "c2":
        out["batched_vs_single"] = batch_leg(torch, np, toom, I, stream)
    if not args.no_serving and args.config == "c2":
        out["serving"] = serving_leg(torch, np, toom, I)
    if args.config == "unb" and not args.no_compare:
        # the same product through the zero-padded balanced plan of 2^20 limbs
        padded = toom.plan_default(n, nv)
        pstep = lambda: toom.mul(du, dv, plan=padded, out=dw)
        for _ in range(2):
            pstep()
        _, pms = time_steps(pstep, max(3, args.steps // 4), stream, torch, np)
        pms /= max(3, args.steps // 4)
        out["padded_plan_ms"] = pms
        out["cut_vs_padded"] = pms / ms
    if cfg.get("square") and not args.no_compare:
        dv2 = toom.to_device(v)
        gstep = lambda: toom.mul(du, dv2, plan=plan, out=dw)
        for _ in range(2):
            gstep()
        _, gms = time_steps(gstep, max(3, args.steps // 4), stream, torch, np)
        gms /= max(3, args.steps // 4)
        out["general_path_ms"] = gms
        out["square_vs_general"] = gms / ms
    if not args.no_configs and args.config == "c2":
        out["configs"] = {}
        log("c1 sub-record")
        out["configs"]["c1"] = single_config_leg(torch, np, toom, I, stream, "c1", 200, 20, 3.0)
        log("c5 sub-record")
        out["configs"]["c5"] = single_config_leg(torch, np, toom, I, stream, "c5", 5, 2, 0.0)
    if not args.no_cpu and args.config != "c5":
        log("cpu baseline")
        kept = []
        out["cpu_baseline"] = cpu_baseline(u, v, plan_list or [], variants, keep=kept)
        if plan_list and args.config == "c2":
            if not np.array_equal(toom.to_host(dw), kept[0]):
                raise RuntimeError("c2: the GPU product differs from the oracle's")
            out["verified"] = "the timed product equals the oracle's"
            for r, w in zip(out.get("toom_over_ntt", []), ntt_prods):
                if not np.array_equal(w, kept[0]):
                    raise RuntimeError("c2: the product over transform leaves differs from "
                                       "the oracle's")
                r["verified"] = "GPU product equals the oracle's"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
