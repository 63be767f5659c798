"""Benchmark of the deep-copy + pointer-chain kernel hot path on one MI355X.

Default workload (the batched MD workload, the largest single-GPU
configuration): 10,000 independent simulations, each a struct pointing to
an array of cells (uniform 8..512 per simulation), each cell pointing to
three double3 arrays (positions, velocities, forces) of Poisson(64) atoms;
~7.75 M arrays, ~12 GB. A step is one replay of a HIP graph that

    attaches every pointer of every structure    -- Figure 2 (d), Algorithm 1
    runs x = fma(x, 1.0001, 0.5) over every leaf, each leaf's address read
    once from its relocated parent slot          -- pointerchain, Section 3
    detaches every pointer again (demarshalling)

in the form the autotuner measured fastest, with the marshalled image
already resident in HBM when the timed region starts. `value` is the
algorithmic bytes of a step over its time. The host-link part of the deep
copy (pack + host-to-device + attach, and the copy back) is timed
separately and reported as `host_link`, never as `value`.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|linear|wide|plain|served|sweep]
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E
LINK_PEAK_GBPS = 63.0       # PCIe Gen5 x16 per direction after encoding (32 GT/s x16)
LINK_WARMUP, LINK_REPS = 2, 5   # untimed, then timed deep copies of the host-link measurements


def traffic(workload, kernel):
    """L2-to-fabric bytes per launch of `kernel` (Infinity Cache hits and HBM
    together) measured by rocprofv3 counters (profiles/hbm_counters.txt), or
    None when there is no entry or the kernel source has changed since the
    counters were taken."""
    import hashlib
    try:
        src = open(os.path.join(ROOT, "paper_1906_01128_amd", "csrc", "dc_kernels.hip"), "rb").read()
        lines = open(os.path.join(ROOT, "profiles", "hbm_counters.txt")).read().splitlines()
    except OSError:
        return None
    sha = hashlib.sha256(src).hexdigest()
    for ln in lines:
        f = ln.split()
        if len(f) == 6 and not ln.startswith("#") and f[0] == workload and f[1] == kernel and f[2] == sha:
            return int(f[5])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched",
                    choices=["linear", "plain", "wide", "batched", "served", "sweep", "copycal"])
    ap.add_argument("--full", action="store_true",
                    help="sweep: the paper's full size range; served: 2000 jobs, leaves up to 256 MiB")
    ap.add_argument("--passes", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-link", action="store_true", help="skip the host-link measurements")
    ap.add_argument("--no-secondary", action="store_true",
                    help="batched: skip the comparisons beside the timed step (forms, kick-drift, linear chain)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q))


def link_peak(torch):
    """Pinned 1 GiB copies in each direction (the host link's achievable peak)."""
    n = 1 << 30
    h = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    out = {}
    for name, fn in (("h2d", lambda: d.copy_(h, non_blocking=True)), ("d2h", lambda: h.copy_(d, non_blocking=True))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(3):
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        out[name] = n / min(ts) / 1e9
    del h, d
    return out


def cpu_baseline_linear(args, passes):
    """The CPU oracle on the same workload, bounded: deep copy, `passes` fma
    passes per mode (the oracle has one result for both modes, so it runs
    once per mode), copy back. Single-threaded."""
    import fixtures as fx
    import oracle as orc
    t = fx.linear()
    chain = [(1, 0)] * 7 + [(0, 0)]
    leaf = 8 << 24
    t0 = time.perf_counter()
    c = orc.OracleCopy(t.types, t.root_type, t.roots, 64, 1 << 40)
    t1 = time.perf_counter()
    c.run_kernel(1.0001, 0.5, iters=passes, select="chain", chain=chain)
    c.run_kernel(1.0001, 0.5, iters=passes, select="chain", chain=chain)
    t2 = time.perf_counter()
    c.copy_back()
    t3 = time.perf_counter()
    kernel_bytes = 2 * 2 * leaf * passes
    return {"value": round(kernel_bytes / (t2 - t1) / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"linear chain k=8, 2^24 FP64: deep copy, {passes} fma passes x 2 modes, copy back; "
                      f"credited with the GPU passes' bytes (2 x leaf per pass), although the oracle keeps each "
                      f"element in a register across its passes and moves the leaf once per run: an fma-latency "
                      f"rate, not memory bandwidth (deep copy {t1 - t0:.3f} s, copy back {t3 - t2:.3f} s)",
            "seconds": round(t3 - t0, 3)}


def bench_linear(args, torch, dc):
    import fixtures as fx
    t = fx.linear()
    ctx = dc.Context(0)
    schema = dc.Schema(t.types)
    plan = dc.Plan(schema, t.root_type, t.roots)
    info = plan.info()
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    chain = [(1, 0)] * 7 + [(0, 0)]
    leaf = info.leaf_bytes
    P = args.passes

    tree = dc.Tree(ctx, plan, arena, scratch)  # pack + H2D + attach
    tree.resolve_chain(chain)
    tree.detach()  # the marshalled image, host pointers in it, resident in HBM
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(rec):
        e = [ev() for _ in range(6)]
        e[0].record(s)
        tree.attach()
        e[1].record(s)
        tree.run_kernel(mode="resolved", select="chain", chain=chain, iters=P, a=1.0001, b=0.5)
        e[2].record(s)
        tree.run_kernel(mode="deref_each", select="chain", chain=chain, iters=P, a=1.0001, b=0.5)
        e[3].record(s)
        tree.detach()
        e[4].record(s)
        rec.append(e)

    for _ in range(args.warmup):
        step([])
    torch.cuda.synchronize()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = [r[0].elapsed_time(r[4]) / 1e3 for r in recs]
    attach_s = [r[0].elapsed_time(r[1]) / 1e3 for r in recs]
    res_s = [r[1].elapsed_time(r[2]) / 1e3 for r in recs]
    der_s = [r[2].elapsed_time(r[3]) / 1e3 for r in recs]
    detach_s = [r[3].elapsed_time(r[4]) / 1e3 for r in recs]
    tree.check()

    reloc_bytes = info.nslots_nonnull * 16 + info.nslots * 8 + info.nobjects * 16
    kernel_bytes = 2 * leaf * P
    step_bytes = 2 * kernel_bytes + 2 * reloc_bytes
    dev_time = sum(step_s)
    value = step_bytes * len(step_s) / dev_time / 1e9
    res_gbps = 2 * leaf / (sum(res_s) / len(res_s) / P) / 1e9
    der_gbps = 2 * leaf / (sum(der_s) / len(der_s) / P) / 1e9
    dominant = "deref_each" if sum(der_s) > sum(res_s) else "resolved"
    dom_t = (sum(der_s) if dominant == "deref_each" else sum(res_s)) / len(step_s) / P
    achieved = 2 * leaf / dom_t / 1e9
    out = {
        "metric": "deep-copy+kernel effective GB/s vs HBM/link roofline; p50/p99 latency",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * dev_time / len(step_s), 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"linear chain: 8 nested structs, LLinit, FP64 leaf of 2^24 elements, "
                               f"{P} fma passes resolved + {P} per-access deref, attach/detach on device",
                   "k": 8, "n": 1 << 24, "passes": P, "leaf_bytes": leaf, "arena_bytes": plan.arena_bytes},
        "roofline": {"bound": "hbm", "kernel": f"k_stream_{'deref' if dominant == 'deref_each' else 'resolved'}",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic("linear", "k_stream_deref" if dominant == "deref_each" else "k_stream_resolved"),
                     "bytes_per_launch": 2 * leaf, "avg_launch_us": round(dom_t * 1e6, 3)},
        "latency_ms": {"p50": round(1e3 * pct(step_s, 50), 4), "p99": round(1e3 * pct(step_s, 99), 4)},
        "modes": {"resolved_GBps": round(res_gbps, 1), "deref_each_GBps": round(der_gbps, 1),
                  "deref_over_resolved_time": round(sum(der_s) / sum(res_s), 3),
                  "attach_us": round(1e6 * pct(attach_s, 50), 2), "detach_us": round(1e6 * pct(detach_s, 50), 2)},
        "wall_s": round(wall, 3),
    }

    # single passes with the 256 MB Infinity Cache flushed before each: a
    # 512 MiB fill between passes evicts the 128 MiB leaf
    tree.attach()
    addr, count, kind = tree.resolve_chain(chain)
    ch = dc.Chain(addr, count, dc.KIND[kind], 0)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    fl = {"resolved": [], "deref_each": []}
    for r in range(2 * 10):
        mode = "resolved" if r % 2 == 0 else "deref_each"
        flush.fill_(r & 0xFF)
        e0, e1 = ev(), ev()
        e0.record(s)
        if mode == "resolved":   # the resolved address, no resolve kernel in the pass
            dc._check(dc.load().dc_chain_run_kernel(ctx.h, ctypes.byref(ch), 1, 1.0001, 0.5,
                                                    float(np.float32(1.0001)), 0.5, s.cuda_stream),
                      "dc_chain_run_kernel")
        else:
            tree.run_kernel(mode="deref_each", select="chain", chain=chain, iters=1, a=1.0001, b=0.5)
        e1.record(s)
        torch.cuda.synchronize()
        fl[mode].append(e0.elapsed_time(e1) / 1e3)
    tree.check()
    tree.detach()
    del flush
    out["mall_flushed"] = {"what": "one pass after a 512 MiB fill (Infinity Cache evicted), median of 10",
                           "resolved_GBps": round(2 * leaf / pct(fl["resolved"], 50) / 1e9, 1),
                           "deref_each_GBps": round(2 * leaf / pct(fl["deref_each"], 50) / 1e9, 1)}

    if not args.no_link:
        # the host-link part: pack + host-to-device + relocation, then copy back;
        # steady state: the first deep copies of a process run slower (8 to
        # 46 GB/s over the first four on this tree), so two untimed ones first
        h2d, d2h, e2e = [], [], []
        peak = link_peak(torch)
        for r in range(LINK_WARMUP + LINK_REPS):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr = dc.Tree(ctx, plan, arena, scratch)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tr.run_kernel(mode="resolved", select="chain", chain=chain, iters=P, a=1.0001, b=0.5)
            tr.run_kernel(mode="deref_each", select="chain", chain=chain, iters=P, a=1.0001, b=0.5)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tr.copy_back()
            t3 = time.perf_counter()
            tr.release()
            if r < LINK_WARMUP:
                continue
            h2d.append(plan.arena_bytes / (t1 - t0) / 1e9)
            d2h.append(leaf / (t3 - t2) / 1e9)
            e2e.append(t3 - t0)
        mh, md_ = pct(h2d, 50), pct(d2h, 50)
        out["host_link"] = {"what": f"median of {LINK_REPS} deep copies after {LINK_WARMUP} untimed",
                            "h2d_GBps": round(mh, 2), "d2h_GBps": round(md_, 2),
                            "h2d_runs": [round(x, 2) for x in h2d], "d2h_runs": [round(x, 2) for x in d2h],
                            "pinned_peak_h2d_GBps": round(peak["h2d"], 2), "pinned_peak_d2h_GBps": round(peak["d2h"], 2),
                            "spec_peak_GBps": LINK_PEAK_GBPS,
                            "h2d_frac_of_spec": round(mh / LINK_PEAK_GBPS, 4),
                            "d2h_frac_of_spec": round(md_ / LINK_PEAK_GBPS, 4),
                            "h2d_frac_of_measured": round(mh / peak["h2d"], 4),
                            "d2h_frac_of_measured": round(md_ / peak["d2h"], 4)}
        job_bytes = plan.arena_bytes + leaf + 2 * kernel_bytes
        out["end_to_end"] = {"what": "pack + H2D + attach + both kernels + copy back, host buffers in and out",
                             "GBps": round(job_bytes / pct(e2e, 50) / 1e9, 2),
                             "p50_ms": round(1e3 * pct(e2e, 50), 3), "p99_ms": round(1e3 * pct(e2e, 99), 3)}
    return out


def bench_wide(args, torch, dc):
    """The wide tree at its stated parameters (leaf lengths up to 65536,
    ~0.28 GB) and the wide-1G variant (up to 2^18, ~0.93 GB)."""
    out = _bench_wide(args, torch, dc, 65536)
    big = _bench_wide(args, torch, dc, 1 << 18)
    out["wide_1g"] = {k: big[k] for k in ("value", "ms_per_step", "config", "roofline", "relocation_us_p50",
                                           "host_link") if k in big}
    return out


def _bench_wide(args, torch, dc, hi):
    """The wide tree (64 x 64 leaves, lengths log-uniform 256..hi, FP32 and
    FP64): step = attach + one fma pass over every leaf + detach."""
    import fixtures as fx
    t = fx.wide(hi=hi)
    ctx = dc.Context(0)
    plan = dc.Plan(dc.Schema(t.types), t.root_type, t.roots)
    info = plan.info()
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    tree = dc.Tree(ctx, plan, arena, scratch)
    tree.detach()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    recs = []
    for i in range(args.warmup + args.steps):
        e = [ev() for _ in range(4)]
        e[0].record(s)
        tree.attach()
        e[1].record(s)
        tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
        e[2].record(s)
        tree.detach()
        e[3].record(s)
        if i >= args.warmup:
            recs.append(e)
    torch.cuda.synchronize()
    tree.check()
    step_s = [r[0].elapsed_time(r[3]) / 1e3 for r in recs]
    ker_s = [r[1].elapsed_time(r[2]) / 1e3 for r in recs]
    rel_s = [(r[0].elapsed_time(r[1]) + r[2].elapsed_time(r[3])) / 1e3 for r in recs]
    kb = 2 * info.leaf_bytes
    rb = 2 * (info.nslots_nonnull * 16 + info.nslots * 8 + info.nobjects * 16)
    out = {"metric": "deep-copy+kernel effective GB/s vs HBM/link roofline; p50/p99 latency",
           "value": round((kb + rb) / (sum(step_s) / len(step_s)) / 1e9, 2), "unit": "GB/s",
           "ms_per_step": round(1e3 * sum(step_s) / len(step_s), 4), "steps": args.steps, "dtype": "f32+f64",
           "config": {"workload": f"wide tree 64x64 leaves, log-uniform 256..{hi} elements, half FP32 half FP64",
                      "leaf_bytes": info.leaf_bytes, "arena_bytes": plan.arena_bytes, "nleaves": info.nleaves},
           "roofline": {"bound": "hbm", "kernel": "k_leaf_tiles", "achieved": round(kb / pct(ker_s, 50) / 1e9, 1),
                        "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": round(kb / pct(ker_s, 50) / 1e9 / HBM_PEAK_GBPS, 4),
                        "traffic": traffic("wide" if hi == 65536 else f"wide_hi{hi}", "k_leaf_tiles")},
           "relocation_us_p50": round(1e6 * pct(rel_s, 50), 2),
           "latency_ms": {"p50": round(1e3 * pct(step_s, 50), 4), "p99": round(1e3 * pct(step_s, 99), 4)}}
    if not args.no_link:
        ts = []
        for r in range(LINK_WARMUP + LINK_REPS):   # steady state, as for the Linear tree
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr = dc.Tree(ctx, plan, arena, scratch)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tr.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tr.copy_back()
            t3 = time.perf_counter()
            tr.release()
            if r >= LINK_WARMUP:
                ts.append((t1 - t0, t2 - t1, t3 - t2))
        h2d = plan.arena_bytes / pct([a for a, _, _ in ts], 50) / 1e9
        d2h = info.leaf_bytes / pct([c for _, _, c in ts], 50) / 1e9
        out["host_link"] = {"h2d_GBps": round(h2d, 2), "h2d_frac_of_spec": round(h2d / LINK_PEAK_GBPS, 4),
                            "d2h_GBps": round(d2h, 2), "d2h_frac_of_spec": round(d2h / LINK_PEAK_GBPS, 4),
                            "end_to_end_ms_p50": round(1e3 * pct([a + b + c for a, b, c in ts], 50), 3)}
    return out


def bench_plain(args, torch, dc, reps=1000):
    """The plain structure (root -> 16 children -> 1024 FP64 each): the whole
    job, host tree in and host tree out (pack + H2D + attach + one fma pass
    over every leaf + copy back), 1000 times. Launch- and latency-bound: 131 KB
    of payload; the plan is made once and reused, as for repeated copies of
    one shape."""
    import fixtures as fx
    t = fx.plain()
    ctx = dc.Context(0)
    plan = dc.Plan(dc.Schema(t.types), t.root_type, t.roots)
    info = plan.info()
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    lat = []
    for r in range(reps + 20):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree = dc.Tree(ctx, plan, arena, scratch)
        tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
        tree.copy_back()
        t1 = time.perf_counter()
        tree.release()
        if r >= 20:
            lat.append(t1 - t0)
    job = info.payload_bytes + info.leaf_bytes + 2 * info.leaf_bytes
    return {"metric": "deep-copy+kernel effective GB/s vs HBM/link roofline; p50/p99 latency",
            "value": round(job / pct(lat, 50) / 1e9, 3), "unit": "GB/s", "steps": reps, "dtype": "f64",
            "config": {"workload": "plain: root -> 16 children -> 1024 FP64 each, whole job host to host",
                       "payload_bytes": info.payload_bytes, "arena_bytes": plan.arena_bytes},
            "latency_ms": {"p50": round(1e3 * pct(lat, 50), 4), "p99": round(1e3 * pct(lat, 99), 4)},
            "note": "launch- and latency-bound; no roofline"}


def _batched_vs_plain(torch, dc, ctx, t, tune, nsub):
    """The first nsub simulations two ways, device-resident and staged: one
    plan over all of them run as the batched form (one graph replay), and one
    plan per simulation, each with its own attach, leaf pass and detach."""
    schema = dc.Schema(t.types)
    s = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    plan = dc.Plan(schema, t.root_type, t.roots[:nsub])
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    if tune is None:   # this plan's own choice
        tune = tree.autotune(reps=2)
    g = tree.graph(a=1.0001, b=0.5, tune=tune)
    g.launch()
    e0, e1 = ev(), ev()
    e0.record(s)
    for _ in range(5):
        g.launch()
    e1.record(s)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / 5
    leaf = plan.info().leaf_bytes
    g.close()
    tree.release()
    del arena, scratch
    trees = []
    for r in t.roots[:nsub]:
        p = dc.Plan(schema, t.root_type, [r])
        a = torch.empty(p.arena_bytes, dtype=torch.uint8, device="cuda")
        sc = torch.empty(p.scratch_bytes, dtype=torch.uint8, device="cuda")
        trees.append((p, a, sc, dc.Tree(ctx, p, a, sc, relocate=False)))
    for _, _, _, tr in trees:   # warm: tile lists built
        tr.attach()
        tr.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
        tr.detach()
    torch.cuda.synchronize()
    e0.record(s)
    for _, _, _, tr in trees:
        tr.attach()
        tr.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
        tr.detach()
    e1.record(s)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    for _, _, _, tr in trees:
        tr.release()
    return {"simulations": nsub, "tune": tune, "batched_ms": round(batched_ms, 3), "per_structure_ms": round(plain_ms, 3),
            "batched_GBps": round(2 * leaf / batched_ms / 1e6, 1), "per_structure_GBps": round(2 * leaf / plain_ms / 1e6, 1),
            "speedup": round(plain_ms / batched_ms, 2)}


def host_cpu():
    """Model name and the number of CPUs this process may run on."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def md_step_bytes(info):
    """Algorithmic bytes of one batched step: every leaf byte read and written
    once, and per relocation (attach, then detach) 8 B read + 8 B written per
    non-null slot, 8 B read per null slot and 16 B per target entry."""
    return 2 * info.leaf_bytes + 2 * (info.nslots_nonnull * 16 + info.nslots * 8 + info.nobjects * 16)


def cpu_baseline_md(t, nsample, max_threads=16):
    """The CPU oracle on the batched MD workload: its deep copy (walk, layout,
    copy into its own buffer, relocation), one fma pass over every leaf and
    the copy back, timed together. One thread over the first `nsample`
    simulations; then every simulation on all the CPUs this process may use
    (at most max_threads), each thread running the oracle on its own
    contiguous share of the simulations (they are independent structures).
    Bytes credited: the GPU step's algorithmic bytes for the same
    simulations (the oracle moves each leaf byte once per pass: one read, one
    write)."""
    import threading
    import fixtures as fx  # noqa: F401  (the tree is already built)
    import oracle as orc
    from paper_1906_01128_amd import dc

    schema = dc.Schema(t.types)

    def step_bytes(roots):
        p = dc.Plan(schema, t.root_type, roots)
        b = md_step_bytes(p.info())
        p.close()
        return b

    def run(roots, out, k):
        t0 = time.perf_counter()
        c = orc.OracleCopy(t.types, t.root_type, roots, 64, 1 << 40)
        t1 = time.perf_counter()
        c.run_kernel(1.0001, 0.5, iters=1, select="all")
        t2 = time.perf_counter()
        c.copy_back()
        t3 = time.perf_counter()
        c.free()
        out[k] = (t1 - t0, t2 - t1, t3 - t2)

    model, ncpu = host_cpu()
    roots1 = t.roots[:nsample]
    r1 = [None]
    run(roots1, r1, 0)
    s1 = sum(r1[0])
    b1 = step_bytes(roots1)
    nth = max(1, min(ncpu, max_threads))
    shares = [t.roots[i * len(t.roots) // nth:(i + 1) * len(t.roots) // nth] for i in range(nth)]
    rn = [None] * nth
    ths = [threading.Thread(target=run, args=(sh, rn, k)) for k, sh in enumerate(shares)]
    t0 = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    sn = time.perf_counter() - t0
    bn = step_bytes(t.roots)
    return {"value": round(bn / sn / 1e9, 3), "unit": "GB/s", "cores": nth, "kind": "oracle",
            "sample": f"all {len(t.roots)} simulations, {nth} threads each running the oracle on its own share "
                      f"(deep copy with relocation + one fma pass + copy back, {sn:.2f} s); credited with the GPU "
                      f"step's algorithmic bytes ({bn} B)",
            "cpu_model": model, "cpus_available": ncpu,
            "single_thread": {"value": round(b1 / s1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                              "sample": f"first {nsample} simulations, one thread",
                              "deep_copy_s": round(r1[0][0], 3), "kernel_s": round(r1[0][1], 3),
                              "copy_back_s": round(r1[0][2], 3), "bytes": b1},
            "seconds": round(s1 + sn, 2)}


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def bench_batched(args, torch, dc):
    """The batched MD workload: 10,000 simulations, ~7.75 M arrays, ~12 GB.
    Step = one replay of the captured graph that attaches every pointer,
    runs fma over every leaf and detaches again, in the form and shape the
    autotuner measured fastest (one persistent launch taking a whole
    relocation unit per item, one persistent launch in three phases, or
    three ordinary launches)."""
    import fixtures as fx
    fx.set_threads(0)
    t0 = time.perf_counter()
    t = fx.md()
    log(args, f"md built in {time.perf_counter() - t0:.1f} s")
    ctx = dc.Context(0)
    schema = dc.Schema(t.types)
    t0 = time.perf_counter()
    plan = dc.Plan(schema, t.root_type, t.roots)
    plan_s = time.perf_counter() - t0
    info = plan.info()
    log(args, f"planned in {plan_s:.2f} s: {info.nobjects} objects, {info.nsegments} units, "
              f"{info.arena_bytes / 1e9:.2f} GB, unit leaf runs {info.unit_leaves}")
    arena = torch.empty(plan.arena_bytes, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    torch.cuda.synchronize()
    stage_s = time.perf_counter() - t0
    tune = tree.autotune(reps=3)
    table = tree.autotune_results()
    log(args, f"autotuner: {tune} ({len(table)} candidates)")
    # the autotuner ran the kernel on the staged image; stage it again so
    # that the timed steps start from the workload's values
    tree.release()
    tree = dc.Tree(ctx, plan, arena, scratch, relocate=False)
    g = tree.graph(a=1.0001, b=0.5, tune=tune)
    step_bytes = md_step_bytes(info)

    # the timed region: W untimed replays, then exactly K, events around each
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    ev = _events(torch, 2 * args.steps)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        ev[2 * i].record(s)
        g.launch()
        ev[2 * i + 1].record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    step_s = [ev[2 * i].elapsed_time(ev[2 * i + 1]) / 1e3 for i in range(args.steps)]
    g.close()
    tree.check()
    mean_s = sum(step_s) / len(step_s)
    value = step_bytes / mean_s / 1e9

    form = {0: "one persistent launch, one relocation unit per item" if info.unit_leaves else
               "one persistent launch in three phases",
            1: "three launches (relocate, every leaf, reverse relocate)",
            2: "one persistent launch in three phases",
            3: "one fused launch: every tile relocates the slots of its own leaves",
            4: "one persistent fused launch: workgroups take tiles, which relocate the slots of their own "
               "leaves, from eight device queues"}[tune["launches"]]
    if tune["launches"] == 1:
        # the compute launch of the graph, timed as separate launches
        kname, kbytes = "k_leaf_tiles", 2 * info.leaf_bytes
        tree.attach()
        tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)  # builds its tile list
        ks = []
        for _ in range(5):
            e = _events(torch, 2)
            e[0].record(s)
            tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.5)
            e[1].record(s)
            torch.cuda.synchronize()
            ks.append(e[0].elapsed_time(e[1]) / 1e3)
        tree.detach()
        k_s = sum(ks) / len(ks)
        k_what = "k_leaf_tiles timed as separate launches beside the graph"
    elif tune["launches"] in (3, 4):
        # the graph's one launch, timed as separate launches of the same form
        # (the persistent one after its one-workgroup queue reset)
        kname, kbytes = ("k_fused" if tune["launches"] == 3 else "k_fused_persistent"), step_bytes
        tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=tune)
        ks = []
        for _ in range(5):
            e = _events(torch, 2)
            e[0].record(s)
            tree.batch_run(a=1.0001, b=0.5, attach=True, detach=True, tune=tune)
            e[1].record(s)
            torch.cuda.synchronize()
            ks.append(e[0].elapsed_time(e[1]) / 1e3)
        k_s = sum(ks) / len(ks)
        k_what = (f"{kname} (relocation and compute in one launch) timed as separate launches beside the graph"
                  + (", each after its queue reset" if tune["launches"] == 4 else ""))
    else:
        kname = "k_batch_units" if (tune["launches"] == 0 and info.unit_leaves) else "k_batch"
        kbytes, k_s = step_bytes, mean_s
        k_what = (f"{kname} is the whole step: its average launch time is the events' time around each graph "
                  f"replay (which also holds a one-thread counter reset)")
    k_ach = kbytes / k_s / 1e9
    out = {"metric": "deep-copy+kernel effective GB/s vs HBM/link roofline; p50/p99 latency",
           "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * mean_s, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched MD: 10,000 structures sim -> cells U{8..512} -> Poisson(64) atoms -> "
                                  "pos/vel/force double3 (~12 GB); step = one HIP graph replay of attach + "
                                  "fma(x, 1.0001, 0.5) over every leaf + detach, image resident in HBM",
                      "simulations": len(t.roots), "objects": info.nobjects, "slots": info.nslots,
                      "slots_nonnull": info.nslots_nonnull, "relocation_units": info.nsegments,
                      "leaf_bytes": info.leaf_bytes, "arena_bytes": plan.arena_bytes, "step_bytes": step_bytes,
                      "form": form, "tune": tune},
           "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(k_ach, 1), "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": round(k_ach / HBM_PEAK_GBPS, 4),
                        "traffic": traffic("batched", kname), "bytes_per_launch": kbytes,
                        "avg_launch_us": round(1e6 * k_s, 1), "how": k_what},
           "latency_ms": {"p50": round(1e3 * pct(step_s, 50), 4), "p99": round(1e3 * pct(step_s, 99), 4)},
           "wall_s": round(wall, 4),
           "autotuner": [dict(tu, us=round(us, 1)) for tu, us in table],
           "host": {"plan_s": round(plan_s, 3), "stage_s": round(stage_s, 3)}}

    if not args.no_secondary:
        out.update(_batched_secondary(args, torch, dc, ctx, t, plan, tree, info, table))
    if not args.no_link:
        out["host_link"] = _md_host_link(torch, dc, ctx, plan, arena, scratch, info)
    tree.release()
    del arena, scratch
    torch.cuda.empty_cache()
    if not args.no_secondary:
        lin = bench_linear(argparse.Namespace(**dict(vars(args), steps=5, warmup=2)), torch, dc)
        out["linear_chain"] = {k: lin[k] for k in ("value", "ms_per_step", "config", "roofline", "modes",
                                                   "mall_flushed", "host_link") if k in lin}
    if not args.no_cpu_baseline:
        log(args, "cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_md(t, nsample=3000)
    return out


def _md_host_link(torch, dc, ctx, plan, arena, scratch, info, reps=3):
    """The deep copy of the whole MD workload over the host link: pack +
    host-to-device + attach (dc_deep_copy_to_device), and the copy back of
    every leaf (device-to-host + scatter into the host tree); medians of
    `reps` after one untimed round."""
    peak = link_peak(torch)
    h2d, d2h = [], []
    for r in range(1 + reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = dc.Tree(ctx, plan, arena, scratch)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tr.copy_back()
        t2 = time.perf_counter()
        tr.release()
        if r:
            h2d.append(plan.arena_bytes / (t1 - t0) / 1e9)
            d2h.append(info.leaf_bytes / (t2 - t1) / 1e9)
    a, b = pct(h2d, 50), pct(d2h, 50)
    return {"what": f"median of {reps}: deep copy (pack + H2D + attach) of the {plan.arena_bytes} B arena, and copy "
                    f"back of the {info.leaf_bytes} B of leaves (D2H + scatter)",
            "h2d_GBps": round(a, 2), "d2h_GBps": round(b, 2), "h2d_runs": [round(x, 2) for x in h2d],
            "d2h_runs": [round(x, 2) for x in d2h],
            "pinned_peak_h2d_GBps": round(peak["h2d"], 2), "pinned_peak_d2h_GBps": round(peak["d2h"], 2),
            "spec_peak_GBps": LINK_PEAK_GBPS, "h2d_frac_of_spec": round(a / LINK_PEAK_GBPS, 4),
            "d2h_frac_of_spec": round(b / LINK_PEAK_GBPS, 4), "h2d_frac_of_measured": round(a / peak["h2d"], 4),
            "d2h_frac_of_measured": round(b / peak["d2h"], 4)}


def _whole_job_graph(torch, tree, plan, info, table, reps=3):
    """The whole batched job as one HIP graph: the staged image host to
    device, the fastest form's attach + pass + detach, the arena device to
    host, each transfer one copy from or into a page-locked buffer of the
    arena's size; medians of `reps` replays after an untimed one."""
    tune = min(table, key=lambda tu_us: tu_us[1])[0]
    s = torch.cuda.current_stream()
    g = tree.graph(a=1.0001, b=0.5, tune=tune, upload=True, download=True)
    ts = []
    for r in range(1 + reps):
        e = _events(torch, 2)
        e[0].record(s)
        g.launch()
        e[1].record(s)
        torch.cuda.synchronize()
        if r:
            ts.append(e[0].elapsed_time(e[1]) / 1e3)
    g.close()
    tree.check()
    t_s = pct(ts, 50)
    link = 2 * plan.arena_bytes / t_s / 1e9
    return {"what": f"one graph replay: {plan.arena_bytes} B image in, attach + pass + detach ({tune}), the "
                    f"arena out; median of {reps} after one untimed",
            "ms": round(1e3 * t_s, 2),
            # the two copies run one after the other: both images' bytes over the replay's time
            "link_GBps": round(link, 2), "link_frac_of_spec": round(link / LINK_PEAK_GBPS, 4)}


def _batched_secondary(args, torch, dc, ctx, t, plan, tree, info, table):
    """Beside the timed step: each batched form's best autotuner time, the
    MD kick-drift kernel and the first 500 simulations one structure per
    call against one graph replay."""
    s = torch.cuda.current_stream()
    step_bytes = md_step_bytes(info)
    best = {}
    for tu, us in table:
        key = {0: "persistent_units" if info.unit_leaves else "persistent_phased", 1: "three_launches",
               2: "persistent_phased", 3: "fused", 4: "persistent_fused"}[tu["launches"]]
        if key not in best or us < best[key]["us"]:
            best[key] = dict(tu, us=round(us, 1), GBps=round(step_bytes / us / 1e3, 1))
    # attach and detach alone (the relocation kernel), medians of 5
    rel = {"attach": [], "detach": []}
    for _ in range(6):
        for what in ("attach", "detach"):
            e = _events(torch, 2)
            e[0].record(s)
            getattr(tree, what)()
            e[1].record(s)
            torch.cuda.synchronize()
            rel[what].append(e[0].elapsed_time(e[1]) / 1e3)
    rel_bytes = info.nslots_nonnull * 16 + info.nslots * 8 + info.nobjects * 16   # algorithmic, as in the step
    att_s, det_s = pct(rel["attach"][1:], 50), pct(rel["detach"][1:], 50)
    tree.check()
    # the MD kick-drift kernel on the same cells: v += f dt/m, x += v dt
    tree.attach()
    dt = 1e-3
    tree.kick_drift(1, 0, 1, 2, dt, dt / 39.948, steps=1)   # builds the element list
    kd = []
    for _ in range(5):
        e = _events(torch, 2)
        e[0].record(s)
        tree.kick_drift(1, 0, 1, 2, dt, dt / 39.948, steps=1)
        e[1].record(s)
        torch.cuda.synchronize()
        kd.append(e[0].elapsed_time(e[1]) / 1e3)
    tree.check()
    tree.detach()
    kd_bytes = 40 * (info.leaf_bytes // 24)    # per double of x: read x, v, f; write x, v
    kd_gbps = kd_bytes / pct(kd, 50) / 1e9
    try:
        whole = _whole_job_graph(torch, tree, plan, info, table)
    except dc.DcError as e:   # two page-locked buffers of the arena's size: reported, not fatal to the line
        whole = {"error": str(e)}
    plain = _batched_vs_plain(torch, dc, ctx, t, None, nsub=500)
    return {"forms": best, "whole_job_graph": whole,
            "relocation": {"kernel": "k_relocate", "attach_us": round(1e6 * att_s, 1), "detach_us": round(1e6 * det_s, 1),
                           "bytes_per_launch": rel_bytes, "achieved_GBps": round(rel_bytes / att_s / 1e9, 1),
                           "frac": round(rel_bytes / att_s / 1e9 / HBM_PEAK_GBPS, 4),
                           "traffic": traffic("batched", "k_relocate"),
                           "bytes": "8 B read + 8 B written per non-null slot, 8 B read per null slot, 16 B per "
                                    "object (its target entry); the 2-byte target index per slot is not counted"},
            "kick_drift": {"kernel": "k_kick_drift", "ms": round(1e3 * pct(kd, 50), 3),
                           "bytes_per_launch": kd_bytes, "achieved_GBps": round(kd_gbps, 1),
                           "frac": round(kd_gbps / HBM_PEAK_GBPS, 4), "traffic": traffic("batched", "k_kick_drift")},
            "one_structure_per_call": plain}


def _served_run(dc, ctx, schema, pool, sizes, jobs, outs, lam, budget):
    """Submits the jobs at Poisson times of rate lam (jobs/s; 0: all at once)
    and waits for all; returns the latencies, the stats and the wall time."""
    import random
    rng = random.Random(7)
    srv = dc.Server(ctx, schema, budget_bytes=budget, max_inflight=16, nstreams=4)
    t0 = time.perf_counter()
    ids = []
    next_t = 0.0
    for si, key, a, b in jobs:
        if lam > 0:
            next_t += rng.expovariate(lam)
            while time.perf_counter() - t0 < next_t:
                time.sleep(0.0002)
        o = outs[si]
        ids.append(srv.submit(pool[si].root_type, pool[si].roots[0], o.ctypes.data, o.nbytes, a, b, key=key))
    res = [srv.wait(i) for i in ids]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return [r.t_done - r.t_submit for r in res], st, wall


def bench_served(args, torch, dc, budget=200 * 10 ** 9):
    """Served jobs: Poisson arrivals of broom structures (depth U{2..8},
    fan-out U{1..64}, leaf bytes log-uniform 4 KiB..bytes_hi, FP32 or FP64),
    half of them reusing a resident structure from a pool of 64: first all at
    once (the server's capacity in jobs/s), then at Poisson offered loads of
    0.5, 0.8 and 0.95 of that capacity (stable queues: latency, not backlog),
    then the same jobs one structure per call. Jobs on one structure share one
    result buffer (results are checked by the tests, not here), written
    before the clock starts."""
    import random
    import fixtures as fx
    njobs = 2000 if args.full else 400
    bytes_hi = (256 << 20) if args.full else (64 << 20)
    rng = random.Random(190601132)
    fx.set_threads(0)
    pool = [fx.broom(seed=190601132 + i, bytes_lo=4096, bytes_hi=bytes_hi) for i in range(64)]
    schema = dc.Schema(pool[0].types)
    ctx = dc.Context(0)
    sizes = []
    for t in pool:
        p = dc.Plan(schema, t.root_type, t.roots)
        sizes.append((p.arena_bytes, p.info().out_bytes))
    jobs = []
    for j in range(njobs):
        si = rng.randrange(64)
        reuse = rng.random() < 0.5
        jobs.append((si, (si + 1) if reuse else 0, rng.choice([1.0001, 0.9999]), rng.choice([0.5, -0.25])))
    outs = [np.ones(max(sz[1], 1), np.uint8) for sz in sizes]
    peak = link_peak(torch)
    cap = min(peak["h2d"], peak["d2h"]) * 1e9      # measured link capacity, bytes/s per direction
    lat, st, wall = _served_run(dc, ctx, schema, pool, sizes, jobs, outs, 0, budget)
    moved = st.h2d_bytes + st.d2h_bytes
    cap_jobs = njobs / wall                        # the server's capacity, jobs/s
    log(args, f"served capacity: {cap_jobs:.1f} jobs/s ({wall:.2f} s)")
    loads = {}
    for rho in (0.5, 0.8, 0.95):
        l2, s2, w2 = _served_run(dc, ctx, schema, pool, sizes, jobs, outs, rho * cap_jobs, budget)
        log(args, f"served rho={rho}: wall {w2:.2f} s, p50 {1e3 * pct(l2, 50):.1f} ms")
        loads[str(rho)] = {"offered_jobs_per_s": round(rho * cap_jobs, 2), "p50_ms": round(1e3 * pct(l2, 50), 3),
                           "p99_ms": round(1e3 * pct(l2, 99), 3), "wall_s": round(w2, 3),
                           "h2d_GBps": round(s2.h2d_bytes / w2 / 1e9, 2), "d2h_GBps": round(s2.d2h_bytes / w2 / 1e9, 2),
                           "reused": s2.reused, "evictions": s2.evictions, "peak_bytes": s2.peak_bytes}
    capacity = {"wall_s": round(wall, 3), "jobs_per_s": round(njobs / wall, 1),
                "h2d_GBps": round(st.h2d_bytes / wall / 1e9, 2), "d2h_GBps": round(st.d2h_bytes / wall / 1e9, 2),
                "busier_direction_frac_of_measured": round(max(st.h2d_bytes, st.d2h_bytes) / wall / cap, 4),
                "busier_direction_frac_of_spec": round(max(st.h2d_bytes, st.d2h_bytes) / wall / 1e9 / LINK_PEAK_GBPS, 4)}
    # the same jobs at capacity with page-locked output buffers, which the
    # server fills by direct copies from the device
    outs_pinned = [torch.zeros(max(sz[1], 1), dtype=torch.uint8, pin_memory=True).numpy() for sz in sizes]
    _, stp, wallp = _served_run(dc, ctx, schema, pool, sizes, jobs, outs_pinned, 0, budget)
    del outs_pinned
    capacity["pinned_outputs"] = {
        "wall_s": round(wallp, 3), "jobs_per_s": round(njobs / wallp, 1),
        "h2d_GBps": round(stp.h2d_bytes / wallp / 1e9, 2), "d2h_GBps": round(stp.d2h_bytes / wallp / 1e9, 2),
        "busier_direction_frac_of_measured": round(max(stp.h2d_bytes, stp.d2h_bytes) / wallp / cap, 4),
        "busier_direction_frac_of_spec": round(max(stp.h2d_bytes, stp.d2h_bytes) / wallp / 1e9 / LINK_PEAK_GBPS, 4)}
    log(args, f"served capacity, pinned outputs: {njobs / wallp:.1f} jobs/s ({wallp:.2f} s)")
    # the plain path: one structure per call, back to back, no residency
    plain_lat = []
    t0 = time.perf_counter()
    for si, key, a, b in jobs[: min(njobs, 200)]:
        ta = time.perf_counter()
        plan = dc.Plan(schema, pool[si].root_type, pool[si].roots)
        arena = torch.empty(max(plan.arena_bytes, 16), dtype=torch.uint8, device="cuda")
        scratch = torch.empty(max(plan.scratch_bytes, 16), dtype=torch.uint8, device="cuda")
        d_out = torch.empty(max(sizes[si][1], 16), dtype=torch.uint8, device="cuda")
        tree = dc.Tree(ctx, plan, arena, scratch)
        tree.run_kernel(mode="resolved", select="all", iters=1, a=a, b=b, out=d_out)
        torch.from_numpy(outs[si][: sizes[si][1]]).copy_(d_out[: sizes[si][1]])
        plain_lat.append(time.perf_counter() - ta)
        tree.release()
        del arena, scratch, d_out
    plain_wall = time.perf_counter() - t0
    main = loads["0.8"]
    return {"metric": "deep-copy+kernel effective GB/s vs HBM/link roofline; p50/p99 latency",
            "value": round((moved + st.kernel_bytes) / wall / 1e9, 2), "unit": "GB/s",
            "config": {"workload": f"served: {njobs} jobs, broom trees depth U{{2..8}} fan-out U{{1..64}}, leaf bytes "
                                   f"log-uniform 4KiB..{bytes_hi}, reuse 0.5 over 64 structures, budget {budget}; "
                                   f"value = all jobs submitted at once (capacity)"},
            "latency_ms": {"p50": main["p50_ms"], "p99": main["p99_ms"],
                           "at_offered_load": "0.8 of the measured capacity in jobs/s"},
            "link": {"measured_capacity_GBps": round(cap / 1e9, 2), "spec_GBps": LINK_PEAK_GBPS, **capacity},
            "offered_load": loads,
            "plain_path": {"jobs": len(plain_lat), "jobs_per_s": round(len(plain_lat) / plain_wall, 1),
                           "p50_ms": round(1e3 * pct(plain_lat, 50), 3), "p99_ms": round(1e3 * pct(plain_lat, 99), 3)},
            "server": {"completed": st.completed, "reused": st.reused, "evictions": st.evictions,
                       "admitted_while_busy": st.batches, "peak_bytes": st.peak_bytes}}


def _time_marshal(torch, dc, ctx, t, chains, allused, reps):
    """Marshalling (Algorithm 1): plan the whole tree, pack, copy to the
    device, relocate; one kernel pass over the used arrays; copy back."""
    s = torch.cuda.current_stream()
    rows = []
    schema = dc.Schema(t.types)
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = dc.Plan(schema, t.root_type, t.roots)
        arena = torch.empty(max(plan.arena_bytes, 16), dtype=torch.uint8, device="cuda")
        scratch = torch.empty(max(plan.scratch_bytes, 16), dtype=torch.uint8, device="cuda")
        t1 = time.perf_counter()
        tree = dc.Tree(ctx, plan, arena, scratch)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        if allused:
            tree.run_kernel(mode="resolved", select="all", iters=1, a=1.0001, b=0.0)
        else:
            for ch in chains:
                tree.run_kernel(mode="resolved", select="chain", chain=ch, iters=1, a=1.0001, b=0.0)
        e1.record(s)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        tree.copy_back()
        t4 = time.perf_counter()
        rows.append({"plan_ms": 1e3 * (t1 - t0), "h2d_ms": 1e3 * (t2 - t1), "kernel_ms": e0.elapsed_time(e1),
                     "d2h_ms": 1e3 * (t4 - t3), "wall_ms": 1e3 * (t4 - t0)})
        tree.release()
        plan.close()
        del tree, arena, scratch
    out = {k: round(pct([r[k] for r in rows], 50), 4) for k in rows[0]}
    out["bytes_to_device"] = plan.arena_bytes
    return out


def _time_pointerchain(torch, dc, ctx, t, chains, reps):
    """pointerchain (Section 3): each chain resolved on the host tree and
    only the array it ends in transferred; one kernel pass per array; copy
    back into the host arrays."""
    s = torch.cuda.current_stream()
    schema = dc.Schema(t.types)
    rows = []
    nbytes = 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ccs = [dc.ChainCopy(ctx, schema, t.root_type, t.roots[0], ch) for ch in chains]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for cc in ccs:
            cc.run_kernel(iters=1, a=1.0001, b=0.0)
        e1.record(s)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for cc in ccs:
            cc.copy_back()
        t3 = time.perf_counter()
        nbytes = sum(cc.count * 8 for cc in ccs)
        rows.append({"h2d_ms": 1e3 * (t1 - t0), "kernel_ms": e0.elapsed_time(e1), "d2h_ms": 1e3 * (t3 - t2),
                     "wall_ms": 1e3 * (t3 - t0)})
        del ccs
    out = {k: round(pct([r[k] for r in rows], 50), 4) for k in rows[0]}
    out["bytes_to_device"] = nbytes
    return out


def bench_sweep(args, torch, dc):
    """The paper's Linear and Dense scenarios (Section 4, Tables 1-2) swept
    over their parameters, marshalling against pointerchain, wall-clock of
    the whole program (plan, transfer in, one kernel pass, transfer back)
    and kernel time. Linear: k levels, n doubles per A array, three layout
    schemes (allinit-allused, allinit-LLused, LLinit-LLused). Dense: q
    children per node, depth 3, n doubles per A array; the kernel scales the
    A array of the last element at every level. Sizes follow equations
    (1)-(3). The kernel scales by a constant: x = fma(x, 1.0001, 0)."""
    import math
    import fixtures as fx
    fx.set_threads(0)
    ctx = dc.Context(0)
    reps = max(1, min(args.steps, 5))
    ks = [2, 4, 6, 8, 10]
    ns = [10 ** e for e in range(2, 9 if args.full else 8)]
    rows = []
    for k in ks:
        for n in ns:
            last = [[(1, 0)] * (k - 1) + [(0, 0)]]
            every = [[(1, 0)] * lv + [(0, 0)] for lv in range(k)]
            t_all = fx.linear(seed=fx.SEED_BASE + 100 + k, k=k, n=n, scheme=0)
            for layout, tree_, chains, allused in (("allinit-allused", t_all, every, True),
                                                   ("allinit-LLused", t_all, last, False)):
                m = _time_marshal(torch, dc, ctx, tree_, chains, allused, reps)
                pc = _time_pointerchain(torch, dc, ctx, tree_, chains, reps)
                rows.append({"scenario": "linear", "layout": layout, "k": k, "n": n, "marshal": m,
                             "pointerchain": pc, "wall_ratio": round(m["wall_ms"] / pc["wall_ms"], 3)})
            del t_all
            t_ll = fx.linear(seed=fx.SEED_BASE + 200 + k, k=k, n=n, scheme=1)
            m = _time_marshal(torch, dc, ctx, t_ll, last, False, reps)
            pc = _time_pointerchain(torch, dc, ctx, t_ll, last, reps)
            rows.append({"scenario": "linear", "layout": "LLinit-LLused", "k": k, "n": n, "marshal": m,
                         "pointerchain": pc, "wall_ratio": round(m["wall_ms"] / pc["wall_ms"], 3)})
            del t_ll
            log(args, f"linear k={k} n={n} done")
    for q in (2, 4, 8, 16):
        for n in (10, 100, 1000, 10 ** 4, 10 ** 5):
            nodes = sum(q ** lv for lv in range(4))
            if nodes * 8 * n > (4 << 30 if args.full else 1 << 30):
                continue
            t = fx.dense(seed=fx.SEED_BASE + 300 + q, q=q, n=n, D=3, packed_last=0)
            chains = [[(1, q - 1)] * lv + [(0, 0)] for lv in range(4)]
            m = _time_marshal(torch, dc, ctx, t, chains, False, reps)
            pc = _time_pointerchain(torch, dc, ctx, t, chains, reps)
            rows.append({"scenario": "dense", "layout": "last element of each level", "q": q, "n": n, "D": 3,
                         "marshal": m, "pointerchain": pc, "wall_ratio": round(m["wall_ms"] / pc["wall_ms"], 3)})
            del t
            log(args, f"dense q={q} n={n} done")
    ratios = [r["wall_ratio"] for r in rows]
    geo = math.exp(sum(math.log(x) for x in ratios) / len(ratios))
    big = max((r for r in rows if r["scenario"] == "linear"), key=lambda r: r["marshal"]["bytes_to_device"])
    kb = 2 * 8 * big["n"] * (big["k"] if big["layout"] == "allinit-allused" else 1)
    kgb = kb / (big["marshal"]["kernel_ms"] / 1e3) / 1e9
    return {"metric": "wall-clock of marshalling over pointerchain (geometric mean over the sweep)",
            "value": round(geo, 3), "unit": "x", "higher_is_better": True, "steps": reps, "dtype": "f64",
            "config": {"workload": "Linear k in {2,4,6,8,10} x n in 10^2..10^%d x 3 layout schemes; Dense q in "
                                   "{2,4,8,16} x n in 10..10^5, D=3 (trees above %s skipped)"
                                   % (8 if args.full else 7, "4 GiB" if args.full else "1 GiB")},
            "roofline": {"bound": "hbm", "kernel": "k_stream_resolved / k_leaf_tiles (largest Linear row)",
                         "achieved": round(kgb, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(kgb / HBM_PEAK_GBPS, 4), "traffic": None},
            "rows": rows}


def bench_copycal(args, torch, dc):
    """Reference kernels of known traffic whose FETCH_SIZE / WRITE_SIZE
    counters calibrate those of the other kernels: a plain device-to-device
    copy of 1 GiB (reads and writes exactly 2^30 bytes), three times, and an
    in-place multiply of 1 GiB of nonzero doubles (reads and writes the same
    2^30 bytes, as the leaf kernels do), three times."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    x = torch.rand(n // 8, dtype=torch.float64, device="cuda").add_(0.5)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(3):
        b.copy_(a)
    e1.record(s)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / 3
    e0.record(s)
    for _ in range(3):
        x.mul_(1.0000001)
    e1.record(s)
    e1.synchronize()
    tm = e0.elapsed_time(e1) / 1e3 / 3
    return {"metric": "device copy GB/s (counter calibration)", "value": round(2 * n / t / 1e9, 1), "unit": "GB/s",
            "config": {"workload": "copy 2^30 bytes device to device, 3 times; in-place multiply of 2^30 bytes of "
                                   "doubles, 3 times"},
            "inplace_multiply_GBps": round(2 * n / tm / 1e9, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}). "
              f"Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1906_01128_amd import dc
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    log(args, f"libdc {dc.version()} on {torch.cuda.get_device_name(0)}")
    if args.workload == "linear":
        out = bench_linear(args, torch, dc)
    elif args.workload == "wide":
        out = bench_wide(args, torch, dc)
    elif args.workload == "batched":
        out = bench_batched(args, torch, dc)
    elif args.workload == "copycal":
        out = bench_copycal(args, torch, dc)
    elif args.workload == "sweep":
        out = bench_sweep(args, torch, dc)
    elif args.workload == "plain":
        out = bench_plain(args, torch, dc)
    else:
        out = bench_served(args, torch, dc)
    out.setdefault("n_gpus", 1)
    out.setdefault("data", "synthetic")
    if not args.no_cpu_baseline and args.workload == "linear":
        log(args, "cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_linear(args, passes=2 * args.passes)   # ~10-15 s of CPU work
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
