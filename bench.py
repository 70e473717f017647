"""Benchmark: trace + collision-check throughput on one MI355X, and proof
latency in the serving loop.

One step = one whole pass of the hot path on one synthetic proof problem:
seed location, manifold tracing over the Coxeter triangulation (batch
triangulation for the d=6 workload: coarse trace, n-coface set, template
subdivision, f evaluation, sign tests, dedup), intersection points, collision
check of every traced cell and gathering of the free points.  Inputs are
uploaded before the timed region; nothing is cached between steps.

`value` is the FP32-certified path (exact: the traced set equals the FP64
one); the plain FP64 path is timed beside it on the same GPU.  The serving
section replays a Poisson stream of mixed proof requests through the
library's server and reports p50/p99 latency.

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector ALU: 256 CUs x 64 lanes x 2 flops (fma) x 2.4 GHz = 78.6
# TFLOP/s for FP64 and for unpacked FP32 (the library is built without
# packed-FP32 instructions; with them FP32 would double to 157.3)
VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

METRIC = "simplices traced/s + cells checked/s at d=6; p50/p99 proof latency in loop"


def workload(name: str):
    from paper_2406_04795_amd import inputs as I
    if name == "d6":
        # 6-DoF arm, 16 obstacles (8 boxes + 8 spheres), 2000 SVs of degree 3,
        # fine scale 0.06, batch triangulation with k = 4
        return I.config_c3(eps=2e-5, k=4)
    if name == "d6direct":
        wl = I.config_c3(eps=2e-5, k=1)
        wl.name = "d6_S2000_p3_lam0.06_direct"
        return wl
    if name == "d5":
        return I.config_c2(eps=3e-4)
    if name == "d3":
        return I.config_c1()
    raise SystemExit(f"unknown config {name}")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "subdivide_d6_k4_traffic.json")


def subdivide_traffic(wl):
    """HBM bytes of one fused subdivision launch from the committed memory
    counter runs (FETCH_SIZE, WRITE_SIZE, each scaled by what it reads for a
    plain copy of known size), or None when they do not describe the kernel
    as built now (its sources changed) or another workload."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    h = hashlib.sha256()
    for rel in rec["sources"]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["sources_sha256_16"] or not rec["workload"].startswith(wl.name):
        return None
    return round(rec["fetch_size_kib"] * 1024 * rec["fetch_factor"] + rec["write_size_kib"] * 1024 * rec["write_factor"])


def nest_flops(d: int, p: int) -> int:
    """FP32 operations per point of the nested (multivariate Horner) form of
    the degree-p polynomial over the monomial basis: one fma (2 flops) per
    non-constant monomial, one add per monomial of degree below p (its
    sub-sum), one final add of the constant term.  194 at d = 6, p = 3."""
    from math import comb
    n = [comb(d + k - 1, k) for k in range(1, p + 1)]
    return 2 * sum(n) + sum(n[:-1]) + 1


def subdivide_flops(st, wl) -> int:
    """Floating-point operations of the fused subdivision launches, from the
    counters of the code that runs: every template point it evaluated
    (n_vertices; in the box, on an active face) costs its FP64 lattice
    coordinates (d^2 fma) and the nested FP32 value."""
    d, p = wl.f.d, wl.f.p
    return st["n_vertices"] * (2 * d * d + nest_flops(d, p))


def prep_flops_per_simplex(wl) -> int:
    """FP64 operations of the preparation kernel per coarse simplex: the
    coordinates of its d + 1 vertices (d^2 fma each) and the region bound
    (per non-constant monomial up to p multiplies and an add).  Its d + 1
    probes of the coarse vertex table are not counted."""
    from math import comb
    d, p = wl.f.d, wl.f.p
    return (d + 1) * 2 * d * d + (p + 1) * (comb(d + p, p) - 1)


def check_flops_per_cell(wl) -> int:
    """FP64 operations of the collision kernel per configuration: per link
    the own sine/cosine (42), the link transform (a rotation about one axis
    after a joint offset: 36), the link ball's world centre (18) and half its
    squared norm (6), and the ball's culling test against a ball around
    every obstacle (c.o - |c|^2/2 as three fma: 6 each).  Early exits are
    ignored; the exact tests of the pairs that pass culling are not
    counted."""
    sc = wl.scene
    d = wl.f.d
    ocyl = getattr(sc, "ocyl_rh", None)
    n_obs = len(sc.osph_r) + len(sc.obox_l) + (0 if ocyl is None else len(ocyl))
    return d * (42 + 36 + 18 + 6) + d * 6 * n_obs


def points_flops_per_cell(wl) -> int:
    """FP64 operations of the intersection-point kernel per traced edge: both
    ends' coordinates (2 x 2 d^2), both ends' FP64 monomial values with their
    bound sums and the bound test (2 x (5 per non-constant monomial + 2)), t
    and the point (3 d + 2)."""
    from math import comb
    d, p = wl.f.d, wl.f.p
    return 2 * (2 * d * d + 5 * (comb(d + p, p) - 1) + 2) + 3 * d + 2


def sigma_bytes(st) -> int:
    """HBM bytes of the coarse n-simplex kernel: each coarse edge record read
    (16 B), one 8 B key probe per n-coface, and per new coarse simplex its
    8 B table write and 8 B list write."""
    return st["n_coarse_edges"] * 16 + st["n_ncofaces"] * 8 + st["n_sigma"] * 16


def expand_bytes(st, wl) -> float:
    """Algorithmic HBM bytes of the direct-mode search kernels, per 2-coface:
    pass 1 vertex-table probe (8 B key) and third-vertex slot write (4 B);
    pass 2 slot read (4 B), f read (8 B) and edge-mask word read (8 B).  Per
    new vertex one 8 B key CAS; per traced edge a 16 B append and 2 x 16 B
    frontier reads."""
    return st["n_cofaces"] * 32 + st["n_vertices"] * 8 + st["n_cells"] * 48


def host_info():
    """The host CPU the oracle ran on: model name and the CPUs this process
    may use (the oracle itself is single-threaded)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def cpu_baseline(wl, budget_s: float = 20.0):
    """The oracle (single thread) on a bounded sample of the same workload:
    the same manifold, scale, coarse factor and scene, traced inside a sub-box
    of the domain centred on the first seed, plus points and collision check
    of those cells."""
    import copy

    import oracle as O
    from paper_2406_04795_amd import inputs as I

    O.build(force=False)
    half = 0.15
    while True:
        sub = copy.copy(wl)
        c = wl.seeds[0]
        sub.dom = I.Domain(lo=np.maximum(wl.dom.lo, c - half), hi=np.minimum(wl.dom.hi, c + half))
        sub.seeds = wl.seeds[:1]
        t0 = time.perf_counter()
        if wl.k > 1:
            v, m, _ = O.trace_batch(sub)
        else:
            v, m = O.trace_direct(sub)
        t_trace = time.perf_counter() - t0
        # the point pass re-evaluates f at both ends of every cell: stop
        # growing the sub-box at about 1/6 of the budget
        if t_trace > budget_s / 6 or half > 1.5:
            break
        half *= 1.25
    t0 = time.perf_counter()
    pts, _ = O.points(sub, v, m)
    t_pts = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.check(wl.scene, pts)
    t_check = time.perf_counter() - t0
    n = len(v)
    total = t_trace + t_pts + t_check
    return {
        "value": n / total if total > 0 else None,
        "unit": "simplices/s",
        "cores": 1,
        "host": host_info(),
        "kind": "oracle",
        "sample": f"same f/scale/k/scene traced in a sub-box of half-width {half:.3f} around the first "
                  f"seed: {n} cells, trace {t_trace:.2f}s + points {t_pts:.2f}s + check {t_check:.2f}s",
    }


def timed_runs(ip, ctx, prob, wl, prec, steps, warmup, budget):
    import torch

    def step():
        c = ip.Cells(ctx, prob, budget=budget, precision=prec)
        nf = c.check(wl.scene)
        st = c.stats()
        c.close()
        return st, nf

    name = "fp32" if prec == ip.IP_FP32_CERTIFY else "fp64"
    for i in range(warmup):
        st, nf = step()
        print(f"[bench] {name} warmup {i}: {st['n_cells']} cells, trace {st['ms_total']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        st, nf = step()
        stats.append(st)
        print(f"[bench] {name} step {i}: {st['n_cells']} cells, trace {st['ms_total']:.1f} ms, "
              f"check {st['ms_check']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return stats, nf, elapsed


def phase(stats, key):
    return float(np.mean([s[key] for s in stats]))


def serving(ip, reqs, slots, rate, precision, seed=1):
    """Replay requests with Poisson arrivals (rate per second; 0 = all at
    once) through a server with `slots` slots; returns per-request results."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(reqs)) if rate > 0 else np.zeros(len(reqs))
    arrivals = np.cumsum(gaps)
    srv = ip.ip_server_create(0, 0, slots)
    try:
        t0 = ip.ip_server_clock(srv)
        ids = []
        for wl, ta in zip(reqs, arrivals):
            while ip.ip_server_clock(srv) - t0 < ta:
                time.sleep(0.0002)
            ids.append(ip.ip_server_submit(srv, wl, precision=precision, scene=wl.scene))
        res = [ip.ip_server_wait(srv, i) for i in ids]
    finally:
        ip.ip_server_destroy(srv)
    bad = [(i, r["error"]) for i, r in enumerate(res) if r["status"] != 0]
    if bad:
        print(f"[bench] {len(bad)} serving requests failed: {bad[:3]}", file=sys.stderr, flush=True)
    return res


def latency_summary(res):
    """Latency over every request; cells (and so simplices/s) over the ones
    that finished; failed requests are counted."""
    lat = np.array([r["t_done"] - r["t_submit"] for r in res]) * 1e3
    t_first = min(r["t_submit"] for r in res)
    t_last = max(r["t_done"] for r in res)
    cells = sum(r["n_cells"] for r in res)
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "simplices_per_s": cells / (t_last - t_first),
            "requests": len(res), "failed": sum(r["status"] != 0 for r in res)}


def timeline(res):
    """Per request: d, cells, submit time, queue wait, admission wait, time
    traced and checked, the trace's own stream time, device allocations that
    missed the context cache (count, bytes), admitted bytes (ms, bytes)."""
    return [[r["d"], r["n_cells"], round(r["t_submit"] * 1e3, 2), round((r["t_start"] - r["t_submit"]) * 1e3, 2),
             round((r["t_admit"] - r["t_start"]) * 1e3, 2), round((r["t_done"] - r["t_admit"]) * 1e3, 2),
             round(r["stats"]["ms_total"], 2), r["stats"]["n_hip_malloc"], r["stats"]["hip_malloc_bytes"],
             r["admitted_bytes"]] for r in res]


def request_sizes(res):
    """Per-request cells and admitted (projected) bytes, as quantiles."""
    q = [0, 10, 50, 90, 100]
    res = [r for r in res if r["status"] == 0]
    n = np.array([r["n_cells"] for r in res], dtype=float)
    b = np.array([r["admitted_bytes"] for r in res], dtype=float)
    return {"cells_quantiles": dict(zip(map(str, q), np.percentile(n, q).round().astype(int).tolist())),
            "admitted_gib_quantiles": dict(zip(map(str, q), np.round(np.percentile(b, q) / 2 ** 30, 4).tolist())),
            "cells_by_d": {str(d): int(sum(r["n_cells"] for r in res if r["d"] == d)) for d in sorted({r["d"] for r in res})}}


def leg(ip, wl, prec, steps, flags=0, budget=0):
    """Warm-up plus `steps` timed traces (and checks, with a scene) of wl."""
    import torch
    ctx = ip.Context(0)
    prob = ip.Problem(ctx, wl)
    try:
        def one():
            c = ip.Cells(ctx, prob, budget=budget, precision=prec, flags=flags)
            if wl.scene is not None:
                c.check(wl.scene)
            st = c.stats()
            c.close()
            return st
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [one() for _ in range(steps)]
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
    finally:
        prob.close()
        ctx.close()
    st = sts[-1]
    return {"simplices_per_s": st["n_cells"] / el, "ms_per_step": round(el * 1e3, 3), "cells": st["n_cells"],
            "vertices_evaluated": st["n_vertices"], "fp64_canonical_evals": st["n_fallback"],
            "settled_by_fp64_monomial": st["n_settled64"],
            "fallback_rate": st["n_fallback"] / max(1, st["n_vertices"]),
            "phases_ms": {"trace": phase(sts, "ms_total"), "refine": phase(sts, "ms_refine"),
                          "check": phase(sts, "ms_check")}}


def cfree_leg(ip, wl, prec, budget, n_free, steps=3):
    """Trace + check + the C_free points to pinned host memory, per step."""
    import torch
    if wl.scene is None:
        return None
    host = torch.empty(max(1, n_free * wl.f.d), dtype=torch.float64, pin_memory=True)
    ctx = ip.Context(0)
    prob = ip.Problem(ctx, wl)
    try:
        def one():
            c = ip.Cells(ctx, prob, budget=budget, precision=prec)
            nf = c.check(wl.scene)
            assert nf * wl.f.d <= host.numel()
            t0 = time.perf_counter()
            ip.ip_cells_download_free(ctx.h, c.h, host.data_ptr())
            t_copy = time.perf_counter() - t0
            n = c.n
            c.close()
            return n, nf, t_copy
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [one() for _ in range(steps)]
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
    finally:
        prob.close()
        ctx.close()
    n, nf, _ = res[-1]
    t_copy = float(np.mean([r[2] for r in res]))
    return {"simplices_per_s": n / el, "ms_per_step": round(el * 1e3, 3), "free_points": nf,
            "d2h_ms": round(t_copy * 1e3, 3), "d2h_gbs": round(nf * wl.f.d * 8 / t_copy / 1e9, 2)}


def per_batch_leg(ip, wl, prec, budgets_gib, steps=3, resident=True):
    """The paper's batch pipeline (trace, check and the C_free points to the
    host batch by batch) at each batch budget: time per step, batches, and
    the device memory the context holds after its first call (free device
    memory before the context minus after), beside the same figure for the
    resident path (cells, points and free points all on the device)."""
    import torch
    if wl.scene is None or wl.k < 2:
        return None

    def held(run):
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx = ip.Context(0)
        prob = ip.Problem(ctx, wl)
        try:
            keep = run(ctx, prob)
            torch.cuda.synchronize()
            used = free0 - torch.cuda.mem_get_info()[0]
            return used, keep, ctx, prob
        except Exception:
            prob.close()
            ctx.close()
            raise

    def resident_run(ctx, prob):
        c = ip.Cells(ctx, prob, precision=prec)
        c.check(wl.scene)
        return c

    out = {}
    if resident:
        used, c, ctx, prob = held(resident_run)
        c.close()
        prob.close()
        ctx.close()
        out["resident_device_gib"] = round(used / 2 ** 30, 2)
    for gib in budgets_gib:
        budget = int(gib * 2 ** 30)
        used, summ, ctx, prob = held(lambda cx, pr: pr.trace_check_batches(wl.scene, budget=budget,
                                                                           precision=prec)[0])
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step_ms, mallocs = [], []
            for _ in range(steps):
                t1 = time.perf_counter()
                summ, _ = prob.trace_check_batches(wl.scene, budget=budget, precision=prec)
                step_ms.append(round((time.perf_counter() - t1) * 1e3, 1))
                mallocs.append(summ["stats"]["n_hip_malloc"])
            el = (time.perf_counter() - t0) / steps
        finally:
            prob.close()
            ctx.close()
        st = summ["stats"]
        out[f"budget_{gib:g}gib"] = {
            "simplices_per_s": summ["n_cells"] / el, "ms_per_step": round(el * 1e3, 3),
            "batches": summ["batches"], "cells": summ["n_cells"], "free_points": summ["n_free"],
            "device_gib": round(used / 2 ** 30, 2), "check_ms": round(st["ms_check"], 3),
            "points_ms": round(st["ms_points"], 3), "subdivide_ms": round(st["ms_subdivide"], 3),
            "step_ms": step_ms, "hip_malloc_per_step": mallocs}
        print(f"[bench] per-batch pipeline, budget {gib:g} GiB: {out[f'budget_{gib:g}gib']}", file=sys.stderr,
              flush=True)
    return out


def extra_legs(ip, wls, main_wl):
    """The other workloads of the suite, one line each: the d=3 planar arm
    (C1), the d=5 arm (C2), the precision stress at its scale (C5, with its
    FP64 fallback rate), an
    RBF-kernel manifold, the iterative intersection on the benchmark
    workload, and the seed search on the benchmark's f."""
    import torch
    out = {}
    for name, wl in wls.items():
        print(f"[bench] leg {name}: d={wl.f.d} S={wl.f.S} k={wl.k} kernel={wl.f.kernel}", file=sys.stderr, flush=True)
        out[name] = {"workload": wl.name,
                     "fp32_certify": leg(ip, wl, ip.IP_FP32_CERTIFY, 3),
                     "fp64": leg(ip, wl, ip.IP_FP64, 2)}
    # iterative intersection: 4 false-position steps on every cell of the
    # benchmark workload (FP32-certified mode: FP64 monomial values)
    print("[bench] leg refine4", file=sys.stderr, flush=True)
    r = leg(ip, main_wl, ip.IP_FP32_CERTIFY, 3, flags=ip.IP_REFINE(4), budget=64 << 30)
    from math import comb
    d, p = main_wl.f.d, main_wl.f.p
    per_edge = 6 * (5 * (comb(d + p, p) - 1) + 2) + 2 * 2 * d * d + 5 * (3 * d + 2)
    ms = r["phases_ms"]["refine"]
    tfs = per_edge * r["cells"] / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    r["refine_kernel"] = {"bound": "alu", "achieved": round(tfs, 3), "peak": VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(tfs / VECTOR_PEAK_TFLOPS, 4), "flops_per_cell": per_edge, "ms": ms}
    out["refine4_bench_workload"] = r
    # seed search: 2^20 starts, 20 Newton steps each, canonical FP64 f + grad
    print("[bench] leg seeds", file=sys.stderr, flush=True)
    n, iters = 1 << 20, 20
    ctx = ip.Context(0)
    prob = ip.Problem(ctx, main_wl)
    try:
        g = torch.Generator(device="cuda")
        g.manual_seed(3)
        lo = torch.tensor(main_wl.dom.lo, device="cuda")
        hi = torch.tensor(main_wl.dom.hi, device="cuda")
        q0 = (lo + (hi - lo) * torch.rand((n, d), generator=g, device="cuda", dtype=torch.float64)).contiguous()
        q = torch.empty_like(q0)
        fq = torch.empty(n, dtype=torch.float64, device="cuda")
        ip.ip_seed_search(ctx.h, prob.h, q0.data_ptr(), n, iters, q.data_ptr(), fq.data_ptr())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ip.ip_seed_search(ctx.h, prob.h, q0.data_ptr(), n, iters, q.data_ptr(), fq.data_ptr())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        scale = float(np.abs(main_wl.f.alpha).sum()) * 1e-9
        on = int((fq.abs() < scale).sum())
    finally:
        prob.close()
        ctx.close()
    per_sv = 4 * d + p + 5
    tfs = n * (iters + 1) * main_wl.f.S * per_sv / el / 1e12
    out["seed_search_bench_f"] = {"starts": n, "iters": iters, "ms": round(el * 1e3, 3),
                                  "starts_per_s": n / el, "on_manifold": on,
                                  "kernel": {"bound": "alu", "achieved": round(tfs, 3), "peak": VECTOR_PEAK_TFLOPS,
                                             "unit": "TFLOP/s", "frac": round(tfs / VECTOR_PEAK_TFLOPS, 4),
                                             "flops_per_sv_step": per_sv}}
    return out


def _gen_requests(span):
    from paper_2406_04795_amd import inputs as I
    return [I.serving_request(i) for i in range(*span)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="d6")
    ap.add_argument("--precision", default="both", choices=["both", "fp32", "fp64"])
    ap.add_argument("--budget-gib", type=float, default=64.0,
                    help="batch-triangulation workspace cap per batch (GiB)")
    ap.add_argument("--serve", type=int, default=256, help="serving requests (0: skip)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--serve-log", default="",
                    help="write every serving request's timeline (JSON, per mode) to this path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--handoff", type=int, default=1,
                    help="run the C_free hand-off lines (resident copy, per-batch pipeline); 0: skip")
    ap.add_argument("--legs", type=int, default=1, help="run the other workloads' lines (0: skip)")
    ap.add_argument("--workload-cache", default="",
                    help="pickle of the generated workload: loaded if present, else written (profiling runs)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run one plain device-to-device copy of this many GiB (counter calibration)")
    ap.add_argument("--per-batch-only", type=float, default=0.0,
                    help="only run the per-batch hand-off line at this budget (GiB) on the cached workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the traced path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return

    # inputs first, on the CPU: the pool forks before anything touches the GPU
    if args.workload_cache and os.path.exists(args.workload_cache):
        import pickle
        with open(args.workload_cache, "rb") as fh:
            wl = pickle.load(fh)
    else:
        wl = workload(args.config)
        if args.workload_cache:
            import pickle
            with open(args.workload_cache, "wb") as fh:
                pickle.dump(wl, fh)
    if args.per_batch_only > 0:
        import torch

        from paper_2406_04795_amd import ip
        assert torch.cuda.is_available(), "bench needs a GPU"
        res = per_batch_leg(ip, wl, ip.IP_FP32_CERTIFY, (args.per_batch_only,), resident=False)
        print(json.dumps(res))
        return
    # the per-batch hand-off in a process of its own, before this one touches
    # the GPU: after a large resident trace has run and been freed in a
    # process, that process's per-batch copies run slower (the line measured
    # after the main steps below shows it)
    fresh = None
    if args.handoff and wl.k >= 2 and wl.scene is not None:
        import pickle
        import subprocess
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "wl.pkl")
            with open(path, "wb") as fh:
                pickle.dump(wl, fh)
            print("[bench] per-batch pipeline in a fresh process", file=sys.stderr, flush=True)
            r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--per-batch-only", "4",
                                "--workload-cache", path], capture_output=True, text=True, timeout=900)
            sys.stderr.write(r.stderr[-2000:])
            if r.returncode == 0 and r.stdout.strip():
                fresh = json.loads(r.stdout.strip().splitlines()[-1])
            else:
                print(f"[bench] fresh-process per-batch line failed ({r.returncode})", file=sys.stderr, flush=True)
    extras = {}
    if args.legs:
        from paper_2406_04795_amd import inputs as I
        extras = {"c1_d3": I.config_c1(), "c2_d5": I.config_c2(eps=3e-4), "c5_stress_d5": I.config_c5(),
                  "rbf_d5": I.rbf_case(5, 500, 0.15, 0.1, seed=1, n_seeds=4)}
    reqs = []
    if args.serve:
        from concurrent.futures import ProcessPoolExecutor
        n = args.serve
        with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
            chunks = list(ex.map(_gen_requests, [(i, min(n, i + 8)) for i in range(0, n, 8)]))
        reqs = [r for c in chunks for r in c]
        print(f"[bench] {len(reqs)} serving requests generated", file=sys.stderr, flush=True)

    import torch

    from paper_2406_04795_amd import ip

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    print(f"[bench] workload {wl.name}: d={wl.f.d} S={wl.f.S} p={wl.f.p} lam={wl.lat.lam} k={wl.k}",
          file=sys.stderr, flush=True)
    budget = int(args.budget_gib * (1 << 30))
    ctx = ip.Context(0)
    prob = ip.Problem(ctx, wl)
    precs = {"both": [ip.IP_FP32_CERTIFY, ip.IP_FP64], "fp32": [ip.IP_FP32_CERTIFY],
             "fp64": [ip.IP_FP64]}[args.precision]
    runs = {}
    for prec in precs:
        runs[prec] = timed_runs(ip, ctx, prob, wl, prec, args.steps, args.warmup, budget)
    prob.close()
    ctx.close()

    main_prec = precs[0]
    stats, nf, elapsed = runs[main_prec]
    n_steps = len(stats)
    n_cells = stats[-1]["n_cells"]
    value = n_cells * n_steps / elapsed

    def summary(prec):
        st, _, el = runs[prec]
        s = st[-1]
        return {"simplices_per_s": s["n_cells"] * len(st) / el, "ms_per_step": el * 1e3 / len(st),
                "phases_ms": {"trace": phase(st, "ms_total"), "search": phase(st, "ms_expand"),
                              "subdivide": phase(st, "ms_subdivide"), "prep": phase(st, "ms_prep"), "feval": phase(st, "ms_feval"),
                              "points": phase(st, "ms_points"), "check": phase(st, "ms_check")},
                "edge_hits": s["n_edge_hits"], "edge_set_probes": s["n_shared_probes"],
                "vertices_evaluated": s["n_vertices"], "fp64_canonical_evals": s["n_fallback"],
                "settled_by_fp64_monomial": s["n_settled64"],
                "hip_malloc_per_step": phase(st, "n_hip_malloc"),
                "step_ms": [round(x["ms_total"] + x["ms_check"], 2) for x in st]}

    # roofline of the dominant kernel of the main run, from the library's HIP
    # events around its launches on the context's stream
    kernels = {}
    s_last = stats[-1]

    def alu(name, flops, ms, **extra):
        tfs = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        kernels[name] = {"bound": "alu", "achieved": round(tfs, 3), "peak": VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tfs / VECTOR_PEAK_TFLOPS, 4),
                         "ms_per_step": round(ms, 3), "flops": int(flops), **extra}

    if wl.scene is not None:
        alu("check_kernel", check_flops_per_cell(wl) * n_cells, phase(stats, "ms_check"),
            flops_per_cell=check_flops_per_cell(wl))
    if wl.k > 1 and main_prec == ip.IP_FP32_CERTIFY:
        ms = phase(stats, "ms_subdivide")
        # one fused launch over every coarse simplex, plus the deferred pass
        # over the few (<1 %) with an unsettled point: the time is the sum
        alu("subdivide_kernel", subdivide_flops(s_last, wl), ms,
            launches_per_step=s_last["subdivide_launches"], points_evaluated=s_last["n_vertices"],
            coarse_simplices=s_last["n_sigma"],
            flops_per_point=2 * wl.f.d ** 2 + nest_flops(wl.f.d, wl.f.p))
        alu("sub_points_kernel", points_flops_per_cell(wl) * n_cells, phase(stats, "ms_points"),
            flops_per_cell=points_flops_per_cell(wl))
        alu("sub_prep_kernel", prep_flops_per_simplex(wl) * s_last["n_sigma"], phase(stats, "ms_prep"),
            flops_per_simplex=prep_flops_per_simplex(wl))
        sg_ms = phase(stats, "ms_sigma")
        gbs = sigma_bytes(s_last) / (sg_ms * 1e-3) / 1e9 if sg_ms > 0 else 0.0
        kernels["sigma_kernel"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                   "ms_per_step": round(sg_ms, 3), "bytes": sigma_bytes(s_last)}
        roof = {"kernel": "subdivide_kernel (fused, FP32-certified)", **kernels["subdivide_kernel"],
                "traffic": subdivide_traffic(wl)}
    else:
        x_ms = phase(stats, "ms_expand")
        gbs = expand_bytes(stats[-1], wl) / (x_ms * 1e-3) / 1e9
        roof = {"kernel": "expand_kernel (2 passes)", "bound": "hbm", "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "ms_per_step": round(x_ms, 3)}
        kernels["expand_kernel"] = dict(roof)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / n_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_prec == ip.IP_FP32_CERTIFY else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "d": wl.f.d, "n_sv": wl.f.S, "degree": wl.f.p,
                   "scale": wl.lat.lam, "coarse_k": wl.k, "batch_budget_gib": args.budget_gib,
                   "cells": n_cells, "free_cells": int(nf), "coarse_simplices": stats[-1]["n_sigma"],
                   "batches": stats[-1]["n_batches"], "levels": stats[-1]["levels"]},
        "roofline": roof,
        "kernels": kernels,
    }
    for prec in precs:
        out["fp32_certify" if prec == ip.IP_FP32_CERTIFY else "fp64"] = summary(prec)

    # the same step with the C_free points copied to pinned host memory (the
    # paper's pipeline hands them to the host): PCIe-inclusive, not `value`
    # the paper's per-batch hand-off: C_free to the host after every batch,
    # device memory bounded by the batch budget (not `value`)
    if args.handoff:
        out["per_batch_cfree_to_host"] = per_batch_leg(ip, wl, main_prec, (4.0, args.budget_gib))
        if out["per_batch_cfree_to_host"] is not None and fresh is not None:
            out["per_batch_cfree_to_host"]["fresh_process"] = fresh
        out["with_cfree_to_host"] = cfree_leg(ip, wl, main_prec, budget, nf)
    if extras:
        out["legs"] = extra_legs(ip, extras, wl)
    if reqs:
        # isolated capacity: every request alone, back to back
        iso = serving(ip, reqs, 1, 0.0, ip.IP_FP32_CERTIFY)
        t_service = float(np.mean([r["t_done"] - r["t_start"] for r in iso if r["status"] == 0]))
        rate = 0.7 / t_service
        print(f"[bench] serving: isolated service {t_service * 1e3:.1f} ms, arrival rate {rate:.1f}/s",
              file=sys.stderr, flush=True)
        srv = {"requests": len(reqs), "slots": args.slots, "arrival_rate_per_s": round(rate, 2),
               "isolated_service_ms": round(t_service * 1e3, 3), "request_sizes": request_sizes(iso)}
        log = {"isolated": timeline(iso)}
        for key, slots, prec in (("fp32_certify", args.slots, ip.IP_FP32_CERTIFY),
                                 ("fp64", args.slots, ip.IP_FP64),
                                 ("queue_only_fp32", 1, ip.IP_FP32_CERTIFY)):
            res = serving(ip, reqs, slots, rate, prec)
            srv[key] = latency_summary(res)
            log[key] = timeline(res)
            print(f"[bench] serving {key}: {srv[key]}", file=sys.stderr, flush=True)
        out["serving"] = srv
        if args.serve_log:
            with open(args.serve_log, "w") as fh:
                json.dump(log, fh)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
