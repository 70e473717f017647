"""Benchmark: trace + collision-check throughput on one MI355X.

One step = one whole pass of the hot path on one synthetic proof problem:
seed location, breadth-first manifold tracing over the Coxeter triangulation
(f evaluation, coface expansion, hash dedup), intersection points, collision
check of every traced cell and gathering of the free points.  Inputs are
uploaded before the timed region; nothing is cached between steps (every step
rebuilds its tables and outputs from the seeds).

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (v_fma_f64), dense
HBM_PEAK_GBS = 8000.0

METRIC = "simplices traced/s + cells checked/s at d=6; p50/p99 proof latency in loop"


def workload(name: str):
    from paper_2406_04795_amd import inputs as I
    if name == "d6":
        # 6-DoF arm, 16 obstacles (8 boxes + 8 spheres), f with 2000 SVs of
        # degree 3, scale 0.06
        wl = I.config_c3(eps=2e-5, k=1)
        wl.name = "d6_S2000_p3_lam0.06_direct"
        return wl
    if name == "d5":
        wl = I.config_c2(eps=3e-4)
        return wl
    if name == "d3":
        return I.config_c1()
    raise SystemExit(f"unknown config {name}")


def flops_per_vertex(f) -> int:
    # per support vector: d fma (dot) + 1 fma (gamma, coef0) + (p-1) mul + 1 fma (alpha)
    return f.S * (2 * f.d + f.p + 3)


def cpu_baseline(wl, budget_s: float = 20.0):
    """The oracle (single thread) on a bounded sample of the same workload:
    the same manifold, scale and scene, traced inside a sub-box of the domain
    centred on the first seed, plus the collision check of those cells."""
    import copy

    import oracle as O
    from paper_2406_04795_amd import inputs as I

    O.build(force=False)
    half = 0.12
    while True:
        sub = copy.copy(wl)
        c = wl.seeds[0]
        sub.dom = I.Domain(lo=np.maximum(wl.dom.lo, c - half), hi=np.minimum(wl.dom.hi, c + half))
        sub.seeds = wl.seeds[:1]
        t0 = time.perf_counter()
        v, m = O.trace_direct(sub)
        t_trace = time.perf_counter() - t0
        # the oracle's point pass re-evaluates f at both ends of every cell,
        # about 2.5x the trace time; stop growing the sub-box at ~1/8 of budget
        if t_trace > budget_s / 8 or half > 1.0:
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
        "kind": "oracle",
        "sample": f"same f/scale/scene traced in a sub-box of half-width {half:.3f} around the first "
                  f"seed: {n} cells, trace {t_trace:.2f}s + points {t_pts:.2f}s + check {t_check:.2f}s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="d6")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the traced path has no multi-GPU mode in this build",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2406_04795_amd import ip

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    wl = workload(args.config)
    prec = ip.IP_FP64 if args.precision == "fp64" else ip.IP_FP32_CERTIFY
    print(f"[bench] workload {wl.name}: d={wl.f.d} S={wl.f.S} p={wl.f.p} lam={wl.lat.lam} k={wl.k}",
          file=sys.stderr, flush=True)

    ctx = ip.Context(0)
    prob = ip.Problem(ctx, wl)

    def step():
        c = ip.Cells(ctx, prob, precision=prec)
        nf = c.check(wl.scene)
        st = c.stats()
        c.close()
        return st, nf

    for i in range(args.warmup):
        st, nf = step()
        print(f"[bench] warmup {i}: {st['n_cells']} cells in {st['ms_total']:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        st, nf = step()
        stats.append(st)
        print(f"[bench] step {i}: {st['n_cells']} cells, trace {st['ms_total']:.1f} ms, "
              f"check {st['ms_check']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prob.close()
    ctx.close()

    n_cells = stats[-1]["n_cells"]
    value = n_cells * args.steps / elapsed
    ms_step = elapsed * 1000 / args.steps

    # dominant kernel class by measured time
    f_ms = float(np.mean([s["ms_feval"] for s in stats]))
    x_ms = float(np.mean([s["ms_expand"] for s in stats]))
    nv = stats[-1]["n_vertices"]
    fl = flops_per_vertex(wl.f) * nv
    feval_tfs = fl / (f_ms * 1e-3) / 1e12 if f_ms > 0 else 0.0
    cof = stats[-1]["n_cofaces"]
    # algorithmic bytes of the two expansion passes per coface: pass 1 vertex
    # probe (8 B key), pass 2 vertex probe + value (16 B) and edge-set probe
    # (8 B); per frontier edge 2 x 8 B key reads; per new vertex / edge one
    # 8 B CAS write and one 4/8 B list append
    xbytes = cof * 32 + n_cells * (16 + 16) + nv * 12
    if f_ms >= x_ms:
        roof = {"kernel": "feval64", "bound": "alu", "achieved": round(feval_tfs, 3),
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(feval_tfs / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                "ms_per_step": round(f_ms, 3)}
    else:
        gbs = xbytes / (x_ms * 1e-3) / 1e9
        roof = {"kernel": "expand", "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "ms_per_step": round(x_ms, 3)}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == ip.IP_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "d": wl.f.d, "n_sv": wl.f.S, "degree": wl.f.p,
                   "scale": wl.lat.lam, "coarse_k": wl.k, "cells": n_cells,
                   "free_cells": int(nf), "vertices": nv, "levels": stats[-1]["levels"],
                   "cofaces": int(cof)},
        "precision": {"fp64_canonical_evals": int(stats[-1]["n_fallback"]),
                      "settled_by_fp64_monomial": int(stats[-1]["n_settled64"])},
        "phases_ms": {"trace": float(np.mean([s["ms_total"] for s in stats])),
                      "feval": f_ms, "expand": x_ms,
                      "points": float(np.mean([s["ms_points"] for s in stats])),
                      "check": float(np.mean([s["ms_check"] for s in stats]))},
        "feval_tflops": round(feval_tfs, 3),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
