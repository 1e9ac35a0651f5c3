#!/usr/bin/env python
"""Throughput benchmark of the MI355X DtN walk estimator.

One step = one pass of the hot path over the workload: for every mesh and
every operator side of the workload, estimate_dtn (start sampling,
Walk-on-Spheres with exact BVH queries, hit basis evaluation, row
accumulation, finalisation) and, when the workload asks for eigenpairs, the
eigen step. Inputs (BVHs, rows, basis tables) are resident on the GPU before
timing starts. Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (dual issue) x 2.4 GHz
NODE_BYTES, TRI_BYTES = 128, 48


def measured_traffic(workload):
    """HBM bytes per walk-kernel launch from the committed rocprofv3 counter
    passes, if they were taken on the current kernel sources (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2606_05581_amd", "csrc")
    sha = hashlib.sha256(open(os.path.join(csrc, "walk.hip"), "rb").read()
                         + open(os.path.join(csrc, "msk_internal.h"), "rb").read()).hexdigest()[:16]
    return rec["traffic_bytes_per_launch"] if rec.get("source_sha") == sha else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(ctx, wl):
    handles = []
    for c in wl.cases:
        mesh = ctx.build_bvh(c.V, c.F)
        rows = ctx.rows(mesh, c.rows)
        basis = ctx.basis(c.basis, c.V.shape[0])
        handles.append((c, mesh, rows, basis))
    return handles


def run_step(ctx, wl, handles, **opts):
    """One pass of the hot path; returns per-launch records."""
    recs = []
    for ext in [m == "exterior" for m in wl.modes]:
        for c, mesh, rows, basis in handles:
            d = ctx.estimate_dtn(mesh, rows, basis, wl.walks, c.eps, c.h, exterior=ext, **opts)
            inf = d.info()
            recs.append(inf)
            d.close()
    return recs


def cpu_baseline(wl, target_s, max_threads=16):
    """The oracle (FP64 walks, its own BVH) on a bounded sample of rows."""
    import numpy as np

    from oracle import oracle as O

    O.build()
    threads = max(1, min(max_threads, os.cpu_count() or 1))
    c = wl.cases[0]
    sc = O.Scene(c.V, c.F, bvh=True)
    modes = [m == "exterior" for m in wl.modes]
    n = c.rows.n_rows

    def run(rows_sel):
        t0 = time.perf_counter()
        walks = 0
        for ext in modes:
            r = O.estimate(sc, c.rows, c.basis, wl.walks, c.eps, c.h, exterior=ext, rows_sel=rows_sel, nthreads=threads)
            walks += int((r["discarded"] == 0).sum()) * wl.walks
        return walks, time.perf_counter() - t0

    pilot = np.arange(0, n, max(1, n // max(1, threads)))[:threads]
    w0, t0 = run(pilot)
    rate = w0 / max(t0, 1e-9)
    want = int(max(threads, min(n, target_s * rate / (wl.walks * len(modes)))))
    sel = np.linspace(0, n - 1, want).astype(np.int32)
    walks, dt = run(sel)
    return {"value": walks / dt, "unit": "walks/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sel)} of {n} rows (evenly spaced) x {wl.walks} walks x {len(modes)} operator(s) "
                      f"of {wl.name}, FP64 oracle with its BVH, {threads} OpenMP threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="soup8_53k")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a device copy of this size first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_05581_amd import msk
    from paper_2606_05581_amd import workloads as W

    t = time.perf_counter()
    wl = W.load(args.workload)
    log(f"[bench] workload {wl.name}: {len(wl.cases)} mesh(es), {sum(c.F.shape[0] for c in wl.cases)} triangles, "
        f"{sum(c.rows.n_rows for c in wl.cases)} rows x {wl.walks} walks, {wl.modes} ({time.perf_counter() - t:.1f} s)")
    ctx = msk.Context(0)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    handles = setup(ctx, wl)
    torch.cuda.synchronize()

    # untimed: traversal statistics (counting kernel) for the per-query work
    st = run_step(ctx, wl, handles, collect_stats=1)
    q_st = sum(r["queries_total"] for r in st)
    nodes_q = sum(r["nodes_visited"] for r in st) / q_st
    tris_q = sum(r["tris_tested"] for r in st) / q_st
    flops_q = sum(r["valu_flops"] for r in st) / q_st
    bytes_q = nodes_q * NODE_BYTES + tris_q * TRI_BYTES
    log(f"[bench] per query: {nodes_q:.2f} nodes, {tris_q:.2f} triangles, {bytes_q:.0f} B, {flops_q:.0f} FP32 ops")

    for i in range(args.warmup):
        run_step(ctx, wl, handles)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        recs += run_step(ctx, wl, handles)
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    walks = sum(r["walks_total"] for r in recs)
    queries = sum(r["queries_total"] for r in recs)
    launches = sum(r["walk_launches"] for r in recs)
    kern_ms = sum(r["walk_kernel_ms"] for r in recs)
    value = walks / elapsed
    avg_ms = kern_ms / launches
    q_per_launch = queries / launches
    flops_ach = q_per_launch * flops_q / (avg_ms * 1e-3) / 1e12
    bytes_ach = q_per_launch * bytes_q / (avg_ms * 1e-3) / 1e9

    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        tp = time.perf_counter()
        pr = run_step(ctx, wl, handles, form=msk.FORM_PLAIN)
        torch.cuda.synchronize()
        plain = sum(r["walks_total"] for r in pr) / (time.perf_counter() - tp)
        log(f"[bench] plain form: {plain:.3e} walks/s")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds)
        log(f"[bench] cpu baseline: {cpu['value']:.3e} walks/s on {cpu['cores']} threads")

    line = {
        "metric": "DtN walks/sec + closest-point queries/sec at fixed std-error; batched vs plain",
        "value": value,
        "unit": "walks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "meshes": len(wl.cases),
            "triangles": int(sum(c.F.shape[0] for c in wl.cases)),
            "rows": int(sum(c.rows.n_rows for c in wl.cases)),
            "walks_per_row": wl.walks,
            "operators": "+".join(wl.modes),
            "form": "persistent",
            "accumulation": "f64",
        },
        "queries_per_s": queries / elapsed,
        "steps_per_walk": queries / max(walks, 1),
        "walk_kernel_ms_avg": avg_ms,
        "plain_walks_per_s": plain,
        "persistent_vs_plain": (value / plain) if plain else None,
        "roofline": {
            "bound": "alu",
            "achieved": flops_ach,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops_ach / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(wl.name),
            "kernel": "walk_persistent_kernel",
            "per_query": {"nodes": nodes_q, "triangles": tris_q, "bytes": bytes_q, "fp32_ops": flops_q},
            "memory_achieved_GBs": bytes_ach,
            "memory_frac_of_hbm": bytes_ach / HBM_PEAK_GBS,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
