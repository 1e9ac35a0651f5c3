#!/usr/bin/env python
"""Throughput benchmark of the MI355X DtN walk estimator.

One step = one pass of the hot path over the workload's input, resident on the
GPU before timing starts:
  * batched workloads (several meshes): one replay of the batch graph -- zeroing,
    discard pass, ONE persistent walk launch over all meshes (start sampling,
    Walk-on-Spheres with exact BVH queries, hit basis evaluation, row
    accumulation), finalisation -- for every operator side;
  * single-mesh workloads: estimate_dtn per operator side, then the eigen step
    when the workload asks for eigenpairs.
The plain form (one mesh per launch, one thread per walk, run to completion)
is timed on the same walks for the batched-vs-plain ratio. Prints one JSON
line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KERNEL_NAME = "walk_stream_kernel"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
CLOCK_GHZ = 2.4                  # MI355X peak engine clock
FP32_VECTOR_PEAK_TFLOPS = 157.3  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (dual issue) x 2.4 GHz
FP64_MATRIX_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix-core peak
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_MATRIX_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix-core peak
NODE_BYTES, TRI_BYTES = 128, 48
DEFAULT_WORKLOAD = "batch64_mixed"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    from paper_2606_05581_amd.build import walk_sources_sha

    return walk_sources_sha()


def laplace_sources_sha():
    csrc = os.path.join(ROOT, "paper_2606_05581_amd", "csrc")
    return hashlib.sha256(open(os.path.join(csrc, "laplace.hip"), "rb").read()
                          + open(os.path.join(csrc, "laplace.h"), "rb").read()).hexdigest()[:16]


def laplace_traffic():
    """HBM bytes of all filter steps of the basis leg's full-mesh solve, from
    the committed counter passes, if taken on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_laplace_sh_sphere_2m.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec["filter_traffic_bytes"] if rec.get("source_sha") == laplace_sources_sha() else None


def measured_traffic(workload):
    """HBM bytes per walk-kernel launch from the committed rocprofv3 counter
    passes, if they were taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec["traffic_bytes_per_launch"] if rec.get("source_sha") == kernel_sources_sha() else None


def traffic_record(workload):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    return json.load(open(path)) if os.path.exists(path) else None


def issue_record(workload):
    """VALU issue of the walk kernel from the committed counter passes
    (instructions and active lanes per launch), if taken on the current
    kernel sources (else None)."""
    rec = traffic_record(workload)
    if not rec or rec.get("source_sha") != kernel_sources_sha() or "valu_insts_per_launch" not in rec:
        return None
    issue_peak = 1024 * CLOCK_GHZ * 1e9 / 4  # 1,024 SIMDs, one wave64 VALU instruction per 4 cycles
    ips = rec["valu_insts_per_launch"] / (rec["launch_ms"] * 1e-3)
    return {"achieved": ips, "peak": issue_peak, "unit": "wave64 VALU instructions/s", "frac": ips / issue_peak,
            "active_lanes": rec["active_lanes_per_valu"], "lane_frac": rec["active_lanes_per_valu"] / 64.0,
            "source": f"profiles/traffic_{workload}.json"}


class Runner:
    """Holds the device-resident inputs and runs one step of the hot path."""

    def __init__(self, ctx, wl):
        self.ctx, self.wl = ctx, wl
        self.handles = []
        for c in wl.cases:
            mesh = ctx.build_bvh(c.V, c.F)
            self.handles.append((c, mesh, ctx.rows(mesh, c.rows), ctx.basis(c.basis, c.V.shape[0])))
        self.batched = len(wl.cases) > 1
        self.batches = {}
        self.opts = {}  # tuned launch settings

    def _batch(self, ext, **opts):
        key = (ext, tuple(sorted(opts.items())))
        if key not in self.batches:
            hs = self.handles
            self.batches[key] = self.ctx.batch([h[1] for h in hs], [h[2] for h in hs], [h[3] for h in hs],
                                               [h[0].eps for h in hs], [h[0].h for h in hs], self.wl.walks,
                                               exterior=ext, **opts)
        return self.batches[key]

    def drop_batches(self):
        for b in self.batches.values():
            b.close()
        self.batches = {}

    def se_sample(self):
        """Mesh indices whose standard errors are compared between forms."""
        n = len(self.handles)
        return sorted(set(int(i) for i in np.linspace(0, n - 1, min(4, n)).astype(int)))

    @staticmethod
    def median_se(dtn):
        from paper_2606_05581_amd import msk

        se = dtn.get(msk.FIELD_SE)
        return float(np.median(se[se > 0])) if np.any(se > 0) else 0.0

    def step(self, with_eigen=True, form=None, se_out=None, **opts):
        """One pass; returns a list of per-launch records. With se_out (a
        dict), the median standard error of each sampled mesh is stored."""
        from paper_2606_05581_amd import msk

        opts = {**self.opts, **opts}
        recs = []
        for ext in [m == "exterior" for m in self.wl.modes]:
            if self.batched and form != msk.FORM_PLAIN:
                b = self._batch(ext, **opts)
                recs.append(b.run())
                if se_out is not None:
                    for i in self.se_sample():
                        se_out[(ext, i)] = self.median_se(b.dtn(i))
                continue
            for i, (c, mesh, rows, basis) in enumerate(self.handles):
                kw = dict(opts)
                if form is not None:
                    kw["form"] = form
                d = self.ctx.estimate_dtn(mesh, rows, basis, self.wl.walks, c.eps, c.h, exterior=ext, mesh_id=i,
                                          **kw)
                inf = d.info()
                if se_out is not None and i in self.se_sample():
                    se_out[(ext, i)] = self.median_se(d)
                if with_eigen and self.wl.k > 0 and c.basis.K == c.rows.n_rows:
                    _, _, est = self.ctx.steklov_modes(d, self.wl.k, vectors=False)
                    inf["eigen_ms"] = est["lanczos_ms"]
                    inf["eigen_converged"] = est["converged"]
                recs.append(inf)
                d.close()
        return recs


def psd_leg(ctx):
    """The PSD estimator (Alg. 2) on its own workload: one untimed warm-up call,
    then one timed call (tangent balls, walks, gathers and products; inputs
    resident). Rooflines: the gather kernel against HBM (algorithmic bytes:
    per pair six table rows read (FP32) and, in the two-pass form, five FP64
    update rows written and read back, per row three
    table rows), the symmetric rank-k products against the FP64 matrix peak
    (5 K (K+1) flops per pair)."""
    import torch

    t = time.perf_counter()
    wl = _psd_workload()
    case = wl.cases[0]
    pairs = wl.walks // 2
    mesh = ctx.build_bvh(case.V, case.F)
    rh = ctx.rows(mesh, case.rows)
    bh = ctx.basis(case.basis, case.V.shape[0])
    torch.cuda.synchronize()
    log(f"[bench] psd workload: {case.F.shape[0]} triangles, {case.rows.n_rows} rows x {pairs} pairs, "
        f"K={case.basis.K} (inputs ready in {time.perf_counter() - t:.1f} s)")
    ctx.estimate_psd(mesh, rh, bh, 4, case.eps)  # untimed warm-up
    # untimed: the same walks through the counting kernel, for the walk
    # kernel's algorithmic work (box nodes, triangle tests, FP32 operations)
    st = ctx.estimate_psd(mesh, rh, bh, pairs, case.eps, collect_stats=1)["info"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.estimate_psd(mesh, rh, bh, pairs, case.eps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = r["info"]
    K, n = int(info["K"]), int(info["n_rows"])
    n_pairs = n * pairs
    flops = 5.0 * K * (K + 1) * n_pairs
    fused = bool(info["fused"])
    # algorithmic bytes: per pair six table rows read (the two terminal
    # triangles) plus, in the two-pass form, five update rows written and read
    # back; per row three table rows (the sample's triangle); walk log entries
    # (the table holds the FP32 basis values: 4 bytes per entry; update rows are FP64)
    gbytes = n_pairs * (6.0 * K * 4 + (0.0 if fused else 10.0 * K * 8) + 2 * 16) + n * 3.0 * K * 4
    prod_tf = flops / (info["product_ms"] * 1e-3) / 1e12
    walk_tf = st["valu_flops"] / (info["walk_kernel_ms"] * 1e-3) / 1e12
    walk_q = max(st["walks_total"], 1)
    gath_ms = info["product_ms"] if fused else info["gather_ms"]
    gath = gbytes / (gath_ms * 1e-3) / 1e9
    log(f"[bench] psd: {info['walks_total'] / el:.3e} walks/s; tangent balls {info['tangent_ms']:.1f} ms, walks "
        f"{info['walk_kernel_ms']:.1f} ms, gathers {info['gather_ms']:.1f} ms, products {info['product_ms']:.1f} ms "
        f"({prod_tf:.1f} TFLOP/s{', fused with the gathers' if fused else ''})")
    return {
        "workload": wl.name, "rows": n, "pairs_per_row": pairs, "K": K, "triangles": int(case.F.shape[0]),
        "value": info["walks_total"] / el, "unit": "walks/s", "pairs_per_s": n_pairs / el, "seconds": el,
        "ms": {k: info[k] for k in ("tangent_ms", "walk_kernel_ms", "gather_ms", "product_ms", "total_ms")},
        "mean_radius": info["mean_radius"], "dropped_rows": info["dropped_rows"], "fused": fused,
        "S_trace": float(np.trace(r["S"])),
        "roofline": {
            "product": {"bound": "mfma", "achieved": prod_tf, "peak": FP64_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": prod_tf / FP64_MATRIX_PEAK_TFLOPS, "dtype": "f64"},
            "gather": {"bound": "hbm", "achieved": gath, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gath / HBM_PEAK_GBS, "kernel": "psd_fused_kernel" if fused else "psd_gather_kernel"},
            # the leg's dominant kernel: the ball-start walks, bound like the
            # main walk kernel by VALU issue; its algorithmic FP32 work from
            # the counting pass over the same walks
            "walk": {"bound": "alu", "achieved": walk_tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": walk_tf / FP32_VECTOR_PEAK_TFLOPS, "kernel": "walk_stream_kernel",
                     "per_walk": {"nodes": st["nodes_visited"] / walk_q, "triangles": st["tris_tested"] / walk_q,
                                  "fp32_ops": st["valu_flops"] / walk_q}},
        },
    }


_PSD_WL = {}


def _psd_workload():
    """The 2M-face SH-sphere PSD workload, built once for the PSD and Kelvin legs."""
    from paper_2606_05581_amd import workloads as W

    if "wl" not in _PSD_WL:
        _PSD_WL["wl"] = W.load("psd_sh_sphere_2m", cache=False)
    return _PSD_WL["wl"]


def kelvin_leg(ctx, pairs=64, kill_walks=1 << 20):
    """The exterior estimate in the Kelvin-inverted domain (Sec. 3.3) on the
    SH-displaced sphere of the PSD workload (2.0M faces, 16,384 point rows,
    K = 128), inverted about the origin (inside the shape): one untimed
    warm-up call, then one timed call with inputs resident (inverted tangent
    balls, jump walks from ball points, killing walks from the origin,
    gathers and FP64 products). The build of the inverted hierarchy is timed
    apart. An untimed pass of the counting walk kernel (the same walks)
    tallies the nearest searches' node visits, element tests and FP64
    operations, for the walk kernel's arithmetic roofline against the FP64
    vector peak and its bytes touched (128 B per node, 120 B per element)."""
    import torch

    wl = _psd_workload()
    case = wl.cases[0]
    mesh = ctx.build_bvh(case.V, case.F)
    rh = ctx.rows(mesh, case.rows)
    bh = ctx.basis(case.basis, case.V.shape[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    kv = ctx.kelvin(mesh, np.zeros(3))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    ki = kv.info()
    eps = 1e-5 * ki["radius"]
    log(f"[bench] kelvin workload: {case.F.shape[0]} triangles inverted in {build_s:.2f} s (depth {ki['depth']}), "
        f"{case.rows.n_rows} rows x {pairs} pairs + {kill_walks} killing walks, K={case.basis.K}")
    ctx.estimate_kelvin(kv, rh, bh, 2, 1024, eps)  # untimed warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.estimate_kelvin(kv, rh, bh, pairs, kill_walks, eps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = r["info"]
    q = info["queries_total"]  # tangent-ball bisection steps, jump walks and killing walks
    q_walk = q - int(info["n_rows"]) * 10  # less the bisection's 10 steps per row
    log(f"[bench] kelvin: {info['walks_total'] / el:.3e} walks/s, {q / el:.3e} queries/s; tangent balls "
        f"{info['tangent_ms']:.1f} ms, walks {info['walk_kernel_ms']:.1f} ms, products {info['product_ms']:.1f} ms")
    cs = ctx.estimate_kelvin(kv, rh, bh, pairs, kill_walks, eps, collect_stats=1)["info"]  # untimed: counting kernel
    wk_s = info["walk_kernel_ms"] * 1e-3
    tf = cs["fp64_ops"] / wk_s / 1e12
    gbs = (128 * cs["nodes_visited"] + 120 * cs["elements_tested"]) / wk_s / 1e9
    roof = {"bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "dtype": "f64", "kernel": "kelvin_walk_kernel",
            "per_query": {"nodes": cs["nodes_visited"] / q_walk, "elements": cs["elements_tested"] / q_walk,
                          "fp64_ops": cs["fp64_ops"] / q_walk},
            "bytes_touched": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK_GBS}}
    log(f"[bench] kelvin walk kernel: {tf:.3f} TFLOP/s FP64 ({roof['frac']:.4f} of peak); per query "
        f"{roof['per_query']['nodes']:.1f} nodes, {roof['per_query']['elements']:.1f} elements, "
        f"{roof['per_query']['fp64_ops']:.0f} FP64 ops")
    return {
        "workload": wl.name + " exterior (Kelvin-inverted)", "rows": int(info["n_rows"]), "pairs_per_row": pairs,
        "kill_walks": kill_walks, "K": int(info["K"]), "triangles": int(case.F.shape[0]),
        "value": info["walks_total"] / el, "unit": "walks/s", "queries_per_s": q / el, "seconds": el,
        "inverted_build_s": build_s, "inverted_depth": int(ki["depth"]),
        "ms": {k: info[k] for k in ("tangent_ms", "walk_kernel_ms", "product_ms")},
        "mean_radius": info["mean_radius"], "dropped_rows": info["dropped_rows"],
        "capped_total": info["capped_total"], "steps_per_walk": q_walk / max(info["walks_total"], 1),
        "S_trace": float(np.trace(r["S"])), "S_kill_trace": float(np.trace(r["S_kill"])), "roofline": roof,
    }


def _cpu_threads():
    """Threads the oracle's scipy/BLAS calls may use (the sparse LU of the
    shift-invert solves runs on one)."""
    try:
        from threadpoolctl import threadpool_info

        return max([1] + [int(p.get("num_threads", 1)) for p in threadpool_info()])
    except Exception:
        return 1


def laplace_leg(ctx, K=160, sample_n=48):
    """The mesh-based Galerkin basis (Sec. 5.1): the K = 160 lowest modes of
    the cotangent Laplacian of the 2.0M-face SH-displaced sphere (128 modes +
    32, the paper's sizing), one untimed call on a small mesh, then one timed
    call (host set-up, assembly, filtered subspace iteration, basis table).
    Roofline of the filter step (sparse block product fused with the
    recurrence) against HBM: algorithmic bytes per step = the filtered columns
    read once (gathered rows), the previous ones read and the new ones written
    (8 bytes per vertex and column each) plus the matrix (12 bytes per entry,
    4 per row), summed by the library over the steps. The oracle
    (shift-invert ARPACK) is timed on a bounded sample, the same family at
    20 sample_n^2 faces, with the GPU timed on that sample too."""
    import torch

    from oracle import laplace as LP  # CPU baseline only
    from paper_2606_05581_amd import workloads as W

    Vs, Fs = W.sh_sphere_mesh(sample_n)
    b, _, _, _ = ctx.basis_laplacian(Vs, Fs, K, want_phi=False)  # untimed warm-up
    b.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b, _, _, info_s = ctx.basis_laplacian(Vs, Fs, K, want_phi=False)
    torch.cuda.synchronize()
    gpu_sample_s = time.perf_counter() - t0
    b.close()
    t0 = time.perf_counter()
    LP.laplacian_basis(Vs.astype(np.float64), Fs, K)
    cpu_sample_s = time.perf_counter() - t0
    t = time.perf_counter()
    V, F = W.sh_sphere_mesh()
    log(f"[bench] laplace leg: {V.shape[0]} vertices, {F.shape[0]} faces, K={K} (mesh in "
        f"{time.perf_counter() - t:.1f} s); sample {Vs.shape[0]} vertices: GPU {gpu_sample_s:.3f} s, "
        f"oracle {cpu_sample_s:.2f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b, lam, _, info = ctx.basis_laplacian(V, F, K, want_phi=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b.close()
    n, m = V.shape[0], info["block"]
    filter_steps = info["spmm_calls"] - 2 * (info["iters"] + 1)  # minus the two plain products per iteration
    step_ms = info["filter_ms"] / max(filter_steps, 1)
    gbs = info["filter_bytes"] / (info["filter_ms"] * 1e-3) / 1e9  # per-step widths shrink as columns lock
    log(f"[bench] laplace: {el:.2f} s ({info['iters']} iterations, {filter_steps} filter steps, {step_ms:.3f} ms "
        f"each on average, {gbs:.0f} GB/s, {info['locked']} columns locked at the end; dense "
        f"{info['dense_ms']:.0f} ms, b {info['bound']:.3e})")
    return {
        "workload": "laplace_sh_sphere_2m", "vertices": int(n), "faces": int(F.shape[0]), "K": K, "block": m,
        "value": el, "unit": "s", "higher_is_better": False, "converged": bool(info["converged"]),
        "iters": info["iters"], "filter_steps": int(filter_steps), "last_degree": info["degree"],
        "bound": info["bound"], "max_residual": info["max_residual"], "lambda_K": float(lam[-1]),
        "ms": {k: info[k] for k in ("setup_ms", "assemble_ms", "filter_ms", "dense_ms", "total_ms")},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "kernel": "cheb_gather_kernel",
                     "filter_bytes": info["filter_bytes"], "traffic": laplace_traffic(),
                     "locked_at_end": info["locked"]},
        "sample": {"vertices": int(Vs.shape[0]), "faces": int(Fs.shape[0]), "gpu_s": gpu_sample_s,
                   "gpu_iters": info_s["iters"]},
        "cpu_baseline": {"value": cpu_sample_s, "unit": "s", "cores": _cpu_threads(), "kind": "oracle",
                         "sample": f"K={K} on the {Fs.shape[0]}-face member of the same mesh family"},
    }


def knn_leg(ctx, walks=1024):
    """The point basis (point-based k-NN interpolator) against the per-vertex
    table on the same walks: sh_sphere_2m's 10,000 point rows, `walks` walks
    each, interior; one untimed call per basis, then one timed call each."""
    import torch

    from paper_2606_05581_amd import msk
    from paper_2606_05581_amd import workloads as W

    t = time.perf_counter()
    wl = W.load("sh_sphere_2m", cache=False)
    case = wl.cases[0]
    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    table = ctx.basis(case.basis, case.V.shape[0])
    sigma = 1.5 * float(np.sqrt(case.rows.w.sum() / case.rows.n_rows))
    point = ctx.basis_knn(mesh, case.rows.p, case.rows.n, k=8, sigma=sigma, tau_n=0.8)
    torch.cuda.synchronize()
    log(f"[bench] point-basis leg: {case.F.shape[0]} triangles, {case.rows.n_rows} rows x {walks} walks "
        f"(inputs ready in {time.perf_counter() - t:.1f} s)")
    out = {"workload": "sh_sphere_2m", "rows": int(case.rows.n_rows), "walks_per_row": walks, "k": 8,
           "sigma": sigma, "tau_n": 0.8}
    for name, b in (("table", table), ("point_basis", point)):
        ctx.estimate_dtn(mesh, rows, b, 64, case.eps, case.h).close()  # untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = ctx.estimate_dtn(mesh, rows, b, walks, case.eps, case.h)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        inf = d.info()
        d.close()
        out[name] = {"walks_per_s": inf["walks_total"] / el, "walk_kernel_ms": inf["walk_kernel_ms"],
                     "seconds": el}
    out["point_over_table"] = out["point_basis"]["walks_per_s"] / out["table"]["walks_per_s"]
    log(f"[bench] point basis {out['point_basis']['walks_per_s']:.3e} walks/s, table {out['table']['walks_per_s']:.3e}")
    return out


def _roofs(per_q, queries, ms):
    """Both rooflines of one walk launch from its algorithmic work per query."""
    if not per_q or ms <= 0:
        return None
    flops = queries * per_q["fp32_ops"] / (ms * 1e-3) / 1e12
    gbs = queries * per_q["bytes"] / (ms * 1e-3) / 1e9
    return {"alu": {"achieved": flops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": flops / FP32_VECTOR_PEAK_TFLOPS},
            "hbm_bytes_touched": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS},
            "per_query": per_q}


def config_leg(ctx, name, accum_forms=(0,), se_target=0.0, eigen=True):
    """One of the other configurations at its full size in the persistent
    single-mesh form: walks/s and queries/s of each operator (after an
    untimed warm-up), per-query work from the counting kernel (untimed), the
    eigen step's time for the workload's k, and for several accumulation
    forms their rates and their difference from the FP64 form on the same
    walks."""
    import torch

    from paper_2606_05581_amd import msk
    from paper_2606_05581_amd import workloads as W

    t = time.perf_counter()
    wl = W.load(name)
    c = wl.cases[0]
    mesh = ctx.build_bvh(c.V, c.F)
    rows = ctx.rows(mesh, c.rows)
    basis = ctx.basis(c.basis, c.V.shape[0])
    torch.cuda.synchronize()
    prep = time.perf_counter() - t
    out = {"workload": name, "triangles": int(c.F.shape[0]), "rows": int(c.rows.n_rows), "walks_per_row": wl.walks,
           "operators": {}}
    kw = {"se_target": se_target} if se_target > 0 else {}
    for mode in wl.modes:
        ext = mode == "exterior"
        st = ctx.estimate_dtn(mesh, rows, basis, wl.walks, c.eps, c.h, exterior=ext, collect_stats=1, **kw)
        si = st.info()
        st.close()
        q = max(si["queries_total"], 1)
        per_q = {"nodes": si["nodes_visited"] / q, "triangles": si["tris_tested"] / q,
                 "fp32_ops": si["valu_flops"] / q}
        per_q["bytes"] = per_q["nodes"] * NODE_BYTES + per_q["triangles"] * TRI_BYTES
        forms = {}
        S0 = None
        for a in accum_forms:
            ctx.estimate_dtn(mesh, rows, basis, wl.walks, c.eps, c.h, exterior=ext, accum=a, **kw).close()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d = ctx.estimate_dtn(mesh, rows, basis, wl.walks, c.eps, c.h, exterior=ext, accum=a, **kw)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            inf = d.info()
            rec = {"walks_per_s": inf["walks_total"] / el, "queries_per_s": inf["queries_total"] / el,
                   "steps_per_walk": inf["queries_total"] / max(inf["walks_total"], 1), "seconds": el,
                   "walk_kernel_ms": inf["walk_kernel_ms"], "walk_launches": inf["walk_launches"],
                   "walks_total": inf["walks_total"],
                   "roofline": _roofs(per_q, inf["queries_total"] / max(inf["walk_launches"], 1),
                                      inf["walk_kernel_ms"] / max(inf["walk_launches"], 1))}
            S = d.get(msk.FIELD_S)
            if S0 is None:
                S0 = S
            else:
                rec["max_abs_diff_vs_f64_rel"] = float(np.abs(S - S0).max() / np.abs(S0).max())
            if eigen and wl.k > 0 and c.basis.K == c.rows.n_rows:
                t1 = time.perf_counter()
                ev, _, est = ctx.steklov_modes(d, wl.k, vectors=False)
                rec["eigen"] = {"k": wl.k, "seconds": time.perf_counter() - t1, "lanczos_ms": est["lanczos_ms"],
                                "converged": bool(est["converged"]), "cycles": est["iterations"],
                                "roofline": _eigen_roofs(est)}
                if a != accum_forms[0] and "ev0" in forms.get("_", {}):
                    rec["eigen"]["max_abs_diff_vs_f64_rel"] = float(np.abs(ev - forms["_"]["ev0"]).max() /
                                                                    np.abs(forms["_"]["ev0"]).max())
                forms.setdefault("_", {}).setdefault("ev0", ev)
            d.close()
            forms[{0: "f64", 1: "f32", 2: "compensated_f32"}[a]] = rec
            log(f"[bench] {name} {mode} accum={a}: {rec['walks_per_s']:.3e} walks/s, "
                f"{rec['queries_per_s']:.3e} queries/s")
        forms.pop("_", None)
        out["operators"][mode] = forms
    out["inputs_s"] = prep
    for h in (basis, rows, mesh):
        h.close()
    return out


def _eigen_roofs(est):
    """Rooflines of the eigen step's dense products from the library's event
    sums: the FP32 products with C against the FP32 matrix peak, the FP64
    basis products against the FP64 matrix peak (algorithmic flops 2 M N K)."""
    out = {}
    for key, peak in (("fp32", FP32_MATRIX_PEAK_TFLOPS), ("fp64", FP64_MATRIX_PEAK_TFLOPS)):
        ms, fl, n = est[key + "_product_ms"], est[key + "_product_flops"], est[key + "_products"]
        tf = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        out[key] = {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                    "products": int(n), "ms": ms, "dtype": "f32" if key == "fp32" else "f64"}
    return out


def plain_leaf_sweep(run, leaves=(2, 4, 8)):
    """The plain form (one lane per walk, one launch per mesh) at each BVH
    leaf width, meshes rebuilt in place; returns the rates and the best."""
    import torch

    from paper_2606_05581_amd import msk

    res = {}
    for leaf in leaves:
        for h in run.handles:
            h[1].rebuild(leaf)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        pr = run.step(with_eigen=False, form=msk.FORM_PLAIN)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        res[leaf] = {"walks_per_s": sum(r["walks_total"] for r in pr) / tp,
                     "walks_per_s_walk_kernels": sum(r["walks_total"] for r in pr) / (
                         sum(r["walk_kernel_ms"] for r in pr) * 1e-3)}
        log(f"[bench] plain form, leaf {leaf}: {res[leaf]['walks_per_s']:.3e} walks/s")
    best = max(res, key=lambda k: res[k]["walks_per_s"])
    return res, best


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    """Threads the oracle may use: the process's CPU share (OMP_NUM_THREADS
    where the host sets it, else 16), at most the CPUs it may run on."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    return max(1, min(share, avail)), avail


def cpu_baseline(wl, target_s, max_meshes=8):
    """The oracle (FP64 walks, its own BVH) on a bounded sample of rows, on
    the process's CPU share and on one core."""
    from oracle import oracle as O

    O.build()
    threads, avail = cpu_threads()
    modes = [m == "exterior" for m in wl.modes]
    picks = np.unique(np.linspace(0, len(wl.cases) - 1, min(max_meshes, len(wl.cases))).astype(int))
    scenes = [(i, wl.cases[i], O.Scene(wl.cases[i].V, wl.cases[i].F, bvh=True)) for i in picks]
    most = max(c.rows.n_rows for _, c, _ in scenes)

    def run(rows_per_mesh, nthreads):
        t0 = time.perf_counter()
        walks = 0
        for i, c, sc in scenes:
            sel = np.linspace(0, c.rows.n_rows - 1, min(rows_per_mesh, c.rows.n_rows)).astype(np.int32)
            for ext in modes:
                r = O.estimate(sc, c.rows, c.basis, wl.walks, c.eps, c.h, exterior=ext, rows_sel=sel,
                               nthreads=nthreads, mesh=int(i))
                walks += int((r["discarded"] == 0).sum()) * wl.walks
        return walks, time.perf_counter() - t0

    def grow(nthreads, budget_s, per_mesh):
        # grow the sample until it takes about budget_s (or covers every row)
        walks, dt = run(per_mesh, nthreads)
        while dt < 0.5 * budget_s and per_mesh < most:
            rate = walks / max(dt, 1e-9)
            per_mesh = int(min(max(2 * per_mesh, budget_s * rate / (wl.walks * len(modes) * len(scenes))), most))
            walks, dt = run(per_mesh, nthreads)
        return walks, dt, per_mesh

    walks, dt, per_mesh = grow(threads, target_s, max(1, threads // len(scenes)))
    walks1, dt1, per_mesh1 = grow(1, target_s / 3, 1)
    rows = sum(min(per_mesh, c.rows.n_rows) for _, c, _ in scenes)
    rows1 = sum(min(per_mesh1, c.rows.n_rows) for _, c, _ in scenes)
    return {"value": walks / dt, "unit": "walks/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} rows (evenly spaced, {len(scenes)} of {len(wl.cases)} meshes) x {wl.walks} walks x "
                      f"{len(modes)} operator(s) of {wl.name}; FP64 oracle with its BVH, {threads} OpenMP threads "
                      f"(the process's CPU share; {avail} CPUs visible), {dt:.1f} s",
            "single_core": {"value": walks1 / dt1, "unit": "walks/s", "rows": rows1, "seconds": dt1},
            "cpu_model": cpu_model(), "cpus_visible": avail,
            "parallel_efficiency": (walks / dt) / (threads * walks1 / dt1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-stats", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (unit sphere, soup, 2M-face sphere, exterior scene)")
    ap.add_argument("--configs-only", action="store_true", help="run only the other configurations")
    ap.add_argument("--no-psd", action="store_true", help="skip the PSD estimator (Alg. 2) leg")
    ap.add_argument("--psd-only", action="store_true", help="run only the PSD estimator leg (profiling)")
    ap.add_argument("--no-knn", action="store_true", help="skip the point-basis (k-NN) leg")
    ap.add_argument("--no-laplace", action="store_true", help="skip the mesh Laplacian basis leg")
    ap.add_argument("--laplace-only", action="store_true", help="run only the mesh Laplacian basis leg")
    ap.add_argument("--knn-only", action="store_true", help="run only the point-basis leg")
    ap.add_argument("--no-kelvin", action="store_true", help="skip the Kelvin-inverted exterior leg")
    ap.add_argument("--kelvin-only", action="store_true", help="run only the Kelvin-inverted exterior leg")
    ap.add_argument("--launch", default="", help="fixed launch settings instead of tuning, e.g. chunk=64,regen_min=16")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2606_05581_amd", "tune_cache.jsonl"),
                    help="autotuner results (JSON lines); a stored entry for this workload is reused, else the "
                         "tuner times the candidates and appends one")
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

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.psd_only:
        print(json.dumps({"psd": psd_leg(msk.Context(0))}), flush=True)
        return
    if args.kelvin_only:
        print(json.dumps({"kelvin": kelvin_leg(msk.Context(0))}), flush=True)
        return
    if args.knn_only:
        print(json.dumps({"knn": knn_leg(msk.Context(0))}), flush=True)
        return
    if args.laplace_only:
        print(json.dumps({"laplace": laplace_leg(msk.Context(0))}), flush=True)
        return
    if args.configs_only:
        c0 = msk.Context(0)
        print(json.dumps({"configs": {
            "unit_sphere_320": config_leg(c0, "unit_sphere_320"),
            "soup8_53k": config_leg(c0, "soup8_53k"),
            "sh_sphere_2m": config_leg(c0, "sh_sphere_2m", accum_forms=(0, 1, 2)),
            "exterior200_301k": config_leg(c0, "exterior200_301k", se_target=1e-3)}}), flush=True)
        return
    t = time.perf_counter()
    wl = W.load(args.workload)
    n_tris = int(sum(c.F.shape[0] for c in wl.cases))
    n_rows = int(sum(c.rows.n_rows for c in wl.cases))
    log(f"[bench] workload {wl.name}: {len(wl.cases)} mesh(es), {n_tris} triangles, {n_rows} rows x {wl.walks} "
        f"walks, {wl.modes} (inputs ready in {time.perf_counter() - t:.1f} s)")
    ctx = msk.Context(0)
    run = Runner(ctx, wl)
    torch.cuda.synchronize()
    log("[bench] inputs on the GPU")
    tuned = None
    if args.launch:
        run.opts = {k: int(v) for k, v in (kv.split("=") for kv in args.launch.split(","))}
        leaf = run.opts.pop("leaf", None)
        if leaf is not None:  # BVH leaf width: rebuild the meshes in place
            for h in run.handles:
                h[1].rebuild(leaf)
        log(f"[bench] launch settings: {run.opts}" + (f", leaf {leaf}" if leaf else ""))
    elif not args.no_tune:  # untimed: pick leaf width / chunk / refill threshold / workgroups per CU
        hs = run.handles
        tuned = ctx.autotune([h[1] for h in hs], [h[2] for h in hs], [h[3] for h in hs], [h[0].eps for h in hs],
                             [h[0].h for h in hs], exterior=(wl.modes[0] == "exterior"),
                             cache_path=args.tune_cache or None, repeats=3)
        run.opts = {"chunk": tuned["chunk"], "regen_min": tuned["regen_min"], "blocks_per_cu": tuned["blocks_per_cu"]}
        log(f"[bench] autotuned: {tuned}")

    per_q = None
    if not args.no_stats:  # untimed: traversal statistics (counting kernel) for the per-query work
        st = run.step(with_eigen=False, collect_stats=1)
        run.drop_batches()
        q_st = sum(r["queries_total"] for r in st)
        per_q = {"nodes": sum(r["nodes_visited"] for r in st) / q_st,
                 "triangles": sum(r["tris_tested"] for r in st) / q_st,
                 "fp32_ops": sum(r["valu_flops"] for r in st) / q_st}
        per_q["bytes"] = per_q["nodes"] * NODE_BYTES + per_q["triangles"] * TRI_BYTES
        log(f"[bench] per query: {per_q['nodes']:.2f} nodes, {per_q['triangles']:.2f} triangles, "
            f"{per_q['bytes']:.0f} B, {per_q['fp32_ops']:.0f} FP32 ops")

    for i in range(args.warmup):
        run.step()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        recs += run.step()
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    se_batched = {}
    run.step(with_eigen=False, se_out=se_batched)  # untimed: standard errors of the same step
    run.drop_batches()

    walks = sum(r["walks_total"] for r in recs)
    queries = sum(r["queries_total"] for r in recs)
    launches = sum(r["walk_launches"] for r in recs)
    kern_ms = sum(r["walk_kernel_ms"] for r in recs)
    value = walks / elapsed
    avg_ms = kern_ms / launches
    q_per_launch = queries / launches

    plain = None
    if not args.no_plain:
        se_plain = {}
        run.step(with_eigen=False, form=msk.FORM_PLAIN, se_out=se_plain)  # untimed: same walks, same se
        # the plain form at its own best BVH leaf width (the walks do not depend on it)
        sweep, best = plain_leaf_sweep(run)
        plain = {"walks_per_s": sweep[best]["walks_per_s"],
                 "walks_per_s_walk_kernels": sweep[best]["walks_per_s_walk_kernels"],
                 "leaf": best, "leaf_sweep": {str(k): v for k, v in sweep.items()},
                 "launches": len(run.handles) * len(wl.modes),
                 "median_se_ratio": float(np.median([se_batched[k] / se_plain[k] for k in se_plain
                                                     if se_plain[k] > 0]))}
        log(f"[bench] plain form at its best leaf width {best}: {plain['walks_per_s']:.3e} walks/s")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds)
        log(f"[bench] cpu baseline: {cpu['value']:.3e} walks/s on {cpu['cores']} threads")

    roof = None
    if per_q is not None:
        # both rooflines of the dominant kernel from its algorithmic work per
        # query; the binding one is the larger fraction of its peak
        flops_ach = q_per_launch * per_q["fp32_ops"] / (avg_ms * 1e-3) / 1e12
        bytes_ach = q_per_launch * per_q["bytes"] / (avg_ms * 1e-3) / 1e9
        mem = {"bound": "hbm", "achieved": bytes_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": bytes_ach / HBM_PEAK_GBS}
        alu = {"bound": "alu", "achieved": flops_ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": flops_ach / FP32_VECTOR_PEAK_TFLOPS}
        # the kernel is bound by VALU issue at a third of the lanes (counters),
        # so the headline is the arithmetic roofline of its algorithmic work;
        # the bytes it touches per query (mostly served by LDS, L2 and MALL)
        # and the measured HBM traffic stand beside it
        roof = dict(alu)
        tr = traffic_record(wl.name)
        roof.update({"traffic": measured_traffic(wl.name), "kernel": KERNEL_NAME, "per_query": per_q,
                     "traffic_source": ({"launch_ms": tr.get("launch_ms"), "launch": tr.get("launch"),
                                         "profile": f"profiles/traffic_{wl.name}.json"} if tr else None),
                     "queries_per_launch": q_per_launch, "launch_ms": avg_ms, "bytes_touched": mem,
                     "valu_issue": issue_record(wl.name)})
    eig = [r["eigen_ms"] for r in recs if "eigen_ms" in r]
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
            "triangles": n_tris,
            "rows": n_rows,
            "walks_per_row": wl.walks,
            "operators": "+".join(wl.modes),
            "form": "batched persistent, one graph" if run.batched else "persistent",
            "accumulation": "f64",
            "eigenpairs": wl.k,
            "tuned": tuned,
        },
        "queries_per_s": queries / elapsed,
        "steps_per_walk": queries / max(walks, 1),
        "walk_kernel_ms_avg": avg_ms,
        "walks_per_s_walk_kernels": walks / (kern_ms * 1e-3),
        "eigen_ms_avg": sum(eig) / len(eig) if eig else None,
        "plain": plain,
        "median_se": {"sample": f"meshes {run.se_sample()}", "per_mesh": [se_batched[k] for k in sorted(se_batched)]},
        "vs_plain": (value / plain["walks_per_s"]) if plain else None,
        "vs_plain_walk_kernels": (walks / (kern_ms * 1e-3) / plain["walks_per_s_walk_kernels"]) if plain else None,
        "roofline": roof,
        "cpu_baseline": cpu,
        "configs": None if args.no_configs else {
            "unit_sphere_320": config_leg(ctx, "unit_sphere_320"),
            "soup8_53k": config_leg(ctx, "soup8_53k"),
            "sh_sphere_2m": config_leg(ctx, "sh_sphere_2m", accum_forms=(0, 1, 2)),
            "exterior200_301k": config_leg(ctx, "exterior200_301k", se_target=1e-3),
        },
        "psd": None if args.no_psd else psd_leg(ctx),
        "kelvin": None if args.no_kelvin else kelvin_leg(ctx),
        "knn": None if args.no_knn else knn_leg(ctx),
        "laplace": None if args.no_laplace else laplace_leg(ctx),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
