"""Shared checks of the GPU parity tests: entries against the oracle's within
4 combined standard errors, and the walk-by-walk divergence report."""
import numpy as np


def terminal_points(V, F, status, tri, bary12):
    """World positions of terminal points (NaN for walks without one)."""
    ok = (status == 0) | (status == 2)
    t = np.where(ok, tri, 0)
    l1, l2 = bary12[..., 0].astype(np.float64), bary12[..., 1].astype(np.float64)
    lam = np.stack([1 - l1 - l2, l1, l2], -1)
    P = np.einsum("...c,...ck->...k", lam, V.astype(np.float64)[F[t]])
    P[~ok] = np.nan
    return P


def parity_report(g, o, label, case):
    """Entries within 4 combined se; a walk diverges from the oracle's when
    its status, query count or terminal point (beyond 1e-5 of the scene
    radius) differ. Terminal points on an edge shared by two triangles are the
    same point whichever triangle a rounding tie names."""
    tol = 4.0 * np.sqrt(g["se"] ** 2 + o["se"] ** 2)
    scale = np.abs(o["S"]).max()
    diff = np.abs(g["S"] - o["S"])
    z = diff / np.maximum(tol / 4.0, 1e-300)
    viol = diff > tol + 1e-12 * scale
    ran = o["log_status"] >= 0
    Pg = terminal_points(case.V, case.F, g["status"], g["tri"], g["bary"])
    Po = terminal_points(case.V, case.F, o["log_status"], o["log_tri"], o["log_bary"])
    R = np.linalg.norm(case.V - 0.5 * (case.V.min(0) + case.V.max(0)), axis=1).max()
    dp = np.linalg.norm(Pg - Po, axis=-1)
    far = np.where(np.isnan(dp), np.isnan(Pg[..., 0]) != np.isnan(Po[..., 0]), dp > 1e-5 * R)
    div_mask = (g["status"] != o["log_status"]) | (g["nq"] != o["log_nquery"]) | far
    div = div_mask[ran].mean()
    other_tri = (g["tri"] != o["log_tri"])[ran & ~div_mask].mean()
    print(f"[{label}] max z {z[np.isfinite(z)].max():.3f}  violations {viol.sum()}/{viol.size}  "
          f"divergent walks {div:.4%}  (same walk, other triangle of a shared edge: {other_tri:.4%})", flush=True)
    return viol, div




def _table_rows(basis, verts, weights, n_out, K, out_rows):
    """Scatter-add weights[i] * table[verts[i]] into an n_out x K array at
    row out_rows[i] (the CSR basis table, vertex by vertex)."""
    acc = np.zeros((n_out, K))
    rp = basis.rowptr.astype(np.int64)
    lens = rp[verts + 1] - rp[verts]
    keep = (lens > 0) & (weights != 0.0)
    verts, weights, out_rows, lens = verts[keep], weights[keep], out_rows[keep], lens[keep]
    if verts.size == 0:
        return acc
    rep = np.repeat(np.arange(verts.size), lens)
    pos = rp[verts][rep] + (np.arange(rep.size) - np.repeat(np.cumsum(lens) - lens, lens))
    np.add.at(acc, (out_rows[rep], basis.col[pos].astype(np.int64)),
              weights[rep] * basis.val[pos].astype(np.float64))
    return acc


def reconstruct_from_log(oracle_mod, case, status, tri, bary, exterior, jump_only=False):
    """S of point rows rebuilt on the CPU from a walk log alone (status,
    terminal triangle and the barycentrics of its vertices 1 and 2, per row and
    walk): the row sum of c = b(s) - b(t) over the walks that hit or were
    capped, plus b(s) for each walk that escaped (0 in the jump-only form),
    finalised by the oracle's Alg. 1 weights. A row whose walks did not run
    (discarded) keeps zero weight."""
    rows = case.rows
    n, W = status.shape
    K = int(case.basis.K)
    F = case.F.astype(np.int64)
    r = np.arange(n)
    lam_s = rows.bary.astype(np.float64)
    bs = sum(_table_rows(case.basis, F[rows.tri, c], lam_s[:, c], n, K, r) for c in range(3))
    ended = (status == 0) | (status == 2)
    run = status >= 0
    n_bs = (run.sum(1) if not jump_only else ended.sum(1)).astype(np.float64)
    l1, l2 = bary[..., 0].astype(np.float64), bary[..., 1].astype(np.float64)
    lam = np.stack([1.0 - l1 - l2, l1, l2], -1)[ended]  # one row per ended walk
    rr = np.broadcast_to(r[:, None], status.shape)[ended]
    t = tri[ended].astype(np.int64)
    bt = sum(_table_rows(case.basis, F[t, c], lam[:, c], n, K, rr) for c in range(3))
    acc = n_bs[:, None] * bs - bt
    disc = (~run).all(1).astype(np.int32)
    S, _ = oracle_mod.finalize(acc, np.zeros_like(acc), rows.w, case.h, W, disc)
    return S


def check_log_reconstruction(oracle_mod, case, g, o, exterior, label, jump_only=False, rtol_gpu=1e-12,
                             rtol_oracle=1e-7):
    """Both estimates equal their own walk logs' reconstruction (the GPU's
    accumulation tables, flushes and finalisation; the oracle's row sums), so
    the remaining GPU-oracle difference is the divergent walks' alone. The GPU
    accumulates the very FP32 barycentrics it logs, in FP64: its bar is FP64
    summation order (1e-12 of the largest entry). The oracle accumulates FP64
    barycentrics and logs them rounded to FP32: its bar is 1e-7. Returns the
    largest relative deviations (GPU, oracle)."""
    scale = max(np.abs(o["S"]).max(), 1e-300)
    Sg = reconstruct_from_log(oracle_mod, case, g["status"], g["tri"], g["bary"], exterior, jump_only)
    So = reconstruct_from_log(oracle_mod, case, o["log_status"], o["log_tri"], o["log_bary"], exterior, jump_only)
    dg = np.abs(g["S"] - Sg).max() / scale
    do = np.abs(o["S"] - So).max() / scale
    print(f"[{label}] S rebuilt from the walk log: GPU within {dg:.2e}, oracle within {do:.2e} of the largest entry",
          flush=True)
    assert dg <= rtol_gpu and do <= rtol_oracle
    return dg, do
