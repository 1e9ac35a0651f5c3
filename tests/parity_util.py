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


