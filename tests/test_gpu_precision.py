"""Precision variants of the row accumulation against the FP64 oracle.

The walks are FP32 geometry in every variant; what differs is how a
wavefront's partial row sums are kept in LDS before they reach the FP64
rows: FP64 (accum 0), plain FP32 (accum 1) or compensated FP32 pairs (accum
2, TwoSum per slot). Each variant is compared entry by entry with the oracle
(4 combined standard errors) and with the FP64 form on the same walks, and
its error is printed.
"""
import numpy as np
import pytest

from paper_2606_05581_amd import workloads as W
from parity_util import parity_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2606_05581_amd import msk

    assert torch.cuda.is_available(), "GPU test needs a visible MI355X"
    c = msk.Context(0)
    yield c
    c.close()


def _run(ctx, case, walks, exterior, **opts):
    from paper_2606_05581_amd import msk

    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    basis = ctx.basis(case.basis, case.V.shape[0])
    d = ctx.estimate_dtn(mesh, rows, basis, walks, case.eps, case.h, exterior=exterior, record_log=1, **opts)
    return dict(S=d.get(msk.FIELD_S), se=d.get(msk.FIELD_SE), status=d.get(msk.FIELD_LOG_STATUS),
                tri=d.get(msk.FIELD_LOG_TRI), bary=d.get(msk.FIELD_LOG_BARY), nq=d.get(msk.FIELD_LOG_QUERIES))


@pytest.fixture(scope="module")
def soup_runs(ctx, oracle_mod):
    wl = W.soup8_53k(N=300, walks=256)
    case = wl.cases[0]
    out = {}
    for exterior in (False, True):
        sc = oracle_mod.Scene(case.V, case.F, bvh=True)
        r = oracle_mod.estimate(sc, case.rows, case.basis, wl.walks, case.eps, case.h, exterior=exterior, log=True)
        S, se = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, wl.walks, r["discarded"])
        r.update(S=S, se=se)
        runs = {a: _run(ctx, case, wl.walks, exterior, accum=a) for a in (0, 1, 2)}
        out[exterior] = (case, r, runs)
    return out


@pytest.mark.parametrize("exterior", [False, True])
@pytest.mark.parametrize("accum", [0, 1, 2])
def test_accumulation_against_oracle(soup_runs, exterior, accum):
    case, o, runs = soup_runs[exterior]
    g = runs[accum]
    name = {0: "FP64", 1: "FP32", 2: "compensated FP32"}[accum]
    label = f"soup8 N=300 x 256 {'exterior' if exterior else 'interior'}, {name} partial sums"
    viol, div = parity_report(g, o, label, case)
    scale = np.abs(o["S"]).max()
    err_o = np.abs(g["S"] - o["S"]).max() / scale
    se_med = np.median(o["se"][o["se"] > 0]) / scale
    print(f"[{label}] max |S - S_oracle| / max|S| = {err_o:.3e} (median se / max|S| = {se_med:.3e})", flush=True)
    assert viol.sum() == 0
    assert div < (0.02 if exterior else 0.01)


@pytest.mark.parametrize("exterior", [False, True])
def test_compensated_sums_match_fp64_to_rounding(soup_runs, exterior):
    """Same walks in all three variants (identical logs). Against the FP64
    form, the plain FP32 partial sums carry an error of order u times the
    chunk length; the compensated pairs stay at FP64 rounding level."""
    case, o, runs = soup_runs[exterior]
    a, b, c = runs[0], runs[1], runs[2]
    for k in ("status", "tri", "nq"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    scale = np.abs(a["S"]).max()
    e1 = np.abs(b["S"] - a["S"]).max() / scale
    e2 = np.abs(c["S"] - a["S"]).max() / scale
    s1 = np.abs(b["se"] - a["se"]).max() / np.abs(a["se"]).max()
    s2 = np.abs(c["se"] - a["se"]).max() / np.abs(a["se"]).max()
    print(f"[precision {'exterior' if exterior else 'interior'}] against the FP64 form: FP32 partial sums "
          f"{e1:.2e} (se {s1:.2e}), compensated FP32 {e2:.2e} (se {s2:.2e}), relative to the largest entry",
          flush=True)
    assert e1 < 1e-5
    assert e2 < 1e-11
    assert s2 < 1e-9
