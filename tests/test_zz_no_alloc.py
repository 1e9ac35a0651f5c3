"""The allocation-free estimate (msk_estimate_dtn_noalloc) against the
allocating one (msk_estimate_dtn), through the C ABI.

Both run the same walks on the same inputs (same Philox streams), so S and
se agree to FP64 rounding of the accumulation order; the fixed workspace is
reused by the second call, which has fewer rows than the first and must not
see the first call's sums. A problem too large for the workspace is refused.
"""
import numpy as np
import pytest

from paper_2606_05581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2606_05581_amd import msk

    assert torch.cuda.is_available(), "GPU test needs a visible MI355X"
    c = msk.Context(0)
    yield c
    c.close()


def _both(ctx, case, walks, exterior, **opts):
    import torch

    from paper_2606_05581_amd import msk

    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    basis = ctx.basis(case.basis, case.V.shape[0])
    ref = ctx.estimate_dtn(mesh, rows, basis, walks, case.eps, case.h, exterior=exterior, **opts)
    S = torch.full((rows.n, basis.K), float("nan"), dtype=torch.float64, device="cuda")
    se = torch.full_like(S, float("nan"))
    info = ctx.estimate_dtn_noalloc(mesh, rows, basis, walks, case.eps, case.h, S, se, exterior=exterior, **opts)
    torch.cuda.synchronize()
    return ref, S.cpu().numpy(), se.cpu().numpy(), info, (mesh, rows, basis)


def _check(ref, S, se, info, label):
    from paper_2606_05581_amd import msk

    S0, se0 = ref.get(msk.FIELD_S), ref.get(msk.FIELD_SE)
    ri = ref.info()
    scale = np.abs(S0).max()
    dS = np.abs(S - S0).max() / scale
    dse = np.abs(se - se0).max() / max(np.abs(se0).max(), 1e-300)
    print(f"[no-alloc] {label}: {info['walks_total']} walks, max |S - S_alloc| / max|S| = {dS:.2e}, "
          f"se {dse:.2e}", flush=True)
    assert np.isfinite(S).all() and np.isfinite(se).all()
    assert dS <= 1e-12 and dse <= 1e-9
    for k in ("walks_total", "queries_total", "escaped_total", "capped_total", "discarded_rows", "n_rows", "K"):
        assert info[k] == ri[k], k


def test_noalloc_matches_the_allocating_estimate_twice(ctx):
    """First the 2,000-row soup (exterior, point rows, 2,000 columns: close to
    the workspace's size), then the 162-row unit sphere (interior, hat rows):
    each equals msk_estimate_dtn on the same inputs."""
    big = W.soup8_53k(N=2000, walks=64).cases[0]
    ref, S, se, info, _ = _both(ctx, big, 64, True)
    _check(ref, S, se, info, "soup8 2,000 rows x 2,000 columns, exterior")
    small = W.unit_sphere_320().cases[0]
    ref, S, se, info, _ = _both(ctx, small, 128, False)
    _check(ref, S, se, info, "unit sphere 162 rows, interior (second call, smaller)")
    assert np.abs(S.sum(1)).max() <= 1e-9 * np.abs(S).max()


def test_noalloc_forms_and_refusals(ctx):
    """The plain form and the compensated accumulation run through it too; a
    workspace too small for the problem, a log or an adaptive walk count is
    refused with INVALID_ARG before any work."""
    import torch

    from paper_2606_05581_amd import msk

    small = W.soup8_53k(N=300, walks=32).cases[0]
    ref, S, se, info, _ = _both(ctx, small, 32, False, form=1)
    _check(ref, S, se, info, "soup8 300 rows, plain form")
    ref, S, se, info, (mesh, rows, basis) = _both(ctx, small, 32, False, accum=2)
    _check(ref, S, se, info, "soup8 300 rows, compensated FP32 partial sums")
    out = torch.zeros((rows.n, basis.K), dtype=torch.float64, device="cuda")
    for bad in ({"record_log": 1}, {"se_target": 1e-3}):
        with pytest.raises(msk.MskError) as ei:
            ctx.estimate_dtn_noalloc(mesh, rows, basis, 8, small.eps, small.h, out, out.clone(), **bad)
        assert ei.value.status == msk.ERR_INVALID_ARG
    # 2,100 rows x 2,100 columns need 16 * 2100^2 + ... > 64 MiB
    over = W.soup8_53k(N=2100, walks=8).cases[0]
    m2 = ctx.build_bvh(over.V, over.F)
    r2 = ctx.rows(m2, over.rows)
    b2 = ctx.basis(over.basis, over.V.shape[0])
    S2 = torch.zeros((r2.n, b2.K), dtype=torch.float64, device="cuda")
    with pytest.raises(msk.MskError) as ei:
        ctx.estimate_dtn_noalloc(m2, r2, b2, 8, over.eps, over.h, S2, S2.clone())
    assert ei.value.status == msk.ERR_INVALID_ARG and "workspace" in str(ei.value)
