"""GPU parity of the exterior estimate without its killing term (Sec. 3.3,
exterior Beurling-Deny form; the paper's default exterior operator, Sec. 4)
against the oracle (whose sphere factor (1-(1+h)^-(l+1))/h - 1/(1+h) is pinned
on the CPU). Bar: every entry within 4 combined standard errors of the
oracle's; on the same walks the result equals the full exterior estimate less
(w_i / (h W_i)) escaped_i b(s_i) to rounding; rows of a partition-of-unity
basis sum to zero."""
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


def test_jump_only_parity_and_identity(ctx, oracle_mod):
    from paper_2606_05581_amd import msk

    case = W.soup8_53k(N=300, walks=64).cases[0]
    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    bh = ctx.basis(case.basis, case.V.shape[0])
    Wk = 64
    dj = ctx.estimate_dtn(mesh, rows, bh, Wk, case.eps, case.h, exterior=True, seed=5, jump_only=1)
    df = ctx.estimate_dtn(mesh, rows, bh, Wk, case.eps, case.h, exterior=True, seed=5)
    Sj, sej, disc = dj.get(msk.FIELD_S), dj.get(msk.FIELD_SE), dj.get(msk.FIELD_ROW_DISCARDED)
    Sf = df.get(msk.FIELD_S)
    esc = dj.get(msk.FIELD_ROW_ESCAPED)
    assert np.array_equal(esc, df.get(msk.FIELD_ROW_ESCAPED)) and esc.sum() > 0
    # identity on the same walks: the killing part of row i is (w_i / (h W)) escaped_i b(s_i)
    tab = case.basis
    Fv = case.F
    bs = np.zeros_like(Sf)
    for i in range(case.rows.n_rows):
        for c in range(3):
            v = Fv[case.rows.tri[i], c]
            for e in range(tab.rowptr[v], tab.rowptr[v + 1]):
                bs[i, tab.col[e]] += float(case.rows.bary[i, c]) * float(tab.val[e])
    scale = np.where(disc == 1, 0.0, case.rows.w / case.h)
    kill = scale[:, None] * (esc / Wk)[:, None] * bs
    assert np.allclose(Sf - Sj, kill, rtol=1e-9, atol=1e-12 * np.abs(Sf).max())
    sc = oracle_mod.Scene(case.V, case.F, bvh=True)
    r = oracle_mod.estimate(sc, case.rows, case.basis, Wk, case.eps, case.h, exterior=True, seed=5, nthreads=8,
                            jump_only=True)
    So, seo = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, Wk, r["discarded"])
    bad = np.abs(Sj - So) > 4 * np.sqrt(sej ** 2 + seo ** 2) + 1e-9 * np.abs(So).max()
    print(f"[jump only] soup exterior: entries outside 4 combined se {int(bad.sum())} of {bad.size}, escaped walks "
          f"{int(esc.sum())}, |killing part| max {np.abs(kill).max():.3e}", flush=True)
    assert np.array_equal(disc, r["discarded"])
    assert not bad.any()


def test_jump_only_rows_sum_to_zero(ctx):
    from paper_2606_05581_amd import msk

    wl = W.unit_sphere_320()
    c = wl.cases[0]
    rows = W.point_rows(c.V.astype(np.float64), c.F, 120, np.random.default_rng(3))
    mesh = ctx.build_bvh(c.V, c.F)
    rh = ctx.rows(mesh, rows)
    bh = ctx.basis(c.basis, c.V.shape[0])  # hat basis: a partition of unity
    d = ctx.estimate_dtn(mesh, rh, bh, 256, c.eps, c.h, exterior=True, seed=2, jump_only=1)
    S = d.get(msk.FIELD_S)
    f = ctx.estimate_dtn(mesh, rh, bh, 256, c.eps, c.h, exterior=True, seed=2)
    Sf = f.get(msk.FIELD_S)
    print(f"[jump only] sphere: max |row sum| {np.abs(S.sum(1)).max():.2e} (full form: "
          f"{np.abs(Sf.sum(1)).max():.2e})", flush=True)
    assert np.abs(S.sum(1)).max() < 1e-6 * np.abs(S).max()
    assert np.abs(Sf.sum(1)).max() > 0.1 * np.abs(Sf).max()  # the killing term does act on constants


def test_jump_only_argument_errors(ctx):
    from paper_2606_05581_amd import msk

    c = W.unit_sphere_320().cases[0]
    mesh = ctx.build_bvh(c.V, c.F)
    hat = ctx.rows(mesh, c.rows)
    bh = ctx.basis(c.basis, c.V.shape[0])
    with pytest.raises(msk.MskError) as e:
        ctx.estimate_dtn(mesh, hat, bh, 16, c.eps, c.h, exterior=True, jump_only=1)
    assert e.value.status == msk.ERR_INVALID_ARG
    pts = ctx.rows(mesh, W.point_rows(c.V.astype(np.float64), c.F, 50, np.random.default_rng(1)))
    with pytest.raises(msk.MskError) as e:
        ctx.estimate_dtn(mesh, pts, bh, 16, c.eps, c.h, exterior=False, jump_only=1)
    assert e.value.status == msk.ERR_INVALID_ARG
