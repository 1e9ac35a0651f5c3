"""Batched estimate (many meshes, one persistent launch in a HIP graph).

Every batch member runs the same walks as a single-mesh estimate with the
member's index in the Philox counter: identical walk counters and queries,
S equal up to the order of floating-point additions. The captured graph is
replayed several times with other GPU work in between, each replay checked.
One member is also checked against the CPU oracle.
"""
import numpy as np
import pytest

from paper_2606_05581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2606_05581_amd import msk

    assert torch.cuda.is_available()
    c = msk.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def small_batch():
    # 6 meshes of the batch workload's four kinds, small enough for the oracle
    return W.batch64_mixed(n_meshes=6, walks=64, face_lo=2e3, face_hi=2e4, rows_lo=64, rows_hi=160, seed=77)


def _handles(ctx, wl):
    hs = []
    for c in wl.cases:
        m = ctx.build_bvh(c.V, c.F)
        hs.append((c, m, ctx.rows(m, c.rows), ctx.basis(c.basis, c.V.shape[0])))
    return hs


def test_batch_matches_single_mesh_runs_and_replays(ctx, small_batch):
    import torch

    from paper_2606_05581_amd import msk

    wl = small_batch
    hs = _handles(ctx, wl)
    eager = []
    for i, (c, m, r, b) in enumerate(hs):
        d = ctx.estimate_dtn(m, r, b, wl.walks, c.eps, c.h, mesh_id=i)
        eager.append((d.get(msk.FIELD_S), d.get(msk.FIELD_ROW_QUERIES), d.get(msk.FIELD_ROW_DISCARDED)))
    B = ctx.batch([h[1] for h in hs], [h[2] for h in hs], [h[3] for h in hs], [c.eps for c in wl.cases],
                  [c.h for c in wl.cases], wl.walks)
    for rep in range(3):
        info = B.run()
        print(f"[batch replay {rep}] walks {info['walks_total']} queries {info['queries_total']} "
              f"walk kernel {info['walk_kernel_ms']:.3f} ms graph {info['total_ms']:.3f} ms", flush=True)
        for i, (S0, q0, d0) in enumerate(eager):
            v = B.dtn(i)
            S = v.get(msk.FIELD_S)
            assert np.array_equal(v.get(msk.FIELD_ROW_QUERIES), q0)
            assert np.array_equal(v.get(msk.FIELD_ROW_DISCARDED), d0)
            assert np.allclose(S, S0, rtol=0, atol=1e-11 * max(1.0, np.abs(S0).max()))
        # unrelated eager GPU work between replays
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert float((x * x).sum()) > 0
    plain = ctx.batch([h[1] for h in hs], [h[2] for h in hs], [h[3] for h in hs], [c.eps for c in wl.cases],
                      [c.h for c in wl.cases], wl.walks, form=msk.FORM_PLAIN)
    plain.run()
    for i, (S0, q0, d0) in enumerate(eager):
        v = plain.dtn(i)
        assert np.array_equal(v.get(msk.FIELD_ROW_QUERIES), q0)
        assert np.allclose(v.get(msk.FIELD_S), S0, rtol=0, atol=1e-11 * max(1.0, np.abs(S0).max()))


def test_batched_one_shot_and_oracle_parity(ctx, oracle_mod, small_batch):
    from paper_2606_05581_amd import msk

    wl = small_batch
    hs = _handles(ctx, wl)
    outs = ctx.estimate_dtn_batched([h[1] for h in hs], [h[2] for h in hs], [h[3] for h in hs],
                                    [c.eps for c in wl.cases], [c.h for c in wl.cases], wl.walks)
    for i in (1, 4):
        c = wl.cases[i]
        sc = oracle_mod.Scene(c.V, c.F, bvh=True)
        r = oracle_mod.estimate(sc, c.rows, c.basis, wl.walks, c.eps, c.h, exterior=False, mesh=i)
        So, seo = oracle_mod.finalize(r["acc"], r["acc2"], c.rows.w, c.h, wl.walks, r["discarded"])
        Sg, seg = outs[i].get(msk.FIELD_S), outs[i].get(msk.FIELD_SE)
        assert np.array_equal(outs[i].get(msk.FIELD_ROW_DISCARDED), r["discarded"])
        tol = 4 * np.sqrt(seg ** 2 + seo ** 2) + 1e-12 * np.abs(So).max()
        bad = np.abs(Sg - So) > tol
        print(f"[batch member {i}] tris {c.F.shape[0]} rows {c.rows.n_rows}: entries outside 4 combined se: "
              f"{bad.sum()}/{bad.size}", flush=True)
        assert bad.sum() == 0


def test_leaf_width_changes_no_walk_and_autotune(ctx):
    """The traversal is exact, so rebuilding the BVH with another leaf width
    leaves every walk (status, triangle, barycentrics, queries) unchanged; the
    autotuner returns settings that run the same walks."""
    from paper_2606_05581_amd import msk

    wl = W.soup8_53k(N=300, walks=64)
    c = wl.cases[0]
    m = ctx.build_bvh(c.V, c.F, leaf_size=4)
    r = ctx.rows(m, c.rows)
    b = ctx.basis(c.basis, c.V.shape[0])

    def run(**kw):
        d = ctx.estimate_dtn(m, r, b, 64, c.eps, c.h, record_log=1, **kw)
        return {k: d.get(f) for k, f in [("st", msk.FIELD_LOG_STATUS), ("tri", msk.FIELD_LOG_TRI),
                                          ("bary", msk.FIELD_LOG_BARY), ("q", msk.FIELD_LOG_QUERIES)]}

    ref = run()
    for leaf in (1, 2, 8):
        ctx._check(msk.lib().msk_mesh_rebuild(ctx.h, m.h, leaf))
        got = run()
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (leaf, k)
    res = ctx.autotune([m], [r], [b], [c.eps], [c.h], trial_rows=256, trial_walks=16, repeats=1,
                       leaf=[2, 4], chunk=[32, 64], regen_min=[1, 16], blocks_per_cu=[4, 8])
    print(f"[autotune soup8 N=300] {res}", flush=True)
    assert res["leaf"] in (2, 4) and res["chunk"] in (32, 64) and res["trials"] >= 8 and res["walks_per_s"] > 0
    got = run(chunk=res["chunk"], regen_min=res["regen_min"], blocks_per_cu=res["blocks_per_cu"])
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k
