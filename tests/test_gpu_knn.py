"""GPU parity of the point basis (Appendix, point-based k-NN interpolator).

The GPU finds the k nearest samples on a uniform grid in FP32; the oracle by
FP64 brute force. Bar: identical neighbour lists (order included) for at least
99.9% of queries, weights within 1e-5 where the lists agree; estimates with
the point basis within 4 combined standard errors of the oracle's, interior
rows summing to zero; plain and persistent forms identical.
"""
import math

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


@pytest.fixture(scope="module")
def soup():
    case = W.soup8_53k(N=300, walks=64).cases[0]
    sigma = 1.5 * math.sqrt(float(case.rows.w.sum()) / case.rows.n_rows)
    knn = dict(points=case.rows.p.astype(np.float64), normals=case.rows.n.astype(np.float64), k=8, sigma=sigma,
               tau=0.8)
    return case, knn


def test_knn_eval_matches_brute_force(ctx, oracle_mod, soup):
    import torch

    case, knn = soup
    mesh = ctx.build_bvh(case.V, case.F)
    b = ctx.basis_knn(mesh, knn["points"], knn["normals"], k=8, sigma=knn["sigma"], tau_n=0.8)
    rng = np.random.default_rng(11)
    Q, tri, _ = W.area_uniform_points(case.V.astype(np.float64), case.F, 3000, rng)
    _, fn = W.face_geometry(case.V.astype(np.float64), case.F)
    Nq = fn[tri]
    # a few queries exactly at sample points and far outside the cloud
    Q = np.concatenate([Q, knn["points"][:50], [[3.0, -2.0, 1.0]]])
    Nq = np.concatenate([Nq, knn["normals"][:50], [[0.0, 0.0, 1.0]]])
    idx, w = ctx.eval_knn(b, torch.tensor(Q, dtype=torch.float32, device="cuda"),
                          torch.tensor(Nq, dtype=torch.float32, device="cuda"))
    idx, w = idx.cpu().numpy(), w.cpu().numpy()
    same, wdiff = 0, 0.0
    for i in range(Q.shape[0]):
        q32 = Q[i].astype(np.float32).astype(np.float64)
        oi, ow = oracle_mod.knn_weights(knn["points"].astype(np.float32).astype(np.float64), knn["normals"], q32,
                                        Nq[i], 8, knn["sigma"], 0.8)
        if list(oi) == list(idx[i]):
            same += 1
            wdiff = max(wdiff, float(np.abs(ow - w[i]).max()))
    frac = same / Q.shape[0]
    print(f"[knn eval] identical neighbour lists {frac:.5f} of {Q.shape[0]}, max weight difference {wdiff:.2e}",
          flush=True)
    assert frac >= 0.999 and wdiff < 1e-5
    assert np.allclose(w.sum(1), 1.0, atol=1e-5)


@pytest.mark.parametrize("exterior", [False, True])
def test_knn_estimate_parity(ctx, oracle_mod, soup, exterior):
    from paper_2606_05581_amd import msk

    case, knn = soup
    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    b = ctx.basis_knn(mesh, knn["points"], knn["normals"], k=8, sigma=knn["sigma"], tau_n=0.8)
    W_ = 64
    d = ctx.estimate_dtn(mesh, rows, b, W_, case.eps, case.h, exterior=exterior, seed=5, record_log=1)
    S, se, disc = d.get(msk.FIELD_S), d.get(msk.FIELD_SE), d.get(msk.FIELD_ROW_DISCARDED)
    d2 = ctx.estimate_dtn(mesh, rows, b, W_, case.eps, case.h, exterior=exterior, seed=5, record_log=1,
                          form=msk.FORM_PLAIN)
    for f in (msk.FIELD_LOG_STATUS, msk.FIELD_LOG_TRI, msk.FIELD_LOG_QUERIES):
        assert np.array_equal(d.get(f), d2.get(f))
    assert np.allclose(d2.get(msk.FIELD_S), S, rtol=0, atol=1e-12 * np.abs(S).max())
    sc = oracle_mod.Scene(case.V, case.F, bvh=True)
    knn32 = dict(knn, points=knn["points"].astype(np.float32).astype(np.float64))
    r = oracle_mod.estimate(sc, case.rows, None, W_, case.eps, case.h, exterior=exterior, seed=5, knn=knn32,
                            nthreads=8)
    So, seo = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, W_, r["discarded"])
    z = np.abs(S - So) / np.maximum(np.sqrt(se ** 2 + seo ** 2), 1e-300)
    bad = (np.abs(S - So) > 4 * np.sqrt(se ** 2 + seo ** 2) + 1e-9 * np.abs(So).max())
    print(f"[knn estimate] exterior={exterior}: entries outside 4 combined se {int(bad.sum())} of {bad.size}, "
          f"max z {np.nanmax(np.where(np.isfinite(z), z, 0)):.2f}, discarded rows {int(disc.sum())}", flush=True)
    assert np.array_equal(disc, r["discarded"])
    assert not bad.any()
    if not exterior:  # partition of unity: every interior row sums to zero
        assert np.abs(S.sum(1)).max() < 1e-6 * np.abs(S).max()


def test_knn_argument_errors(ctx, soup):
    from paper_2606_05581_amd import msk

    case, knn = soup
    mesh = ctx.build_bvh(case.V, case.F)
    with pytest.raises(msk.MskError):
        ctx.basis_knn(mesh, knn["points"], knn["normals"], k=0)
    with pytest.raises(msk.MskError):
        ctx.basis_knn(mesh, knn["points"][:4], knn["normals"][:4], k=8)
    b = ctx.basis_knn(mesh, knn["points"], knn["normals"], k=8, sigma=knn["sigma"])
    rows = ctx.rows(mesh, case.rows)
    with pytest.raises(msk.MskError) as e:
        ctx.estimate_dtn(mesh, rows, b, 16, case.eps, case.h, collect_stats=1)
    assert e.value.status == msk.ERR_INVALID_ARG
    with pytest.raises(msk.MskError) as e:
        ctx.estimate_psd(mesh, rows, b, 4, 1e-4)
    assert e.value.status == msk.ERR_INVALID_ARG
    other = ctx.build_bvh(case.V, case.F)
    with pytest.raises(msk.MskError):
        ctx.estimate_dtn(other, ctx.rows(other, case.rows), b, 16, case.eps, case.h)
