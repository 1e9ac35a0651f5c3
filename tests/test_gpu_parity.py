"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bar: nearest-triangle indices, distances and barycentrics bit-exact against
the oracle's FP32 brute force; DtN entries within 4 combined standard errors
of the oracle's (same Philox streams, same inputs); eigenvalues of the
symmetrised estimates within 2%; the fraction of walks whose terminal triangle
or status differs from the oracle's walk (FP32 vs FP64 paths) is reported and
bounded. For point rows the bar is also deterministic: each side's S equals
its own walk log summed and finalised on the CPU (the GPU's to 1e-12 of the
largest entry, the oracle's to 1e-7: it logs its FP64 barycentrics rounded to
FP32), so the GPU-oracle difference is that of the divergent walks alone.
"""
import math

import numpy as np
import pytest

from paper_2606_05581_amd import workloads as W
from parity_util import check_log_reconstruction
from parity_util import parity_report as _parity_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2606_05581_amd import msk

    assert torch.cuda.is_available(), "GPU test needs a visible MI355X"
    c = msk.Context(0)
    yield c
    c.close()


def _tiny_meshes():
    out = []
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    F = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]])
    out.append(("tetrahedron", V, F))
    V, F = W.box_grid(1)
    out.append(("cube", V, F))
    V, F = W.icosphere_recursive(2)
    out.append(("icosphere320", V, F))
    V, F = W.icosphere_recursive(4)
    out.append(("icosphere5120", V * np.array([1.0, 0.6, 0.3]), F))
    # a cube with zero-area triangles: a segment, a point, a doubled-vertex segment
    V, F = W.box_grid(1)
    nv = V.shape[0]
    V = np.concatenate([V, [[0.2, 0.3, 0.4], [0.6, 0.9, 1.2], [1.0, 1.5, 2.0], [0.1, 0.1, 0.1]]], 0)
    F = np.concatenate([F, [[nv, nv + 1, nv + 2], [nv + 3, nv + 3, nv + 3], [nv, nv, nv + 1]]], 0)
    out.append(("degenerate", V, F))
    return out


def _queries(V, F, rng, n_random=2000):
    area, fn = W.face_geometry(V, F)
    lo, hi = V.min(0), V.max(0)
    pts = [rng.uniform(lo - 0.3, hi + 0.3, size=(n_random, 3))]
    pts.append(V)  # every vertex: ties between all faces of its ring
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    pts.append(0.5 * (V[e[:, 0]] + V[e[:, 1]]))  # edge midpoints: ties of two faces
    cen = V[F].mean(1)
    for off in (0.0, 1e-5, -1e-5, 1e-3, -1e-3):
        pts.append(cen + off * fn)
    pts.append(np.zeros((1, 3)))
    return np.concatenate(pts, 0)


@pytest.mark.parametrize("name", ["tetrahedron", "cube", "degenerate", "icosphere320", "icosphere5120", "soup"])
def test_closest_points_bit_exact(ctx, oracle_mod, name):
    import torch

    rng = np.random.default_rng(21)
    if name == "soup":
        c = W.soup8_53k(N=200, walks=8).cases[0]
        V, F = c.V.astype(np.float64), c.F
        keep = rng.choice(F.shape[0], 6000, replace=False)
        F = F[keep]
    else:
        V, F = dict((n, (v, f)) for n, v, f in _tiny_meshes())[name]
    print(f"[closest_points] mesh={name} tris={F.shape[0]}", flush=True)
    mesh = ctx.build_bvh(V.astype(np.float32), F)
    Q = _queries(V, F, rng)
    sc = oracle_mod.Scene(V.astype(np.float32), F, bvh=False)
    Qt = torch.tensor(Q.astype(np.float32), device="cuda")
    # the oracle takes float32 world points too: feed it the same values
    t_o, d_o, b_o = sc.nearest_f32(Q.astype(np.float32).astype(np.float64))
    t_g, d_g, b_g = (x.cpu().numpy() for x in ctx.closest_points(mesh, Qt))
    assert np.array_equal(t_g, t_o), np.nonzero(t_g != t_o)[0][:10]
    assert np.array_equal(d_g, d_o)
    assert np.array_equal(b_g, b_o)


# ------------------------------------------------------------ estimates


def _gpu_estimate(ctx, case, walks, exterior, seed=0, log=True, **opts):
    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    basis = ctx.basis(case.basis, case.V.shape[0])
    d = ctx.estimate_dtn(mesh, rows, basis, walks, case.eps, case.h, exterior=exterior, seed=seed,
                         record_log=1 if log else 0, **opts)
    from paper_2606_05581_amd import msk

    out = dict(S=d.get(msk.FIELD_S), se=d.get(msk.FIELD_SE), disc=d.get(msk.FIELD_ROW_DISCARDED),
               esc=d.get(msk.FIELD_ROW_ESCAPED), cap=d.get(msk.FIELD_ROW_CAPPED), q=d.get(msk.FIELD_ROW_QUERIES),
               info=d.info())
    if log:
        out.update(status=d.get(msk.FIELD_LOG_STATUS), tri=d.get(msk.FIELD_LOG_TRI), bary=d.get(msk.FIELD_LOG_BARY),
                   nq=d.get(msk.FIELD_LOG_QUERIES))
    return out


def _oracle_estimate(oracle_mod, case, walks, exterior, seed=0):
    sc = oracle_mod.Scene(case.V, case.F, bvh=True)
    r = oracle_mod.estimate(sc, case.rows, case.basis, walks, case.eps, case.h, exterior=exterior, seed=seed, log=True)
    S, se = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, walks, r["discarded"])
    r.update(S=S, se=se)
    return r


@pytest.mark.parametrize("exterior", [False, True])
def test_unit_sphere_hat_rows_parity(ctx, oracle_mod, exterior):
    """Unit icosphere (320 faces), hat basis, 162 vertex rows x 256 walks."""
    wl = W.unit_sphere_320()
    case = wl.cases[0]
    label = f"unit_sphere_320 {'exterior' if exterior else 'interior'}"
    print(f"[{label}] start", flush=True)
    g = _gpu_estimate(ctx, case, wl.walks, exterior)
    o = _oracle_estimate(oracle_mod, case, wl.walks, exterior)
    viol, div = _parity_report(g, o, label, case)
    assert viol.sum() == 0
    assert div < 0.01
    # walk counters and identities
    assert g["info"]["walks_total"] == case.rows.n_rows * wl.walks
    assert g["cap"].sum() == 0
    if not exterior:
        assert g["esc"].sum() == 0
        assert np.abs(g["S"].sum(1)).max() <= 1e-9 * (case.rows.w / case.h).max()
    else:
        rs = case.rows.w / case.h * g["esc"] / wl.walks
        assert np.abs(g["S"].sum(1) - rs).max() <= 1e-9 * (case.rows.w / case.h).max()
    # eigenvalues of the two symmetrised estimates
    lg, _, _ = oracle_mod.steklov_modes(g["S"], case.rows.w, wl.k)
    lo, _, _ = oracle_mod.steklov_modes(o["S"], case.rows.w, wl.k)
    assert np.all(np.abs(lg - lo) <= 0.02 * np.maximum(1.0, np.abs(lo)))


@pytest.mark.parametrize("exterior", [False, True])
def test_soup_point_rows_parity(ctx, oracle_mod, exterior):
    """Overlapping 8-shape soup (53,249 faces), point k-NN basis, 300 rows x 128 walks."""
    wl = W.soup8_53k(N=300, walks=128)
    case = wl.cases[0]
    label = f"soup8 N=300 {'exterior' if exterior else 'interior'}"
    print(f"[{label}] start", flush=True)
    g = _gpu_estimate(ctx, case, wl.walks, exterior)
    o = _oracle_estimate(oracle_mod, case, wl.walks, exterior)
    assert np.array_equal(g["disc"], o["discarded"])
    viol, div = _parity_report(g, o, label, case)
    assert viol.sum() == 0
    assert div < (0.02 if exterior else 0.01)
    assert g["cap"].sum() == o["n_capped"].sum() == 0
    # deterministic: each side's S is its own walk log summed (to rounding),
    # so the GPU-oracle difference is the divergent walks' alone
    check_log_reconstruction(oracle_mod, case, g, o, exterior, label)


def test_plain_and_persistent_forms_agree(ctx):
    """Both kernel forms run the same walks: identical logs, sums equal up to
    the order of floating-point additions."""
    case = W.unit_sphere_320().cases[0]
    a = _gpu_estimate(ctx, case, 64, False, form=1)
    b = _gpu_estimate(ctx, case, 64, False, form=0)
    for k in ("status", "tri", "bary", "nq"):
        assert np.array_equal(a[k], b[k])
    assert np.allclose(a["S"], b["S"], rtol=0, atol=1e-12 * np.abs(a["S"]).max())


@pytest.mark.parametrize("exterior", [False, True])
@pytest.mark.parametrize("mesh", ["soup", "degenerate"])
def test_wavefront_and_lane_private_tests_agree(ctx, mesh, exterior):
    """The persistent form tests each query's triangles cooperatively (whole
    wavefront, lexicographic LDS minimum), the plain form one lane at a time:
    over every query of these walks (tens of millions of triangle tests,
    zero-area triangles included) both must pick the same nearest triangle
    with the same distance and barycentrics, so the logs are identical."""
    if mesh == "soup":
        case = W.soup8_53k(N=300, walks=128).cases[0]
    else:
        V, F = _tiny_meshes()[4][1:]
        case = W._point_case(V, F, 200, np.random.default_rng(17))
    a = _gpu_estimate(ctx, case, 128, exterior, form=1)
    b = _gpu_estimate(ctx, case, 128, exterior, form=0)
    for k in ("status", "tri", "bary", "nq"):
        assert np.array_equal(a[k], b[k]), k
    print(f"[cooperative vs lane-private] {mesh} exterior={exterior}: {int(a['nq'].sum())} queries identical",
          flush=True)


def test_split_walk_ranges(ctx):
    """walk_offset continues the Philox walk counter: [0,40) + [40,96) = [0,96)."""
    case = W.unit_sphere_320().cases[0]
    a = _gpu_estimate(ctx, case, 96, True)
    b1 = _gpu_estimate(ctx, case, 40, True)
    b2 = _gpu_estimate(ctx, case, 56, True, walk_offset=40)
    for k in ("status", "tri", "bary", "nq"):
        assert np.array_equal(a[k], np.concatenate([b1[k], b2[k]], 1))


def test_fp32_partial_sums_within_rounding(ctx):
    """Mixed precision: FP32 partial sums per chunk, FP64 rows. Same walks as
    the FP64 form; every entry within 1e-5 of the FP64 estimate's scale."""
    wl = W.soup8_53k(N=300, walks=128)
    case = wl.cases[0]
    a = _gpu_estimate(ctx, case, 128, False, accum=0)
    b = _gpu_estimate(ctx, case, 128, False, accum=1)
    for k in ("status", "tri", "nq"):
        assert np.array_equal(a[k], b[k])
    scale = np.abs(a["S"]).max()
    err = np.abs(a["S"] - b["S"]).max() / scale
    print(f"[fp32 partial sums] max |S_f32 - S_f64| / max|S| = {err:.2e}", flush=True)
    assert err < 1e-5


def test_nonfinite_estimate_reports_numeric(ctx):
    """Basis values near 1e30 square past the FP32 range in the mixed-precision
    partial sums: the call reports NUMERIC, hands the estimate back and counts
    the non-finite entries; the FP64 form of the same walks stays finite."""
    import dataclasses

    from paper_2606_05581_amd import msk

    wl = W.soup8_53k(N=300, walks=64)
    case = wl.cases[0]
    big = dataclasses.replace(case.basis, val=(case.basis.val.astype(np.float64) * 1e30).astype(np.float32))
    assert np.isfinite(big.val).all()
    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    basis = ctx.basis(big, case.V.shape[0])
    d = ctx.estimate_dtn(mesh, rows, basis, 64, case.eps, case.h, accum=0)
    assert d.info()["nonfinite_entries"] == 0
    assert np.isfinite(d.get(msk.FIELD_S)).all() and np.isfinite(d.get(msk.FIELD_SE)).all()
    with pytest.raises(msk.MskNumericError) as ei:
        ctx.estimate_dtn(mesh, rows, basis, 64, case.eps, case.h, accum=1)
    r = ei.value.result
    S, se = r.get(msk.FIELD_S), r.get(msk.FIELD_SE)
    n_bad = int((~np.isfinite(S)).sum() + (~np.isfinite(se)).sum())
    print(f"[numeric] non-finite entries {n_bad} of {2 * S.size}", flush=True)
    assert n_bad > 0 and r.info()["nonfinite_entries"] == n_bad
    assert S.shape[0] == S.shape[1]
    with pytest.raises(msk.MskError) as ee:
        ctx.steklov_modes(r, 4)
    assert ee.value.status == msk.ERR_NUMERIC


@pytest.mark.parametrize("exterior", [False, True])
def test_capped_walks_parity(ctx, oracle_mod, exterior):
    """A step cap of 4 ends most walks CAPPED: each ends at the nearest surface
    point of its last position and is counted. The GPU's capped walks, their
    terminal triangles and query counts follow the oracle's walk for walk,
    and the entries stay within 4 combined standard errors."""
    wl = W.soup8_53k(N=200, walks=64)
    case = wl.cases[0]
    label = f"soup8 N=200 capped at 4 steps {'exterior' if exterior else 'interior'}"
    print(f"[{label}] start", flush=True)
    g = _gpu_estimate(ctx, case, wl.walks, exterior, max_steps=4)
    sc = oracle_mod.Scene(case.V, case.F, bvh=True)
    r = oracle_mod.estimate(sc, case.rows, case.basis, wl.walks, case.eps, case.h, exterior=exterior, log=True,
                            max_steps=4)
    S, se = oracle_mod.finalize(r["acc"], r["acc2"], case.rows.w, case.h, wl.walks, r["discarded"])
    r.update(S=S, se=se)
    viol, div = _parity_report(g, r, label, case)
    ran = r["log_status"] >= 0
    capped_o = (r["log_status"] == oracle_mod.CAPPED)[ran].mean()
    capped_g = (g["status"] == oracle_mod.CAPPED)[ran].mean()
    print(f"[{label}] capped walks: GPU {capped_g:.2%}, oracle {capped_o:.2%}; "
          f"per-row counts GPU {int(g['cap'].sum())}, oracle {int(r['n_capped'].sum())}", flush=True)
    assert capped_o > 0.3  # the cap is exercised
    assert viol.sum() == 0
    assert div < 0.01
    assert abs(capped_g - capped_o) <= 0.01
    assert int(g["cap"].sum()) == int((g["status"] == oracle_mod.CAPPED).sum())
    check_log_reconstruction(oracle_mod, case, g, r, exterior, label)
    # a capped walk makes exactly max_steps + 1 queries (the cap's query included)
    assert np.all(g["nq"][g["status"] == oracle_mod.CAPPED] == 5)


def test_eps_at_the_floor_is_refused(ctx):
    """eps must exceed msk_eps_floor(R): at the floor a walk inside the shell
    could take a step of non-positive length. On a sphere of radius 3 the
    default floor is the FP32 resolution 3 * 2^-18."""
    from paper_2606_05581_amd import msk

    V, F = W.icosphere_recursive(2)
    case = W._point_case(3.0 * V, F, 64, np.random.default_rng(5))
    mesh = ctx.build_bvh(case.V, case.F)
    rows = ctx.rows(mesh, case.rows)
    basis = ctx.basis(case.basis, case.V.shape[0])
    R = mesh.info()["radius"]
    floor = msk.lib().msk_eps_floor(R, None)
    assert floor == R * 2.0 ** -18
    with pytest.raises(msk.MskError) as ei:
        ctx.estimate_dtn(mesh, rows, basis, 8, floor, case.h)
    assert ei.value.status == msk.ERR_INVALID_ARG and "eps must exceed" in str(ei.value)
    d = ctx.estimate_dtn(mesh, rows, basis, 8, floor * 1.01, case.h)
    assert d.info()["walks_total"] > 0
