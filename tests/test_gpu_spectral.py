"""GPU parity of Steklov heat and heat kernel signatures (Sec. 5, eqs.
steklovHeat and spectralSteklovHeat) against the oracle (oracle/spectral.py),
on the same FP32 table values: every entry within 1e-12 of the largest
magnitude (FP64 sums in another order). End to end on the unit sphere: the
PSD estimate in the GPU Laplacian basis gives a signature close to the
closed form of the exact spectrum (addition theorem)."""
import math

import numpy as np
import pytest

from oracle import laplace as LP
from oracle import spectral as SP
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


@pytest.mark.parametrize("K,n_modes", [(40, 40), (150, 96), (9, 5)])
def test_spectral_parity(ctx, K, n_modes):
    V, F = W.icosphere_recursive(3)
    rng = np.random.default_rng(K)
    tab = rng.normal(size=(V.shape[0], K)).astype(np.float32)
    if K == 9:  # a sparse table: three entries per vertex
        tab[:, 3:] = 0.0
    bh = ctx.basis(W.dense_basis(tab), V.shape[0])
    C = np.linalg.qr(rng.normal(size=(K, K)))[0][:, :n_modes]
    lam = np.sort(rng.uniform(0, 10, size=n_modes))
    times = np.array([0.0, 0.01, 0.1, 1.0, 3.0])
    mass = rng.uniform(0.5, 1.5, size=V.shape[0])
    u0 = rng.normal(size=V.shape[0])
    hks, heat = ctx.spectral_heat(bh, lam, C, times, mass=mass, u0=u0)
    Phi = tab.astype(np.float64)
    h_o = SP.heat_kernel_signature(Phi, C, lam, times)
    u_o = SP.steklov_heat(Phi, C, lam, times, mass, u0)
    dh = np.abs(hks - h_o).max() / np.abs(h_o).max()
    du = np.abs(heat - u_o).max() / np.abs(u_o).max()
    print(f"[spectral] K={K} modes={n_modes}: rel diff hks {dh:.1e} heat {du:.1e}", flush=True)
    assert dh < 1e-12 and du < 1e-12
    h_only, none = ctx.spectral_heat(bh, lam, C, times)
    assert none is None and np.array_equal(h_only, hks)


def test_spectral_argument_errors(ctx):
    from paper_2606_05581_amd import msk

    V, F = W.icosphere_recursive(2)
    tab = np.ones((V.shape[0], 4), dtype=np.float32)
    bh = ctx.basis(W.dense_basis(tab), V.shape[0])
    C = np.eye(4)
    for lam, CC, t in ((np.zeros(5), np.eye(4, 5), [0.1]), (np.zeros(4), C, [-1.0]), (np.array([0, 1, np.nan, 2.0]), C, [1.0])):
        with pytest.raises(msk.MskError) as e:
            ctx.spectral_heat(bh, lam, CC, np.array(t))
        assert e.value.status == msk.ERR_INVALID_ARG


def test_sphere_signature_end_to_end(ctx):
    """Laplacian basis (K = 16, degrees <= 3) on the unit icosphere, PSD
    estimate, Galerkin Steklov pairs, signature: within a few percent of
    sum_l (2l+1)/(4 pi) exp(-l t) (Steklov eigenvalues l, addition theorem),
    the gap being the faceting, the cap and Monte Carlo noise."""
    V, F = W.icosphere_recursive(4)
    V = (V / np.linalg.norm(V, axis=1, keepdims=True)).astype(np.float32)
    F = F.astype(np.int32)
    rows = W.point_rows(V.astype(np.float64), F, 1500, np.random.default_rng(21))
    mesh = ctx.build_bvh(V, F)
    rh = ctx.rows(mesh, rows)
    bl, lam_l, Phi, _ = ctx.basis_laplacian(V, F, 16, seed=1)
    g = ctx.estimate_psd(mesh, rh, bl, 64, 1e-4, seed=3)
    lam, C = SP.galerkin_steklov(g["S"])
    times = np.array([0.05, 0.5, 2.0])
    hks, _ = ctx.spectral_heat(bl, lam, C, times)
    want = np.array([sum((2 * l + 1) / (4 * math.pi) * math.exp(-l * t) for l in range(4)) for t in times])
    rel = np.abs(hks.mean(0) - want) / want
    spread = hks.std(0) / hks.mean(0)
    print(f"[spectral sphere] Steklov eigenvalues {lam.round(3)}; mean hks {hks.mean(0).round(4)} vs {want.round(4)}, "
          f"relative spread over vertices {spread.round(4)}", flush=True)
    assert np.all(rel < 0.05)
    assert np.all(spread < 0.05)
