"""Input generators: the spherical harmonics that displace the large sphere
workload agree with scipy's complex harmonics, and the generators are
deterministic."""
import numpy as np

from paper_2606_05581_amd import workloads as W


def test_real_sh_matches_scipy():
    from scipy.special import sph_harm_y

    rng = np.random.default_rng(0)
    D = rng.normal(size=(500, 3))
    D[:3] = [[0, 0, 1], [0, 0, -1], [1, 0, 0]]  # poles and the equator
    L = 16
    Y = W.real_sh(L, D)
    d = D / np.linalg.norm(D, axis=1, keepdims=True)
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    col = 0
    for l in range(L + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), th, ph)
            ref = np.sqrt(2) * (-1) ** m * (y.real if m > 0 else y.imag) if m != 0 else y.real
            assert np.allclose(Y[:, col], ref, rtol=0, atol=1e-12), (l, m)
            col += 1
    # orthonormal on the sphere: quadrature over a fine geodesic grid
    V, F = W.geodesic_sphere(40)
    area, _ = W.face_geometry(V, F)
    c = V[F].mean(1)
    Yc = W.real_sh(6, c)
    G = (Yc * area[:, None]).T @ Yc
    assert np.abs(G - np.eye(G.shape[0])).max() < 2e-2


def test_generators_are_deterministic():
    a = W.batch64_mixed(n_meshes=3, walks=8, face_lo=2e3, face_hi=4e3, rows_lo=32, rows_hi=40, seed=5)
    b = W.batch64_mixed(n_meshes=3, walks=8, face_lo=2e3, face_hi=4e3, rows_lo=32, rows_hi=40, seed=5)
    for x, y in zip(a.cases, b.cases):
        assert np.array_equal(x.V, y.V) and np.array_equal(x.F, y.F)
        assert np.array_equal(x.rows.p, y.rows.p) and np.array_equal(x.basis.val, y.basis.val)
