"""Pins of the oracle's mesh-based Galerkin basis (Sec. 5.1, mesh-based
Galerkin basis: low modes of the cotangent Laplacian).

* the stiffness matrix against the Dirichlet energy computed from
  barycentric gradients (an independent route; equal quadratic forms fix a
  symmetric matrix), its null vector and linear precision on a flat mesh;
* the mass against the surface area;
* the regular icosahedron, whose spectrum is closed-form (every angle 60
  degrees: L is the graph Laplacian over sqrt(3), M = 5 sqrt(3) a^2 / 12);
* the unit sphere, where the modes approach the spherical harmonics
  (eigenvalue l(l+1), multiplicity 2l+1) at second order in the edge length;
* zero-area triangles and unreferenced vertices leave the spectrum alone.
"""
import math

import numpy as np
import pytest
from scipy.spatial import Delaunay

from oracle import laplace as LP
from paper_2606_05581_amd import workloads as W


def _jittered_sphere(level, amp, seed):
    V, F = W.icosphere_recursive(level)
    rng = np.random.default_rng(seed)
    V = V * (1.0 + amp * rng.uniform(-1, 1, size=(V.shape[0], 1))) + 0.5 * amp * rng.normal(size=V.shape)
    return V, F


def test_stiffness_is_dirichlet_energy():
    V, F = _jittered_sphere(2, 0.15, 1)  # irregular, with obtuse angles
    L, m, skipped = LP.cotan_laplacian(V, F)
    assert skipped == 0
    ang = []
    for c in range(3):
        u = V[F[:, (c + 1) % 3]] - V[F[:, c]]
        v = V[F[:, (c + 2) % 3]] - V[F[:, c]]
        ang.append(np.arccos(np.einsum("ij,ij->i", u, v) / np.linalg.norm(u, axis=1) / np.linalg.norm(v, axis=1)))
    assert np.max(ang) > math.pi / 2  # the mesh has obtuse corners (negative weights)
    assert abs(L - L.T).max() == 0.0
    rng = np.random.default_rng(2)
    for _ in range(4):
        u = rng.normal(size=V.shape[0])
        assert float(u @ (L @ u)) == pytest.approx(LP.dirichlet_energy(V, F, u), rel=1e-12)
    assert np.abs(L @ np.ones(V.shape[0])).max() < 1e-12 * abs(L).max()


def test_linear_precision_on_a_flat_mesh():
    rng = np.random.default_rng(3)
    P2 = np.concatenate([rng.uniform(0, 1, size=(300, 2)), [[0, 0], [1, 0], [0, 1], [1, 1]]])
    tri = Delaunay(P2)
    V = np.concatenate([P2, np.zeros((P2.shape[0], 1))], 1)
    F = tri.simplices
    L, m, _ = LP.cotan_laplacian(V, F)
    hull = np.unique(tri.convex_hull)
    interior = np.setdiff1d(np.arange(V.shape[0]), hull)
    for d in range(2):  # a linear function is harmonic: zero at every interior vertex
        assert np.abs((L @ V[:, d])[interior]).max() < 1e-12
    e1, e2 = P2[F[:, 1]] - P2[F[:, 0]], P2[F[:, 2]] - P2[F[:, 0]]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]).sum()
    assert m.sum() == pytest.approx(area, rel=1e-13) and area == pytest.approx(1.0, rel=1e-12)


def test_icosahedron_closed_form():
    V, F = W.icosahedron()
    a = np.linalg.norm(V[F[0, 0]] - V[F[0, 1]])
    L, m, _ = LP.cotan_laplacian(V, F)
    assert np.allclose(m, 5 * math.sqrt(3) * a * a / 12, rtol=1e-14)
    s5 = math.sqrt(5)
    mu = np.array([0] + [5 - s5] * 3 + [6] * 5 + [5 + s5] * 3)  # graph Laplacian spectrum
    want = 4 * mu / (5 * a * a)
    lam, Phi, mm = LP.laplacian_basis(V, F, 11)
    assert np.allclose(lam, want[:11], rtol=1e-10, atol=1e-12)
    assert np.allclose(Phi.T @ (mm[:, None] * Phi), np.eye(11), atol=1e-12)


def test_unit_sphere_modes_approach_spherical_harmonics():
    errs = []
    for level in (3, 4):
        V, F = W.icosphere_recursive(level)
        lam, Phi, m = LP.laplacian_basis(V, F, 25)
        want = np.concatenate([[l * (l + 1)] * (2 * l + 1) for l in range(5)])
        errs.append(np.abs(lam - want).max())
        # clusters of 2l+1 below the next degree
        for l in range(4):
            assert lam[(l + 1) ** 2 - 1] < 0.5 * (l * (l + 1) + (l + 1) * (l + 2)) < lam[(l + 1) ** 2]
        L, _, _ = LP.cotan_laplacian(V, F)
        R = L @ Phi - m[:, None] * Phi * lam[None, :]
        assert np.abs(R).max() < 1e-9 * max(1.0, lam.max())
        # the degree-1 modes span the coordinate functions
        Q = Phi[:, 1:4]
        coef = np.linalg.lstsq(Q, V, rcond=None)[0]
        assert np.abs(Q @ coef - V).max() < 0.02
    assert errs[1] < errs[0] / 3.0  # second order in the edge length


def test_degenerate_faces_and_isolated_vertices():
    V, F = W.icosphere_recursive(2)
    lam0, _, _ = LP.laplacian_basis(V, F, 9)
    # a zero-area triangle (repeated vertex) and a collinear one, plus an unreferenced vertex
    V2 = np.concatenate([V, [[0.5 * (V[0, 0] + V[1, 0]), 0.5 * (V[0, 1] + V[1, 1]), 0.5 * (V[0, 2] + V[1, 2])],
                             [3.0, 3.0, 3.0]]])
    F2 = np.concatenate([F, [[0, 0, 5], [0, 1, V.shape[0]]]])
    L, m, skipped = LP.cotan_laplacian(V2, F2)
    assert skipped == 2
    assert m[-1] == 0.0 and m[-2] == 0.0
    lam, Phi, _ = LP.laplacian_basis(V2, F2, 9)
    assert np.allclose(lam, lam0, rtol=1e-10, atol=1e-12)
    assert np.all(Phi[-2:] == 0.0)
