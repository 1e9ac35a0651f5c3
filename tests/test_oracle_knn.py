"""Pins of the oracle's point basis (Appendix, point-based k-NN interpolator).

The neighbour search is checked against SciPy's KD-tree (an independent
implementation); the weights against closed-form special cases; the estimator
built on them against the partition of unity (rows of the interior estimate
sum to zero).
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2606_05581_amd import workloads as W


def test_knn_set_matches_kdtree(oracle_mod):
    rng = np.random.default_rng(3)
    P = rng.normal(size=(2000, 3))
    N = P / np.linalg.norm(P, axis=1, keepdims=True)
    tree = cKDTree(P)
    for q in rng.normal(size=(200, 3)):
        idx, w = oracle_mod.knn_weights(P, N, q, np.array([0.0, 0.0, 1.0]), 8, 0.3, 0.8)
        d, ref = tree.query(q, k=8)
        assert list(idx) == list(ref)
        assert w.sum() == pytest.approx(1.0, abs=1e-14) and np.all(w > 0)


def test_knn_weights_closed_forms(oracle_mod):
    sigma, tau = 0.2, 0.8
    # equal normals: weights go as exp(-d^2 / (2 sigma^2))
    P = np.array([[0.1, 0, 0], [0, 0.25, 0], [0, 0, -0.4]])
    N = np.tile([0.0, 0.0, 1.0], (3, 1))
    idx, w = oracle_mod.knn_weights(P, N, np.zeros(3), np.array([0.0, 0, 1]), 3, sigma, tau)
    assert list(idx) == [0, 1, 2]
    g = np.exp(-np.array([0.01, 0.0625, 0.16]) / (2 * sigma ** 2))
    assert np.allclose(w, g / g.sum(), rtol=1e-14)
    # equidistant points: weights go as exp(-(1 - cos angle) / tau)
    ang = np.array([0.0, 0.5, 1.2])
    P = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    N = np.stack([np.zeros(3), np.sin(ang), np.cos(ang)], 1)
    idx, w = oracle_mod.knn_weights(P, N, np.zeros(3), np.array([0.0, 0, 1]), 3, sigma, tau)
    g = np.exp(-(1 - np.cos(ang)) / tau)
    assert list(idx) == [0, 1, 2]  # ties in distance: lower index first
    assert np.allclose(w, g / g.sum(), rtol=1e-14)
    # very wide falloffs: the k neighbours share equally
    rng = np.random.default_rng(1)
    P = rng.normal(size=(50, 3))
    N = rng.normal(size=(50, 3))
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    idx, w = oracle_mod.knn_weights(P, N, rng.normal(size=3), np.array([1.0, 0, 0]), 8, 1e6, 1e9)
    assert np.allclose(w, 1 / 8, rtol=1e-9)


def test_point_basis_estimator_rows_sum_to_zero(oracle_mod):
    """Every basis evaluation is a partition of unity, so each walk's
    c = b(s) - b(t) sums to zero and so does every interior row."""
    V, F = W.icosphere_recursive(3)
    rng = np.random.default_rng(5)
    rows = W.point_rows(V, F, 200, rng)
    P = rows.p.astype(np.float64)
    knn = dict(points=P, normals=rows.n.astype(np.float64), k=8, sigma=1.5 * math.sqrt(4 * math.pi / 200), tau=0.8)
    sc = oracle_mod.Scene(V.astype(np.float32), F, bvh=True)
    r = oracle_mod.estimate(sc, rows, None, 32, 1e-3, 0.05, exterior=False, seed=2, knn=knn, nthreads=8)
    assert r["acc"].shape == (200, 200)
    assert np.abs(r["acc"].sum(1)).max() < 1e-9 * 32
    S, se = oracle_mod.finalize(r["acc"], r["acc2"], rows.w, 0.05, 32, r["discarded"])
    # the diagonal (each sample's own weight at s) dominates its row
    assert np.all(np.diag(S)[r["discarded"] == 0] > 0)
