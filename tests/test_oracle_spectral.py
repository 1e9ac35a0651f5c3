"""Pins of the oracle's spectral quantities (Sec. 5, eqs. steklovHeat and
spectralSteklovHeat; heat kernel signatures).

* On the unit sphere the Steklov eigenfunctions are the spherical harmonics
  with eigenvalue l, and by the addition theorem sum_m Y_lm(x)^2 =
  (2l+1)/(4 pi) at every point: the HKS is sum_l (2l+1)/(4 pi) exp(-l t),
  independent of x (the basis is evaluated exactly at the points, so this
  holds to rounding).
* The heat of a single eigenfunction decays as exp(-lambda t) and keeps its
  shape; heat is linear in u0 and conserves nothing else.
* A rotation of the basis inside an eigenspace leaves both unchanged.
"""
import math

import numpy as np

from oracle import spectral as SP
from paper_2606_05581_amd import workloads as W


def _sphere_basis(L, n=400, seed=0):
    rng = np.random.default_rng(seed)
    P = rng.normal(size=(n, 3))
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    Y = W.real_sh(L, P)  # (n, (L+1)^2), orthonormal on the unit sphere
    deg = np.concatenate([[l] * (2 * l + 1) for l in range(L + 1)])
    return P, Y, deg.astype(np.float64)


def test_hks_addition_theorem():
    L = 6
    P, Y, deg = _sphere_basis(L)
    K = Y.shape[1]
    times = np.array([0.0, 0.1, 0.5, 2.0])
    hks = SP.heat_kernel_signature(Y, np.eye(K), deg, times)
    want = np.array([sum((2 * l + 1) / (4 * math.pi) * math.exp(-l * t) for l in range(L + 1)) for t in times])
    assert np.allclose(hks, want[None, :], rtol=1e-12)


def test_rotation_inside_eigenspaces_changes_nothing():
    L = 4
    P, Y, deg = _sphere_basis(L, seed=1)
    K = Y.shape[1]
    rng = np.random.default_rng(2)
    Q = np.zeros((K, K))
    for l in range(L + 1):  # a random orthogonal block per degree
        a, b = l * l, (l + 1) ** 2
        Q[a:b, a:b] = np.linalg.qr(rng.normal(size=(b - a, b - a)))[0]
    times = np.array([0.05, 0.3])
    m = rng.uniform(0.5, 1.5, size=P.shape[0])
    u0 = rng.normal(size=P.shape[0])
    h1 = SP.heat_kernel_signature(Y, np.eye(K), deg, times)
    h2 = SP.heat_kernel_signature(Y, Q, deg, times)
    assert np.allclose(h1, h2, rtol=1e-12)
    u1 = SP.steklov_heat(Y, np.eye(K), deg, times, m, u0)
    u2 = SP.steklov_heat(Y, Q, deg, times, m, u0)
    assert np.allclose(u1, u2, rtol=1e-11, atol=1e-13)


def test_heat_of_one_mode_decays_exponentially():
    # an M-orthonormal basis on random points: Phi = orthonormalised columns under weights m
    rng = np.random.default_rng(3)
    n, K = 300, 12
    m = rng.uniform(0.5, 2.0, size=n)
    A = rng.normal(size=(n, K))
    Qm, _ = np.linalg.qr(np.sqrt(m)[:, None] * A)
    Phi = Qm / np.sqrt(m)[:, None]
    S = rng.normal(size=(K, K))
    S = S @ S.T
    lam, C = SP.galerkin_steklov(S)
    Psi = Phi @ C
    k0 = 5
    times = np.array([0.0, 0.2, 1.0])
    u = SP.steklov_heat(Phi, C, lam, times, m, Psi[:, k0])
    for j, t in enumerate(times):
        assert np.allclose(u[:, j], math.exp(-lam[k0] * t) * Psi[:, k0], rtol=1e-10, atol=1e-12)
    # linear in u0
    v0 = rng.normal(size=n)
    w0 = rng.normal(size=n)
    lhs = SP.steklov_heat(Phi, C, lam, times, m, 2.0 * v0 - 3.0 * w0)
    rhs = 2.0 * SP.steklov_heat(Phi, C, lam, times, m, v0) - 3.0 * SP.steklov_heat(Phi, C, lam, times, m, w0)
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12)
