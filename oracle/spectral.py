"""CPU oracle for the spectral quantities built on Steklov eigenpairs in a
Galerkin basis (arXiv 2606.05581, Sec. 5: eqs. steklovHeat and
spectralSteklovHeat, and the heat kernel signatures compared there).

TEST INFRASTRUCTURE ONLY: the plain FP64 reference that the GPU library is
checked against. Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the GPU product path never does.

With an M-orthonormal basis Phi (Phi^T M Phi = I) the Galerkin Steklov
problem S c = lambda c is an ordinary symmetric one, and the eigenfunctions
psi_k = Phi c_k are M-orthonormal. Then
* Steklov heat from u0: u_t = sum_k exp(-lambda_k t) a_k psi_k with
  a_k = <u0, psi_k>_M = sum_v m_v u0(v) psi_k(v);
* heat kernel signature: HKS(v, t) = sum_k exp(-lambda_k t) psi_k(v)^2.
"""
from __future__ import annotations

import numpy as np


def galerkin_steklov(S):
    """(lambda ascending, C): eigenpairs of the symmetrised K x K estimate,
    for an M-orthonormal basis (Alg. 1 / Alg. 2 output)."""
    lam, C = np.linalg.eigh(0.5 * (S + S.T))
    return lam, C


def heat_kernel_signature(Phi, C, lam, times):
    """nv x T: sum_k exp(-lambda_k t) (Phi C)_vk^2."""
    Psi = np.asarray(Phi, dtype=np.float64) @ np.asarray(C, dtype=np.float64)
    E = np.exp(-np.outer(lam, times))
    return (Psi * Psi) @ E


def steklov_heat(Phi, C, lam, times, mass, u0):
    """nv x T: sum_k exp(-lambda_k t) a_k psi_k, a_k = sum_v m_v u0_v psi_k(v)."""
    Psi = np.asarray(Phi, dtype=np.float64) @ np.asarray(C, dtype=np.float64)
    a = Psi.T @ (np.asarray(mass, dtype=np.float64) * np.asarray(u0, dtype=np.float64))
    E = np.exp(-np.outer(lam, times))
    return Psi @ (a[:, None] * E)
