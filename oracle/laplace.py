"""CPU oracle for the mesh-based Galerkin basis (arXiv 2606.05581, Sec. 5.1,
"Mesh-based Galerkin basis"): the low-frequency eigenmodes of the cotangent
Laplacian of the boundary mesh, evaluated in a triangle by barycentric
interpolation.

TEST INFRASTRUCTURE ONLY: the plain FP64 reference that the GPU library is
checked against. Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the GPU product path never does.

Definitions (the paper names the operator, not its discretisation; these are
the textbook piecewise-linear finite-element forms):

* stiffness L: for every triangle of nonzero area and each of its corners
  with angle theta opposite the edge (i, j), L_ij and L_ji gain
  -cot(theta)/2 and L_ii, L_jj gain +cot(theta)/2 (so L 1 = 0 and
  u^T L u is the Dirichlet energy of the piecewise-linear u);
* lumped mass M = diag(m), m_i = one third of the area of the triangles at i;
* basis: the K smallest eigenpairs of L phi = lambda M phi, phi normalised
  so that Phi^T M Phi = I (orthonormal in the mass inner product).

Triangles of (numerically) zero area contribute to neither matrix: a
triangle is left out when twice its area, |(b - a) x (c - a)| from its first
corner, is at most DEGENERATE_REL times its longest squared edge (a relative
test, so that exactly collinear corners, whose cross product rounds to a tiny
nonzero value, are left out whichever corner it is taken from). Vertices of
zero mass
(unreferenced, or only in zero-area triangles) are not part of the
eigenproblem; their basis values are zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


DEGENERATE_REL = 1e-12


def face_area2(V, F):
    """Twice the area of every triangle (|e1 x e2|), FP64."""
    P = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    return np.linalg.norm(np.cross(b - a, c - a), axis=1)


def live_faces(V, F):
    """Mask of the triangles that enter the matrices (see the module header)."""
    P = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    l2 = np.maximum(np.maximum(((b - a) ** 2).sum(1), ((c - b) ** 2).sum(1)), ((a - c) ** 2).sum(1))
    return face_area2(P, F) > DEGENERATE_REL * l2


def cotan_laplacian(V, F):
    """(L, m, skipped): the cotangent stiffness matrix (scipy CSR, FP64), the
    lumped mass vector and the number of zero-area triangles left out."""
    P = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    nv = P.shape[0]
    area2 = face_area2(P, F)
    live = live_faces(P, F)
    Fl, A2 = F[live], area2[live]
    rows, cols, vals = [], [], []
    for c in range(3):  # corner c, opposite edge (i, j)
        k = Fl[:, c]
        i = Fl[:, (c + 1) % 3]
        j = Fl[:, (c + 2) % 3]
        u = P[i] - P[k]
        v = P[j] - P[k]
        cot = np.einsum("ij,ij->i", u, v) / A2  # cos / sin, |u x v| = twice the area
        half = 0.5 * cot
        rows += [i, j, i, j]
        cols += [j, i, i, j]
        vals += [-half, -half, half, half]
    L = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nv, nv)).tocsr()
    L.sum_duplicates()
    m = np.zeros(nv)
    for c in range(3):
        np.add.at(m, Fl[:, c], A2 / 6.0)
    return L, m, int((~live).sum())


def dirichlet_energy(V, F, u):
    """sum over triangles of area * |grad u|^2 for the piecewise-linear u,
    with grad u from the barycentric gradients grad(lambda_i) = (n x e_i) / (2A),
    e_i the edge opposite vertex i (an independent route to u^T L u)."""
    P = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    nrm = np.cross(b - a, c - a)
    A2 = np.linalg.norm(nrm, axis=1)
    live = live_faces(P, F)
    n = nrm[live] / A2[live, None]
    e0, e1, e2 = (c - b)[live], (a - c)[live], (b - a)[live]
    Fl = F[live]
    g = (np.cross(n, e0) * u[Fl[:, 0], None] + np.cross(n, e1) * u[Fl[:, 1], None]
         + np.cross(n, e2) * u[Fl[:, 2], None]) / A2[live, None]
    return float(np.sum(0.5 * A2[live] * np.einsum("ij,ij->i", g, g)))


def laplacian_basis(V, F, K, sigma=None):
    """(evals ascending (K,), Phi (nv, K) with Phi^T M Phi = I, m).

    The generalised problem over the vertices of positive mass is solved by
    ARPACK in shift-invert mode about a small negative shift (scipy eigsh) for
    more pairs than K, the K smallest kept, and the eigenvectors
    M-normalised."""
    L, m, _ = cotan_laplacian(V, F)
    act = np.nonzero(m > 0)[0]
    La = L[act][:, act].tocsc()
    Ma = sp.diags(m[act]).tocsc()
    if sigma is None:
        P = np.asarray(V, dtype=np.float64)[act]
        R = np.max(np.linalg.norm(P - P.mean(0), axis=1))
        sigma = -1e-3 / max(R * R, 1e-300)
    # extra pairs beyond K so that whole clusters of repeated eigenvalues at
    # the cut are found (Krylov methods may miss copies at the edge of a block)
    k_solve = min(La.shape[0] - 1, K + max(10, K // 4))
    lam, X = spla.eigsh(La, k=k_solve, M=Ma, sigma=sigma, which="LM", tol=1e-13)
    order = np.argsort(lam)[:K]
    lam, X = lam[order], X[:, order]
    G = X.T @ (m[act, None] * X)
    X = X / np.sqrt(np.diag(G))[None, :]
    Phi = np.zeros((np.asarray(V).shape[0], K))
    Phi[act] = X
    return lam, Phi, m


def eigen_clusters(lam, rel_gap=1e-6):
    """Index ranges [a, b) of eigenvalues closer than rel_gap * max(|lam|, 1)."""
    out, a = [], 0
    scale = max(float(np.abs(lam).max()), 1.0)
    for i in range(1, len(lam) + 1):
        if i == len(lam) or lam[i] - lam[i - 1] > rel_gap * scale:
            out.append((a, i))
            a = i
    return out
