"""Seeded synthetic inputs for the DtN walk estimator.

This module only builds *inputs*: triangle meshes, boundary samples (rows),
quadrature weights and per-vertex basis tables. It contains none of the
estimator's arithmetic (no walks, no distance queries, no accumulation), so
both the HIP path and the CPU oracle may consume what it produces.

What the inputs stand for (Monte Carlo Steklov operators, arXiv 2606.05581):
  * the piecewise-linear hat basis of the naive estimator (Sec. 3.1, Alg. 1);
  * the point basis of Sec. 3.4 ("Point-based Galerkin basis") with the
    bilateral k-NN interpolator of Appendix B (k=8, tau_n=0.8), tabulated at
    mesh vertices and interpolated barycentrically at walk hits;
  * uniform boundary samples s ~ U(dOmega) (Alg. 1), thinned to blue noise by
    farthest-point selection, as the paper's point sets are (Sec. 3.4);
  * meshes standing in for the paper's in-the-wild inputs (Sec. 5,
    Appendix A): soups with overlaps, open seams and a non-manifold fin,
    a ~2M-face scan-sized surface, batches of uneven meshes and a
    200-component exterior scene.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os
from typing import List, Optional

import numpy as np

# --------------------------------------------------------------------------
# basic shapes
# --------------------------------------------------------------------------


def icosahedron():
    """Regular icosahedron with outward-oriented faces (vertices on the unit sphere)."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-p, p):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # faces = triples of mutually adjacent vertices (edge = shortest distance)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    e = d[d > 1e-9].min()
    adj = np.abs(d - e) < 1e-6
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    f = [i, j, k]
                    n = np.cross(v[j] - v[i], v[k] - v[i])
                    if np.dot(n, v[i] + v[j] + v[k]) < 0:
                        f = [i, k, j]
                    faces.append(f)
    return v, np.array(faces, dtype=np.int64)


def icosphere_recursive(level: int):
    """Icosahedron refined by `level` recursive 4-way splits, projected to the unit sphere.

    level 2 -> 162 vertices / 320 faces; level 5 -> 10242 / 20480.
    """
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = (np.array(verts[a]) + np.array(verts[b])) * 0.5
                m /= np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    return np.array(verts, dtype=np.float64), f


def geodesic_sphere(n: int):
    """Frequency-n geodesic sphere: 20 n^2 faces, 10 n^2 + 2 vertices, unit radius.

    Every icosahedron face is split into an n x n triangular grid; grid points
    shared by neighbouring faces are welded through an exact integer key.
    """
    iv, ifc = icosahedron()
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    m = (ii + jj) <= n
    gi, gj = ii[m], jj[m]  # local grid coords, weights (n-i-j, i, j) on (A,B,C)
    gk = n - gi - gj
    lid = -np.ones((n + 1, n + 1), dtype=np.int64)
    lid[gi, gj] = np.arange(gi.size)
    # local triangles (orientation follows (A, B, C))
    up_i, up_j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    um = (up_i + up_j) <= n - 1
    ui, uj = up_i[um], up_j[um]
    tri_up = np.stack([lid[ui, uj], lid[ui + 1, uj], lid[ui, uj + 1]], 1)
    dm = (up_i + up_j) <= n - 2
    di, dj = up_i[dm], up_j[dm]
    tri_dn = np.stack([lid[di + 1, dj], lid[di + 1, dj + 1], lid[di, dj + 1]], 1)
    ltri = np.concatenate([tri_up, tri_dn], 0)

    keys, pos, faces = [], [], []
    npts = gi.size
    for fi, (a, b, c) in enumerate(ifc):
        w = np.stack([gk, gi, gj], 1)  # weights on a, b, c
        vid = np.array([a, b, c])
        # canonical key: (vertex id, weight) pairs sorted by vertex id, zero weights dropped
        vv = np.broadcast_to(vid, w.shape).copy()
        vv[w == 0] = 15
        ww = np.where(w == 0, 0, w)
        order = np.argsort(vv, axis=1, kind="stable")
        vv = np.take_along_axis(vv, order, 1)
        ww = np.take_along_axis(ww, order, 1)
        key = np.zeros(npts, dtype=np.int64)
        for c_ in range(3):
            key = (key << 13) | (vv[:, c_].astype(np.int64) << 9) | ww[:, c_].astype(np.int64)
        keys.append(key)
        p = (w[:, 0:1] * iv[a] + w[:, 1:2] * iv[b] + w[:, 2:3] * iv[c]) / float(n)
        pos.append(p)
        faces.append(ltri + fi * npts)
    keys = np.concatenate(keys)
    pos = np.concatenate(pos, 0)
    faces = np.concatenate(faces, 0)
    uk, first, inv = np.unique(keys, return_index=True, return_inverse=True)
    V = pos[first]
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = inv[faces]
    return V, F


def torus_grid(nu: int, nv: int, R: float, r: float, weld_seam: bool = False):
    """Torus as an nu x nv quad grid (2 nu nv triangles), outward winding.

    With weld_seam=False the u and v seams keep duplicated vertices (an open
    seam in the connectivity, geometrically closed).
    """
    cu, cv = (nu, nv) if weld_seam else (nu + 1, nv + 1)
    u = np.arange(cu) * (2 * np.pi / nu)
    v = np.arange(cv) * (2 * np.pi / nv)
    U, Vv = np.meshgrid(u, v, indexing="ij")
    X = np.stack([(R + r * np.cos(Vv)) * np.cos(U), (R + r * np.cos(Vv)) * np.sin(U), r * np.sin(Vv)], -1)
    V = X.reshape(-1, 3)

    def idx(i, j):
        if weld_seam:
            return (i % nu) * cv + (j % nv)
        return i * cv + j

    I, J = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    I, J = I.ravel(), J.ravel()
    a, b, c, d = idx(I, J), idx(I + 1, J), idx(I + 1, J + 1), idx(I, J + 1)
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
    # orient outward: check against the tube direction
    cen = V[F].mean(1)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    ring = cen.copy()
    rr = np.linalg.norm(cen[:, :2], axis=1, keepdims=True)
    ring[:, :2] = cen[:, :2] / rr * R
    ring[:, 2] = 0
    flip = np.einsum("ij,ij->i", n, cen - ring) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def box_grid(m: int, half=(1.0, 1.0, 1.0)):
    """Axis-aligned box, each face an m x m quad grid: 12 m^2 triangles, outward winding."""
    Vs, Fs, off = [], [], 0
    t = np.linspace(-1.0, 1.0, m + 1)
    A, B = np.meshgrid(t, t, indexing="ij")
    I, J = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    I, J = I.ravel(), J.ravel()
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            P = np.zeros((m + 1, m + 1, 3))
            o = [k for k in range(3) if k != axis]
            P[..., axis] = sgn
            P[..., o[0]] = A
            P[..., o[1]] = B
            V = P.reshape(-1, 3)
            a = I * (m + 1) + J
            b = (I + 1) * (m + 1) + J
            c = (I + 1) * (m + 1) + J + 1
            d = I * (m + 1) + J + 1
            F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
            n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
            if np.mean(n[:, axis] * sgn) < 0:
                F = F[:, [0, 2, 1]]
            Vs.append(V)
            Fs.append(F + off)
            off += V.shape[0]
    V = np.concatenate(Vs, 0) * np.asarray(half, dtype=np.float64)
    return V, np.concatenate(Fs, 0)


def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def real_sh(L: int, dirs: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonics Y_lm, l <= L, at unit directions.

    Columns are ordered (l, m) with m = -l..l; returns (n, (L+1)^2).
    Y_l0 = K_l0 P_l(cos t); Y_lm = sqrt(2) K_lm P_l^|m|(cos t) cos(m p) for
    m > 0 and sin(|m| p) for m < 0, with P_l^m the associated Legendre
    functions without the Condon-Shortley phase and K_lm the normalisation
    sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). The normalised functions K_lm P_l^m
    come from the standard three-term recurrence in l (started from the
    diagonal l = m), which stays stable at high degree.
    """
    d = dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
    x = np.clip(d[:, 2], -1.0, 1.0)
    sxy = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    phi = np.arctan2(d[:, 1], d[:, 0])
    out = np.empty((d.shape[0], (L + 1) ** 2))
    col = lambda l, m: l * l + l + m
    qmm = np.full(x.shape, 1.0 / math.sqrt(4.0 * math.pi))  # K_00 P_0^0
    for m in range(L + 1):
        if m > 0:
            qmm = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sxy * qmm
        cm, sm = (np.cos(m * phi), np.sin(m * phi)) if m > 0 else (None, None)
        q_prev, q = None, qmm
        for l in range(m, L + 1):
            if l == m + 1:
                q_prev, q = q, math.sqrt(2.0 * m + 3.0) * x * q
            elif l > m + 1:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                q_prev, q = q, a * (x * q - b * q_prev)
            if m == 0:
                out[:, col(l, 0)] = q
            else:
                out[:, col(l, m)] = math.sqrt(2.0) * q * cm
                out[:, col(l, -m)] = math.sqrt(2.0) * q * sm
    return out


def sh_displaced_sphere(n: int, L: int, amp: float, rng):
    """Radial graph r = max(0.2, 1 + sum_{1<=l<=L} a_lm Y_lm), a_lm ~ N(0, amp^2), on a 20 n^2 geodesic sphere."""
    V, F = geodesic_sphere(n)
    ncoef = (L + 1) ** 2 - 1
    a = rng.normal(0.0, amp, size=ncoef)
    r = np.ones(V.shape[0])
    # evaluate in chunks to bound memory
    step = 200_000
    for s in range(0, V.shape[0], step):
        Y = real_sh(L, V[s : s + step])[:, 1:]
        r[s : s + step] += Y @ a
    r = np.maximum(0.2, r)
    return V * r[:, None], F


# --------------------------------------------------------------------------
# mesh helpers
# --------------------------------------------------------------------------


def face_geometry(V, F):
    """Face areas and unit normals (FP64) of an indexed mesh."""
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    c = np.cross(e1, e2)
    ln = np.linalg.norm(c, axis=1)
    area = 0.5 * ln
    n = np.where(ln[:, None] > 0, c / np.maximum(ln, 1e-300)[:, None], 0.0)
    return area, n


def vertex_normals(V, F):
    area, n = face_geometry(V, F)
    vn = np.zeros_like(V)
    for k in range(3):
        np.add.at(vn, F[:, k], n * area[:, None])
    ln = np.linalg.norm(vn, axis=1, keepdims=True)
    return np.where(ln > 0, vn / np.maximum(ln, 1e-300), 0.0)


def as_soup(V, F):
    """Unweld an indexed mesh into a triangle soup (V' = 3F vertices)."""
    V2 = V[F].reshape(-1, 3)
    F2 = np.arange(V2.shape[0], dtype=np.int64).reshape(-1, 3)
    return V2, F2


def concat_meshes(parts):
    Vs, Fs, off = [], [], 0
    for V, F in parts:
        Vs.append(V)
        Fs.append(F + off)
        off += V.shape[0]
    return np.concatenate(Vs, 0), np.concatenate(Fs, 0)


def normalise_unit_ball(V):
    """Translate to the bounding-box centre and scale so max |v| = 1."""
    c = 0.5 * (V.min(0) + V.max(0))
    V = V - c
    return V / np.linalg.norm(V, axis=1).max()


# --------------------------------------------------------------------------
# rows (boundary samples) and bases
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Rows:
    """Boundary rows of one operator estimate.

    mode 'point': row i is a surface point p[i] on face tri[i] with barycentrics
    bary[i] and unit normal n[i] (the face normal), quadrature weight w[i].
    mode 'hat_ring': row i is vertex i; its start points are drawn on the
    vertex's one-ring (ring_ptr/ring_tri/ring_cum = cumulative face areas),
    with face normals fn, and weight w[i] = (one-ring area)/3.
    """

    mode: str
    w: np.ndarray
    p: Optional[np.ndarray] = None
    n: Optional[np.ndarray] = None
    tri: Optional[np.ndarray] = None
    bary: Optional[np.ndarray] = None
    ring_ptr: Optional[np.ndarray] = None
    ring_tri: Optional[np.ndarray] = None
    ring_cum: Optional[np.ndarray] = None
    fn: Optional[np.ndarray] = None

    @property
    def n_rows(self):
        return self.w.shape[0]


@dataclasses.dataclass
class Basis:
    """Per-vertex CSR table: b(p) = sum_v lambda_v(p) * table[v] (K columns)."""

    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    K: int


def hat_rows(V, F):
    """Vertex rows for the hat basis: one-ring CSR with cumulative face areas, weights A_i."""
    area, fn = face_geometry(V, F)
    nv = V.shape[0]
    vert = F.ravel()
    faces = np.repeat(np.arange(F.shape[0]), 3)
    order = np.lexsort((faces, vert))
    vert, faces = vert[order], faces[order]
    counts = np.bincount(vert, minlength=nv)
    ptr = np.zeros(nv + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    a = area[faces]
    cum = np.empty_like(a)
    for i in range(nv):  # per-vertex running sums (small meshes only)
        cum[ptr[i] : ptr[i + 1]] = np.cumsum(a[ptr[i] : ptr[i + 1]])
    w = np.array([cum[ptr[i + 1] - 1] / 3.0 if ptr[i + 1] > ptr[i] else 0.0 for i in range(nv)])
    return Rows(mode="hat_ring", w=w, ring_ptr=ptr.astype(np.int32), ring_tri=faces.astype(np.int32),
                ring_cum=cum, fn=fn.astype(np.float32))


def hat_basis(nv):
    return Basis(rowptr=np.arange(nv + 1, dtype=np.int32), col=np.arange(nv, dtype=np.int32),
                 val=np.ones(nv, dtype=np.float32), K=nv)


def dense_basis(table: np.ndarray):
    """Dense per-vertex table (nv, K), e.g. coordinates or spherical harmonics."""
    nv, K = table.shape
    return Basis(rowptr=(np.arange(nv + 1) * K).astype(np.int32),
                 col=np.tile(np.arange(K, dtype=np.int32), nv),
                 val=table.astype(np.float32).ravel(), K=K)


def area_uniform_points(V, F, count, rng):
    """count points uniform in area: face chosen by area, point by sqrt-warped barycentrics."""
    area, _ = face_geometry(V, F)
    cdf = np.cumsum(area)
    u = rng.random(count) * cdf[-1]
    tri = np.minimum(np.searchsorted(cdf, u, side="right"), F.shape[0] - 1)
    u1, u2 = rng.random(count), rng.random(count)
    s = np.sqrt(u1)
    bary = np.stack([1.0 - s, s * (1.0 - u2), s * u2], 1)
    p = np.einsum("ij,ijk->ik", bary, V[F[tri]])
    return p, tri, bary


def farthest_point_indices(P, count):
    """Greedy farthest-point selection from pool index 0; ties go to the lowest index."""
    n = P.shape[0]
    count = min(count, n)
    idx = np.empty(count, dtype=np.int64)
    X = np.ascontiguousarray(P, dtype=np.float32)
    x, y, z = X[:, 0].copy(), X[:, 1].copy(), X[:, 2].copy()
    d = np.full(n, np.inf, dtype=np.float32)
    t = np.empty(n, dtype=np.float32)
    u = np.empty(n, dtype=np.float32)
    cur = 0
    for k in range(count):
        idx[k] = cur
        np.subtract(x, x[cur], out=t)
        np.multiply(t, t, out=t)
        np.subtract(y, y[cur], out=u)
        np.multiply(u, u, out=u)
        np.add(t, u, out=t)
        np.subtract(z, z[cur], out=u)
        np.multiply(u, u, out=u)
        np.add(t, u, out=t)
        np.minimum(d, t, out=d)
        cur = int(np.argmax(d))
    return idx


def point_rows(V, F, N, rng, pool_factor=16):
    """N farthest-point boundary samples (from an area-uniform pool), equal weights |dOmega|/N."""
    area, fn = face_geometry(V, F)
    total = area.sum()
    p, tri, bary = area_uniform_points(V, F, pool_factor * N, rng)
    sel = farthest_point_indices(p, N)
    p, tri, bary = p[sel], tri[sel], bary[sel]
    return Rows(mode="point", w=np.full(N, total / N), p=p.astype(np.float32),
                n=fn[tri].astype(np.float32), tri=tri.astype(np.int32), bary=bary.astype(np.float32))


def knn_point_basis(V, F, rows: Rows, k=8, tau_n=0.8, sigma=None, vnormals=None):
    """Point basis of the rows' sample points, tabulated at mesh vertices.

    Column j is the k-NN bilateral interpolation weight of sample j
    (Appendix B): w~ = exp(-|q-x_j|^2 / 2 sigma^2) exp(-(1 - <n_q, n_j>) / tau_n),
    normalised over the k nearest samples of the vertex q. Every vertex row
    sums to one, so barycentric interpolation keeps a partition of unity.
    """
    from scipy.spatial import cKDTree

    area, _ = face_geometry(V, F)
    N = rows.n_rows
    if sigma is None:
        sigma = 1.5 * math.sqrt(area.sum() / N)
    if vnormals is None:
        vnormals = vertex_normals(V, F)
    P = rows.p.astype(np.float64)
    Pn = rows.n.astype(np.float64)
    kk = min(k, N)
    tree = cKDTree(P)
    d, j = tree.query(V, k=kk)
    if kk == 1:
        d, j = d[:, None], j[:, None]
    wsp = np.exp(-(d ** 2) / (2.0 * sigma ** 2))
    wn = np.exp(-(1.0 - np.einsum("vc,vkc->vk", vnormals, Pn[j])) / tau_n)
    wt = wsp * wn
    s = wt.sum(1, keepdims=True)
    bad = ~(s[:, 0] > 0)
    wt = np.where(bad[:, None], 0.0, wt / np.where(s > 0, s, 1.0))
    wt[bad, 0] = 1.0  # isolated vertex: fall back to its nearest sample
    # sort columns within each row
    order = np.argsort(j, axis=1)
    j = np.take_along_axis(j, order, 1)
    wt = np.take_along_axis(wt, order, 1)
    nv = V.shape[0]
    return Basis(rowptr=(np.arange(nv + 1) * kk).astype(np.int32), col=j.astype(np.int32).ravel(),
                 val=wt.astype(np.float32).ravel(), K=N)


def morton_order(P):
    """Row order along a 3D Z-order curve of the sample positions (Sec. 4, sample sort)."""
    lo, hi = P.min(0), P.max(0)
    q = ((P - lo) / np.maximum(hi - lo, 1e-30) * 1023.0).astype(np.int64).clip(0, 1023)

    def spread(x):
        x = (x | (x << 16)) & 0x030000FF
        x = (x | (x << 8)) & 0x0300F00F
        x = (x | (x << 4)) & 0x030C30C3
        x = (x | (x << 2)) & 0x09249249
        return x

    code = spread(q[:, 0]) | (spread(q[:, 1]) << 1) | (spread(q[:, 2]) << 2)
    return np.argsort(code, kind="stable")


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------


@dataclasses.dataclass
class MeshCase:
    V: np.ndarray  # (nv,3) float32 world coordinates
    F: np.ndarray  # (nf,3) int32
    rows: Rows
    basis: Basis
    eps: float
    h: float


@dataclasses.dataclass
class Workload:
    name: str
    cases: List[MeshCase]
    walks: int
    modes: List[str]  # 'interior' / 'exterior'
    k: int  # eigenpairs (0 = none)
    note: str = ""


def _point_case(V, F, N, rng, k=8, pool_factor=16):
    V = V.astype(np.float64)
    rows = point_rows(V, F, N, rng, pool_factor=pool_factor)
    area, _ = face_geometry(V, F)
    h = 0.25 * math.sqrt(area.sum() / N)
    eps = min(1e-3, h / 10.0)
    basis = knn_point_basis(V, F, rows, k=k)
    return MeshCase(V=V.astype(np.float32), F=F.astype(np.int32), rows=rows, basis=basis, eps=eps, h=h)


def unit_sphere_320():
    """Unit icosphere (2 recursive splits: 162 V / 320 F), hat basis, vertex rows, 256 walks."""
    V, F = icosphere_recursive(2)
    rows = hat_rows(V, F)
    case = MeshCase(V=V.astype(np.float32), F=F.astype(np.int32), rows=rows,
                    basis=hat_basis(V.shape[0]), eps=1e-3, h=0.05)
    return Workload("unit_sphere_320", [case], walks=256, modes=["interior", "exterior"], k=25)


def soup8_53k(N=2000, walks=1024):
    """5 ellipsoids + 3 tori + 1 fin triangle as one unindexed soup (53,249 faces), 2,000 rows."""
    rng = np.random.default_rng(1001)
    parts = []
    centres = []
    for i in range(8):
        while True:
            c = rng.normal(size=3)
            c = c / np.linalg.norm(c) * 0.6 * rng.random() ** (1 / 3)
            break
        centres.append(c)
    # forced overlaps: ellipsoid 0 and 1; torus 0 (shape 5) through ellipsoid 2
    centres[1] = centres[0] + np.array([0.15, 0.05, 0.0])
    centres[5] = centres[2] + np.array([0.0, 0.1, 0.05])
    for i in range(5):
        V, F = icosphere_recursive(4)
        ax = rng.uniform(0.15, 0.4, size=3)
        R = random_rotation(rng)
        V = (V * ax) @ R.T + centres[i]
        if i == 3:  # non-manifold fin on one edge of ellipsoid 3
            a, b = F[0, 0], F[0, 1]
            nrm = np.cross(V[F[0, 1]] - V[F[0, 0]], V[F[0, 2]] - V[F[0, 0]])
            nrm /= np.linalg.norm(nrm)
            tip = 0.5 * (V[a] + V[b]) + 0.08 * nrm
            V = np.concatenate([V, tip[None]], 0)
            F = np.concatenate([F, np.array([[a, b, V.shape[0] - 1]])], 0)
        parts.append((V, F))
    for i in range(3):
        Rr, rr = rng.uniform(0.2, 0.35), rng.uniform(0.05, 0.12)
        V, F = torus_grid(96, 48, Rr, rr, weld_seam=False)
        R = random_rotation(rng)
        V = V @ R.T + centres[5 + i]
        parts.append((V, F))
    V, F = concat_meshes(parts)
    V, F = as_soup(V, F)
    V = normalise_unit_ball(V)
    case = _point_case(V, F, N, rng)
    return Workload("soup8_53k", [case], walks=walks, modes=["interior", "exterior"], k=32)


def sh_sphere_2m(n=316, N=10000, walks=4096):
    """Sphere displaced by random SH (l<=16, a_lm~N(0,0.05^2)) on a 20 n^2 geodesic grid (~2.0M faces)."""
    rng = np.random.default_rng(1002)
    V, F = sh_displaced_sphere(n, 16, 0.05, rng)
    V = normalise_unit_ball(V)
    case = _point_case(V, F, N, rng)
    return Workload("sh_sphere_2m", [case], walks=walks, modes=["interior"], k=64)


def batch64_mixed(n_meshes=64, walks=1024, face_lo=5e3, face_hi=5e5, rows_lo=512, rows_hi=4096, seed=1003):
    """64 meshes cycling SH-sphere / ellipsoid / torus / box, faces log-uniform in [5e3, 5e5]."""
    rng = np.random.default_rng(seed)
    cases = []
    for m in range(n_meshes):
        target = math.exp(rng.uniform(math.log(face_lo), math.log(face_hi)))
        kind = m % 4
        if kind == 0:
            n = max(2, round(math.sqrt(target / 20)))
            V, F = sh_displaced_sphere(n, 8, 0.05, rng)
        elif kind == 1:
            n = max(2, round(math.sqrt(target / 20)))
            V, F = geodesic_sphere(n)
            V = V * rng.uniform(0.3, 1.0, size=3)
        elif kind == 2:
            nv = max(3, round(math.sqrt(target / 4)))
            V, F = torus_grid(2 * nv, nv, 1.0, rng.uniform(0.2, 0.45), weld_seam=True)
        else:
            mm = max(1, round(math.sqrt(target / 12)))
            V, F = box_grid(mm, half=rng.uniform(0.4, 1.0, size=3))
        V = V @ random_rotation(rng).T
        V = normalise_unit_ball(V)
        N = int(rng.integers(rows_lo, rows_hi + 1))
        cases.append(_point_case(V, F, N, rng, pool_factor=4))
    return Workload("batch64_mixed", cases, walks=walks, modes=["interior"], k=0)


def exterior200_301k(N=20000, walks=256):
    """100 ellipsoids (1,280 F) + 100 boxes (1,728 F), bounding spheres disjoint, exterior operator."""
    rng = np.random.default_rng(1004)
    shapes = []
    for i in range(200):
        if i < 100:
            V, F = icosphere_recursive(3)
            V = V * rng.uniform(0.5, 1.5, size=3)
        else:
            V, F = box_grid(12, half=rng.uniform(0.5, 1.5, size=3))
        V = V @ random_rotation(rng).T
        shapes.append((V, F, np.linalg.norm(V, axis=1).max()))
    placed = []
    parts = []
    for V, F, r in shapes:
        for _ in range(100000):
            c = rng.uniform(-20.0, 20.0, size=3)
            if all(np.linalg.norm(c - c2) > r + r2 + 0.5 for c2, r2 in placed):
                break
        placed.append((c, r))
        parts.append((V + c, F))
    V, F = concat_meshes(parts)
    V = normalise_unit_ball(V)
    case = _point_case(V, F, N, rng, pool_factor=8)
    return Workload("exterior200_301k", [case], walks=walks, modes=["exterior"], k=128)


def sh_sphere_mesh(n=316, seed=1002):
    """The SH-displaced sphere of sh_sphere_2m alone (20 n^2 faces; n = 316:
    998,562 vertices, 1,997,120 faces), FP32 positions in the unit ball."""
    rng = np.random.default_rng(seed)
    V, F = sh_displaced_sphere(n, 16, 0.05, rng)
    V = normalise_unit_ball(V)
    return V.astype(np.float32), F.astype(np.int32)


def psd_sh_sphere_2m(n=316, N=16384, pairs=320, K=128):
    """PSD estimator (Alg. 2) workload at the scale of the paper's runtime study
    (2^14 sample points, about 10M walks, the first 128 basis functions): the
    SH-displaced sphere of sh_sphere_2m (~2.0M faces), N farthest-point rows,
    and a dense basis of the first K real spherical harmonics of the vertex
    directions (standing in for the surface Laplacian's low modes)."""
    rng = np.random.default_rng(1002)
    V, F = sh_displaced_sphere(n, 16, 0.05, rng)
    V = normalise_unit_ball(V)
    rows = point_rows(V, F, N, rng, pool_factor=4)
    area, _ = face_geometry(V, F)
    h = 0.25 * math.sqrt(area.sum() / N)
    eps = 1e-5  # the PSD walks start next to the surface: a fine termination shell (the paper's is 1e-6)
    L = int(math.ceil(math.sqrt(K))) - 1
    table = real_sh(L, V)[:, :K]
    case = MeshCase(V=V.astype(np.float32), F=F.astype(np.int32), rows=rows, basis=dense_basis(table), eps=eps, h=h)
    return Workload("psd_sh_sphere_2m", [case], walks=2 * pairs, modes=["interior"], k=0,
                    note=f"PSD estimator: {N} rows x {pairs} antithetic pairs, K={K}")


WORKLOADS = {
    "unit_sphere_320": unit_sphere_320,
    "soup8_53k": soup8_53k,
    "sh_sphere_2m": sh_sphere_2m,
    "batch64_mixed": batch64_mixed,
    "exterior200_301k": exterior200_301k,
    "psd_sh_sphere_2m": psd_sh_sphere_2m,
}


def _cache_dir():
    d = os.environ.get("MSK_WORKLOAD_CACHE")
    if d is None:
        d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".workload_cache")
    os.makedirs(d, exist_ok=True)
    return d


def _save(path, wl: Workload):
    blob = {"name": wl.name, "walks": wl.walks, "modes": ",".join(wl.modes), "k": wl.k, "ncases": len(wl.cases)}
    arrs = {}
    for i, c in enumerate(wl.cases):
        arrs[f"{i}_V"], arrs[f"{i}_F"] = c.V, c.F
        arrs[f"{i}_eps"], arrs[f"{i}_h"] = np.array(c.eps), np.array(c.h)
        for f in dataclasses.fields(Rows):
            v = getattr(c.rows, f.name)
            if v is not None:
                arrs[f"{i}_rows_{f.name}"] = np.array(v)
        for f in dataclasses.fields(Basis):
            arrs[f"{i}_basis_{f.name}"] = np.array(getattr(c.basis, f.name))
    np.savez(path, **{k: np.array(v) for k, v in blob.items()}, **arrs)


def _load(path) -> Workload:
    z = np.load(path, allow_pickle=False)
    cases = []
    for i in range(int(z["ncases"])):
        rk = {f.name: (z[f"{i}_rows_{f.name}"] if f"{i}_rows_{f.name}" in z else None) for f in dataclasses.fields(Rows)}
        rk["mode"] = str(rk["mode"])
        bk = {f.name: z[f"{i}_basis_{f.name}"] for f in dataclasses.fields(Basis)}
        bk["K"] = int(bk["K"])
        cases.append(MeshCase(V=z[f"{i}_V"], F=z[f"{i}_F"], rows=Rows(**rk), basis=Basis(**bk),
                              eps=float(z[f"{i}_eps"]), h=float(z[f"{i}_h"])))
    return Workload(str(z["name"]), cases, int(z["walks"]), str(z["modes"]).split(","), int(z["k"]))


def load(name: str, cache: bool = True, **kw) -> Workload:
    """Build (or load from the local cache) a named workload."""
    fn = WORKLOADS[name]
    if not cache:
        return fn(**kw)
    key = hashlib.sha1((name + repr(sorted(kw.items())) + "v3").encode()).hexdigest()[:12]
    path = os.path.join(_cache_dir(), f"{name}_{key}.npz")
    if os.path.exists(path):
        return _load(path)
    wl = fn(**kw)
    tmp = path + ".tmp.npz"
    _save(tmp, wl)
    os.replace(tmp, path)
    return wl
