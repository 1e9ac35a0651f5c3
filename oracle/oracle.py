"""CPU oracle for the Monte Carlo DtN walk estimator (arXiv 2606.05581).

TEST INFRASTRUCTURE ONLY: the plain FP64 reference that the GPU library is
checked against. Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the GPU product path never does.

The walks run in ``oracle.c`` (built to ``liboracle.so`` with gcc); this file
binds it and adds the dense post-processing steps, each written from its
definition:

* ``finalize`` -- Alg. 1's scaling of the accumulated rank-one updates by
  |dOmega| / (N h) (Sec. 3.1), here per row i as w_i / (h W), and the sample
  standard error of every entry;
* ``symmetrise`` -- Alg. 1's last step S <- (S + S^T) / 2;
* ``steklov_modes`` -- the Steklov eigenproblem (Sec. 2, eq.
  steklov-eigenproblem) discretised with a lumped mass M = diag(w): the
  smallest k eigenpairs of M^-1/2 (S + S^T)/2 M^-1/2 by LAPACK (numpy.eigh),
  eigenvectors mapped back by M^-1/2;
* ``psd_estimate`` -- the PSD estimator of Sec. 3.2 (Alg. 2), run in
  ``oracle.c``, with ``psd_standard_error`` for its entries;
* ``kelvin_estimate`` -- the exterior estimator of Sec. 3.3 in the
  Kelvin-inverted exterior (jump term from tangent balls, killing term from
  walks started at the image of infinity), run in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# walk status codes
HIT, ESCAPED, CAPPED = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no fused multiply-adds, OpenMP over rows)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _P(t):
    return C.POINTER(t)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_P(C.c_uint32), _P(C.c_uint32), _P(C.c_uint32)]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_closest_tri.argtypes = [_P(C.c_double)] * 5
        L.orc_closest_tri.restype = C.c_double
        L.orc_closest_tri_f32.argtypes = [_P(C.c_float)] * 5
        L.orc_closest_tri_f32.restype = C.c_float
        L.orc_scene_frame.argtypes = [_P(C.c_float), C.c_int64, _P(C.c_double), _P(C.c_double)]
        L.orc_scene_create.argtypes = [_P(C.c_float), C.c_int64, _P(C.c_int32), C.c_int64, C.c_int]
        L.orc_scene_create.restype = C.c_void_p
        L.orc_scene_destroy.argtypes = [C.c_void_p]
        L.orc_scene_info.argtypes = [C.c_void_p, _P(C.c_double), _P(C.c_double)]
        L.orc_nearest.argtypes = [C.c_void_p, _P(C.c_double), C.c_int64, C.c_int, _P(C.c_int64),
                                  _P(C.c_double), _P(C.c_double)]
        L.orc_nearest_f32.argtypes = [_P(C.c_float), _P(C.c_int32), C.c_int64, _P(C.c_float), C.c_int64,
                                      _P(C.c_int32), _P(C.c_float), _P(C.c_float)]
        L.orc_reentry_mu.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_reentry_mu.restype = C.c_double
        L.orc_walks_from.argtypes = [C.c_void_p, _P(C.c_double), C.c_int64, C.c_double, C.c_double, C.c_double,
                                     C.c_int64, C.c_uint64, _P(C.c_int32), _P(C.c_int64), _P(C.c_double),
                                     _P(C.c_int64)]
        L.orc_estimate.argtypes = (
            [C.c_void_p, C.c_int, C.c_int, C.c_int64, _P(C.c_int32)]
            + [_P(C.c_float), _P(C.c_float), _P(C.c_int32), _P(C.c_float)]
            + [_P(C.c_int32), _P(C.c_int32), _P(C.c_double), _P(C.c_float)]
            + [_P(C.c_int32), _P(C.c_int32), _P(C.c_float), C.c_int64]
            + [C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_uint64,
               C.c_uint32, C.c_int]
            + [_P(C.c_double), _P(C.c_double), _P(C.c_int64), _P(C.c_int64), _P(C.c_int64), _P(C.c_int32)]
            + [_P(C.c_int32), _P(C.c_int64), _P(C.c_float), _P(C.c_int64), _P(C.c_int32), _P(C.c_float)]
            + [_P(C.c_double), _P(C.c_double), C.c_int64, C.c_int, C.c_double, C.c_double, C.c_int]
        )
        L.orc_knn_weights.argtypes = [_P(C.c_double), _P(C.c_double), C.c_int64, C.c_int, C.c_double, C.c_double,
                                      _P(C.c_double), _P(C.c_double), _P(C.c_int32), _P(C.c_double)]
        L.orc_knn_weights.restype = C.c_int
        L.orc_tangent_ball.argtypes = [C.c_void_p, _P(C.c_double), _P(C.c_double), C.c_double, C.c_int, C.c_double]
        L.orc_tangent_ball.restype = C.c_double
        L.orc_ball_jump_mass.argtypes = [C.c_double, C.c_double]
        L.orc_ball_jump_mass.restype = C.c_double
        L.orc_ball_point.argtypes = [_P(C.c_double), C.c_double, _P(C.c_double), C.c_double, C.c_double, C.c_double,
                                     C.c_int, _P(C.c_double)]
        L.orc_psd_estimate.argtypes = (
            [C.c_void_p, C.c_int64, _P(C.c_float), _P(C.c_float), _P(C.c_int32), _P(C.c_float), _P(C.c_double),
             _P(C.c_double), C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_double,
             C.c_double, C.c_double, C.c_int64, C.c_uint64, C.c_uint32, C.c_int]
            + [_P(C.c_double), _P(C.c_double), _P(C.c_double), _P(C.c_double), _P(C.c_int64)]
            + [_P(C.c_int32), _P(C.c_int64), _P(C.c_float), _P(C.c_int64)]
        )
        L.orc_kelvin_tri_d2.argtypes = [_P(C.c_double)] * 6
        L.orc_kelvin_tri_d2.restype = C.c_double
        L.orc_kelvin_create.argtypes = [_P(C.c_float), C.c_int64, _P(C.c_int32), C.c_int64, _P(C.c_double)]
        L.orc_kelvin_create.restype = C.c_void_p
        L.orc_kelvin_destroy.argtypes = [C.c_void_p]
        L.orc_kelvin_info.argtypes = [C.c_void_p, _P(C.c_double), _P(C.c_double), _P(C.c_double)]
        L.orc_kelvin_nearest.argtypes = [C.c_void_p, _P(C.c_double), C.c_int64, C.c_int, _P(C.c_int64),
                                         _P(C.c_double), _P(C.c_double), _P(C.c_double)]
        L.orc_kelvin_tangent_ball.argtypes = [C.c_void_p, _P(C.c_double), _P(C.c_double), C.c_double, C.c_int,
                                              C.c_double]
        L.orc_kelvin_tangent_ball.restype = C.c_double
        L.orc_kelvin_point_normal.argtypes = [_P(C.c_double)] * 4
        L.orc_kelvin_estimate.argtypes = (
            [C.c_void_p, C.c_int64, _P(C.c_float), _P(C.c_float), _P(C.c_int32), _P(C.c_float), _P(C.c_double),
             _P(C.c_double), C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_double,
             C.c_double, C.c_double, C.c_int64, C.c_uint64, C.c_uint32, C.c_int]
            + [_P(C.c_double)] * 6 + [_P(C.c_int64), _P(C.c_int64), _P(C.c_int32), _P(C.c_int64), _P(C.c_float)]
        )
        _lib = L
    return _lib


def _ptr(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(_P(t))


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


# ----------------------------------------------------------------- primitives


def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC 2011) of a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def uniform(r):
    return lib().orc_uniform(int(r))


def closest_tri(p, a, b, c):
    """FP64 squared distance from p to triangle abc and the closest point's barycentrics."""
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (p, a, b, c)]
    l = np.zeros(3)
    d2 = lib().orc_closest_tri(*[_ptr(x, C.c_double) for x in args], _ptr(l, C.c_double))
    return d2, l


def closest_tri_f32(p, a, b, c):
    args = [np.ascontiguousarray(x, dtype=np.float32) for x in (p, a, b, c)]
    l = np.zeros(2, dtype=np.float32)
    d2 = lib().orc_closest_tri_f32(*[_ptr(x, C.c_float) for x in args], _ptr(l, C.c_float))
    return np.float32(d2), l


def reentry_mu(rho, R, u):
    return lib().orc_reentry_mu(float(rho), float(R), float(u))


def scene_frame(V):
    V = _c(V, np.float32)
    c = np.zeros(3)
    r = np.zeros(1)
    lib().orc_scene_frame(_ptr(V, C.c_float), V.shape[0], _ptr(c, C.c_double), _ptr(r, C.c_double))
    return c, float(r[0])


class Scene:
    """Mesh in the oracle's FP64 scene frame (optionally with a BVH that
    returns exactly the brute-force minimum)."""

    def __init__(self, V, F, bvh: bool = True):
        self.V = _c(V, np.float32)
        self.F = _c(F, np.int32)
        self.h = lib().orc_scene_create(_ptr(self.V, C.c_float), self.V.shape[0], _ptr(self.F, C.c_int32),
                                        self.F.shape[0], int(bvh))
        c = np.zeros(3)
        r = np.zeros(1)
        lib().orc_scene_info(self.h, _ptr(c, C.c_double), _ptr(r, C.c_double))
        self.centre, self.radius = c, float(r[0])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    def nearest(self, Q, bvh: bool = True):
        Q = _c(Q, np.float64).reshape(-1, 3)
        n = Q.shape[0]
        tri = np.zeros(n, dtype=np.int64)
        d2 = np.zeros(n)
        bary = np.zeros((n, 3))
        lib().orc_nearest(self.h, _ptr(Q, C.c_double), n, int(bvh), _ptr(tri, C.c_int64), _ptr(d2, C.c_double),
                          _ptr(bary, C.c_double))
        return tri, d2, bary

    def rel32(self, X):
        """World points to float offsets from the scene centre (the single-precision frame)."""
        return (np.asarray(X, dtype=np.float64) - self.centre).astype(np.float32)

    def nearest_f32(self, Q):
        """Brute-force FP32 nearest triangle (index, d2, barycentrics of vertices 1, 2)."""
        Vr = self.rel32(self.V.astype(np.float64))
        Qr = np.ascontiguousarray(self.rel32(np.asarray(Q).reshape(-1, 3)))
        n = Qr.shape[0]
        tri = np.zeros(n, dtype=np.int32)
        d2 = np.zeros(n, dtype=np.float32)
        b = np.zeros((n, 2), dtype=np.float32)
        lib().orc_nearest_f32(_ptr(Vr, C.c_float), _ptr(self.F, C.c_int32), self.F.shape[0], _ptr(Qr, C.c_float),
                              n, _ptr(tri, C.c_int32), _ptr(d2, C.c_float), _ptr(b, C.c_float))
        return tri, d2, b

    def walks_from(self, X, eps, seed=0, kappa=2.0 ** -20, delta_rel=2.0 ** -21, max_steps=100000):
        """Walk-on-Spheres from world points X: (status, terminal triangle, barycentrics, queries)."""
        X = _c(X, np.float64).reshape(-1, 3)
        n = X.shape[0]
        st = np.zeros(n, dtype=np.int32)
        tri = np.zeros(n, dtype=np.int64)
        bary = np.zeros((n, 3))
        nq = np.zeros(n, dtype=np.int64)
        lib().orc_walks_from(self.h, _ptr(X, C.c_double), n, eps, kappa, delta_rel * self.radius, max_steps,
                             C.c_uint64(seed), _ptr(st, C.c_int32), _ptr(tri, C.c_int64), _ptr(bary, C.c_double),
                             _ptr(nq, C.c_int64))
        return st, tri, bary, nq

    def hit_points(self, tri, bary):
        """World-space positions of (triangle, barycentric) pairs."""
        P = np.einsum("ij,ijk->ik", bary, self.V.astype(np.float64)[self.F[tri]])
        return P


DEFAULT_MAX_STEPS = {"interior": 1024, "exterior": 8192}


def estimate(scene: Scene, rows, basis, walks: int, eps: float, h: float, exterior: bool, seed: int = 0,
             w0: int = 0, rows_sel=None, kappa=2.0 ** -20, delta_rel=2.0 ** -21, max_steps=None, mesh: int = 0,
             log: bool = False, nthreads: int = 1, knn=None, jump_only: bool = False):
    """Accumulate the naive estimator's per-walk contributions c = b(s) - b(t).

    ``jump_only`` (exterior): drop the killing term of the exterior form
    (Sec. 3.3, eq. exterior-dtn-beurling-deny-form; the paper's default,
    Sec. 4): an escaped walk then contributes nothing instead of b(s).

    ``knn`` (point rows only) replaces the per-vertex table by the point
    basis: a dict with ``points`` (N,3 world), ``normals`` (N,3 unit), ``k``,
    ``sigma``, ``tau``; the K = N columns are the points.

    Returns a dict with ``acc`` (sum of c), ``acc2`` (sum of c^2), each
    (n_rows_selected, K), per-row query / escape / capped counts, discard
    flags and (optionally) a walk log of status, terminal triangle,
    barycentrics of the terminal triangle's second and third vertices, query
    count, start triangle and start barycentrics (second and third vertices).
    """
    if max_steps is None:
        max_steps = DEFAULT_MAX_STEPS["exterior" if exterior else "interior"]
    mode = 0 if rows.mode == "point" else 1
    sel = None if rows_sel is None else np.ascontiguousarray(rows_sel, dtype=np.int32)
    n = rows.n_rows if sel is None else sel.shape[0]
    if knn is not None:
        if mode != 0 or not (1 <= int(knn["k"]) <= 32):
            raise ValueError("the point basis takes point rows and 1 <= k <= 32")
        kx, kn = _c(knn["points"], np.float64), _c(knn["normals"], np.float64)
        K = kx.shape[0]
    else:
        kx = kn = None
        K = int(basis.K)
    acc = np.zeros((n, K))
    acc2 = np.zeros((n, K))
    nq = np.zeros(n, dtype=np.int64)
    nesc = np.zeros(n, dtype=np.int64)
    ncap = np.zeros(n, dtype=np.int64)
    disc = np.zeros(n, dtype=np.int32)
    if log:
        # walks of discarded rows never run: status and triangle stay -1
        ls = np.full((n, walks), -1, dtype=np.int32)
        lt = np.full((n, walks), -1, dtype=np.int64)
        lb = np.zeros((n, walks, 2), dtype=np.float32)
        lq = np.zeros((n, walks), dtype=np.int64)
        lst = np.full((n, walks), -1, dtype=np.int32)
        lsb = np.zeros((n, walks, 2), dtype=np.float32)
    else:
        ls = lt = lb = lq = lst = lsb = None
    p, nn, tri, bary = (_c(rows.p, np.float32), _c(rows.n, np.float32), _c(rows.tri, np.int32),
                        _c(rows.bary, np.float32))
    rp, rt, rc, fn = (_c(rows.ring_ptr, np.int32), _c(rows.ring_tri, np.int32), _c(rows.ring_cum, np.float64),
                      _c(rows.fn, np.float32))
    if basis is not None:
        brp, bc, bv = _c(basis.rowptr, np.int32), _c(basis.col, np.int32), _c(basis.val, np.float32)
    else:
        brp = bc = bv = None
    lib().orc_estimate(
        scene.h, mode, int(exterior), n, _ptr(sel, C.c_int32),
        _ptr(p, C.c_float), _ptr(nn, C.c_float), _ptr(tri, C.c_int32), _ptr(bary, C.c_float),
        _ptr(rp, C.c_int32), _ptr(rt, C.c_int32), _ptr(rc, C.c_double), _ptr(fn, C.c_float),
        _ptr(brp, C.c_int32), _ptr(bc, C.c_int32), _ptr(bv, C.c_float), K,
        walks, w0, eps, h, kappa, delta_rel * scene.radius, max_steps, C.c_uint64(seed), mesh, nthreads,
        _ptr(acc, C.c_double), _ptr(acc2, C.c_double), _ptr(nq, C.c_int64), _ptr(nesc, C.c_int64),
        _ptr(ncap, C.c_int64), _ptr(disc, C.c_int32),
        _ptr(ls, C.c_int32), _ptr(lt, C.c_int64), _ptr(lb, C.c_float), _ptr(lq, C.c_int64),
        _ptr(lst, C.c_int32), _ptr(lsb, C.c_float),
        _ptr(kx, C.c_double), _ptr(kn, C.c_double), 0 if kx is None else kx.shape[0],
        0 if knn is None else int(knn["k"]), 0.0 if knn is None else float(knn["sigma"]),
        0.0 if knn is None else float(knn["tau"]), int(bool(jump_only)))
    out = dict(acc=acc, acc2=acc2, n_query=nq, n_escaped=nesc, n_capped=ncap, discarded=disc, walks=walks)
    if log:
        out.update(log_status=ls, log_tri=lt, log_bary=lb, log_nquery=lq, log_stri=lst, log_sbary=lsb)
    return out


# ----------------------------------------------------------- dense post-steps


def finalize(acc, acc2, w, h, W, discarded=None):
    """Row i of the estimate: S_i = w_i / (h W) * sum_w c_w (Alg. 1's |dOmega|/(N h)
    weight, stratified by row), and the standard error of each entry's mean,
    se_ij = (w_i / h) * sqrt(var_ij / W) with the unbiased sample variance."""
    w = np.asarray(w, dtype=np.float64).copy()
    if discarded is not None:
        w[np.asarray(discarded) != 0] = 0.0
    mean = acc / W
    var = np.maximum(0.0, (acc2 / W - mean ** 2)) * (W / (W - 1.0))
    S = (w / h)[:, None] * mean
    se = (w / h)[:, None] * np.sqrt(var / W)
    return S, se


def symmetrise(S):
    """Alg. 1, last step: S <- (S + S^T) / 2."""
    return 0.5 * (S + S.T)


def steklov_modes(S, w, k):
    """Smallest-k eigenpairs of the generalised problem (S+S^T)/2 psi = lambda M psi, M = diag(w).

    Rows with zero weight (discarded samples) are removed first. Returns
    (eigenvalues ascending, eigenvectors psi (n_kept, k), kept row indices).
    """
    w = np.asarray(w, dtype=np.float64)
    keep = np.nonzero(w > 0)[0]
    Ss = symmetrise(S[np.ix_(keep, keep)])
    m = 1.0 / np.sqrt(w[keep])
    Cm = m[:, None] * Ss * m[None, :]
    lam, V = np.linalg.eigh(Cm)
    k = min(k, lam.shape[0])
    return lam[:k], m[:, None] * V[:, :k], keep


# ------------------------------------------------- PSD estimator (Sec. 3.2)

PSD_CAP_DEG = 2.5          # excluded cap about s (Sec. 3.2, Implementation), angle at the ball centre
PSD_BISECT_ITERS = 10      # tangent-ball bisection steps (Sec. 3.2, Implementation)


def psd_r_max(V):
    """Largest tangent-ball radius: half the shortest side of the mesh's bounding box
    (the diameter clamp of Appendix A, unbounded tangent balls)."""
    V = np.asarray(V, dtype=np.float64)
    return 0.5 * float((V.max(0) - V.min(0)).min())


def tangent_ball(scene: Scene, s, n, r_max, iters=PSD_BISECT_ITERS, tol=5e-5):
    """Radius of the largest ball inside the domain tangent at world point s (outward unit normal n),
    overlapping the surface by less than tol."""
    sr = _c(np.asarray(s, dtype=np.float64) - scene.centre, np.float64)
    nn = _c(n, np.float64)
    return float(lib().orc_tangent_ball(scene.h, _ptr(sr, C.c_double), _ptr(nn, C.c_double), r_max, iters, tol))


def ball_jump_mass(r, theta0):
    """Integral of the ball jump kernel 1/(2 pi |s-z|^3) over the sphere minus the cap of angle theta0."""
    return float(lib().orc_ball_jump_mass(r, theta0))


def ball_point(c, r, n, theta0, xi, eta, partner=0):
    """The ball point drawn from uniforms (xi, eta), or its antithetic partner."""
    cc, nn = _c(c, np.float64), _c(n, np.float64)
    z = np.zeros(3)
    lib().orc_ball_point(_ptr(cc, C.c_double), r, _ptr(nn, C.c_double), theta0, xi, eta, int(partner),
                         _ptr(z, C.c_double))
    return z


def psd_estimate(scene: Scene, rows, table, pairs: int, eps: float, seed: int = 0, cap_deg=PSD_CAP_DEG,
                 r_max=None, bisect_iters=PSD_BISECT_ITERS, kappa=2.0 ** -20, delta_rel=2.0 ** -21,
                 max_steps=None, mesh: int = 0, log: bool = False, nthreads: int = 1):
    """Alg. 2 over point rows with a dense per-vertex basis table (n_verts x K).

    Returns S (K x K, the estimate), Q (sum of squared per-pair terms), se (its
    standard error per entry), per-row tangent-ball radius (0 = dropped), the
    jump-kernel mass Z, query counts and an optional walk log (n_rows x
    2 pairs)."""
    if rows.mode != "point":
        raise ValueError("the PSD estimator takes point rows")
    if max_steps is None:
        max_steps = DEFAULT_MAX_STEPS["interior"]
    if r_max is None:
        r_max = psd_r_max(scene.V)
    tab = _c(table, np.float64)
    nv, K = tab.shape
    n = rows.n_rows
    S = np.zeros((K, K))
    Q = np.zeros((K, K))
    rad = np.zeros(n)
    Z = np.zeros(n)
    nq = np.zeros(n, dtype=np.int64)
    W2 = 2 * pairs
    if log:
        ls = np.full((n, W2), -1, dtype=np.int32)
        lt = np.full((n, W2), -1, dtype=np.int64)
        lb = np.zeros((n, W2, 2), dtype=np.float32)
        lq = np.zeros((n, W2), dtype=np.int64)
    else:
        ls = lt = lb = lq = None
    p, nn, tri, bary = (_c(rows.p, np.float32), _c(rows.n, np.float32), _c(rows.tri, np.int32),
                        _c(rows.bary, np.float32))
    w = _c(rows.w, np.float64)
    lib().orc_psd_estimate(scene.h, n, _ptr(p, C.c_float), _ptr(nn, C.c_float), _ptr(tri, C.c_int32),
                           _ptr(bary, C.c_float), _ptr(w, C.c_double), _ptr(tab, C.c_double), K, pairs,
                           np.deg2rad(cap_deg), r_max, bisect_iters, eps, kappa, delta_rel * scene.radius,
                           max_steps, C.c_uint64(seed), mesh, nthreads, _ptr(S, C.c_double), _ptr(Q, C.c_double),
                           _ptr(rad, C.c_double), _ptr(Z, C.c_double), _ptr(nq, C.c_int64),
                           _ptr(ls, C.c_int32), _ptr(lt, C.c_int64), _ptr(lb, C.c_float), _ptr(lq, C.c_int64))
    out = dict(S=S, Q=Q, se=psd_standard_error(S, Q, n * pairs), radius=rad, Z=Z, n_query=nq, pairs=pairs)
    if log:
        out.update(log_status=ls, log_tri=lt, log_bary=lb, log_nquery=lq)
    return out


def psd_standard_error(S, Q, n_pairs):
    """Standard error of S = sum_p X_p over n_pairs pair terms, the pairs taken as
    independent draws of n_pairs X_p: se^2 = (n_pairs Q - S^2) / (n_pairs - 1)."""
    return np.sqrt(np.maximum(0.0, n_pairs * Q - S * S) / (n_pairs - 1.0))


# ------------------------------------- Kelvin-inverted exterior (Sec. 3.3)


def kelvin(x):
    """Kelvin transform about the origin, x -> x / |x|^2 (Sec. 3.3, The Kelvin Transform)."""
    x = np.asarray(x, dtype=np.float64)
    return x / np.sum(x * x, axis=-1, keepdims=True)


def kelvin_tri_d2(p, a, b, c):
    """Squared distance from p to the image of triangle abc under the Kelvin
    transform (all relative to the inversion centre), the nearest point q
    and the barycentrics of its image in abc."""
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (p, a, b, c)]
    q, l = np.zeros(3), np.zeros(3)
    d2 = lib().orc_kelvin_tri_d2(*[_ptr(x, C.c_double) for x in args], _ptr(q, C.c_double), _ptr(l, C.c_double))
    return d2, q, l


def kelvin_point_normal(s, ns):
    """s~ = kappa(s) and the unit normal there pointing out of the inverted
    exterior (s relative to the centre, ns the primal outward unit normal)."""
    s, ns = _c(s, np.float64), _c(ns, np.float64)
    st, nt = np.zeros(3), np.zeros(3)
    lib().orc_kelvin_point_normal(_ptr(s, C.c_double), _ptr(ns, C.c_double), _ptr(st, C.c_double),
                                  _ptr(nt, C.c_double))
    return st, nt


class KelvinScene:
    """A mesh seen through the Kelvin transform about a centre inside it: the
    inverted exterior, bounded by the images of the triangles (spherical
    patches), with brute-force nearest-patch queries."""

    def __init__(self, V, F, centre):
        self.V = _c(V, np.float32)
        self.F = _c(F, np.int32)
        self.centre = _c(centre, np.float64)
        self.h = lib().orc_kelvin_create(_ptr(self.V, C.c_float), self.V.shape[0], _ptr(self.F, C.c_int32),
                                         self.F.shape[0], _ptr(self.centre, C.c_double))
        lo, hi, r = np.zeros(3), np.zeros(3), np.zeros(1)
        lib().orc_kelvin_info(self.h, _ptr(lo, C.c_double), _ptr(hi, C.c_double), _ptr(r, C.c_double))
        self.lo, self.hi, self.radius = lo, hi, float(r[0])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_kelvin_destroy(self.h)
            self.h = None

    def nearest(self, Q, bvh: bool = True):
        """Nearest inverted triangle of points Q (inverted space, relative to
        the centre): (index, squared distance, nearest point, primal
        barycentrics); the BVH returns the brute-force minimum."""
        Q = _c(Q, np.float64).reshape(-1, 3)
        n = Q.shape[0]
        tri, d2, q, l = np.zeros(n, dtype=np.int64), np.zeros(n), np.zeros((n, 3)), np.zeros((n, 3))
        lib().orc_kelvin_nearest(self.h, _ptr(Q, C.c_double), n, int(bvh), _ptr(tri, C.c_int64),
                                 _ptr(d2, C.c_double), _ptr(q, C.c_double), _ptr(l, C.c_double))
        return tri, d2, q, l

    def r_max(self):
        """Largest tangent-ball radius: half the shortest side of the inverted
        surface's bounding box (Appendix, unbounded tangent balls, for the
        exterior), here the box of the inverted vertices."""
        return 0.5 * float((self.hi - self.lo).min())


def kelvin_estimate(ks: KelvinScene, rows, table, pairs: int, kill_walks: int, eps: float, seed: int = 0,
                    cap_deg=PSD_CAP_DEG, r_max=None, bisect_iters=PSD_BISECT_ITERS, kappa=2.0 ** -20,
                    delta_rel=2.0 ** -21, max_steps=None, mesh: int = 0, log: bool = False, nthreads: int = 1):
    """The exterior estimate of Sec. 3.3 (eq. main-exterior-estimator) in the
    Kelvin-inverted exterior, over point rows with a dense per-vertex table.
    eps is the shell width in inverted-space units; the step guard is
    delta_rel times the inverted domain's bound. Returns the jump term
    ``S_jump`` and the killing term ``S_kill`` (K x K each) with their standard
    errors, the full operator ``S = S_jump + S_kill``, per-row radii and query
    counts."""
    if rows.mode != "point":
        raise ValueError("the exterior estimator takes point rows")
    if max_steps is None:
        max_steps = DEFAULT_MAX_STEPS["interior"]
    if r_max is None:
        r_max = ks.r_max()
    tab = _c(table, np.float64)
    K = tab.shape[1]
    n = rows.n_rows
    Sj, Qj, Sk, Qk = (np.zeros((K, K)) for _ in range(4))
    rad, Z = np.zeros(n), np.zeros(n)
    nq = np.zeros(n, dtype=np.int64)
    kq = np.zeros(1, dtype=np.int64)
    if log:
        ls = np.full((n, 2 * pairs), -1, dtype=np.int32)
        lt = np.full((n, 2 * pairs), -1, dtype=np.int64)
        lb = np.zeros((n, 2 * pairs, 2), dtype=np.float32)
    else:
        ls = lt = lb = None
    p, nn, tri, bary = (_c(rows.p, np.float32), _c(rows.n, np.float32), _c(rows.tri, np.int32),
                        _c(rows.bary, np.float32))
    w = _c(rows.w, np.float64)
    lib().orc_kelvin_estimate(ks.h, n, _ptr(p, C.c_float), _ptr(nn, C.c_float), _ptr(tri, C.c_int32),
                              _ptr(bary, C.c_float), _ptr(w, C.c_double), _ptr(tab, C.c_double), K, pairs,
                              kill_walks, np.deg2rad(cap_deg), r_max, bisect_iters, eps, kappa,
                              delta_rel * ks.radius, max_steps, C.c_uint64(seed), mesh, nthreads,
                              _ptr(Sj, C.c_double), _ptr(Qj, C.c_double), _ptr(Sk, C.c_double), _ptr(Qk, C.c_double),
                              _ptr(rad, C.c_double), _ptr(Z, C.c_double), _ptr(nq, C.c_int64), _ptr(kq, C.c_int64),
                              _ptr(ls, C.c_int32), _ptr(lt, C.c_int64), _ptr(lb, C.c_float))
    se_j = psd_standard_error(Sj, Qj, n * pairs)
    se_k = psd_standard_error(Sk, Qk, kill_walks) if kill_walks > 1 else np.zeros_like(Sk)
    out = dict(S_jump=Sj, se_jump=se_j, S_kill=Sk, se_kill=se_k, S=Sj + Sk, se=np.sqrt(se_j ** 2 + se_k ** 2),
               radius=rad, Z=Z, n_query=nq, kill_queries=int(kq[0]), pairs=pairs, kill_walks=kill_walks)
    if log:
        out.update(log_status=ls, log_tri=lt, log_bary=lb)
    return out


# ------------------------------------------------------- point basis (k-NN)


def knn_weights(points, normals, q, nq, k, sigma, tau):
    """Bilateral k-NN weights at query q with normal nq (Appendix, point-based
    k-NN interpolator): (indices of the k nearest points, ties by index, and
    their normalised weights)."""
    x, n = _c(points, np.float64), _c(normals, np.float64)
    qq, nn = _c(q, np.float64), _c(nq, np.float64)
    idx = np.zeros(k, dtype=np.int32)
    w = np.zeros(k)
    m = lib().orc_knn_weights(_ptr(x, C.c_double), _ptr(n, C.c_double), x.shape[0], k, sigma, tau,
                              _ptr(qq, C.c_double), _ptr(nn, C.c_double), _ptr(idx, C.c_int32), _ptr(w, C.c_double))
    return idx[:m], w[:m]
