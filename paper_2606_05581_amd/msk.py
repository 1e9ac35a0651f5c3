"""Python binding of libmsk (include/msk.h): argument marshalling only.

Every step of the estimator runs in the HIP library; this module turns numpy
arrays and torch tensors into the plain pointers and sizes of the C ABI. It
raises if the library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MSK_LIBRARY selects another build of the library (tuning experiments)
LIB_PATH = os.environ.get("MSK_LIBRARY", os.path.join(HERE, "libmsk.so"))

OK, ERR_INVALID_ARG, ERR_OOM, ERR_DEVICE, ERR_NOT_CONVERGED, ERR_NUMERIC = range(6)
ROWS_POINT, ROWS_HAT_RING = 0, 1
INTERIOR, EXTERIOR = 0, 1
FORM_PERSISTENT, FORM_PLAIN = 0, 1
(FIELD_S, FIELD_SE, FIELD_ROW_WALKS, FIELD_ROW_QUERIES, FIELD_ROW_ESCAPED, FIELD_ROW_CAPPED, FIELD_ROW_DISCARDED,
 FIELD_LOG_STATUS, FIELD_LOG_TRI, FIELD_LOG_BARY, FIELD_LOG_QUERIES) = range(11)

_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "DEVICE", 4: "NOT_CONVERGED", 5: "NUMERIC"}


class MskError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class MskNumericError(MskError):
    """A call that produced non-finite entries; `result` still holds its output."""

    def __init__(self, status, msg, result):
        super().__init__(status, msg)
        self.result = result


class BvhOpts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("top_nodes", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("centre", C.c_double * 3), ("radius", C.c_double), ("area", C.c_double), ("n_verts", C.c_int64),
                ("n_tris", C.c_int64), ("n_nodes", C.c_int64), ("node_bytes", C.c_int64), ("tri_bytes", C.c_int64),
                ("depth", C.c_int32), ("leaf_size", C.c_int32)]


class RowsDesc(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_rows", C.c_int64), ("w", C.c_void_p), ("p", C.c_void_p), ("n", C.c_void_p),
                ("tri", C.c_void_p), ("bary", C.c_void_p), ("ring_ptr", C.c_void_p), ("ring_tri", C.c_void_p),
                ("ring_cum", C.c_void_p), ("face_normals", C.c_void_p)]


class DtnOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("max_steps", C.c_int64), ("walk_offset", C.c_int64), ("kappa", C.c_double),
                ("delta_rel", C.c_double), ("form", C.c_int32), ("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("chunk", C.c_int32), ("regen_min", C.c_int32), ("record_log", C.c_int32), ("se_target", C.c_double),
                ("walks_max", C.c_int64), ("collect_stats", C.c_int32), ("mesh_id", C.c_int32),
                ("accum", C.c_int32), ("jump_only", C.c_int32)]


class DtnInfo(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("K", C.c_int64), ("walks_total", C.c_int64), ("queries_total", C.c_int64),
                ("escaped_total", C.c_int64), ("capped_total", C.c_int64), ("discarded_rows", C.c_int64),
                ("walk_kernel_ms", C.c_double), ("total_ms", C.c_double), ("walk_launches", C.c_int32),
                ("nodes_visited", C.c_int64), ("tris_tested", C.c_int64), ("valu_flops", C.c_int64),
                ("nonfinite_entries", C.c_int64)]


class EigStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("block", C.c_int32), ("max_residual", C.c_double),
                ("lanczos_ms", C.c_double), ("fp32_products", C.c_int64), ("fp32_product_ms", C.c_double),
                ("fp32_product_flops", C.c_double), ("fp64_products", C.c_int64), ("fp64_product_ms", C.c_double),
                ("fp64_product_flops", C.c_double)]


class TuneSpace(C.Structure):
    _fields_ = [("n_leaf", C.c_int32), ("leaf", C.c_int32 * 4), ("n_chunk", C.c_int32), ("chunk", C.c_int32 * 4),
                ("n_regen", C.c_int32), ("regen_min", C.c_int32 * 4), ("n_bpc", C.c_int32),
                ("blocks_per_cu", C.c_int32 * 4), ("trial_rows", C.c_int64), ("trial_walks", C.c_int64),
                ("repeats", C.c_int32), ("cache_path", C.c_char_p)]


class TuneResult(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("chunk", C.c_int32), ("regen_min", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("walks_per_s", C.c_double), ("trials", C.c_int32), ("from_cache", C.c_int32)]


class PsdOpts(C.Structure):
    _fields_ = [("cap_deg", C.c_double), ("bisect_iters", C.c_int32), ("r_max", C.c_double),
                ("chunk_pairs", C.c_int64)]


class PsdInfo(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("K", C.c_int64), ("pairs", C.c_int64), ("walks_total", C.c_int64),
                ("queries_total", C.c_int64), ("escaped_total", C.c_int64), ("capped_total", C.c_int64),
                ("dropped_rows", C.c_int64), ("mean_radius", C.c_double), ("r_max", C.c_double),
                ("tangent_ms", C.c_double), ("walk_kernel_ms", C.c_double), ("gather_ms", C.c_double),
                ("product_ms", C.c_double), ("total_ms", C.c_double), ("nonfinite_entries", C.c_int64),
                ("fused", C.c_int32), ("nodes_visited", C.c_int64), ("tris_tested", C.c_int64),
                ("valu_flops", C.c_int64)]


class PsdLog(C.Structure):
    _fields_ = [("status", C.c_void_p), ("tri", C.c_void_p), ("bary", C.c_void_p), ("queries", C.c_void_p)]


class KelvinInfo(C.Structure):
    _fields_ = [("centre", C.c_double * 3), ("radius", C.c_double), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3), ("r_max", C.c_double), ("n_tris", C.c_int64), ("n_nodes", C.c_int64),
                ("depth", C.c_int32), ("leaf_size", C.c_int32)]


class KelvinLog(C.Structure):
    _fields_ = [("status", C.c_void_p), ("tri", C.c_void_p), ("bary", C.c_void_p), ("queries", C.c_void_p)]


class KelvinEstInfo(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("K", C.c_int64), ("pairs", C.c_int64), ("kill_walks", C.c_int64),
                ("walks_total", C.c_int64), ("queries_total", C.c_int64), ("kill_queries", C.c_int64),
                ("dropped_rows", C.c_int64), ("capped_total", C.c_int64), ("mean_radius", C.c_double),
                ("r_max", C.c_double), ("tangent_ms", C.c_double), ("walk_kernel_ms", C.c_double),
                ("product_ms", C.c_double), ("nonfinite_entries", C.c_int64), ("nodes_visited", C.c_int64),
                ("elements_tested", C.c_int64), ("fp64_ops", C.c_int64)]


class LaplaceOpts(C.Structure):
    _fields_ = [("block", C.c_int32), ("degree", C.c_int32), ("max_iters", C.c_int32), ("max_degree", C.c_int32),
                ("tol", C.c_double), ("seed", C.c_uint64), ("no_locking", C.c_int32), ("reserved", C.c_int32)]


class LaplaceInfo(C.Structure):
    _fields_ = [("active_vertices", C.c_int64), ("skipped_faces", C.c_int64), ("nnz", C.c_int64),
                ("spmm_calls", C.c_int64), ("block", C.c_int32), ("degree", C.c_int32), ("iters", C.c_int32),
                ("converged", C.c_int32), ("grams", C.c_int32), ("rotates", C.c_int32), ("rank_drops", C.c_int32),
                ("locked", C.c_int32), ("bound", C.c_double), ("filter_lower", C.c_double),
                ("max_residual", C.c_double), ("setup_ms", C.c_double), ("assemble_ms", C.c_double),
                ("filter_ms", C.c_double), ("dense_ms", C.c_double), ("total_ms", C.c_double),
                ("filter_bytes", C.c_double)]


_lib = None

# symbol name -> (argtypes, restype); the C ABI declared in include/msk.h
SIGNATURES = {
    "msk_create": ([C.c_int, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "msk_destroy": ([C.c_void_p], None),
    "msk_last_error": ([C.c_void_p], C.c_char_p),
    "msk_build_bvh": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.POINTER(BvhOpts),
                       C.POINTER(C.c_void_p)], C.c_int),
    "msk_mesh_get_info": ([C.c_void_p, C.POINTER(MeshInfo)], C.c_int),
    "msk_mesh_destroy": ([C.c_void_p], None),
    "msk_closest_points": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
                           C.c_int),
    "msk_rows_create": ([C.c_void_p, C.c_void_p, C.POINTER(RowsDesc), C.POINTER(C.c_void_p)], C.c_int),
    "msk_rows_destroy": ([C.c_void_p], None),
    "msk_basis_create": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                          C.POINTER(C.c_void_p)], C.c_int),
    "msk_basis_destroy": ([C.c_void_p], None),
    "msk_basis_create_knn": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_double,
                              C.c_double, C.POINTER(C.c_void_p)], C.c_int),
    "msk_basis_eval_knn": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
                           C.c_int),
    "msk_dtn_opts_default": ([C.POINTER(DtnOpts)], None),
    "msk_eps_floor": ([C.c_double, C.POINTER(DtnOpts)], C.c_double),
    "msk_estimate_dtn": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_int32,
                          C.POINTER(DtnOpts), C.POINTER(C.c_void_p)], C.c_int),
    "msk_estimate_dtn_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                  C.c_int32, C.POINTER(DtnOpts), C.c_void_p, C.c_void_p, C.POINTER(DtnInfo)], C.c_int),
    "msk_estimate_dtn_batched": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64,
                                  C.c_int32, C.POINTER(DtnOpts), C.POINTER(C.c_void_p)], C.c_int),
    "msk_dtn_get_info": ([C.c_void_p, C.POINTER(DtnInfo)], C.c_int),
    "msk_dtn_get": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_int32], C.c_int),
    "msk_dtn_destroy": ([C.c_void_p], None),
    "msk_steklov_modes": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(EigStats)], C.c_int),
    "msk_batch_create": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                          C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64, C.c_int32, C.POINTER(DtnOpts),
                          C.POINTER(C.c_void_p)], C.c_int),
    "msk_batch_run": ([C.c_void_p], C.c_int),
    "msk_batch_dtn": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "msk_batch_get_info": ([C.c_void_p, C.POINTER(DtnInfo)], C.c_int),
    "msk_batch_destroy": ([C.c_void_p], None),
    "msk_tune_space_default": ([C.POINTER(TuneSpace)], None),
    "msk_mesh_rebuild": ([C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
    "msk_psd_opts_default": ([C.POINTER(PsdOpts)], None),
    "msk_laplace_opts_default": ([C.POINTER(LaplaceOpts)], None),
    "msk_spectral_heat": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "msk_basis_create_laplacian": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                    C.POINTER(LaplaceOpts), C.c_void_p, C.c_void_p, C.POINTER(LaplaceInfo),
                                    C.POINTER(C.c_void_p)], C.c_int),
    "msk_estimate_psd": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.POINTER(DtnOpts),
                          C.POINTER(PsdOpts), C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PsdLog),
                          C.POINTER(PsdInfo)], C.c_int),
    "msk_kelvin_create": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "msk_kelvin_get_info": ([C.c_void_p, C.POINTER(KelvinInfo)], C.c_int),
    "msk_kelvin_destroy": ([C.c_void_p], None),
    "msk_kelvin_closest_points": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p], C.c_int),
    "msk_estimate_kelvin": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_double,
                             C.POINTER(DtnOpts), C.POINTER(PsdOpts), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.POINTER(KelvinLog), C.POINTER(KelvinEstInfo)], C.c_int),
    "msk_autotune": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.POINTER(TuneSpace),
                      C.POINTER(TuneResult)], C.c_int),
}


def lib():
    """Load libmsk.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (paper_2606_05581_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _np(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, a.ctypes.data


def _dev_ptr(t, dtype):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous CUDA tensor of {dtype}")
    return t.data_ptr()


class Context:
    """A library context on one device, queuing work on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = C.c_void_p()
        st = lib().msk_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != OK:
            raise MskError(st, "msk_create failed")
        self.h = h

    def _check(self, st):
        if st != OK:
            raise MskError(st, lib().msk_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().msk_destroy(self.h)
            self.h = None

    # -- mesh
    def build_bvh(self, V, F, leaf_size: int = 4, top_nodes: int = 85) -> "Mesh":
        V, pv = _np(V, np.float32)
        F, pf = _np(F, np.int32)
        h = C.c_void_p()
        o = BvhOpts(leaf_size, top_nodes)
        self._check(lib().msk_build_bvh(self.h, pv, V.shape[0], pf, F.shape[0], C.byref(o), C.byref(h)))
        return Mesh(self, h)

    def closest_points(self, mesh: "Mesh", Q):
        """Q: CUDA float32 (n,3) world points -> (tri int32, d2 float32, bary (n,2) float32) CUDA tensors."""
        import torch

        n = Q.shape[0]
        tri = torch.empty(n, dtype=torch.int32, device=Q.device)
        d2 = torch.empty(n, dtype=torch.float32, device=Q.device)
        bary = torch.empty((n, 2), dtype=torch.float32, device=Q.device)
        self._check(lib().msk_closest_points(self.h, mesh.h, _dev_ptr(Q, torch.float32), n,
                                             tri.data_ptr(), d2.data_ptr(), bary.data_ptr()))
        return tri, d2, bary

    # -- rows / basis
    def rows(self, mesh: "Mesh", rows) -> "RowsHandle":
        keep = []

        def p(a, dt):
            if a is None:
                return None
            arr, ptr = _np(a, dt)
            keep.append(arr)
            return ptr

        mode = ROWS_POINT if rows.mode == "point" else ROWS_HAT_RING
        d = RowsDesc(mode, int(rows.w.shape[0]), p(rows.w, np.float64), p(rows.p, np.float32), p(rows.n, np.float32),
                     p(rows.tri, np.int32), p(rows.bary, np.float32), p(rows.ring_ptr, np.int32),
                     p(rows.ring_tri, np.int32), p(rows.ring_cum, np.float64), p(rows.fn, np.float32))
        h = C.c_void_p()
        self._check(lib().msk_rows_create(self.h, mesh.h, C.byref(d), C.byref(h)))
        return RowsHandle(self, h, int(rows.w.shape[0]))

    def basis(self, basis, n_verts: int) -> "BasisHandle":
        rp, prp = _np(basis.rowptr, np.int32)
        cl, pcl = _np(basis.col, np.int32)
        vl, pvl = _np(basis.val, np.float32)
        h = C.c_void_p()
        self._check(lib().msk_basis_create(self.h, prp, pcl, pvl, n_verts, int(basis.K), C.byref(h)))
        return BasisHandle(self, h, int(basis.K), int(n_verts))

    def basis_knn(self, mesh, points, normals, k: int = 8, sigma: float = 0.025, tau_n: float = 0.8) -> "BasisHandle":
        """Point basis: bilateral k-NN interpolation over the sample points (K = number of points)."""
        P, pp = _np(points, np.float32)
        Nn, pn = _np(normals, np.float32)
        h = C.c_void_p()
        self._check(lib().msk_basis_create_knn(self.h, mesh.h, pp, pn, int(P.shape[0]), int(k), float(sigma),
                                               float(tau_n), C.byref(h)))
        bh = BasisHandle(self, h, int(P.shape[0]))
        bh.k = int(k)
        return bh

    def basis_laplacian(self, V, F, K: int, want_phi: bool = True, **opts):
        """Mesh-based Galerkin basis: the K lowest modes of the cotangent
        Laplacian (Sec. 5.1), computed on the GPU. Returns (basis handle,
        eigenvalues (K,), Phi (nv, K) FP64 or None, info dict). Raises
        MskError(NOT_CONVERGED) with .result = that tuple when the residual
        target was not met (the handle must still be closed)."""
        Vv, pv = _np(V, np.float32)
        Ff, pf = _np(F, np.int32)
        o = LaplaceOpts()
        lib().msk_laplace_opts_default(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        nv = int(Vv.shape[0])
        ev = np.zeros(int(K))
        phi = np.zeros((nv, int(K))) if want_phi else None
        inf = LaplaceInfo()
        h = C.c_void_p()
        st = lib().msk_basis_create_laplacian(self.h, pv, nv, pf, int(Ff.shape[0]), int(K), C.byref(o),
                                              ev.ctypes.data, phi.ctypes.data if want_phi else None, C.byref(inf),
                                              C.byref(h))
        info = {f: getattr(inf, f) for f, _ in LaplaceInfo._fields_ if f != "reserved"}
        if st == ERR_NOT_CONVERGED and h.value:
            err = MskError(st, lib().msk_last_error(self.h).decode())
            err.result = (BasisHandle(self, h, int(K), nv), ev, phi, info)
            raise err
        self._check(st)
        return BasisHandle(self, h, int(K), nv), ev, phi, info

    def spectral_heat(self, basis, evals, coeffs, times, mass=None, u0=None, hks: bool = True):
        """Steklov heat and heat kernel signatures on the vertices from eigenpairs
        in a table basis (eqs. steklovHeat and spectralSteklovHeat): returns
        (hks (nv, T) or None, heat (nv, T) or None); heat needs mass and u0."""
        ev, pe = _np(evals, np.float64)
        Cc, pc = _np(coeffs, np.float64)
        tt, pt = _np(times, np.float64)
        n_modes, T = int(ev.shape[0]), int(tt.shape[0])
        nv = int(basis.nv)
        out_h = np.zeros((nv, T)) if hks else None
        out_u = None
        pm = pu = None
        if u0 is not None:
            mm, pm = _np(mass, np.float64)
            uu, pu = _np(u0, np.float64)
            out_u = np.zeros((nv, T))
        self._check(lib().msk_spectral_heat(self.h, basis.h, n_modes, pe, pc, pt, T, pm, pu,
                                            out_h.ctypes.data if hks else None,
                                            out_u.ctypes.data if out_u is not None else None))
        return out_h, out_u

    def eval_knn(self, basis, Q, Nq):
        """The point basis at queries (torch tensors on the GPU, n x 3 float32): (indices, weights), n x k."""
        import torch

        n = int(Q.shape[0])
        idx = torch.empty((n, basis.k), dtype=torch.int32, device=Q.device)
        w = torch.empty((n, basis.k), dtype=torch.float32, device=Q.device)
        self._check(lib().msk_basis_eval_knn(self.h, basis.h, Q.data_ptr(), Nq.data_ptr(), n, idx.data_ptr(),
                                             w.data_ptr()))
        return idx, w

    # -- estimate
    @staticmethod
    def default_opts(**kw) -> DtnOpts:
        o = DtnOpts()
        lib().msk_dtn_opts_default(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def estimate_dtn(self, mesh, rows, basis, walks: int, eps: float, inset_h: float, exterior: bool = False,
                     **opts) -> "Dtn":
        o = self.default_opts(**opts)
        h = C.c_void_p()
        st = lib().msk_estimate_dtn(self.h, mesh.h, rows.h, basis.h, walks, eps, inset_h,
                                    EXTERIOR if exterior else INTERIOR, C.byref(o), C.byref(h))
        if st == ERR_NUMERIC and h.value:
            raise MskNumericError(st, lib().msk_last_error(self.h).decode(), Dtn(self, h, rows.n, basis.K, walks))
        self._check(st)
        return Dtn(self, h, rows.n, basis.K, walks)

    def estimate_dtn_noalloc(self, mesh, rows, basis, walks: int, eps: float, inset_h: float, S, se,
                             exterior: bool = False, **opts) -> dict:
        """msk_estimate_dtn into caller-provided device arrays S and se (torch
        CUDA float64 tensors, n_rows x K, contiguous) with no device
        allocation; returns the counters."""
        for t in (S, se):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()
                    and tuple(t.shape) == (rows.n, basis.K)):
                raise ValueError("S and se must be contiguous float64 CUDA tensors of shape (n_rows, K)")
        o = self.default_opts(**opts)
        info = DtnInfo()
        st = lib().msk_estimate_dtn_noalloc(self.h, mesh.h, rows.h, basis.h, walks, eps, inset_h,
                                            EXTERIOR if exterior else INTERIOR, C.byref(o), C.c_void_p(S.data_ptr()),
                                            C.c_void_p(se.data_ptr()), C.byref(info))
        self._check(st)
        return {f: getattr(info, f) for f, _ in DtnInfo._fields_}

    def estimate_dtn_batched(self, meshes, rows, bases, eps, insets, walks: int, exterior: bool = False, **opts):
        n = len(meshes)
        o = self.default_opts(**opts)
        arr = lambda xs: (C.c_void_p * n)(*[x.h for x in xs])
        outs = (C.c_void_p * n)()
        e = (C.c_double * n)(*eps)
        hh = (C.c_double * n)(*insets)
        st = lib().msk_estimate_dtn_batched(self.h, n, arr(meshes), arr(rows), arr(bases), e, hh, walks,
                                            EXTERIOR if exterior else INTERIOR, C.byref(o), outs)
        if st == ERR_NUMERIC:
            res = [Dtn(self, C.c_void_p(outs[i]), rows[i].n, bases[i].K, walks) for i in range(n)]
            raise MskNumericError(st, lib().msk_last_error(self.h).decode(), res)
        self._check(st)
        return [Dtn(self, C.c_void_p(outs[i]), rows[i].n, bases[i].K, walks) for i in range(n)]

    def batch(self, meshes, rows, bases, eps, insets, walks: int, exterior: bool = False, **opts) -> "Batch":
        """A reusable batch plan (one captured graph over all meshes)."""
        n = len(meshes)
        o = self.default_opts(**opts)
        arr = lambda xs: (C.c_void_p * n)(*[x.h for x in xs])
        h = C.c_void_p()
        self._check(lib().msk_batch_create(self.h, n, arr(meshes), arr(rows), arr(bases), (C.c_double * n)(*eps),
                                           (C.c_double * n)(*insets), walks, EXTERIOR if exterior else INTERIOR,
                                           C.byref(o), C.byref(h)))
        return Batch(self, h, [r.n for r in rows], [b.K for b in bases], walks)

    def autotune(self, meshes, rows, bases, eps, insets, exterior: bool = False, cache_path=None, **space) -> dict:
        """Tune leaf width / chunk / refill threshold / workgroups per CU; meshes are rebuilt in place."""
        n = len(meshes)
        sp = TuneSpace()
        lib().msk_tune_space_default(C.byref(sp))
        for k, v in space.items():
            if k in ("leaf", "chunk", "regen_min", "blocks_per_cu"):
                cnt = {"leaf": "n_leaf", "chunk": "n_chunk", "regen_min": "n_regen", "blocks_per_cu": "n_bpc"}[k]
                setattr(sp, cnt, len(v))
                arr = getattr(sp, k)
                for i, x in enumerate(v):
                    arr[i] = x
            else:
                setattr(sp, k, v)
        keep = cache_path.encode() if cache_path else None
        sp.cache_path = keep
        res = TuneResult()
        arr = lambda xs: (C.c_void_p * n)(*[x.h for x in xs])
        self._check(lib().msk_autotune(self.h, n, arr(meshes), arr(rows), arr(bases), (C.c_double * n)(*eps),
                                       (C.c_double * n)(*insets), EXTERIOR if exterior else INTERIOR, C.byref(sp),
                                       C.byref(res)))
        return {f: getattr(res, f) for f, _ in TuneResult._fields_}

    # -- exterior in the Kelvin-inverted domain
    def kelvin(self, mesh, centre, leaf_size: int = 0) -> "Kelvin":
        """The mesh seen through the Kelvin transform about `centre` (world, inside the shape)."""
        c = (C.c_double * 3)(*[float(x) for x in centre])
        h = C.c_void_p()
        self._check(lib().msk_kelvin_create(self.h, mesh.h, c, leaf_size, C.byref(h)))
        return Kelvin(self, h)

    def kelvin_closest_points(self, kv, Q):
        """Nearest inverted elements of Q (torch float64 CUDA tensor, n x 3, inverted space):
        (tri, d2, nearest point, barycentrics of its image) as CUDA tensors."""
        import torch

        Q = Q.contiguous()
        n = Q.shape[0]
        tri = torch.empty(n, dtype=torch.int32, device=Q.device)
        d2 = torch.empty(n, dtype=torch.float64, device=Q.device)
        qp = torch.empty((n, 3), dtype=torch.float64, device=Q.device)
        bary = torch.empty((n, 3), dtype=torch.float64, device=Q.device)
        self._check(lib().msk_kelvin_closest_points(self.h, kv.h, Q.data_ptr(), n, tri.data_ptr(), d2.data_ptr(),
                                                    qp.data_ptr(), bary.data_ptr()))
        return tri, d2, qp, bary

    def estimate_kelvin(self, kv, rows, basis, pairs: int, kill_walks: int, eps: float, cap_deg: float = 2.5,
                        bisect_iters: int = 10, r_max: float = 0.0, chunk_pairs: int = 262144, log: bool = False,
                        **walk_opts) -> dict:
        """The exterior estimate in the Kelvin-inverted domain: jump and killing terms (K x K)
        with standard errors, inverted tangent radii, info and optionally the walk log."""
        o = self.default_opts(**walk_opts)
        po = PsdOpts()
        lib().msk_psd_opts_default(C.byref(po))
        po.cap_deg, po.bisect_iters, po.r_max, po.chunk_pairs = cap_deg, bisect_iters, r_max, chunk_pairs
        K, n = int(basis.K), int(rows.n)
        nw = n * 2 * int(pairs) + int(kill_walks)
        Sj, sej, Sk, sek = (np.zeros((K, K)) for _ in range(4))
        rad = np.zeros(n)
        info = KelvinEstInfo()
        lg = None
        out = {}
        if log:
            out = dict(status=np.zeros(nw, dtype=np.int32), tri=np.zeros(nw, dtype=np.int32),
                       bary=np.zeros((nw, 2), dtype=np.float32), nq=np.zeros(nw, dtype=np.int32))
            lg = KelvinLog(out["status"].ctypes.data, out["tri"].ctypes.data, out["bary"].ctypes.data,
                           out["nq"].ctypes.data)
        st = lib().msk_estimate_kelvin(self.h, kv.h, rows.h, basis.h, pairs, kill_walks, eps, C.byref(o),
                                       C.byref(po), Sj.ctypes.data, sej.ctypes.data,
                                       Sk.ctypes.data if kill_walks > 0 else None,
                                       sek.ctypes.data if kill_walks > 0 else None, rad.ctypes.data,
                                       C.byref(lg) if lg is not None else None, C.byref(info))
        self._check(st)
        res = dict(S_jump=Sj, se_jump=sej, S_kill=Sk, se_kill=sek, S=Sj + Sk, se=np.sqrt(sej ** 2 + sek ** 2),
                   radius=rad, info={f: getattr(info, f) for f, _ in KelvinEstInfo._fields_}, **out)
        return res

    def estimate_psd(self, mesh, rows, basis, pairs: int, eps: float, cap_deg: float = 2.5, bisect_iters: int = 10,
                     r_max: float = 0.0, chunk_pairs: int = 262144, log: bool = False, **walk_opts) -> dict:
        """The PSD estimator (Alg. 2) over point rows: S, se (K x K), tangent radii, info and optionally the walk log."""
        o = self.default_opts(**walk_opts)
        po = PsdOpts()
        lib().msk_psd_opts_default(C.byref(po))
        po.cap_deg, po.bisect_iters, po.r_max, po.chunk_pairs = cap_deg, bisect_iters, r_max, chunk_pairs
        K, n, W = int(basis.K), int(rows.n), 2 * int(pairs)
        S = np.zeros((K, K))
        se = np.zeros((K, K))
        rad = np.zeros(n, dtype=np.float32)
        info = PsdInfo()
        lg = None
        out = {}
        if log:
            out = dict(status=np.zeros((n, W), dtype=np.int32), tri=np.zeros((n, W), dtype=np.int32),
                       bary=np.zeros((n, W, 2), dtype=np.float32), nq=np.zeros((n, W), dtype=np.int32))
            lg = PsdLog(out["status"].ctypes.data, out["tri"].ctypes.data, out["bary"].ctypes.data,
                        out["nq"].ctypes.data)
        st = lib().msk_estimate_psd(self.h, mesh.h, rows.h, basis.h, int(pairs), eps, C.byref(o), C.byref(po),
                                    S.ctypes.data, se.ctypes.data, rad.ctypes.data,
                                    C.byref(lg) if lg is not None else None, C.byref(info))
        res = dict(S=S, se=se, radius=rad, info={f: getattr(info, f) for f, _ in PsdInfo._fields_}, **out)
        if st == ERR_NUMERIC:
            raise MskNumericError(st, lib().msk_last_error(self.h).decode(), res)
        self._check(st)
        return res

    def steklov_modes(self, dtn: "Dtn", k: int, vectors: bool = True):
        evals = np.zeros(k)
        evecs = np.zeros((dtn.n, k)) if vectors else None
        stats = EigStats()
        st = lib().msk_steklov_modes(self.h, dtn.h, k, evals.ctypes.data,
                                     evecs.ctypes.data if vectors else None, C.byref(stats))
        if st not in (OK, ERR_NOT_CONVERGED):
            self._check(st)
        return evals, evecs, dict(converged=st == OK, **{f: getattr(stats, f) for f, _ in EigStats._fields_})


class _Handle:
    _destroy = None

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def close(self):
        if getattr(self, "h", None):
            getattr(lib(), self._destroy)(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh(_Handle):
    _destroy = "msk_mesh_destroy"

    def rebuild(self, leaf_size: int):
        """Rebuild the BVH in place with another leaf width (walks do not change)."""
        self.ctx._check(lib().msk_mesh_rebuild(self.ctx.h, self.h, leaf_size))

    def info(self) -> dict:
        i = MeshInfo()
        self.ctx._check(lib().msk_mesh_get_info(self.h, C.byref(i)))
        return {f: (list(getattr(i, f)) if f == "centre" else getattr(i, f)) for f, _ in MeshInfo._fields_}


class Kelvin(_Handle):
    _destroy = "msk_kelvin_destroy"

    def info(self) -> dict:
        i = KelvinInfo()
        self.ctx._check(lib().msk_kelvin_get_info(self.h, C.byref(i)))
        return {f: (list(getattr(i, f)) if f in ("centre", "box_lo", "box_hi") else getattr(i, f))
                for f, _ in KelvinInfo._fields_}


class RowsHandle(_Handle):
    _destroy = "msk_rows_destroy"

    def __init__(self, ctx, h, n):
        super().__init__(ctx, h)
        self.n = n


class BasisHandle(_Handle):
    _destroy = "msk_basis_destroy"

    def __init__(self, ctx, h, K, nv=None):
        super().__init__(ctx, h)
        self.K = K
        self.nv = nv


_FIELD_SHAPE = {
    FIELD_S: ("nk", np.float64), FIELD_SE: ("nk", np.float64), FIELD_ROW_WALKS: ("n", np.int64),
    FIELD_ROW_QUERIES: ("n", np.int64), FIELD_ROW_ESCAPED: ("n", np.int64), FIELD_ROW_CAPPED: ("n", np.int64),
    FIELD_ROW_DISCARDED: ("n", np.int32), FIELD_LOG_STATUS: ("nw", np.int32), FIELD_LOG_TRI: ("nw", np.int32),
    FIELD_LOG_BARY: ("nw2", np.float32), FIELD_LOG_QUERIES: ("nw", np.int32),
}


class Dtn(_Handle):
    _destroy = "msk_dtn_destroy"

    def __init__(self, ctx, h, n, K, W):
        super().__init__(ctx, h)
        self.n, self.K, self.W = n, K, W

    def info(self) -> dict:
        i = DtnInfo()
        self.ctx._check(lib().msk_dtn_get_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in DtnInfo._fields_}

    def get(self, field: int, device: bool = False):
        kind, dt = _FIELD_SHAPE[field]
        shape = {"nk": (self.n, self.K), "n": (self.n,), "nw": (self.n, self.W), "nw2": (self.n, self.W, 2)}[kind]
        if device:
            import torch

            tdt = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32,
                   np.float32: torch.float32}[dt]
            out = torch.empty(shape, dtype=tdt, device=f"cuda:{self.ctx.device}")
            self.ctx._check(lib().msk_dtn_get(self.h, field, out.data_ptr(), 1))
            return out
        out = np.empty(shape, dtype=dt)
        self.ctx._check(lib().msk_dtn_get(self.h, field, out.ctypes.data, 0))
        return out


class _DtnView(Dtn):
    """A result owned by a batch (not destroyed on its own)."""

    def close(self):
        self.h = None


class Batch(_Handle):
    _destroy = "msk_batch_destroy"

    def __init__(self, ctx, h, ns, Ks, W):
        super().__init__(ctx, h)
        self.ns, self.Ks, self.W = ns, Ks, W

    def run(self) -> dict:
        self.ctx._check(lib().msk_batch_run(self.h))
        return self.info()

    def info(self) -> dict:
        i = DtnInfo()
        self.ctx._check(lib().msk_batch_get_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in DtnInfo._fields_}

    def dtn(self, i: int) -> Dtn:
        h = C.c_void_p()
        self.ctx._check(lib().msk_batch_dtn(self.h, i, C.byref(h)))
        return _DtnView(self.ctx, h, self.ns[i], self.Ks[i], self.W)
