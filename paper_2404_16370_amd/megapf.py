"""ctypes binding of libmegapf (include/megapf.h): argument marshalling only.

Every computation happens in the library's HIP kernels.  Arrays may be numpy
arrays (host memory) or torch tensors (host or device memory: their data
pointers are passed through unchanged); streams are taken from torch's
current stream when torch has a GPU.  If the shared library is missing the
import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmegapf.so")

MP_OK, MP_E_ARG, MP_E_STATE, MP_E_OOM, MP_E_HIP, MP_E_UNSUPPORTED, MP_E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
MP_NNF_AUTO, MP_NNF_HASH, MP_NNF_DENSE = 0, 1, 2
MP_INIT_UNIFORM_BOX, MP_INIT_EXPLICIT, MP_INIT_GAUSSIAN = 0, 1, 2
(MP_STAGE_PREDICT, MP_STAGE_LSH, MP_STAGE_SORT, MP_STAGE_REFRESH, MP_STAGE_LIK, MP_STAGE_SVGD,
 MP_STAGE_POSTERIOR, MP_STAGE_SCAN, MP_STAGE_LIK_CORE) = range(9)
MP_NUM_STAGES = 9
STAGE_NAMES = ["predict", "lsh", "sort", "refresh", "likelihood", "svgd", "posterior", "scan", "likelihood_core"]


class MegaPFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("status %d: %s" % (status, msg))
        self.status = status


class mp_map_params(C.Structure):
    _fields_ = [("voxel", C.c_float), ("nnf_radius", C.c_int32), ("min_points", C.c_int32),
                ("cov_eps", C.c_float), ("backend", C.c_int32), ("gauss_mode", C.c_int32), ("point_k", C.c_int32),
                ("point_search", C.c_int32)]


class mp_map_info(C.Structure):
    _fields_ = [("num_gauss", C.c_int64), ("num_band", C.c_int64), ("grid_origin", C.c_int32 * 3),
                ("grid_dim", C.c_int32 * 3), ("box_min", C.c_float * 3), ("box_max", C.c_float * 3),
                ("backend", C.c_int32), ("table_slots", C.c_int64), ("device_bytes", C.c_int64)]


class mp_filter_params(C.Structure):
    _fields_ = [("n_particles", C.c_int32), ("k", C.c_int32), ("lsh_bits", C.c_int32), ("svgd_iters", C.c_int32),
                ("post_iters", C.c_int32), ("window_c", C.c_int32), ("scan_k", C.c_int32),
                ("sigma_r", C.c_float), ("sigma_t", C.c_float), ("lsh_alpha", C.c_float),
                ("lsh_sigma", C.c_float), ("c_max", C.c_float), ("d_max", C.c_float),
                ("lambda_rel", C.c_float), ("lambda_abs", C.c_float), ("temperature", C.c_float),
                ("prior_floor", C.c_float), ("cov_eps", C.c_float), ("lik_chunks", C.c_int32),
                ("lik_batch", C.c_int32), ("lik_layout", C.c_int32), ("scorer", C.c_int32), ("sigma_s", C.c_float),
                ("lsh_tangent", C.c_int32), ("lsh_tables", C.c_int32), ("svgd_grad", C.c_int32),
                ("svgd_transport", C.c_int32), ("final_rescore", C.c_int32), ("seed", C.c_uint64)]


class mp_odometry_params(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("d_max", C.c_float), ("lambda_rel", C.c_float),
                ("lambda_abs", C.c_float), ("cov_scale", C.c_float)]


class mp_odometry_result(C.Structure):
    _fields_ = [("H", C.c_double * 21), ("b", C.c_double * 6), ("cost", C.c_double), ("inliers", C.c_int32),
                ("iterations", C.c_int32), ("cov_ok", C.c_int32), ("dT64", C.c_double * 7)]


class mp_smoother_params(C.Structure):
    _fields_ = [("window", C.c_int32), ("jump_m", C.c_float), ("jump_rad", C.c_float), ("switch_frames", C.c_int32)]


class mp_batch_info(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("captures", C.c_int32), ("evals_per_step", C.c_int64),
                ("queued_instances", C.c_int32), ("queue_batch", C.c_int32), ("queue_workgroups", C.c_int32),
                ("pad", C.c_int32), ("queue_tiles_per_step", C.c_int64)]


class mp_surrogate_params(C.Structure):
    _fields_ = [("box_min", C.c_float * 3), ("box_max", C.c_float * 3), ("f_max", C.c_float),
                ("sigma_s", C.c_float), ("d_max", C.c_float), ("c_max", C.c_float), ("lr", C.c_float),
                ("lr_min", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float),
                ("total_steps", C.c_int32), ("batch", C.c_int32), ("seed", C.c_uint64)]


class mp_surrogate_info(C.Structure):
    _fields_ = [("n_params", C.c_int64), ("n_data", C.c_int64), ("steps", C.c_int64), ("lo", C.c_float * 3),
                ("inv_ext", C.c_float * 3), ("freqs", C.c_float * 32), ("r_scale", C.c_float),
                ("g_scale", C.c_float), ("weight_bytes", C.c_int32)]


class mp_init_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("box_min", C.c_float * 3), ("box_max", C.c_float * 3),
                ("poses", C.c_void_p), ("mean", C.c_float * 7), ("cov", C.c_float * 36)]


class mp_posterior(C.Structure):
    _fields_ = [("map_pose", C.c_float * 7), ("map_index", C.c_int32), ("map_weight", C.c_double),
                ("n_eff", C.c_double), ("log_evidence", C.c_double), ("max_loglik", C.c_double),
                ("frame", C.c_int32), ("fp64_resolves", C.c_int32), ("fallback_steps", C.c_int32),
                ("sur_checks", C.c_int32), ("sur_check_ds", C.c_float)]


EXPORTS = ["mp_map_default_params", "mp_map_build", "mp_map_get_info", "mp_map_get_gauss", "mp_map_lookup",
           "mp_map_destroy", "mp_filter_default_params", "mp_filter_init", "mp_filter_destroy", "mp_scan_upload",
           "mp_filter_step", "mp_posterior_query", "mp_last_error", "mp_stage_times", "mp_debug_get",
           "mp_debug_set", "mp_debug_stage", "mp_debug_map_point_knn", "mp_debug_sort_u32", "mp_surrogate_default_params", "mp_surrogate_create",
           "mp_surrogate_destroy", "mp_surrogate_get_info", "mp_surrogate_label", "mp_surrogate_eval",
           "mp_surrogate_set_data", "mp_surrogate_train", "mp_surrogate_grad", "mp_surrogate_get_params",
           "mp_surrogate_set_params", "mp_filter_set_surrogate", "mp_filter_set_surrogate_check", "mp_odometry_default_params", "mp_odometry", "mp_odometry_noalloc", "mp_smoother_default_params",
           "mp_smoother_create", "mp_smoother_push", "mp_smoother_destroy", "mp_batch_create", "mp_batch_step",
           "mp_batch_get_info", "mp_batch_destroy"]

MP_SCORER_PLAIN, MP_SCORER_SCOREFIELD, MP_SCORER_SURROGATE = 0, 1, 2
MP_LIK_LAYOUT_AUTO, MP_LIK_LAYOUT_PARTICLE, MP_LIK_LAYOUT_GROUPED = 0, 1, 2
MP_GAUSS_VOXEL, MP_GAUSS_POINT = 0, 1
MP_DEBUG_RESCORE = 100
MP_LSH_TANGENT_DECOUPLED, MP_LSH_TANGENT_SE3 = 0, 1
MP_SVGD_GRAD_APPROX, MP_SVGD_GRAD_EXACT = 0, 1
MP_SVGD_TRANSPORT_NONE, MP_SVGD_TRANSPORT_ADJOINT = 0, 1
MP_SUR_NPARAMS = 41732

_lib = None


def lib():
    """Load libmegapf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmegapf.so is not built: run `python -m paper_2404_16370_amd.build`")
    # torch bundles its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that one instance instead of a second
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.mp_map_default_params.argtypes = [C.POINTER(mp_map_params)]
    L.mp_map_default_params.restype = None
    L.mp_map_build.argtypes = [vp, i64, C.POINTER(mp_map_params), vp, C.POINTER(vp)]
    L.mp_map_get_info.argtypes = [vp, C.POINTER(mp_map_info)]
    L.mp_map_get_gauss.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mp_map_lookup.argtypes = [vp, vp, i64, vp, vp]
    L.mp_map_destroy.argtypes = [vp]
    L.mp_filter_default_params.argtypes = [C.POINTER(mp_filter_params)]
    L.mp_filter_default_params.restype = None
    L.mp_filter_init.argtypes = [vp, C.POINTER(mp_filter_params), C.POINTER(mp_init_desc), vp, C.POINTER(vp)]
    L.mp_filter_destroy.argtypes = [vp]
    L.mp_scan_upload.argtypes = [vp, vp, vp, i32, vp]
    L.mp_filter_step.argtypes = [vp, vp, vp, vp]
    L.mp_posterior_query.argtypes = [vp, C.POINTER(mp_posterior), vp, vp, vp]
    L.mp_last_error.argtypes = []
    L.mp_last_error.restype = C.c_char_p
    L.mp_stage_times.argtypes = [vp, vp, vp]
    L.mp_debug_get.argtypes = [vp, C.c_char_p, vp, i64, vp]
    L.mp_debug_set.argtypes = [vp, C.c_char_p, vp, i64, vp]
    L.mp_debug_stage.argtypes = [vp, i32, i32, vp, vp, vp]
    L.mp_debug_map_point_knn.argtypes = [vp, i64, C.POINTER(mp_map_params), vp, vp]
    L.mp_debug_sort_u32.argtypes = [vp, i64, i32, vp, vp, vp]
    L.mp_surrogate_default_params.argtypes = [C.POINTER(mp_surrogate_params)]
    L.mp_surrogate_default_params.restype = None
    L.mp_surrogate_create.argtypes = [vp, C.POINTER(mp_surrogate_params), vp, C.POINTER(vp)]
    L.mp_surrogate_destroy.argtypes = [vp]
    L.mp_surrogate_get_info.argtypes = [vp, C.POINTER(mp_surrogate_info)]
    L.mp_surrogate_label.argtypes = [vp, vp, i64, vp, vp]
    L.mp_surrogate_eval.argtypes = [vp, vp, i64, vp, vp]
    L.mp_surrogate_set_data.argtypes = [vp, vp, i64, vp]
    L.mp_surrogate_train.argtypes = [vp, i32, vp, vp]
    L.mp_surrogate_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.mp_surrogate_get_params.argtypes = [vp, vp, vp]
    L.mp_surrogate_set_params.argtypes = [vp, vp, vp]
    L.mp_filter_set_surrogate.argtypes = [vp, vp]
    L.mp_filter_set_surrogate_check.argtypes = [vp, i32, i32, C.c_float, i32]
    L.mp_odometry_default_params.argtypes = [C.POINTER(mp_odometry_params)]
    L.mp_odometry_default_params.restype = None
    L.mp_odometry.argtypes = [vp, C.POINTER(mp_odometry_params), vp, vp, vp, C.POINTER(mp_odometry_result), vp]
    L.mp_odometry_noalloc.argtypes = L.mp_odometry.argtypes
    L.mp_smoother_default_params.argtypes = [C.POINTER(mp_smoother_params)]
    L.mp_smoother_default_params.restype = None
    L.mp_smoother_create.argtypes = [C.POINTER(mp_smoother_params), C.POINTER(vp)]
    L.mp_smoother_push.argtypes = [vp, vp, vp, vp]
    L.mp_smoother_destroy.argtypes = [vp]
    L.mp_batch_create.argtypes = [vp, i32, i32, vp, C.POINTER(vp)]
    L.mp_batch_step.argtypes = [vp, vp, vp, vp]
    L.mp_batch_get_info.argtypes = [vp, C.POINTER(mp_batch_info), vp, vp]
    L.mp_batch_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("mp_map_default_params", "mp_filter_default_params", "mp_last_error",
                        "mp_surrogate_default_params"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def _check(status):
    if status != MP_OK:
        raise MegaPFError(status, lib().mp_last_error().decode())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(0)


def _ptr(a, dtype=None, keep=None):
    """Data pointer of a numpy array or torch tensor (contiguous); None -> NULL."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):  # torch tensor
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr())
    arr = np.ascontiguousarray(a, dtype=dtype)
    if keep is not None:
        keep.append(arr)
    return C.c_void_p(arr.ctypes.data)


def _nrows(a):
    return int(a.shape[0]) if hasattr(a, "shape") else len(a)


# ------------------------------------------------------------------ map
def mp_map_default_params():
    p = mp_map_params()
    lib().mp_map_default_params(C.byref(p))
    return p


class Map:
    """Owner of an mp_map handle (mp_map_build / mp_map_destroy)."""

    def __init__(self, xyz, voxel=0.5, nnf_radius=2, min_points=5, cov_eps=1e-3, backend=MP_NNF_AUTO, stream=None,
                 gauss_mode=None, point_k=10, point_search=2):
        p = mp_map_default_params()
        p.voxel, p.nnf_radius, p.min_points, p.cov_eps, p.backend = voxel, nnf_radius, min_points, cov_eps, backend
        if gauss_mode is not None:
            p.gauss_mode = gauss_mode
        p.point_k, p.point_search = point_k, point_search
        keep = []
        h = C.c_void_p()
        n = _nrows(xyz)
        _check(lib().mp_map_build(_ptr(xyz, np.float32, keep), n, C.byref(p), _stream(stream), C.byref(h)))
        self.handle = h
        self.params = p

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().mp_map_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().mp_map_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def info(self):
        i = mp_map_info()
        _check(lib().mp_map_get_info(self.handle, C.byref(i)))
        return dict(num_gauss=i.num_gauss, num_band=i.num_band, grid_origin=list(i.grid_origin),
                    grid_dim=list(i.grid_dim), box_min=list(i.box_min), box_max=list(i.box_max),
                    backend=i.backend, table_slots=i.table_slots, device_bytes=i.device_bytes)

    def gauss(self, stream=None):
        G = self.info()["num_gauss"]
        mu = np.zeros((G, 3), np.float32); nrm = np.zeros((G, 3), np.float32)
        vox = np.zeros((G, 3), np.int32); cnt = np.zeros(G, np.int32)
        if G:
            _check(lib().mp_map_get_gauss(self.handle, _ptr(mu), _ptr(nrm), _ptr(vox), _ptr(cnt), _stream(stream)))
        return dict(mu=mu, normal=nrm, vox=vox, count=cnt)

    def lookup(self, xyz, out=None, stream=None):
        n = _nrows(xyz)
        keep = []
        res = np.zeros(n, np.int32) if out is None else out
        if n:
            _check(lib().mp_map_lookup(self.handle, _ptr(xyz, np.float32, keep), n, _ptr(res), _stream(stream)))
        return res


def debug_map_point_knn(xyz, voxel, point_k=10, point_search=2, nnf_radius=2, min_points=5, cov_eps=1e-3,
                        stream=None):
    """Neighbour lists of a per-point map build (mp_debug_map_point_knn):
    n x point_k int32, ranked as the build ranks them, -1 pads."""
    p = mp_map_default_params()
    p.voxel, p.nnf_radius, p.min_points, p.cov_eps = voxel, nnf_radius, min_points, cov_eps
    p.gauss_mode, p.point_k, p.point_search = MP_GAUSS_POINT, point_k, point_search
    n = _nrows(xyz)
    keep = []
    out = np.zeros((n, point_k), np.int32)
    _check(lib().mp_debug_map_point_knn(_ptr(xyz, np.float32, keep), n, C.byref(p), _ptr(out), _stream(stream)))
    return out


def debug_sort_u32(keys, bits, stream=None):
    """Stable sort of uint32 keys by their low `bits` bits with the library's
    bucket sort (mp_debug_sort_u32): (sorted keys, input index of each)."""
    keep = []
    n = _nrows(keys)
    ko = np.zeros(n, np.uint32)
    order = np.zeros(n, np.int32)
    _check(lib().mp_debug_sort_u32(_ptr(keys, np.uint32, keep), n, bits, _ptr(ko), _ptr(order), _stream(stream)))
    return ko, order


# ------------------------------------------------------------------ filter
def mp_filter_default_params(**kw):
    p = mp_filter_params()
    lib().mp_filter_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


_DEBUG_LAYOUT = {  # name -> (dtype, shape as a function of (n, K, scan_n))
    "poses": (np.float32, lambda n, K, s: (n, 8)),
    "psi": (np.float32, lambda n, K, s: (n, 8)),
    "hb": (np.float32, lambda n, K, s: (n, 28)),
    "solve": (np.int32, lambda n, K, s: (n,)),
    "codes": (np.uint32, lambda n, K, s: (n,)),
    "sorted": (np.int32, lambda n, K, s: (n,)),
    "scodes": (np.uint32, lambda n, K, s: (n,)),
    "head": (np.int32, lambda n, K, s: (n,)),
    "end": (np.int32, lambda n, K, s: (n,)),
    "nbr": (np.int32, lambda n, K, s: (K, n)),
    "kval": (np.float32, lambda n, K, s: (K, n)),
    "cnt": (np.int32, lambda n, K, s: (n,)),
    "prior": (np.float32, lambda n, K, s: (n,)),
    "post": (np.float32, lambda n, K, s: (n,)),
    "post0": (np.float32, lambda n, K, s: (n,)),
    "scan": (np.float32, lambda n, K, s: (s, 12)),
    "scan_walk": (np.float32, lambda n, K, s: (s, 12)),
    "odo_nn": (np.int32, lambda n, K, s: (s,)),
    "tlsh": (np.float32, lambda n, K, s: (8,)),
    "sort_wait": (np.uint32, lambda n, K, s: (1,)),
}


class Filter:
    """Owner of an mp_filter handle."""

    def __init__(self, map_: Map, params=None, poses=None, box=None, stream=None, gaussian=None, **kw):
        """poses: explicit N x 7; gaussian: (mean pose 7, covariance 6 x 6); else uniform over `box`
        (default: the map's box)"""
        self.map = map_
        self.params = params if params is not None else mp_filter_default_params(**kw)
        init = mp_init_desc()
        keep = []
        if gaussian is not None:
            init.kind = MP_INIT_GAUSSIAN
            mean, cov = gaussian
            mean = np.asarray(mean, np.float32).reshape(7)
            cov = np.asarray(cov, np.float32).reshape(36)
            for a in range(7):
                init.mean[a] = mean[a]
            for a in range(36):
                init.cov[a] = cov[a]
        elif poses is not None:
            init.kind = MP_INIT_EXPLICIT
            p = poses
            if not hasattr(p, "data_ptr"):
                p = np.ascontiguousarray(np.asarray(poses, np.float32)[:, :7])
            init.poses = _ptr(p, np.float32, keep)
        else:
            init.kind = MP_INIT_UNIFORM_BOX
            lo, hi = box if box is not None else (map_.info()["box_min"], map_.info()["box_max"])
            for a in range(3):
                init.box_min[a] = lo[a]
                init.box_max[a] = hi[a]
        h = C.c_void_p()
        _check(lib().mp_filter_init(map_.handle, C.byref(self.params), C.byref(init), _stream(stream), C.byref(h)))
        self.handle = h
        self.n = self.params.n_particles
        self.K = self.params.k
        self.scan_n = 0

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().mp_filter_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().mp_filter_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def set_surrogate(self, sur):
        _check(lib().mp_filter_set_surrogate(self.handle, sur.handle if sur is not None else None))
        self._sur = sur   # keeps the network alive while attached

    def set_surrogate_check(self, period=10, stride=100, threshold=0.5, fallback=10):
        """mp_filter_set_surrogate_check (period 0 turns the check off)"""
        _check(lib().mp_filter_set_surrogate_check(self.handle, int(period), int(stride), float(threshold),
                                                   int(fallback)))

    def odometry(self, init=None, stream=None, noalloc=False, **kw):
        """mp_odometry (mp_odometry_noalloc with noalloc=True): dT (7),
        Sigma^dT (6 x 6) and the match's H, b, cost, inliers between the last
        two non-empty scans; keywords override mp_odometry_params fields"""
        p = mp_odometry_params()
        lib().mp_odometry_default_params(C.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError("unknown odometry parameter %r" % k)
            setattr(p, k, v)
        keep = []
        dT = np.zeros(7, np.float32)
        cov = np.zeros(36, np.float32)
        res = mp_odometry_result()
        fn = lib().mp_odometry_noalloc if noalloc else lib().mp_odometry
        _check(fn(self.handle, C.byref(p), _ptr(init, np.float32, keep), _ptr(dT), _ptr(cov), C.byref(res),
                  _stream(stream)))
        return dict(dT=dT, cov=cov.reshape(6, 6), H21=np.array(res.H[:]), b=np.array(res.b[:]), cost=res.cost,
                    inliers=res.inliers, iterations=res.iterations, cov_ok=bool(res.cov_ok),
                    dT64=np.array(res.dT64[:]))

    def scan_upload(self, xyz, cov6=None, stream=None):
        n = _nrows(xyz) if xyz is not None else 0
        keep = []
        _check(lib().mp_scan_upload(self.handle, _ptr(xyz, np.float32, keep) if n else None,
                                    _ptr(cov6, np.float32, keep), n, _stream(stream)))
        self.scan_n = n

    def step(self, dT=None, cov_dT=None, stream=None):
        keep = []
        _check(lib().mp_filter_step(self.handle, _ptr(dT, np.float32, keep), _ptr(cov_dT, np.float32, keep),
                                    _stream(stream)))

    def posterior_query(self, poses=False, weights=False, stream=None):
        out = mp_posterior()
        P = np.zeros((self.n, 7), np.float32) if poses else None
        W = np.zeros(self.n, np.float64) if weights else None
        _check(lib().mp_posterior_query(self.handle, C.byref(out), _ptr(P), _ptr(W), _stream(stream)))
        res = dict(map_pose=np.array(out.map_pose[:], np.float32), map_index=out.map_index,
                   map_weight=out.map_weight, n_eff=out.n_eff, log_evidence=out.log_evidence,
                   max_loglik=out.max_loglik, frame=out.frame, fp64_resolves=out.fp64_resolves,
                   fallback_steps=out.fallback_steps, sur_checks=out.sur_checks, sur_check_ds=out.sur_check_ds)
        if poses:
            res["poses"] = P
        if weights:
            res["weights"] = W
        return res

    def stage_times(self):
        ms = np.zeros(MP_NUM_STAGES, np.float32)
        cnt = np.zeros(MP_NUM_STAGES, np.int32)
        _check(lib().mp_stage_times(self.handle, _ptr(ms), _ptr(cnt)))
        return {STAGE_NAMES[k]: (float(ms[k]), int(cnt[k])) for k in range(MP_NUM_STAGES)}

    def debug_get(self, name, stream=None):
        dt, shp = _DEBUG_LAYOUT[name]
        out = np.zeros(shp(self.n, self.K, self.scan_n), dt)
        _check(lib().mp_debug_get(self.handle, name.encode(), _ptr(out), out.nbytes, _stream(stream)))
        return out

    def debug_set(self, name, value, stream=None):
        if name == "capture_hb":
            v = np.array([int(value)], np.int32)
            _check(lib().mp_debug_set(self.handle, b"capture_hb", _ptr(v), 4, _stream(stream)))
            return
        dt, shp = _DEBUG_LAYOUT[name]
        arr = np.ascontiguousarray(value, dt).reshape(shp(self.n, self.K, self.scan_n))
        _check(lib().mp_debug_set(self.handle, name.encode(), _ptr(arr), arr.nbytes, _stream(stream)))

    def debug_stage(self, stage, iteration=0, dT=None, cov_dT=None, stream=None):
        keep = []
        _check(lib().mp_debug_stage(self.handle, stage, iteration, _ptr(dT, np.float32, keep),
                                    _ptr(cov_dT, np.float32, keep), _stream(stream)))


# ------------------------------------------------------------------ surrogate
def mp_surrogate_default_params(**kw):
    p = mp_surrogate_params()
    lib().mp_surrogate_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k in ("box_min", "box_max"):
            for a in range(3):
                getattr(p, k)[a] = v[a]
        else:
            setattr(p, k, v)
    return p


class Surrogate:
    """Owner of an mp_surrogate handle (network replacing the map's per-point score)."""

    def __init__(self, map_: Map, params=None, stream=None, **kw):
        self.map = map_
        self.params = params if params is not None else mp_surrogate_default_params(**kw)
        h = C.c_void_p()
        _check(lib().mp_surrogate_create(map_.handle, C.byref(self.params), _stream(stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().mp_surrogate_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().mp_surrogate_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def info(self):
        i = mp_surrogate_info()
        _check(lib().mp_surrogate_get_info(self.handle, C.byref(i)))
        return dict(n_params=i.n_params, n_data=i.n_data, steps=i.steps, lo=np.array(i.lo[:], np.float32),
                    inv_ext=np.array(i.inv_ext[:], np.float32), freqs=np.array(i.freqs[:], np.float32),
                    r_scale=i.r_scale, g_scale=i.g_scale, weight_bytes=i.weight_bytes)

    def _points_call(self, fn, xyz, stream):
        n = _nrows(xyz)
        keep = []
        if hasattr(xyz, "data_ptr"):
            import torch
            out = torch.empty((n, 4), dtype=torch.float32, device=xyz.device)
        else:
            out = np.zeros((n, 4), np.float32)
        _check(fn(self.handle, _ptr(xyz, np.float32, keep), n, _ptr(out), _stream(stream)))
        return out

    def label(self, xyz, stream=None):
        return self._points_call(lib().mp_surrogate_label, xyz, stream)

    def eval(self, xyz, stream=None):
        return self._points_call(lib().mp_surrogate_eval, xyz, stream)

    def set_data(self, xyz, stream=None):
        keep = []
        _check(lib().mp_surrogate_set_data(self.handle, _ptr(xyz, np.float32, keep), _nrows(xyz), _stream(stream)))

    def train(self, steps, losses=True, stream=None):
        out = np.zeros(max(steps, 1), np.float32) if losses else None
        _check(lib().mp_surrogate_train(self.handle, steps, _ptr(out), _stream(stream)))
        return out[:steps] if losses else None

    def grad(self, xyz, target4, stream=None):
        keep = []
        g = np.zeros(MP_SUR_NPARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        _check(lib().mp_surrogate_grad(self.handle, _ptr(xyz, np.float32, keep), _ptr(target4, np.float32, keep),
                                       _nrows(xyz), _ptr(g), _ptr(loss), _stream(stream)))
        return float(loss[0]), g

    def get_params(self, stream=None):
        P = np.zeros(MP_SUR_NPARAMS, np.float32)
        _check(lib().mp_surrogate_get_params(self.handle, _ptr(P), _stream(stream)))
        return P

    def set_params(self, P, stream=None):
        keep = []
        P = np.ascontiguousarray(P, np.float32)
        if P.shape != (MP_SUR_NPARAMS,):
            raise ValueError("expected %d parameters" % MP_SUR_NPARAMS)
        _check(lib().mp_surrogate_set_params(self.handle, _ptr(P, np.float32, keep), _stream(stream)))


# ------------------------------------------------------------------ batch
class Batch:
    """Owner of an mp_batch handle: several filters stepped by one graph replay."""

    def __init__(self, filters, autotune=True, stream=None):
        self.filters = list(filters)
        arr = (C.c_void_p * len(self.filters))(*[f.handle.value for f in self.filters])
        h = C.c_void_p()
        _check(lib().mp_batch_create(arr, len(self.filters), int(bool(autotune)), _stream(stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().mp_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().mp_batch_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def step(self, dT=None, cov_dT=None, stream=None):
        keep = []
        n = len(self.filters)
        d = None if dT is None else np.ascontiguousarray(np.asarray(dT, np.float32).reshape(n, 7))
        c = None if cov_dT is None else np.ascontiguousarray(np.asarray(cov_dT, np.float32).reshape(n, 36))
        _check(lib().mp_batch_step(self.handle, _ptr(d, np.float32, keep), _ptr(c, np.float32, keep),
                                   _stream(stream)))

    def info(self):
        i = mp_batch_info()
        lb = np.zeros(len(self.filters), np.int32)
        ll = np.zeros(len(self.filters), np.int32)
        _check(lib().mp_batch_get_info(self.handle, C.byref(i), _ptr(lb), _ptr(ll)))
        return dict(n_instances=i.n_instances, captures=i.captures, evals_per_step=i.evals_per_step,
                    lik_batch=[int(x) for x in lb], lik_layout=[int(x) for x in ll],
                    queued_instances=i.queued_instances, queue_batch=i.queue_batch,
                    queue_workgroups=i.queue_workgroups, queue_tiles_per_step=i.queue_tiles_per_step)


class Smoother:
    """mp_smoother_*: smoothing of the representative pose"""

    def __init__(self, **kw):
        p = mp_smoother_params()
        lib().mp_smoother_default_params(C.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError("unknown smoother parameter %r" % k)
            setattr(p, k, v)
        h = C.c_void_p()
        _check(lib().mp_smoother_create(C.byref(p), C.byref(h)))
        self.handle = h

    def push(self, pose, dT=None):
        keep = []
        out = np.zeros(7, np.float32)
        _check(lib().mp_smoother_push(self.handle, _ptr(pose, np.float32, keep), _ptr(dT, np.float32, keep),
                                      _ptr(out)))
        return out

    def close(self):
        if self.handle:
            _check(lib().mp_smoother_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
