"""ctypes binding of libqpscatter.so (include/qpscatter.h).

Argument marshalling only: every step of the solver runs in the HIP library.  Host arrays
are numpy arrays (complex128 / float64, column-major where the C ABI says so); device
arrays are torch CUDA tensors, passed by data pointer together with the current stream.
Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpscatter.so")

if not os.path.exists(LIB_PATH):
    raise RuntimeError(f"{LIB_PATH} is missing: run paper_1301_1247_amd/build.py (or __graft_entry__.build())")

_lib = C.CDLL(LIB_PATH)

HBS_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "NONFINITE", -3: "OOM", -4: "DEVICE", -6: "SINGULAR", -7: "NOT_CONVERGED",
          -8: "ALPHA_MISMATCH", -9: "WOOD"}
QUAD = {"kr6": 0, "kress": 1, "alpert": 2}
COMPRESS = {"proxy": 0, "exact": 1}
PTR_HOST, PTR_DEVICE = 0, 1


class HBSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class HbsOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("quad", C.c_int32), ("compress", C.c_int32), ("leaf_size", C.c_int32),
                ("proxy_ratio", C.c_double), ("proxy_min", C.c_int32), ("ptr_mode", C.c_int32),
                ("curvature", C.c_void_p), ("stream", C.c_void_p), ("seed", C.c_uint64),
                ("far_radius", C.c_double), ("precision", C.c_int32), ("fp64_top_levels", C.c_int32),
                ("rank_predictor", C.c_int32), ("rank_scale", C.c_double), ("rank_model", C.c_void_p),
                ("root_level", C.c_int32), ("graph", C.c_int32), ("mem_limit", C.c_uint64),
                ("image_period", C.c_double), ("defer_root", C.c_int32), ("index", C.c_double)]


class QpOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("P", C.c_int32), ("M", C.c_int32), ("K", C.c_double), ("h", C.c_double),
                ("ca", C.c_double), ("cb", C.c_double), ("y0", C.c_double), ("wood_min_kn", C.c_double),
                ("refine_max_iter", C.c_int32), ("refine_tol", C.c_double), ("compress_walls", C.c_int32),
                ("wood", C.c_int32), ("wood_shift", C.c_double), ("wood_samples", C.c_int32)]


class HbsStats(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("levels", C.c_int32), ("N", C.c_int64), ("root_size", C.c_int32),
                ("max_rank", C.c_int32), ("factor_bytes", C.c_int64), ("build_seconds", C.c_double),
                ("ranks_per_level_max", C.c_int32 * 32), ("ranks_per_level_mean", C.c_double * 32),
                ("refine_iters", C.c_int32), ("refine_residual", C.c_double), ("contour_M", C.c_int32),
                ("walls_compressed", C.c_int32), ("rank_fallbacks", C.c_int32), ("sketch_bytes_max", C.c_int64),
                ("cpqr_work", C.c_double), ("root_level", C.c_int32), ("graph_captures", C.c_int64),
                ("graph_replays", C.c_int64), ("device_bytes_peak", C.c_int64), ("wood_angles", C.c_int32),
                ("wood_orders", C.c_int32), ("wood_shift", C.c_double), ("image_samples", C.c_int64),
                ("unknowns", C.c_int64)]


_P = C.c_void_p
_sig = {
    "hbs_opts_init": (None, [C.POINTER(HbsOpts)]),
    "qp_opts_init": (None, [C.POINTER(QpOpts)]),
    "hbs_build": (C.c_int, [_P, _P, _P, C.c_int64, C.c_double, C.c_double, C.POINTER(HbsOpts), C.POINTER(_P)]),
    "hbs_apply": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32]),
    "hbs_forward": (C.c_int, [_P, _P, C.c_int64, _P]),
    "hbs_apply_noalloc": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32]),
    "qp_solve": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, _P, C.c_int64, C.POINTER(QpOpts), _P, _P, _P, _P,
                           _P, _P]),
    "qp_solve_many": (C.c_int, [_P, C.c_double, _P, C.c_int64, C.POINTER(QpOpts), _P, _P, _P, _P, _P, _P]),
    "qp_contour_size": (C.c_int32, [_P, C.c_double, C.POINTER(QpOpts)]),
    "qp_max_modes": (C.c_int32, [C.c_double, C.c_double]),
    "hbs_stats": (C.c_int, [_P, C.POINTER(HbsStats)]),
    "hbs_free": (None, [_P]),
    "hbs_last_error": (C.c_char_p, []),
    "qps_hankel01": (C.c_int, [_P, C.c_int64, _P, C.c_int32]),
    "qps_kr6_corrections": (C.c_int, [_P]),
    "qps_alpert_rule": (C.c_int, [C.c_int32, C.c_int32, _P, _P]),
    "qps_matrix_entries": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "qps_zgemm": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "qps_zinv": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32]),
    "qps_cgemm": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "qps_cinv": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32]),
    "qps_rank_model_size": (C.c_int32, []),
    "qps_rank_model_default": (C.c_int, [_P]),
    "qps_rank_features": (C.c_int, [_P, _P, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "qps_mlp_forward": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32]),
    "qps_mlp_grad": (C.c_int, [_P, _P, _P, C.c_int64, C.c_float, _P, _P, C.c_int32]),
    "qps_mlp_train": (C.c_int, [_P, _P, _P, C.c_int64, C.c_float, C.c_int32, C.c_float, _P, C.c_int32]),
    "qps_pool_release": (C.c_int, []),
    "qps_pool_cached_bytes": (C.c_int64, []),
    "qps_profile_enable": (C.c_int, [C.c_int32]),
    "qps_profile_read": (C.c_int, [C.c_char_p, _P, _P, _P, _P]),
    "qps_gemm_class": (C.c_int, [C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int64, _P]),
    "qps_gemm_tune_lookup": (C.c_int, [C.c_int32, _P]),
    "qps_gemm_tune_set": (C.c_int, [_P, _P, C.c_int32]),
    "qps_gemm_tune_get": (C.c_int, [_P, _P, C.c_int32, _P]),
    "qps_gemm_tune_begin": (C.c_int, [C.c_int32]),
    "qps_gemm_tune_end": (C.c_int, [_P, _P, _P, C.c_int32, _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(rc):
    if rc != HBS_OK:
        raise HBSError(rc, _lib.hbs_last_error().decode())


def _ptr(a):
    """Data pointer of a C-contiguous numpy array or a contiguous torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"] and not a.flags["F_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return a.ctypes.data
    if not a.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return a.data_ptr()


def _cmat(a):
    """Complex (rows, cols) numpy matrix -> column-major complex128 buffer."""
    a = np.asarray(a, dtype=np.complex128)
    if a.ndim == 1:
        a = a[:, None]
    return np.asfortranarray(a)


def hbs_opts(**kw) -> HbsOpts:
    o = HbsOpts()
    _lib.hbs_opts_init(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def qp_opts(**kw) -> QpOpts:
    o = QpOpts()
    _lib.qp_opts_init(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Handle:
    """A built compressed inverse (hbs_build) with its apply / solve calls."""

    def __init__(self, nodes, weights, normals, omega, tol, quad="kr6", compress=None, leaf_size=64,
                 curvature=None, device=False, stream=None, proxy_ratio=2.0, proxy_min=64, seed=0x5EED1301,
                 far_radius=0.0, precision="fp64", fp64_top_levels=0, rank_predictor=False, rank_scale=1.0,
                 rank_model=None, root_level=0, graph=False, mem_limit=0, image_period=0.0, defer_root=False,
                 index=0.0):
        if compress is None:
            compress = "exact" if quad == "kress" else "proxy"
        self.device = bool(device)
        if self.device:
            import torch
            self._torch = torch
            self._keep = [nodes, weights, normals, curvature]
            N = int(weights.shape[0])
            st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        else:
            nodes = np.ascontiguousarray(nodes, dtype=np.float64)
            weights = np.ascontiguousarray(weights, dtype=np.float64)
            normals = np.ascontiguousarray(normals, dtype=np.float64)
            curvature = None if curvature is None else np.ascontiguousarray(curvature, dtype=np.float64)
            self._keep = [nodes, weights, normals, curvature]
            N = int(weights.shape[0])
            st = stream
        self.N = N
        # unknowns: two densities per node for the transmission problem (index > 0), interlaced
        self.NU = 2 * N if index > 0 else N
        self.omega = float(omega)
        o = hbs_opts(quad=QUAD[quad], compress=COMPRESS[compress], leaf_size=int(leaf_size),
                     proxy_ratio=float(proxy_ratio), proxy_min=int(proxy_min),
                     ptr_mode=PTR_DEVICE if self.device else PTR_HOST,
                     curvature=_ptr(curvature), stream=st, seed=int(seed), far_radius=float(far_radius),
                     precision={"fp64": 0, "fp32": 1}[precision], fp64_top_levels=int(fp64_top_levels),
                     rank_predictor=1 if rank_predictor else 0, rank_scale=float(rank_scale),
                     root_level=int(root_level), graph=1 if graph else 0, mem_limit=int(mem_limit),
                     image_period=float(image_period), defer_root=1 if defer_root else 0, index=float(index))
        if rank_model is not None:
            rank_model = np.ascontiguousarray(rank_model, dtype=np.float32)
            o.rank_model = rank_model.ctypes.data
        self._model = rank_model
        h = C.c_void_p()
        _check(_lib.hbs_build(_ptr(nodes), _ptr(weights), _ptr(normals), N, float(omega), float(tol), C.byref(o),
                              C.byref(h)))
        self._h = h

    def __del__(self):
        self.free()

    def free(self, _free=_lib.hbs_free):
        # the library function is bound at definition time: at interpreter shutdown the module's
        # globals may already be cleared when the last handles are collected
        if getattr(self, "_h", None) is not None and self._h.value:
            _free(self._h)
            self._h = None

    # -- apply / forward
    def _alloc_like(self, rows, cols):
        if self.device:
            return self._torch.empty((cols, rows), dtype=self._torch.complex128, device="cuda")
        return np.empty((rows, cols), dtype=np.complex128, order="F")

    def apply(self, rhs, refine=0):
        """A^{-1} rhs (NU x r, NU = the handle's unknowns).  Host: numpy (NU,) or (NU, r); device: torch (r, NU)
        complex128 (column-major NU x r)."""
        if self.device:
            r = rhs.shape[0] if rhs.dim() == 2 else 1
            out = self._torch.empty_like(rhs)
            _check(_lib.hbs_apply(self._h, _ptr(rhs), r, _ptr(out), int(refine)))
            return out
        b = _cmat(rhs)
        out = np.empty_like(b)
        _check(_lib.hbs_apply(self._h, _ptr(b), b.shape[1], _ptr(out), int(refine)))
        return out[:, 0] if np.ndim(rhs) == 1 else out

    def apply_noalloc(self, rhs, refine=0, out=None):
        """hbs_apply_noalloc: device handles only; rhs torch (r, N) complex128 (column-major N x r)."""
        if not self.device:
            raise ValueError("apply_noalloc needs a handle built with device=True")
        r = rhs.shape[0] if rhs.dim() == 2 else 1
        if out is None:
            out = self._torch.empty_like(rhs)
        _check(_lib.hbs_apply_noalloc(self._h, _ptr(rhs), r, _ptr(out), int(refine)))
        return out

    def forward(self, x):
        if self.device:
            r = x.shape[0] if x.dim() == 2 else 1
            out = self._torch.empty_like(x)
            _check(_lib.hbs_forward(self._h, _ptr(x), r, _ptr(out)))
            return out
        b = _cmat(x)
        out = np.empty_like(b)
        _check(_lib.hbs_forward(self._h, _ptr(b), b.shape[1], _ptr(out)))
        return out[:, 0] if np.ndim(x) == 1 else out

    # -- quasi-periodic solve
    def contour_size(self, period, **qkw):
        q = qp_opts(**qkw)
        return int(_lib.qp_contour_size(self._h, float(period), C.byref(q)))

    def qp_solve_many(self, period, thetas, alpha=None, **qkw):
        """Solve for all angles.  Returns dict(eta (N, n), xi (2M, n), bragg (2*maxm, n), nlo, nmodes, flux).
        Device handles take thetas as a torch float64 CUDA tensor and return torch tensors (n, N) etc."""
        q = qp_opts(**qkw)
        M = self.contour_size(period, **qkw)
        maxm = int(_lib.qp_max_modes(self.omega, float(period)))
        if self.device:
            torch = self._torch
            th = thetas.to(device="cuda", dtype=torch.float64).contiguous()
            n = th.shape[0]
            eta = torch.empty((n, self.NU), dtype=torch.complex128, device="cuda")
            xi = torch.empty((n, 2 * M), dtype=torch.complex128, device="cuda")
            bragg = torch.empty((n, 2 * maxm), dtype=torch.complex128, device="cuda")
        else:
            th = np.ascontiguousarray(thetas, dtype=np.float64)
            n = th.shape[0]
            eta = np.empty((self.NU, n), dtype=np.complex128, order="F")
            xi = np.empty((2 * M, n), dtype=np.complex128, order="F")
            bragg = np.empty((2 * maxm, n), dtype=np.complex128, order="F")
        nlo = np.zeros(n, dtype=np.int32)
        nm = np.zeros(n, dtype=np.int32)
        flux = np.zeros(n, dtype=np.float64)
        if alpha is None:
            rc = _lib.qp_solve_many(self._h, float(period), _ptr(th), n, C.byref(q), _ptr(eta), _ptr(xi), _ptr(bragg),
                                    _ptr(nlo), _ptr(nm), _ptr(flux))
        else:
            rc = _lib.qp_solve(self._h, float(period), float(np.real(alpha)), float(np.imag(alpha)), _ptr(th), n,
                               C.byref(q), _ptr(eta), _ptr(xi), _ptr(bragg), _ptr(nlo), _ptr(nm), _ptr(flux))
        _check(rc)
        return dict(eta=eta, xi=xi, bragg=bragg, nlo=nlo, nmodes=nm, flux=flux, M=M, maxmodes=maxm)

    def stats(self):
        s = HbsStats()
        _check(_lib.hbs_stats(self._h, C.byref(s)))
        return s

    def rank_features(self):
        """(features n x 16, CPQR ranks, levels, predicted ranks) of every box, leaves first."""
        cnt = C.c_int64()
        _check(_lib.qps_rank_features(self._h, None, None, None, None, 0, C.byref(cnt)))
        n = cnt.value
        f = np.empty((n, 16), dtype=np.float32)
        k = np.empty(n, dtype=np.int32)
        lv = np.empty(n, dtype=np.int32)
        pr = np.empty(n, dtype=np.float32)
        _check(_lib.qps_rank_features(self._h, _ptr(f), _ptr(k), _ptr(lv), _ptr(pr), n, C.byref(cnt)))
        return f, k, lv, pr

    def matrix_entries(self, rows, cols):
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        out = np.empty(rows.shape[0], dtype=np.complex128)
        _check(_lib.qps_matrix_entries(self._h, _ptr(rows), _ptr(cols), rows.shape[0], _ptr(out)))
        return out


def hankel01(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(2 * x.shape[0], dtype=np.complex128)
    _check(_lib.qps_hankel01(_ptr(x), x.shape[0], _ptr(out), PTR_HOST))
    return out[: x.shape[0]], out[x.shape[0]:]


def alpert_rule(m=5, a=6):
    """Nodes and weights of the library's Alpert correction (derived on the host)."""
    x = np.zeros(m)
    w = np.zeros(m)
    _check(_lib.qps_alpert_rule(int(m), int(a), _ptr(x), _ptr(w)))
    return x, w


def kr6_corrections():
    out = np.empty(6, dtype=np.float64)
    _check(_lib.qps_kr6_corrections(_ptr(out)))
    return out


def zgemm(A, B, transA=False, precision="fp64"):
    """Batched C = op(A) B on the GPU: A (b, m, k) or (b, k, m) if transA, B (b, k, n).

    precision "fp64": complex128 (FP64 MFMA); "fp32": complex64 (FP32 MFMA)."""
    dt, fn = (np.complex128, _lib.qps_zgemm) if precision == "fp64" else (np.complex64, _lib.qps_cgemm)
    A = np.asarray(A, dtype=dt)
    B = np.asarray(B, dtype=dt)
    nb = A.shape[0]
    if transA:
        k, m = A.shape[1], A.shape[2]
    else:
        m, k = A.shape[1], A.shape[2]
    n = B.shape[2]
    Af = np.array(np.transpose(A, (0, 2, 1)), order="C", copy=True)  # column-major per batch entry
    Bf = np.array(np.transpose(B, (0, 2, 1)), order="C", copy=True)
    Cf = np.zeros((nb, n, m), dtype=dt)
    _check(fn(_ptr(Af), _ptr(Bf), _ptr(Cf), m, n, k, nb, int(transA), 0, PTR_HOST))
    return np.transpose(Cf, (0, 2, 1))


def zinv(A, precision="fp64"):
    """Batched in-place Gauss-Jordan inverse on the GPU (complex128, or complex64 for "fp32")."""
    dt, fn = (np.complex128, _lib.qps_zinv) if precision == "fp64" else (np.complex64, _lib.qps_cinv)
    A = np.asarray(A, dtype=dt)
    nb, n = A.shape[0], A.shape[1]
    Af = np.array(np.transpose(A, (0, 2, 1)), order="C", copy=True)
    _check(fn(_ptr(Af), n, nb, PTR_HOST))
    return np.transpose(Af, (0, 2, 1))


def rank_model_size():
    return int(_lib.qps_rank_model_size())


def rank_model_default():
    out = np.empty(rank_model_size(), dtype=np.float32)
    _check(_lib.qps_rank_model_default(_ptr(out)))
    return out


def mlp_forward(params, x):
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(x.shape[0], dtype=np.float32)
    _check(_lib.qps_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(y), PTR_HOST))
    return y


def mlp_grad(params, x, t, tau=0.9):
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    g = np.empty_like(params)
    loss = np.zeros(1, dtype=np.float32)
    _check(_lib.qps_mlp_grad(_ptr(params), _ptr(x), _ptr(t), x.shape[0], float(tau), _ptr(g), _ptr(loss), PTR_HOST))
    return g, float(loss[0])


def mlp_train(params, x, t, tau=0.9, steps=1000, lr=1e-3):
    """Adam on the mean pinball loss; returns (new params, per-step mean loss)."""
    p = np.array(params, dtype=np.float32, copy=True)
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    hist = np.zeros(max(1, steps), dtype=np.float32)
    _check(_lib.qps_mlp_train(_ptr(p), _ptr(x), _ptr(t), x.shape[0], float(tau), int(steps), float(lr), _ptr(hist),
                              PTR_HOST))
    return p, hist[:steps]


def pool_release():
    """Return the device memory cached by the library's pool (current device) to HIP."""
    _check(_lib.qps_pool_release())


def pool_cached_bytes():
    return int(_lib.qps_pool_cached_bytes())


def profile_enable(on=True):
    _check(_lib.qps_profile_enable(1 if on else 0))


def profile_read(family):
    ms = C.c_double()
    la = C.c_int64()
    fl = C.c_double()
    by = C.c_double()
    _check(_lib.qps_profile_read(family.encode(), C.byref(ms), C.byref(la), C.byref(fl), C.byref(by)))
    return dict(ms=ms.value, launches=la.value, flops=fl.value, bytes=by.value)


GEMM_CONFIGS = {0: (64, 64), 1: (32, 32), 2: (64, 32), 3: (32, 64)}  # output tile (rows, cols) per config


def gemm_class(max_m, max_n, max_k, count, complex64=False):
    """Shape-class key of a batched GEMM launch (largest m, n, k of its entries, entry count)."""
    key = C.c_int32()
    _check(_lib.qps_gemm_class(1 if complex64 else 0, int(max_m), int(max_n), int(max_k), int(count), C.byref(key)))
    return key.value


def gemm_class_fields(key):
    """(complex64, ceil log2 m, n, k, count) of a class key."""
    return (key >> 24) & 1, (key >> 18) & 63, (key >> 12) & 63, (key >> 6) & 63, key & 63


def gemm_tune_lookup(key):
    """The tuning table's configuration for a class key, or -1 (configuration 0 is used)."""
    cfg = C.c_int32()
    _check(_lib.qps_gemm_tune_lookup(int(key), C.byref(cfg)))
    return cfg.value


def gemm_tune_set(table):
    """Replace the tuning table by {key: cfg}; None restores the built-in table."""
    if table is None:
        _check(_lib.qps_gemm_tune_set(None, None, -1))
        return
    keys = np.ascontiguousarray(list(table.keys()), dtype=np.int32)
    cfgs = np.ascontiguousarray([table[k] for k in table], dtype=np.int32)
    _check(_lib.qps_gemm_tune_set(_ptr(keys) if len(keys) else None, _ptr(cfgs) if len(cfgs) else None, len(keys)))


def gemm_tune_get():
    """The active tuning table as {key: cfg}."""
    n = C.c_int32()
    _check(_lib.qps_gemm_tune_get(None, None, 0, C.byref(n)))
    keys = np.zeros(max(1, n.value), dtype=np.int32)
    cfgs = np.zeros(max(1, n.value), dtype=np.int32)
    _check(_lib.qps_gemm_tune_get(_ptr(keys), _ptr(cfgs), n.value, C.byref(n)))
    return {int(k): int(c) for k, c in zip(keys[: n.value], cfgs[: n.value])}


def gemm_tune_begin(cfg):
    """Start a sweep: every GEMM launch uses configuration cfg and is timed per shape class."""
    _check(_lib.qps_gemm_tune_begin(int(cfg)))


def gemm_tune_end(cap=4096):
    """End the sweep: {key: (ms, launches)} of the classes timed since gemm_tune_begin."""
    keys = np.zeros(cap, dtype=np.int32)
    ms = np.zeros(cap, dtype=np.float64)
    la = np.zeros(cap, dtype=np.int64)
    n = C.c_int32()
    _check(_lib.qps_gemm_tune_end(_ptr(keys), _ptr(ms), _ptr(la), cap, C.byref(n)))
    m = min(n.value, cap)
    return {int(keys[i]): (float(ms[i]), int(la[i])) for i in range(m)}
