"""Python binding of the MI355X worldline Wilson-loop library (libwl.so).

Argument marshalling only: every step of the evaluation runs in the HIP
kernels behind the C ABI of ``include/wl.h``; the functions here carry the
same names.  Host arrays are numpy; device arrays are torch tensors on the
context's device (torch supplies device memory and streams).

If ``libwl.so`` has not been built the import raises: there is no CPU
fallback.  Build it with ``python -m paper_1407_7486_amd.build`` or
``__graft_entry__.build()``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwl.so")

WL_OK, WL_EINVAL, WL_ENOMEM, WL_EHIP, WL_ENODEV = 0, -1, -2, -3, -4
WL_CONST, WL_SECH2, WL_GAUSS, WL_RATIONAL = 0, 1, 2, 3
WL_FP32C, WL_FP32, WL_FP64, WL_FP32K = 0, 1, 2, 3
WL_HOST_PTR, WL_DEVICE_PTR = 0, 1
WL_DISC_PAPER, WL_DISC_FULL = 0, 1
WL_SUB_CIRCLE, WL_SUB_SQUARE, WL_SUB_TRIANGLE = 0, 1, 2
WL_NOALLOC_SCRATCH_BYTES = 256 << 20

# every entry point declared in include/wl.h
EXPORTS = (
    "wl_create", "wl_destroy", "wl_last_error", "wl_strerror", "wl_version",
    "wl_ensemble_upload", "wl_ensemble_free", "wl_ensemble_info",
    "wl_average", "wl_average_async", "wl_per_loop", "wl_set_timing",
    "wl_last_kernel_ms", "wl_kernel_ms_total", "wl_average_batch",
    "wl_server_create", "wl_server_submit", "wl_server_poll", "wl_server_wait",
    "wl_server_release", "wl_server_timing", "wl_server_info", "wl_server_last_error", "wl_server_destroy",
    "wl_discretisation", "wl_subloop_per_loop", "wl_action_grids", "wl_action",
    "wl_ensemble_generate", "wl_ensemble_download", "wl_ensemble_set_groups",
    "wl_correlation", "wl_regroup", "wl_average_async_noalloc", "wl_average_ex",
)


class WLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class wl_field(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eB0", ctypes.c_double), ("lambda_", ctypes.c_double)]


class wl_request(ctypes.Structure):
    _fields_ = [("field", wl_field), ("rho", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("n_rho", ctypes.c_int32), ("n_T", ctypes.c_int32),
                ("spin", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("err", ctypes.c_void_p),
                ("group_sums", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("fp_err", ctypes.c_void_p), ("escalated", ctypes.c_void_p)]


class wl_result(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "mean", "err", "group_sums", "scale", "fp_err", "escalated")]


class wl_action_spec(ctypes.Structure):
    _fields_ = [("m2", ctypes.c_double), ("a", ctypes.c_double), ("T_max", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("n_T", ctypes.c_int32),
                ("n_rho", ctypes.c_int32)]


class wl_action_out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "density", "density_mean", "density_err", "action", "action_mean", "action_err",
        "lcf_density", "lcf_action")]


class wl_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("input_bytes", ctypes.c_size_t), ("result_bytes", ctypes.c_size_t),
                ("in_order", ctypes.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: the HIP library has not been built "
        "(run python -m paper_1407_7486_amd.build)")

# torch ships its own HIP runtime (libamdhip64.so).  Loading torch first
# makes libwl.so bind to that same runtime, so that torch streams and device
# pointers are valid here; loaded the other way round the process would hold
# two HIP runtimes competing for the device.
try:
    import torch  # noqa: F401
except ImportError:  # no torch: libwl.so uses the system HIP runtime
    pass

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_sigs = {
    "wl_create": ([ctypes.POINTER(_vp), ctypes.c_int, _vp], ctypes.c_int),
    "wl_destroy": ([_vp], ctypes.c_int),
    "wl_last_error": ([_vp], ctypes.c_char_p),
    "wl_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "wl_version": ([], ctypes.c_char_p),
    "wl_ensemble_upload": ([_vp, _vp, _vp, _i64, _i32, _i32, _i32,
                            ctypes.POINTER(_vp)], ctypes.c_int),
    "wl_ensemble_free": ([_vp], ctypes.c_int),
    "wl_ensemble_generate": ([_vp, ctypes.c_uint64, _i64, _i64, _i32, _i32,
                              ctypes.POINTER(_vp)], ctypes.c_int),
    "wl_ensemble_download": ([_vp, _vp, _vp, _i64, _i64], ctypes.c_int),
    "wl_ensemble_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                          ctypes.POINTER(_i32)], ctypes.c_int),
    "wl_average": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp, _i32,
                    _i32, _i32, _vp, _vp, _vp], ctypes.c_int),
    "wl_average_async": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp,
                          _i32, _i32, _i32, _vp, _vp, _vp], ctypes.c_int),
    "wl_average_ex": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp, _i32, _i32, _i32,
                       _i32, ctypes.POINTER(wl_result)], ctypes.c_int),
    "wl_average_async_noalloc": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp,
                                  _i32, _i32, _i32, _vp, _vp, _vp], ctypes.c_int),
    "wl_per_loop": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp, _i32,
                     _i32, _i32, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
    "wl_discretisation": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp, _i32,
                           _i32, _i32, _i32, _vp, _vp, _vp, _vp], ctypes.c_int),
    "wl_subloop_per_loop": ([_vp, _vp, ctypes.POINTER(wl_field), _vp, _i32, _vp, _i32,
                             _i32, _i32, _i32, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
    "wl_action_grids": ([ctypes.POINTER(wl_action_spec), _vp, _vp], ctypes.c_int),
    "wl_action": ([_vp, ctypes.POINTER(wl_action_spec), ctypes.POINTER(wl_field), _i32, _vp,
                   _i32, _i64, _i32, ctypes.POINTER(wl_action_out)], ctypes.c_int),
    "wl_ensemble_set_groups": ([_vp, _i32], ctypes.c_int),
    "wl_correlation": ([_vp, _vp, _i64, _i32, _i32, _vp], ctypes.c_int),
    "wl_regroup": ([_vp, _vp, _i64, _i32, _vp, _i32, _vp, _i32, _i32, _vp], ctypes.c_int),
    "wl_set_timing": ([_vp, _i32], ctypes.c_int),
    "wl_last_kernel_ms": ([_vp, ctypes.POINTER(_d)], ctypes.c_int),
    "wl_kernel_ms_total": ([_vp, ctypes.POINTER(_d), ctypes.POINTER(_i64)],
                           ctypes.c_int),
    "wl_average_batch": ([_vp, _vp, ctypes.POINTER(wl_request), _i32], ctypes.c_int),
    "wl_server_create": ([_vp, _vp, ctypes.POINTER(wl_server_config), ctypes.POINTER(_vp)],
                         ctypes.c_int),
    "wl_server_submit": ([_vp, ctypes.POINTER(wl_request), ctypes.POINTER(_i64)], ctypes.c_int),
    "wl_server_poll": ([_vp, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_d)], ctypes.c_int),
    "wl_server_wait": ([_vp, _i64, _d, ctypes.POINTER(_i32), ctypes.POINTER(_d)], ctypes.c_int),
    "wl_server_release": ([_vp, _i64], ctypes.c_int),
    "wl_server_timing": ([_vp, _i64, ctypes.POINTER(_d), ctypes.POINTER(_d)], ctypes.c_int),
    "wl_server_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
                       ctypes.c_int),
    "wl_server_last_error": ([_vp], ctypes.c_char_p),
    "wl_server_destroy": ([_vp], ctypes.c_int),
}
for _name, (_args, _res) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def _check(rc, ctx=None):
    if rc != WL_OK:
        msg = _lib.wl_last_error(ctx).decode() if ctx else ""
        raise WLError(rc, msg or _lib.wl_strerror(rc).decode())


def _ptr(a):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _host_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def field(kind, eB0, lam=1.0):
    return wl_field(int(kind), 0, float(eB0), float(lam))


def wl_version():
    return _lib.wl_version().decode()


def wl_strerror(code):
    return _lib.wl_strerror(code).decode()


def wl_create(device=0, stream=None):
    """Context on HIP device `device`; `stream` is a raw hipStream_t value
    (e.g. torch.cuda.current_stream().cuda_stream) or None."""
    ctx = _vp()
    rc = _lib.wl_create(ctypes.byref(ctx), int(device), stream)
    if rc != WL_OK:
        raise WLError(rc, wl_strerror(rc))
    return ctx


def wl_destroy(ctx):
    _check(_lib.wl_destroy(ctx))


def wl_last_error(ctx):
    return _lib.wl_last_error(ctx).decode()


def wl_ensemble_upload(ctx, y_x, y_y, n_groups):
    """Upload unit loops [n_loops][n_ppl] (FP32).  numpy arrays are host
    memory; torch CUDA tensors are device memory."""
    dev = not isinstance(y_x, np.ndarray)
    if dev:
        if y_x.dtype != _torch().float32 or not y_x.is_contiguous() \
                or not y_y.is_contiguous() or y_x.shape != y_y.shape:
            raise ValueError("device coordinates must be contiguous float32 of one shape")
    else:
        y_x = np.ascontiguousarray(y_x, dtype=np.float32)
        y_y = np.ascontiguousarray(y_y, dtype=np.float32)
        if y_x.shape != y_y.shape or y_x.ndim != 2:
            raise ValueError("coordinates must be two arrays of shape (n_loops, n_ppl)")
    n_loops, n_ppl = y_x.shape
    ens = _vp()
    _check(_lib.wl_ensemble_upload(ctx, _ptr(y_x), _ptr(y_y), n_loops, n_ppl,
                                   int(n_groups),
                                   WL_DEVICE_PTR if dev else WL_HOST_PTR,
                                   ctypes.byref(ens)), ctx)
    return ens


def wl_ensemble_generate(ctx, seed, first_loop, n_loops, n_ppl, n_groups):
    """d-loop ensemble generated on the device (see include/wl.h)."""
    ens = _vp()
    _check(_lib.wl_ensemble_generate(ctx, int(seed), int(first_loop), int(n_loops),
                                     int(n_ppl), int(n_groups), ctypes.byref(ens)), ctx)
    return ens


def wl_ensemble_download(ens, loop0, n_loops):
    """Loops loop0 .. loop0+n_loops-1 as FP32 numpy arrays (x, y)."""
    _, n_ppl, _ = wl_ensemble_info(ens)
    x = np.zeros((n_loops, n_ppl), dtype=np.float32)
    y = np.zeros((n_loops, n_ppl), dtype=np.float32)
    rc = _lib.wl_ensemble_download(ens, _ptr(x), _ptr(y), int(loop0), int(n_loops))
    if rc != WL_OK:
        raise WLError(rc, "wl_ensemble_download failed")
    return x, y


def wl_ensemble_set_groups(ens, n_groups):
    rc = _lib.wl_ensemble_set_groups(ens, int(n_groups))
    if rc != WL_OK:
        raise WLError(rc, "wl_ensemble_set_groups failed")


def wl_correlation(ctx, values):
    """Correlation matrix (n_pts, n_pts) of the columns of host values
    (n_units, n_pts) over the rows."""
    X = np.ascontiguousarray(values, dtype=np.float64)
    n_units, n_pts = X.shape
    out = np.zeros((n_pts, n_pts))
    _check(_lib.wl_correlation(ctx, _ptr(X), n_units, n_pts, WL_HOST_PTR, _ptr(out)), ctx)
    return out


def wl_regroup(ctx, per_unit, perms, n_groups, point_perm=None):
    """Group sums (n_groups, n_pts) of host per-unit values (n_units, n_pts)
    under the permutations perms (n_perms, n_units); point_perm (n_pts,)
    picks the permutation of each column (None: row 0 everywhere)."""
    X = np.ascontiguousarray(per_unit, dtype=np.float64)
    P = np.ascontiguousarray(np.atleast_2d(perms), dtype=np.int64)
    Q = None if point_perm is None else np.ascontiguousarray(point_perm, dtype=np.int32)
    n_units, n_pts = X.shape
    out = np.zeros((n_groups, n_pts))
    _check(_lib.wl_regroup(ctx, _ptr(X), n_units, n_pts, _ptr(P), P.shape[0], _ptr(Q),
                           int(n_groups), WL_HOST_PTR, _ptr(out)), ctx)
    return out


def wl_ensemble_free(ens):
    _check(_lib.wl_ensemble_free(ens))


def wl_ensemble_info(ens):
    nl, npl, ng = _i64(), _i32(), _i32()
    _check(_lib.wl_ensemble_info(ens, ctypes.byref(nl), ctypes.byref(npl),
                                 ctypes.byref(ng)))
    return nl.value, npl.value, ng.value


def wl_average(ctx, ens, fld, rho, T, spin, precision=WL_FP32C):
    """Synchronous average; returns (mean, err, group_sums) as numpy arrays
    of shapes (n_rho, n_T), (n_rho, n_T), (G, n_rho, n_T)."""
    rho = _host_f64(rho)
    T = _host_f64(T)
    _, _, G = wl_ensemble_info(ens)
    mean = np.zeros((rho.size, T.size))
    err = np.zeros((rho.size, T.size))
    sums = np.zeros((G, rho.size, T.size))
    _check(_lib.wl_average(ctx, ens, ctypes.byref(fld), _ptr(rho), rho.size,
                           _ptr(T), T.size, int(spin), int(precision),
                           _ptr(mean), _ptr(err), _ptr(sums)), ctx)
    return mean, err, sums


RESULT_KEYS = ("mean", "err", "group_sums", "scale", "fp_err", "escalated")


def _result_arrays(G, n_rho, n_T):
    return {"mean": np.zeros((n_rho, n_T)), "err": np.zeros((n_rho, n_T)),
            "group_sums": np.zeros((G, n_rho, n_T)), "scale": np.zeros((n_rho, n_T)),
            "fp_err": np.zeros((n_rho, n_T)),
            "escalated": np.zeros((n_rho, n_T), dtype=np.uint8)}


def wl_average_ex(ctx, ens, fld, rho, T, spin, precision=WL_FP32C):
    """Synchronous average with every output of wl_result; returns a dict
    of numpy arrays: mean, err, scale, fp_err, escalated (n_rho, n_T) and
    group_sums (G, n_rho, n_T)."""
    rho = _host_f64(rho)
    T = _host_f64(T)
    _, _, G = wl_ensemble_info(ens)
    out = _result_arrays(G, rho.size, T.size)
    res = wl_result(*[_ptr(out[k]) for k in RESULT_KEYS])
    _check(_lib.wl_average_ex(ctx, ens, ctypes.byref(fld), _ptr(rho), rho.size, _ptr(T),
                              T.size, int(spin), int(precision), WL_HOST_PTR,
                              ctypes.byref(res)), ctx)
    return out


def wl_average_ex_device(ctx, ens, fld, d_rho, d_T, spin, precision, outs):
    """Enqueue an average on the context stream; d_rho, d_T and the values
    of `outs` (keys of RESULT_KEYS, group_sums required) are torch device
    tensors."""
    res = wl_result(*[_ptr(outs.get(k)) for k in RESULT_KEYS])
    _check(_lib.wl_average_ex(ctx, ens, ctypes.byref(fld), _ptr(d_rho), d_rho.numel(),
                              _ptr(d_T), d_T.numel(), int(spin), int(precision),
                              WL_DEVICE_PTR, ctypes.byref(res)), ctx)


def wl_discretisation(ctx, ens, fld, rho, T, spin, precision=WL_FP32C, mode=WL_DISC_PAPER):
    """Discretisation estimate (levels N, N/2, N/4, extrapolated); returns
    (mean, err, delta, group_sums) of shapes (4, n_rho, n_T), (4, n_rho,
    n_T), (n_rho, n_T), (4, G, n_rho, n_T)."""
    rho = _host_f64(rho)
    T = _host_f64(T)
    _, _, G = wl_ensemble_info(ens)
    mean = np.zeros((4, rho.size, T.size))
    err = np.zeros((4, rho.size, T.size))
    delta = np.zeros((rho.size, T.size))
    sums = np.zeros((4, G, rho.size, T.size))
    _check(_lib.wl_discretisation(ctx, ens, ctypes.byref(fld), _ptr(rho), rho.size,
                                  _ptr(T), T.size, int(spin), int(precision), int(mode),
                                  _ptr(mean), _ptr(err), _ptr(delta), _ptr(sums)), ctx)
    return mean, err, delta, sums


def wl_subloop_per_loop(ctx, ens, fld, rho, T, spin, precision, subloop, loop0, n_loops):
    """Per-loop (phase, spin_exp, w) of one sub-loop (WL_SUB_*), each of
    shape (n_loops, n_rho, n_T)."""
    rho = _host_f64(rho)
    T = _host_f64(T)
    out = [np.zeros((n_loops, rho.size, T.size)) for _ in range(3)]
    _check(_lib.wl_subloop_per_loop(ctx, ens, ctypes.byref(fld), _ptr(rho), rho.size,
                                    _ptr(T), T.size, int(spin), int(precision), int(subloop),
                                    int(loop0), int(n_loops), *[_ptr(a) for a in out]), ctx)
    return tuple(out)


def action_spec(m2, a, T_max, n_T, rho_max, n_rho):
    return wl_action_spec(float(m2), float(a), float(T_max), float(rho_max), int(n_T),
                          int(n_rho))


def wl_action_grids(spec):
    """(T[n_T], rho[n_rho]) of the action integrals."""
    T = np.zeros(spec.n_T)
    rho = np.zeros(spec.n_rho)
    rc = _lib.wl_action_grids(ctypes.byref(spec), _ptr(T), _ptr(rho))
    if rc != WL_OK:
        raise WLError(rc, "invalid action spec")
    return T, rho


def wl_action(ctx, spec, fld, spin, group_sums, n_loops):
    """Effective action from host group sums (G, n_rho, n_T); returns a dict
    of numpy arrays (density (G, n_rho), density_mean, density_err, action
    (G,), action_mean, action_err, lcf_density, lcf_action)."""
    S = _host_f64(group_sums)
    G = S.shape[0]
    nr = spec.n_rho
    res = {"density": np.zeros((G, nr)), "density_mean": np.zeros(nr),
           "density_err": np.zeros(nr), "action": np.zeros(G), "action_mean": np.zeros(1),
           "action_err": np.zeros(1), "lcf_density": np.zeros(nr), "lcf_action": np.zeros(1)}
    out = wl_action_out(*[_ptr(res[n]) for n, _ in wl_action_out._fields_])
    _check(_lib.wl_action(ctx, ctypes.byref(spec), ctypes.byref(fld), int(spin), _ptr(S), G,
                          int(n_loops), WL_HOST_PTR, ctypes.byref(out)), ctx)
    for n in ("action_mean", "action_err", "lcf_action"):
        res[n] = float(res[n][0])
    return res


def wl_average_async(ctx, ens, fld, d_rho, d_T, spin, precision, d_mean,
                     d_err, d_group_sums):
    """Enqueue an average on the context stream; all arrays are torch
    float64 device tensors (d_mean / d_err may be None)."""
    _check(_lib.wl_average_async(ctx, ens, ctypes.byref(fld), _ptr(d_rho),
                                 d_rho.numel(), _ptr(d_T), d_T.numel(),
                                 int(spin), int(precision), _ptr(d_mean),
                                 _ptr(d_err), _ptr(d_group_sums)), ctx)


def wl_average_async_noalloc(ctx, ens, fld, d_rho, d_T, spin, precision, d_mean,
                             d_err, d_group_sums):
    """As wl_average_async, through the allocation-free entry point (partial
    sums in the library's static device scratch)."""
    _check(_lib.wl_average_async_noalloc(ctx, ens, ctypes.byref(fld), _ptr(d_rho),
                                         d_rho.numel(), _ptr(d_T), d_T.numel(),
                                         int(spin), int(precision), _ptr(d_mean),
                                         _ptr(d_err), _ptr(d_group_sums)), ctx)


def _request(q, G, keep):
    rho = _host_f64(q["rho"])
    T = _host_f64(q["T"])
    out = _result_arrays(G, rho.size, T.size)
    keep += [rho, T]
    req = wl_request(field(q["kind"], q["eB0"], q.get("lam", 1.0)), _ptr(rho), _ptr(T),
                     rho.size, T.size, int(q["spin"]), int(q.get("precision", WL_FP32C)),
                     *[_ptr(out[k]) for k in RESULT_KEYS])
    return req, out


def wl_average_batch(ctx, ens, requests, full=False):
    """Batched evaluation.  requests: list of dicts with keys kind, eB0, lam,
    rho, T, spin, precision.  Returns a list of (mean, err, group_sums), or
    with full=True of dicts with every output of wl_result."""
    _, _, G = wl_ensemble_info(ens)
    arr = (wl_request * max(1, len(requests)))()
    keep, outs = [], []
    for i, q in enumerate(requests):
        arr[i], out = _request(q, G, keep)
        outs.append(out)
    _check(_lib.wl_average_batch(ctx, ens, arr, len(requests)), ctx)
    if full:
        return outs
    return [(o["mean"], o["err"], o["group_sums"]) for o in outs]


class Server:
    """Continuous-batching server (wl_server_*).  submit() keeps the request's
    numpy outputs alive until the ticket is released."""

    def __init__(self, ctx, ens, slots=2, max_batch=1024, input_bytes=8 << 20,
                 result_bytes=512 << 20, in_order=False):
        self.ctx, self.ens = ctx, ens
        self.G = wl_ensemble_info(ens)[2]
        cfg = wl_server_config(slots, max_batch, input_bytes, result_bytes, int(in_order))
        self.h = _vp()
        _check(_lib.wl_server_create(ctx, ens, ctypes.byref(cfg), ctypes.byref(self.h)), ctx)
        self._live = {}

    def _check(self, rc):
        if rc != WL_OK:
            raise WLError(rc, _lib.wl_server_last_error(self.h).decode() or wl_strerror(rc))

    def submit(self, q):
        """q: dict with kind, eB0, lam, rho, T, spin, precision.  Returns a
        ticket; outputs via result()."""
        keep = []
        req, out = _request(q, self.G, keep)
        t = _i64()
        self._check(_lib.wl_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = out
        return t.value

    def poll(self, ticket):
        st, lat = _i32(), _d()
        self._check(_lib.wl_server_poll(self.h, ticket, ctypes.byref(st), ctypes.byref(lat)))
        return st.value, lat.value

    def wait(self, ticket, timeout_s=-1.0):
        st, lat = _i32(), _d()
        self._check(_lib.wl_server_wait(self.h, ticket, float(timeout_s), ctypes.byref(st),
                                        ctypes.byref(lat)))
        return st.value, lat.value

    def timing(self, ticket):
        """(queue_ms, service_ms) of a finished ticket: submission to its
        batch's launch, launch to completion (-1, -1 if it did not run)."""
        q, sv = _d(), _d()
        self._check(_lib.wl_server_timing(self.h, ticket, ctypes.byref(q), ctypes.byref(sv)))
        return q.value, sv.value

    def result(self, ticket, release=True, full=False):
        """(mean, err, group_sums) of a finished ticket, or with full=True the
        dict of every output of wl_result."""
        out = self._live[ticket]
        if release:
            self._check(_lib.wl_server_release(self.h, ticket))
            del self._live[ticket]
        if full:
            return out
        return out["mean"], out["err"], out["group_sums"]

    def info(self):
        a, b, c = _i64(), _i64(), _i64()
        self._check(_lib.wl_server_info(self.h, ctypes.byref(a), ctypes.byref(b),
                                        ctypes.byref(c)))
        return {"pending": a.value, "running": b.value, "batches": c.value}

    def close(self):
        if self.h:
            _lib.wl_server_destroy(self.h)
            self.h = None


def wl_per_loop(ctx, ens, fld, rho, T, spin, precision, loop0, n_loops):
    """Per-loop (phase, spin exponent, w), each (n_loops, n_rho, n_T)."""
    rho = _host_f64(rho)
    T = _host_f64(T)
    shape = (n_loops, rho.size, T.size)
    ph, sp, w = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    _check(_lib.wl_per_loop(ctx, ens, ctypes.byref(fld), _ptr(rho), rho.size,
                            _ptr(T), T.size, int(spin), int(precision),
                            int(loop0), int(n_loops), _ptr(ph), _ptr(sp),
                            _ptr(w)), ctx)
    return ph, sp, w


def wl_set_timing(ctx, enable=True):
    _check(_lib.wl_set_timing(ctx, int(bool(enable))), ctx)


def wl_last_kernel_ms(ctx):
    ms = _d()
    _check(_lib.wl_last_kernel_ms(ctx, ctypes.byref(ms)), ctx)
    return ms.value


def wl_kernel_ms_total(ctx):
    """(sum of recorded main-kernel durations in ms, number of launches)."""
    ms = _d()
    n = _i64()
    _check(_lib.wl_kernel_ms_total(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def _torch():
    import torch
    return torch


def raw_function(name):
    """The ctypes function object of an exported symbol."""
    return getattr(_lib, name)
