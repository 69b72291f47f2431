"""ctypes binding of libwilson.so (include/wilson.h): same names, argument marshalling only.

Arrays may be torch tensors (CPU or GPU) or numpy arrays holding complex128 (or the
equivalent float64 pairs) in the canonical layout; their data pointers are passed
through unchanged.  Every computation happens in the HIP library; if the library has
not been built this module raises ImportError instead of falling back to anything.

torch is imported before the library is loaded so that the process holds one HIP
runtime: libwilson.so's dependency on libamdhip64.so.7 then resolves to the runtime
torch already loaded, and torch streams and allocations are valid in library calls.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must be loaded first; see module docstring)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwilson.so")

WILSON_OK = 0
WILSON_NOT_CONVERGED = 1
WILSON_INVALID_ARG = -1
WILSON_OUT_OF_MEMORY = -2
WILSON_DEVICE_ERROR = -3
WILSON_BREAKDOWN = -4
WILSON_NONFINITE = -5
WILSON_REJECTED = -6
WILSON_BUSY = -7

WILSON_FP64, WILSON_FP32, WILSON_FP16, WILSON_FP16_L32 = 0, 1, 2, 3
WILSON_GAUGE_FP64, WILSON_GAUGE_FP32, WILSON_GAUGE_FP16 = 1, 2, 4
WILSON_SOLVER_BICGSTAB_EO, WILSON_SOLVER_CGNR_EO, WILSON_SOLVER_BLOCK_BICGSTAB_EO = 0, 1, 2
WILSON_KERNEL_HOP, WILSON_KERNEL_BLAS = 0, 1
WILSON_LAYOUT_SOA, WILSON_LAYOUT_AOS, WILSON_LAYOUT_AOSOA, WILSON_LAYOUT_VNODE = 0, 1, 2, 3

EXPORTS = [
    "wilson_dslash", "wilson_solve", "wilson_context_create", "wilson_context_destroy", "wilson_gauge_load",
    "wilson_gauge_free", "wilson_gauge_bytes", "wilson_dslash_ex", "wilson_solve_ex", "wilson_footprint_bytes",
    "wilson_batch_create", "wilson_batch_destroy", "wilson_batch_attach", "wilson_batch_step", "wilson_batch_poll",
    "wilson_batch_detach", "wilson_timing_enable", "wilson_timing_read", "wilson_stream_copy", "wilson_strerror",
    "wilson_last_error", "wilson_version", "wilson_stream_read", "wilson_gauge_attach_clover",
    "wilson_gauge_detach_clover", "wilson_layout_hop", "wilson_solve_noalloc", "wilson_gauge_footprint_bytes",
    "wilson_index_check",
]


class wilson_solve_opts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("precision", ctypes.c_int32), ("maxiter", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int32),
                ("poll_every", ctypes.c_int32), ("mixed_update", ctypes.c_int32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class wilson_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer_cycles", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("true_residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("hop_launches", ctypes.c_double), ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_d = ctypes.c_double
_SIGS = {
    "wilson_dslash": (_i32, [_vp, _vp, _vp, _d, _vp, _i32]),
    "wilson_solve": (_i32, [_vp, _vp, _vp, _d, _vp, _d, _i32]),
    "wilson_context_create": (_i32, [ctypes.POINTER(_vp), _vp]),
    "wilson_context_destroy": (_i32, [_vp]),
    "wilson_gauge_load": (_i32, [_vp, ctypes.POINTER(_vp), _vp, _vp, ctypes.c_uint32]),
    "wilson_gauge_free": (_i32, [_vp, _vp]),
    "wilson_gauge_bytes": (ctypes.c_size_t, [_vp]),
    "wilson_gauge_footprint_bytes": (ctypes.c_size_t, [_vp, ctypes.c_uint32, _i32]),
    "wilson_index_check": (_i32, [_vp]),
    "wilson_gauge_attach_clover": (_i32, [_vp, _vp, _vp]),
    "wilson_gauge_detach_clover": (_i32, [_vp, _vp]),
    "wilson_dslash_ex": (_i32, [_vp, _vp, _vp, _vp, _d, _i32, _i32, _i32]),
    "wilson_solve_ex": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(wilson_solve_opts),
                               ctypes.POINTER(wilson_solve_info)]),
    "wilson_solve_noalloc": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(wilson_solve_opts),
                                    ctypes.POINTER(wilson_solve_info)]),
    "wilson_footprint_bytes": (ctypes.c_size_t, [_vp, _i32, ctypes.POINTER(wilson_solve_opts)]),
    "wilson_batch_create": (_i32, [_vp, _vp, _i32, ctypes.POINTER(wilson_solve_opts), ctypes.POINTER(_vp)]),
    "wilson_batch_destroy": (_i32, [_vp]),
    "wilson_batch_attach": (_i32, [_vp, _i32, _vp, _d, _d, _i32]),
    "wilson_batch_step": (_i32, [_vp, _i32]),
    "wilson_batch_poll": (_i32, [_vp, _vp, _vp]),
    "wilson_batch_detach": (_i32, [_vp, _i32, _vp, ctypes.POINTER(wilson_solve_info)]),
    "wilson_timing_enable": (_i32, [_vp, _i32]),
    "wilson_timing_read": (_i32, [_vp, _i32, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(_d)]),
    "wilson_stream_copy": (_i32, [_vp, _vp, _vp, ctypes.c_size_t]),
    "wilson_stream_read": (_i32, [_vp, _vp, ctypes.c_size_t]),
    "wilson_layout_hop": (_i32, [_vp, _vp, _vp, _vp, _vp, _d, _i32, _i32, _i32, _i32, _i32, ctypes.POINTER(_d)]),
    "wilson_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "wilson_last_error": (ctypes.c_char_p, []),
    "wilson_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libwilson.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(handle, name)
            f.restype = res
            f.argtypes = args
        _lib = handle
    return _lib


class WilsonError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = lib().wilson_strerror(code).decode()
        detail = lib().wilson_last_error().decode()
        super().__init__(f"{where}: {msg} ({code}); {detail}")


def check(code, where=""):
    if code < 0:
        raise WilsonError(code, where)
    return code


# ---- marshalling helpers ----
def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        assert a.is_contiguous(), "tensor must be contiguous"
        return ctypes.c_void_p(a.data_ptr())
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
        return ctypes.c_void_p(a.ctypes.data)
    raise TypeError(f"unsupported array type {type(a)}")


def _nbytes(a):
    if isinstance(a, torch.Tensor):
        return a.numel() * a.element_size()
    return a.nbytes


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,)
    return d


def _check_size(a, dims, nrhs, what, per_site=24):
    need = per_site * 8 * int(np.prod(dims)) * nrhs
    if _nbytes(a) != need:
        raise ValueError(f"{what}: expected {need} bytes, got {_nbytes(a)}")


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _opts(opts):
    if opts is None:
        return None
    o = wilson_solve_opts()
    o.solver = int(opts.get("solver", WILSON_SOLVER_BICGSTAB_EO))
    o.precision = int(opts.get("precision", WILSON_FP64))
    o.maxiter = int(opts.get("maxiter", 10000))
    o.max_restarts = int(opts.get("max_restarts", -1))
    o.inner_tol = float(opts.get("inner_tol", 0.0))
    o.use_x0 = int(bool(opts.get("use_x0", False)))
    o.poll_every = int(opts.get("poll_every", 0))
    o.mixed_update = int(opts.get("mixed_update", 0))
    ws = opts.get("workspace")
    if ws is not None:  # a device tensor (its storage) or a raw address
        o.workspace = ws.data_ptr() if isinstance(ws, torch.Tensor) else int(ws)
        o.workspace_bytes = int(opts.get("workspace_bytes", _nbytes(ws) if isinstance(ws, torch.Tensor) else 0))
    return ctypes.byref(o)


# ---- entry points (same names as the C ABI) ----
def wilson_version():
    return lib().wilson_version().decode()


def wilson_strerror(code):
    return lib().wilson_strerror(code).decode()


def wilson_last_error():
    return lib().wilson_last_error().decode()


def wilson_dslash(out, in_, U, kappa, dims, parity):
    d = _dims(dims)
    _check_size(out, d, 1, "out"); _check_size(in_, d, 1, "in"); _check_size(U, d, 1, "U", per_site=72)
    return lib().wilson_dslash(_ptr(out), _ptr(in_), _ptr(U), float(kappa), d.ctypes.data, int(parity))


def wilson_solve(x, b, U, kappa, dims, tol, maxiter):
    d = _dims(dims)
    _check_size(x, d, 1, "x"); _check_size(b, d, 1, "b"); _check_size(U, d, 1, "U", per_site=72)
    return lib().wilson_solve(_ptr(x), _ptr(b), _ptr(U), float(kappa), d.ctypes.data, float(tol), int(maxiter))


def wilson_context_create(stream=None):
    h = ctypes.c_void_p()
    check(lib().wilson_context_create(ctypes.byref(h), _stream_handle(stream)), "wilson_context_create")
    return h


def wilson_context_destroy(ctx):
    return check(lib().wilson_context_destroy(ctx), "wilson_context_destroy")


def wilson_gauge_load(ctx, U, dims, precisions=WILSON_GAUGE_FP64):
    d = _dims(dims)
    _check_size(U, d, 1, "U", per_site=72)
    h = ctypes.c_void_p()
    check(lib().wilson_gauge_load(ctx, ctypes.byref(h), _ptr(U), d.ctypes.data, int(precisions)),
          "wilson_gauge_load")
    return h


def wilson_gauge_free(ctx, g):
    return check(lib().wilson_gauge_free(ctx, g), "wilson_gauge_free")


def wilson_gauge_bytes(g):
    return int(lib().wilson_gauge_bytes(g))


def wilson_index_check(dims):
    """Host replay of the kernels' site indexing on one lattice: 0, a negative error code,
    or the number of violations (the first in wilson_last_error())."""
    if dims is None:
        return int(lib().wilson_index_check(None))
    d = np.ascontiguousarray(dims, dtype=np.int32)
    return int(lib().wilson_index_check(d.ctypes.data))


def wilson_gauge_footprint_bytes(dims, precisions=WILSON_GAUGE_FP64, link_reals=18):
    d = _dims(dims)
    return int(lib().wilson_gauge_footprint_bytes(d.ctypes.data, int(precisions), int(link_reals)))


def wilson_gauge_attach_clover(ctx, g, F, dims):
    """Attach the clover term F (V x 12 x 12 complex128, canonical) to gauge field g."""
    _check_size(F, _dims(dims), 1, "F", per_site=288)
    return lib().wilson_gauge_attach_clover(ctx, g, _ptr(F))


def wilson_gauge_detach_clover(ctx, g):
    return check(lib().wilson_gauge_detach_clover(ctx, g), "wilson_gauge_detach_clover")


def wilson_dslash_ex(ctx, g, out, in_, kappa, parity, precision=WILSON_FP64, nrhs=1):
    return lib().wilson_dslash_ex(ctx, g, _ptr(out), _ptr(in_), float(kappa), int(parity), int(precision), int(nrhs))


def wilson_layout_hop(ctx, out, in_, U, dims, kappa, parity, precision, layout, link_reals=18, reps=0):
    """Returns (status, mean microseconds of the `reps` timed launches)."""
    d = _dims(dims)
    _check_size(out, d, 1, "out"); _check_size(in_, d, 1, "in"); _check_size(U, d, 1, "U", per_site=72)
    us = ctypes.c_double(0.0)
    st = lib().wilson_layout_hop(ctx, _ptr(out), _ptr(in_), _ptr(U), d.ctypes.data, float(kappa), int(parity),
                                 int(precision), int(layout), int(link_reals), int(reps), ctypes.byref(us))
    return st, us.value


def wilson_solve_ex(ctx, g, x, b, nrhs, kappa, tol, opts=None):
    """Returns (status, [info dict per RHS])."""
    kap = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, np.float64), (nrhs,)))
    tl = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, np.float64), (nrhs,)))
    infos = (wilson_solve_info * nrhs)()
    st = lib().wilson_solve_ex(ctx, g, _ptr(x), _ptr(b), int(nrhs), kap.ctypes.data, tl.ctypes.data, _opts(opts),
                               infos)
    return st, [i.as_dict() for i in infos]


def wilson_solve_noalloc(ctx, g, x, b, nrhs, kappa, tol, opts=None):
    """wilson_solve_ex without device allocations (x, b device tensors).  Returns
    (status, [info dict per RHS])."""
    kap = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, np.float64), (nrhs,)))
    tl = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, np.float64), (nrhs,)))
    infos = (wilson_solve_info * nrhs)()
    st = lib().wilson_solve_noalloc(ctx, g, _ptr(x), _ptr(b), int(nrhs), kap.ctypes.data, tl.ctypes.data,
                                    _opts(opts), infos)
    return st, [i.as_dict() for i in infos]


def wilson_footprint_bytes(dims, nrhs, opts=None):
    d = _dims(dims)
    return int(lib().wilson_footprint_bytes(d.ctypes.data, int(nrhs), _opts(opts)))


def wilson_batch_create(ctx, g, nslots, opts=None):
    h = ctypes.c_void_p()
    check(lib().wilson_batch_create(ctx, g, int(nslots), _opts(opts), ctypes.byref(h)), "wilson_batch_create")
    return h


def wilson_batch_destroy(batch):
    return check(lib().wilson_batch_destroy(batch), "wilson_batch_destroy")


def wilson_batch_attach(batch, slot, b, kappa, tol, maxiter=10000):
    return lib().wilson_batch_attach(batch, int(slot), _ptr(b), float(kappa), float(tol), int(maxiter))


def wilson_batch_step(batch, iters):
    return check(lib().wilson_batch_step(batch, int(iters)), "wilson_batch_step")


def wilson_batch_poll(batch, nslots):
    state = np.zeros(nslots, np.int32)
    status = np.zeros(nslots, np.int32)
    check(lib().wilson_batch_poll(batch, state.ctypes.data, status.ctypes.data), "wilson_batch_poll")
    return state, status


def wilson_batch_detach(batch, slot, x):
    info = wilson_solve_info()
    st = lib().wilson_batch_detach(batch, int(slot), _ptr(x), ctypes.byref(info))
    return st, info.as_dict()


def wilson_timing_enable(ctx, enable=True):
    return check(lib().wilson_timing_enable(ctx, int(bool(enable))), "wilson_timing_enable")


def wilson_timing_read(ctx, kernel_class=WILSON_KERNEL_HOP):
    ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    check(lib().wilson_timing_read(ctx, int(kernel_class), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
          "wilson_timing_read")
    return ms.value, n.value, b.value


def wilson_stream_copy(ctx, dst, src, nbytes):
    return check(lib().wilson_stream_copy(ctx, _ptr(dst), _ptr(src), int(nbytes)), "wilson_stream_copy")


def wilson_stream_read(ctx, src, nbytes):
    return check(lib().wilson_stream_read(ctx, _ptr(src), int(nbytes)), "wilson_stream_read")
