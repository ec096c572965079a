"""ctypes binding of the serving loop (include/md_server.h): argument
marshalling only; admission, batching and completion run in the library's
scheduler thread."""
import ctypes

import numpy as np

from . import _lib

_DTN = {np.dtype(np.float32): "s", np.dtype(np.float64): "d", np.dtype(np.complex64): "c",
        np.dtype(np.complex128): "z", np.dtype(np.float16): "h"}


def _dt_name(X):
    from .inputs import HALF_COMPLEX
    return "hc" if X.dtype == HALF_COMPLEX else _DTN[X.dtype]


class MdServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("slots", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("big_flops", ctypes.c_double), ("big_lanes", ctypes.c_int)]


class MdRequest(ctypes.Structure):
    _fields_ = [("transa", ctypes.c_char), ("transb", ctypes.c_char),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("alpha", _lib.MdScalar), ("a", ctypes.c_int64), ("b", ctypes.c_int64),
                ("beta", _lib.MdScalar), ("c_in", ctypes.c_int64),
                ("dtc", ctypes.c_int), ("comp", ctypes.c_int), ("keep_output", ctypes.c_int)]


class MdResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("done", ctypes.c_int),
                ("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double), ("output", ctypes.c_int64),
                ("batch_size", ctypes.c_int), ("flops", ctypes.c_double)]


class MdServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("refused", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("grouped_launches", ctypes.c_int64), ("plain_launches", ctypes.c_int64),
                ("inflight_bytes", ctypes.c_int64), ("peak_inflight_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("pool_bytes", ctypes.c_int64), ("device_mallocs", ctypes.c_int64),
                ("max_concurrent_batches", ctypes.c_int)]


def _bind():
    L = _lib.lib()
    if getattr(L, "_md_server_bound", False):
        return L
    vp, i64, ci, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.md_server_create.argtypes = [ctypes.POINTER(MdServerConfig), ctypes.POINTER(vp)]
    L.md_server_destroy.argtypes = [vp]
    L.md_server_put.argtypes = [vp, vp, ci, i64, i64, ctypes.POINTER(i64)]
    L.md_server_drop.argtypes = [vp, i64]
    L.md_server_fetch.argtypes = [vp, i64, vp]
    L.md_server_submit.argtypes = [vp, ctypes.POINTER(MdRequest), ctypes.POINTER(i64)]
    L.md_server_poll.argtypes = [vp, i64, ctypes.POINTER(MdResult)]
    L.md_server_wait.argtypes = [vp, i64, ctypes.POINTER(MdResult), dbl]
    L.md_server_forget.argtypes = [vp, i64]
    L.md_server_stats.argtypes = [vp, ctypes.POINTER(MdServerStats)]
    for f in ("create", "destroy", "put", "drop", "fetch", "submit", "poll", "wait", "forget", "stats"):
        getattr(L, "md_server_" + f).restype = ci
    L._md_server_bound = True
    return L


class ServerError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed with status %d" % (what, status))


class Server:
    """Continuous-batching request loop over mdgemm on the current device."""

    def __init__(self, budget_bytes, slots=4, max_batch=64, big_flops=2e9, big_lanes=1):
        self.L = _bind()
        self.h = None
        cfg = MdServerConfig(int(budget_bytes), slots, max_batch, float(big_flops), big_lanes)
        h = ctypes.c_void_p()
        st = self.L.md_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != 0:
            raise ServerError(st, "md_server_create")
        self.h = h

    def close(self):
        if self.h:
            self.L.md_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def put(self, X, rows=None, cols=None):
        """Upload a column-major numpy matrix (shape (rows, cols)); returns a handle."""
        X = np.asfortranarray(X)
        rows = X.shape[0] if rows is None else rows
        cols = X.shape[1] if cols is None else cols
        h = ctypes.c_int64()
        st = self.L.md_server_put(self.h, X.ctypes.data, _lib.tag(_dt_name(X)), rows, cols, ctypes.byref(h))
        if st != 0:
            raise ServerError(st, "md_server_put")
        return h.value

    def drop(self, handle):
        return self.L.md_server_drop(self.h, handle)

    def fetch(self, handle, rows, cols, dt):
        from .inputs import NP_DTYPE
        out = np.empty((rows, cols), dtype=NP_DTYPE[dt], order="F")
        st = self.L.md_server_fetch(self.h, handle, out.ctypes.data)
        if st != 0:
            raise ServerError(st, "md_server_fetch")
        return out

    def submit(self, transa, transb, m, n, k, alpha, a, b, beta, c_in, dtc, comp=None, keep_output=False):
        r = MdRequest(transa.encode(), transb.encode(), m, n, k, _lib.scalar(alpha), a, b, _lib.scalar(beta),
                      -1 if c_in is None else c_in, _lib.tag(dtc), _lib.comp_tag(comp), 1 if keep_output else 0)
        t = ctypes.c_int64()
        st = self.L.md_server_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        return st, t.value

    def poll(self, ticket):
        r = MdResult()
        st = self.L.md_server_poll(self.h, ticket, ctypes.byref(r))
        return st, r

    def wait(self, ticket, timeout=60.0):
        r = MdResult()
        st = self.L.md_server_wait(self.h, ticket, ctypes.byref(r), timeout)
        return st, r

    def forget(self, ticket):
        return self.L.md_server_forget(self.h, ticket)

    def stats(self):
        s = MdServerStats()
        self.L.md_server_stats(self.h, ctypes.byref(s))
        return {f[0]: getattr(s, f[0]) for f in MdServerStats._fields_}
