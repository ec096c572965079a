"""Torch-facing wrappers over the C ABI (marshalling only).

``gemm`` takes 2-D torch tensors stored by columns (``stride(0) == 1``) or by
rows (``stride(1) == 1``, torch's default) and passes their row and column
strides to ``mdgemm_strided`` (the strided interface sketched in Section 3 of
the paper).  ``plan`` and grouped calls take column-major tensors, the BLAS
layout of Section 1 (leading dimension ``stride(1)``); ``colmajor`` makes one.
The storage type follows the tensor dtype: float32 -> s, float64 -> d,
complex64 -> c, complex128 -> z, float16 -> h, complex32 -> hc (binary16).  op is one of N, T, C (conjugate transpose)
and R (conjugate without transposing).
"""
import torch

from . import _lib

_DT = {torch.float32: "s", torch.float64: "d", torch.complex64: "c", torch.complex128: "z",
       torch.float16: "h", torch.complex32: "hc"}
_TORCH = {v: k for k, v in _DT.items()}


class MdgemmError(RuntimeError):
    def __init__(self, status, msg=None):
        self.status = status
        super().__init__(msg or "mdgemm failed with status %d (%s)" % (status, _lib.strerror(status)))


def dt_of(t):
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError("unsupported dtype %s (use float32/float64/complex64/complex128/float16/complex32)"
                        % t.dtype)


def torch_dtype(dt):
    return _TORCH[dt]


def colmajor(rows, cols, dt, device="cuda", ld=None):
    """A zero-initialised column-major (rows x cols) tensor with leading dimension ld."""
    ld = max(1, rows) if ld is None else ld
    return torch.zeros((max(cols, 1), ld), dtype=_TORCH[dt], device=device).t()[:rows, :cols]


def _layout(t, name):
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    rows, cols = t.shape
    if rows > 1 and t.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1)" % name)
    ld = t.stride(1) if cols > 1 else max(1, rows)
    return t.data_ptr(), dt_of(t), max(ld, 1), rows, cols


def _dims(A, B, C, transa, transb):
    m, n = C.shape
    a_plain, b_plain = transa.upper() in ("N", "R"), transb.upper() in ("N", "R")
    k = A.shape[1] if a_plain else A.shape[0]
    am = A.shape[0] if a_plain else A.shape[1]
    bk, bn = (B.shape[0], B.shape[1]) if b_plain else (B.shape[1], B.shape[0])
    if am != m or bn != n or bk != k:
        raise ValueError("shape mismatch: op(A) %dx%d, op(B) %dx%d, C %dx%d" % (am, k, bk, bn, m, n))
    return m, n, k


def _args(A, B, C, alpha, beta, transa, transb, comp):
    m, n, k = _dims(A, B, C, transa, transb)
    pa, dta, lda, _, _ = _layout(A, "A")
    pb, dtb, ldb, _, _ = _layout(B, "B")
    pc, dtc, ldc, _, _ = _layout(C, "C")
    return (transa, transb, m, n, k, alpha, pa, dta, lda, pb, dtb, ldb, beta, pc, dtc, ldc, comp)


def _strides(t, name):
    """(pointer, type, row stride, column stride); a stride along an extent of
    at most one element is never used and is passed as 1."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    rows, cols = t.shape
    rs = t.stride(0) if rows > 1 else 1
    cs = t.stride(1) if cols > 1 else 1
    return t.data_ptr(), dt_of(t), rs, cs


def gemm(A, B, C, alpha=1.0, beta=0.0, transa="N", transb="N", comp=None, stream=None,
         literal_alpha=False):
    """C := beta*C + alpha*op(A)*op(B) on the GPU, enqueued on `stream` (default:
    torch's current stream for C's device).  Each tensor may be stored by rows
    or by columns.  `comp` is None (C's precision), "s", "d" or "bf16x3".
    literal_alpha: apply a complex alpha as given in the mixed-domain cases
    (the literal interpretation of Section 7.2) instead of refusing it.
    Returns C."""
    if literal_alpha and not (isinstance(comp, str) and comp.endswith("+literal")):
        if comp is None:
            comp = ("d" if C.dtype in (torch.float64, torch.complex128)
                    else "h" if C.dtype in (torch.float16, torch.complex32) else "s")
        comp = comp + "+literal"
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        if not t.is_cuda:
            raise ValueError("%s must be a device tensor" % nm)
    if stream is None:
        stream = torch.cuda.current_stream(C.device).cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    pa, dta, rsa, csa = _strides(A, "A")
    pb, dtb, rsb, csb = _strides(B, "B")
    pc, dtc, rsc, csc = _strides(C, "C")
    m, n, k = _dims(A, B, C, transa, transb)
    st = _lib.mdgemm_strided(transa, transb, m, n, k, alpha, pa, dta, rsa, csa, pb, dtb, rsb, csb,
                             beta, pc, dtc, rsc, csc, comp, stream=stream)
    if st != 0:
        raise MdgemmError(st)
    return C


def plan(A, B, C, alpha=1.0, beta=0.0, transa="N", transb="N", comp=None):
    """What gemm() would do (host only; tensors may live anywhere)."""
    st, d = _lib.mdgemm_plan(*_args(A, B, C, alpha, beta, transa, transb, comp))
    return d


class GroupedCall:
    """One product of a grouped launch (same arguments as gemm())."""

    def __init__(self, A, B, C, alpha=1.0, beta=0.0, transa="N", transb="N", comp=None):
        self.args = _args(A, B, C, alpha, beta, transa, transb, comp)
        self.tensors = (A, B, C)

    def desc(self):
        return _lib.make_desc(*self.args)


def grouped(calls, stream=None):
    """Enqueue many products as one persistent kernel launch."""
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    st = _lib.mdgemm_grouped([c.desc() for c in calls], stream)
    if st != 0:
        raise MdgemmError(st)
