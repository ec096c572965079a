"""Oracle for mixed-datatype GEMM -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU evaluation of C := beta*C + alpha*op(A)*op(B) for operands
independently stored as s/d/c/z (Van Zee, Parikh, van de Geijn: Section 1 for
the operation, Figure "mixeddom" for the domain cases, Section 7 for scalars).
The arithmetic lives in ``md_oracle.c``; this module only marshals numpy
buffers into it.  Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the GPU library never does.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "libmdoracle.so")

OK = 0
ERR_ALPHA_IMAG = 1
ERR_ARG = -1

CASE_NAMES = ("0", "1b", "1a", "2ab", "1c", "2bc", "2ac", "3")

_TAG = {"s": 0, "d": 1, "c": 2, "z": 3, "h": 4, "hc": 5}


def build(src=_SRC, out=_LIB):
    """Compile the oracle with plain gcc -O2 (no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", src, "-o", out, "-lm"]
    subprocess.check_call(cmd)
    return out


def tag(dt):
    """Storage tag 0..5 from 's','d','c','z','h','hc' or an int."""
    return _TAG[dt] if isinstance(dt, str) else int(dt)


class Oracle:
    """ctypes handle on one compiled copy of the oracle."""

    def __init__(self, path=_LIB):
        if path == _LIB and (not os.path.exists(path)
                             or os.path.getmtime(path) < os.path.getmtime(_SRC)):
            build(out=path)
        self.path = path
        lib = ctypes.CDLL(path)
        i64, dbl, vp, ci, cc = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int, ctypes.c_char
        common = [cc, cc, i64, i64, i64, dbl, dbl, vp, ci, i64, vp, ci, i64, dbl, dbl, vp, ci, i64]
        lib.md_oracle_gemm.argtypes = common + [vp, vp]
        lib.md_oracle_gemm.restype = ci
        lib.md_oracle_gemm_literal.argtypes = common + [vp, vp]
        lib.md_oracle_gemm_literal.restype = ci
        lib.md_oracle_gemm_at.argtypes = common + [i64, vp, vp, vp, vp]
        lib.md_oracle_gemm_at.restype = ci
        lib.md_oracle_gemm_gs.argtypes = [cc, cc, i64, i64, i64, dbl, dbl, vp, ci, i64, i64, vp, ci, i64, i64,
                                          dbl, dbl, vp, ci, i64, i64, vp, vp]
        lib.md_oracle_gemm_gs.restype = ci
        lib.md_oracle_case.argtypes = [ci, ci, ci]
        lib.md_oracle_case.restype = ci
        lib.md_oracle_flops.argtypes = [ci, ci, ci, i64, i64, i64]
        lib.md_oracle_flops.restype = dbl
        self.lib = lib

    def case(self, dtc, dta, dtb):
        return CASE_NAMES[self.lib.md_oracle_case(tag(dtc), tag(dta), tag(dtb))]

    def flops(self, dtc, dta, dtb, m, n, k):
        return self.lib.md_oracle_flops(tag(dtc), tag(dta), tag(dtb), m, n, k)

    @staticmethod
    def _args(transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb, beta, C, dtc, ldc):
        alpha = complex(alpha)
        beta = complex(beta)

        def ptr(X):
            if X is None:
                return None
            assert X.flags["F_CONTIGUOUS"] or X.flags["C_CONTIGUOUS"]
            return X.ctypes.data

        return (transa.encode() if isinstance(transa, str) else transa,
                transb.encode() if isinstance(transb, str) else transb,
                m, n, k, alpha.real, alpha.imag,
                ptr(A), tag(dta), lda, ptr(B), tag(dtb), ldb,
                beta.real, beta.imag, ptr(C), tag(dtc), ldc)

    def gemm(self, transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb,
             beta, C, dtc, ldc, want_bound=True, literal_alpha=False):
        """Full reference.  Returns (status, cref complex128 (m, n), g float64 (m, n)).
        literal_alpha: apply a complex alpha as given in every case (the literal
        interpretation of Section 7.2) instead of refusing it in the mixed cases."""
        cref = np.zeros((max(m, 0), max(n, 0)), dtype=np.complex128, order="F")
        g = np.zeros((max(m, 0), max(n, 0)), dtype=np.float64, order="F") if want_bound else None
        fn = self.lib.md_oracle_gemm_literal if literal_alpha else self.lib.md_oracle_gemm
        st = fn(*self._args(transa, transb, m, n, k, alpha, A, dta, lda,
                                                 B, dtb, ldb, beta, C, dtc, ldc),
                                     cref.ctypes.data, g.ctypes.data if g is not None else None)
        return st, cref, g

    def gemm_at(self, transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb,
                beta, C, dtc, ldc, rows, cols):
        """The definition at selected entries.  Returns (status, values complex128, g)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.zeros(rows.shape[0], dtype=np.complex128)
        g = np.zeros(rows.shape[0], dtype=np.float64)
        st = self.lib.md_oracle_gemm_at(*self._args(transa, transb, m, n, k, alpha, A, dta, lda,
                                                    B, dtb, ldb, beta, C, dtc, ldc),
                                        rows.shape[0], rows.ctypes.data, cols.ctypes.data,
                                        out.ctypes.data, g.ctypes.data)
        return st, out, g


    def gemm_gs(self, transa, transb, m, n, k, alpha, A, dta, rsa, csa, B, dtb, rsb, csb,
                beta, C, dtc, rsc, csc, want_bound=True):
        """The definition with row/column strides (elements) for every operand:
        A, B, C are flat numpy buffers of their storage type.  Returns (status,
        cref complex128 (m, n), g float64 (m, n))."""
        alpha, beta = complex(alpha), complex(beta)
        cref = np.zeros((max(m, 0), max(n, 0)), dtype=np.complex128, order="F")
        g = np.zeros((max(m, 0), max(n, 0)), dtype=np.float64, order="F") if want_bound else None
        ptr = lambda X: None if X is None else X.ctypes.data
        st = self.lib.md_oracle_gemm_gs(transa.encode(), transb.encode(), m, n, k, alpha.real, alpha.imag,
                                        ptr(A), tag(dta), rsa, csa, ptr(B), tag(dtb), rsb, csb,
                                        beta.real, beta.imag, ptr(C), tag(dtc), rsc, csc,
                                        cref.ctypes.data, g.ctypes.data if g is not None else None)
        return st, cref, g


_default = None


def get():
    """The oracle built from this directory's source (compiled on first use)."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
