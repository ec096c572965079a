"""ctypes binding of libmdgemm (argument marshalling only).

The names follow the C ABI in include/mdgemm.h.  Torch tensors provide device
pointers, storage types, leading dimensions and the current stream; every
step of the computation runs in the library's HIP kernels.  If the library
has not been built this module raises -- there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MDGEMM_LIBRARY may name another build of the same library (for example one
# compiled with different tuning knobs).
LIB_PATH = os.environ.get("MDGEMM_LIBRARY", os.path.join(HERE, "libmdgemm.so"))

MD_S, MD_D, MD_C, MD_Z, MD_H, MD_HC = 0, 1, 2, 3, 4, 5
MD_COMP_DEFAULT, MD_COMP_S, MD_COMP_D, MD_COMP_S_BF16X3, MD_COMP_H = -1, 0, 1, 2, 3
MD_OK, MD_ERR_ALPHA_IMAG, MD_ERR_HIP, MD_ERR_BUDGET, MD_ERR_STATE, MD_ERR_UNSUPPORTED = 0, 1, 2, 3, 4, 5
MD_ERR_SCRATCH = 6
MD_GROUPED_NOALLOC_BYTES = 8 << 20
CASE_NAMES = ("0", "1a", "1b", "1c", "2ab", "2ac", "2bc", "3")
DT_TAG = {"s": MD_S, "d": MD_D, "c": MD_C, "z": MD_Z, "h": MD_H, "hc": MD_HC}
COMP_TAG = {None: MD_COMP_DEFAULT, "default": MD_COMP_DEFAULT, "s": MD_COMP_S, "d": MD_COMP_D,
            "bf16x3": MD_COMP_S_BF16X3, "h": MD_COMP_H}


class MdScalar(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class MdPlan(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("domain_case", ctypes.c_int), ("comp", ctypes.c_int),
                ("quick", ctypes.c_int), ("flops", ctypes.c_double),
                ("m_real", ctypes.c_int64), ("n_real", ctypes.c_int64), ("k_real", ctypes.c_int64),
                ("a_parts", ctypes.c_int), ("b_parts", ctypes.c_int),
                ("tile_m", ctypes.c_int), ("tile_n", ctypes.c_int), ("tile_k", ctypes.c_int),
                ("workgroups", ctypes.c_int64), ("kernel", ctypes.c_char * 48)]


class MdGemmDesc(ctypes.Structure):
    _fields_ = [("transa", ctypes.c_char), ("transb", ctypes.c_char),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("alpha", MdScalar),
                ("A", ctypes.c_void_p), ("dta", ctypes.c_int), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("dtb", ctypes.c_int), ("ldb", ctypes.c_int64),
                ("beta", MdScalar),
                ("C", ctypes.c_void_p), ("dtc", ctypes.c_int), ("ldc", ctypes.c_int64),
                ("comp", ctypes.c_int)]


_lib = None


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmdgemm.so is not built (run __graft_entry__.build() or "
                               "python -m paper_1901_06015_amd.build); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, ci, cc = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_char
        args = [cc, cc, i64, i64, i64, MdScalar, vp, ci, i64, vp, ci, i64, MdScalar, vp, ci, i64, ci]
        L.mdgemm.argtypes = args + [vp]
        L.mdgemm.restype = ci
        L.mdgemm_plan.argtypes = args + [ctypes.POINTER(MdPlan)]
        L.mdgemm_strided.argtypes = [cc, cc, i64, i64, i64, MdScalar, vp, ci, i64, i64, vp, ci, i64, i64,
                                     MdScalar, vp, ci, i64, i64, ci, vp]
        L.mdgemm_strided.restype = ci
        L.mdgemm_plan.restype = ci
        L.mdgemm_grouped.argtypes = [i64, ctypes.POINTER(MdGemmDesc), vp]
        L.mdgemm_grouped.restype = ci
        L.mdgemm_grouped_noalloc.argtypes = [i64, ctypes.POINTER(MdGemmDesc), vp]
        L.mdgemm_grouped_noalloc.restype = ci
        L.mdgemm_tune_load.argtypes = [ctypes.c_char_p]
        L.mdgemm_tune_load.restype = ci
        L.mdgemm_tune_set.argtypes = [ci, ci, ci, ci, ci]
        L.mdgemm_tune_set.restype = ci
        L.mdgemm_tune_get.argtypes = [ci, ci, ci, ci]
        L.mdgemm_tune_get.restype = ci
        L.mdgemm_strerror.argtypes = [ci]
        L.mdgemm_strerror.restype = ctypes.c_char_p
        L.mdgemm_version.argtypes = []
        L.mdgemm_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def scalar(x):
    x = complex(x)
    return MdScalar(x.real, x.imag)


def tag(dt):
    return DT_TAG[dt] if isinstance(dt, str) else int(dt)


MD_COMP_LITERAL_ALPHA = 0x100


def comp_tag(comp):
    """None/"default", "s", "d", "bf16x3", or one of the last three with
    "+literal" (MD_COMP_LITERAL_ALPHA: a complex alpha applied as given in the
    mixed cases), or an int passed through."""
    if comp is None or not isinstance(comp, str):
        return COMP_TAG[comp] if comp is None else int(comp)
    if comp.endswith("+literal"):
        base = comp[:-len("+literal")]
        if base not in ("s", "d", "bf16x3", "h"):
            raise ValueError("the literal-alpha flag needs an explicit precision (s, d, bf16x3 or h)")
        return COMP_TAG[base] | MD_COMP_LITERAL_ALPHA
    return COMP_TAG[comp]


def _ch(t):
    return t.encode() if isinstance(t, str) else t


def mdgemm(transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb, beta, C, dtc, ldc,
           comp=None, stream=None):
    """The C entry point with raw device pointers (ints)."""
    return lib().mdgemm(_ch(transa), _ch(transb), m, n, k, scalar(alpha), A, tag(dta), lda,
                        B, tag(dtb), ldb, scalar(beta), C, tag(dtc), ldc, comp_tag(comp), stream)


def mdgemm_strided(transa, transb, m, n, k, alpha, A, dta, rsa, csa, B, dtb, rsb, csb,
                   beta, C, dtc, rsc, csc, comp=None, stream=None):
    """The strided C entry point: each operand with its row and column strides."""
    return lib().mdgemm_strided(_ch(transa), _ch(transb), m, n, k, scalar(alpha), A, tag(dta), rsa, csa,
                                B, tag(dtb), rsb, csb, scalar(beta), C, tag(dtc), rsc, csc,
                                comp_tag(comp), stream)


def mdgemm_plan(transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb, beta, C, dtc, ldc,
                comp=None):
    """Host-only description of what mdgemm would do.  Returns (status, dict)."""
    p = MdPlan()
    st = lib().mdgemm_plan(_ch(transa), _ch(transb), m, n, k, scalar(alpha), A, tag(dta), lda,
                           B, tag(dtb), ldb, scalar(beta), C, tag(dtc), ldc, comp_tag(comp),
                           ctypes.byref(p))
    d = {f[0]: getattr(p, f[0]) for f in MdPlan._fields_}
    d["kernel"] = p.kernel.decode()
    d["case"] = CASE_NAMES[p.domain_case] if 0 <= p.domain_case < 8 else None
    return st, d


def make_desc(transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb, beta, C, dtc, ldc,
              comp=None):
    return MdGemmDesc(_ch(transa), _ch(transb), m, n, k, scalar(alpha), A, tag(dta), lda,
                      B, tag(dtb), ldb, scalar(beta), C, tag(dtc), ldc, comp_tag(comp))


def mdgemm_grouped(descs, stream=None):
    arr = (MdGemmDesc * len(descs))(*descs)
    return lib().mdgemm_grouped(len(descs), arr, stream)


def mdgemm_grouped_noalloc(descs, stream=None):
    arr = (MdGemmDesc * len(descs))(*descs)
    return lib().mdgemm_grouped_noalloc(len(descs), arr, stream)


def strerror(status):
    return lib().mdgemm_strerror(status).decode()


def tune_load(path):
    return lib().mdgemm_tune_load(None if path is None else path.encode())


# Grouped tile configurations (md_gtile), by their table-file names.
GTILE_NAMES = ("64x64", "128x128", "128x64", "64x128", "64x64k")
TUNE_BUCKETS = 5


def tune_set(comp, case, bucket_m, bucket_n, config):
    """Set one tile-table entry; `config` is an md_gtile value or its name."""
    cfg = GTILE_NAMES.index(config) if isinstance(config, str) else config
    return lib().mdgemm_tune_set(comp_tag(comp), CASE_NAMES.index(case) if isinstance(case, str) else case,
                                 bucket_m, bucket_n, cfg)


def tune_get(comp, case, bucket_m, bucket_n):
    """The md_gtile value of one tile-table entry (-1 if invalid)."""
    return lib().mdgemm_tune_get(comp_tag(comp), CASE_NAMES.index(case) if isinstance(case, str) else case,
                                 bucket_m, bucket_n)


def tune_bucket(dim):
    """Size bucket of a real-product dimension (<=64, <=128, <=256, <=512, larger)."""
    b, lim = 0, 64
    while b < TUNE_BUCKETS - 1 and dim > lim:
        b, lim = b + 1, lim * 2
    return b
