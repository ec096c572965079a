"""Seeded synthetic operands for mixed-datatype GEMM.

Random numbers only: nothing in this module multiplies, accumulates or
converts the way the product does.  Tests, the benchmark and the smoke check
draw operands here, then hand the same host buffers to the GPU library and to
the CPU oracle.

A matrix is returned as a Fortran-ordered numpy array of shape (ld, cols) in
its storage type (float32, float64, complex64, complex128, float16, or the
structured pair of float16 ``HALF_COMPLEX`` for complex half); the logical
matrix is its first ``rows`` rows.  Rows beyond ``rows`` (the ld padding) are
filled with ``pad`` so that tests can check they are never written.

Distributions (the paper's experiments use random column-stored matrices;
the workloads add the variants below):
  * "uniform":  real and imaginary parts iid U[-1, 1] drawn in float64 by
                numpy's PCG64 and rounded to nearest to the storage type;
  * "loguniform": magnitude 10**U(-3, 3) with a random sign, per part;
  * "int":      integers drawn uniformly from [-4, 4] (exactly representable
                in every storage and computation type, bf16 included).
"""
import numpy as np

# complex binary16: interleaved (re, im) pairs, 4 bytes per element
HALF_COMPLEX = np.dtype([("re", np.float16), ("im", np.float16)])
NP_DTYPE = {"s": np.float32, "d": np.float64, "c": np.complex64, "z": np.complex128,
            "h": np.float16, "hc": HALF_COMPLEX}
REAL_OF = {"s": np.float32, "d": np.float64, "c": np.float32, "z": np.float64,
           "h": np.float16, "hc": np.float16}
TAGS = ("s", "d", "c", "z")
HALF_TAGS = ("h", "hc")


def is_complex(dt):
    return dt in ("c", "z", "hc")


def to_complex128(X):
    """The stored values of any storage type as complex128 (exact)."""
    if X.dtype == HALF_COMPLEX:
        return X["re"].astype(np.float64) + 1j * X["im"].astype(np.float64)
    return np.asarray(X, dtype=np.complex128)


def _parts(rng, shape, dist):
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=shape)
    if dist == "loguniform":
        mag = 10.0 ** rng.uniform(-3.0, 3.0, size=shape)
        sign = np.where(rng.integers(0, 2, size=shape) == 0, -1.0, 1.0)
        return mag * sign
    if dist == "int":
        return rng.integers(-4, 5, size=shape).astype(np.float64)
    raise ValueError("unknown distribution %r" % (dist,))


def matrix(rows, cols, dt, seed, ld=None, dist="uniform", pad=0.0):
    """A (ld x cols) column-major buffer whose leading rows x cols block is random."""
    ld = max(1, rows) if ld is None else ld
    assert ld >= max(1, rows)
    rng = np.random.Generator(np.random.PCG64(seed))
    if dt == "hc":
        out = np.zeros((ld, cols), dtype=HALF_COMPLEX, order="F")
        out["re"] = pad
        out["im"] = pad
    else:
        out = np.full((ld, cols), pad, dtype=NP_DTYPE[dt], order="F")
    if rows == 0 or cols == 0:
        return out
    re = _parts(rng, (cols, rows), dist).T
    if dt == "hc":
        im = _parts(rng, (cols, rows), dist).T
        out["re"][:rows, :] = re.astype(np.float16)
        out["im"][:rows, :] = im.astype(np.float16)
    elif is_complex(dt):
        im = _parts(rng, (cols, rows), dist).T
        out[:rows, :] = (re.astype(REAL_OF[dt]) + 1j * im.astype(REAL_OF[dt])).astype(NP_DTYPE[dt])
    else:
        out[:rows, :] = re.astype(NP_DTYPE[dt])
    return out


def operand_seed(base, label, which):
    """Deterministic per-(combination, operand) seed."""
    h = base * 1000003
    for ch in label + "/" + which:
        h = (h * 131 + ord(ch)) % (2 ** 63 - 1)
    return h


def loguniform_dims(count, seed, lo=16, hi=1024):
    """Integers floor(exp(U(ln lo, ln(hi+1)))), i.e. log-uniform on [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=count))).astype(np.int64)
    return np.clip(d, lo, hi)
