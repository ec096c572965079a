"""Helpers for the GPU parity tests: run one product on the device through the
C ABI and compare it with the CPU oracle on the same seeded host buffers.

Tolerance (elementwise):
    |C_gpu - C_ref| <= 4 * k * u_x * (|A||B|)_ij + 4 * u_C * |C_ref_ij|
with u_x the unit roundoff of the computation precision (2^-24 single,
2^-53 double), u_C that of C's storage precision, |.| the complex modulus,
(|A||B|)_ij = sum_p |op(A)_ip| |op(B)_pj| as returned by the oracle, and C_ref
the oracle's exact-input FP64 result.  BF16x3 adds its split term
3 * 2^-16 * (|A||B|)_ij (BF16X3_SPLIT).  `extra` adds documented terms where
a test leaves the regime the bound is stated for.
"""
import numpy as np
import torch

import oracle
from paper_1901_06015_amd import _lib, api, inputs

U = {"s": 2.0 ** -24, "d": 2.0 ** -53, "h": 2.0 ** -11}
# BF16x3 forms each product a*b of FP32 values from bf16 halves, a = ha + la + ea
# with |la| <= 2^-8 |a| and |ea| <= 2^-16 |a| (bf16 keeps 8 significant bits),
# as ha*hb + ha*lb + la*hb: the dropped la*lb and the residuals ea, eb leave
# at most about 3 * 2^-16 |a||b| per product (the BF16x3 reading of the
# single-precision bound), which 4 k u_s covers only from k ~ 192 on.  The
# bound of the BF16x3 tests adds this term, so they hold at any k.
BF16X3_SPLIT = 3.0 * 2.0 ** -16
PREC = {"s": "s", "d": "d", "c": "s", "z": "d", "h": "h", "hc": "h"}
SENTINEL = 777.25


def to_device(X):
    """Copy a Fortran-ordered host buffer into a device tensor with the same
    column-major strides (complex binary16 as torch.complex32)."""
    ld, cols = X.shape
    if X.dtype == inputs.HALF_COMPLEX:
        raw = np.ascontiguousarray(X.T).view(np.float16)  # (cols, 2 ld): re, im pairs down each column
        return torch.from_numpy(raw).to("cuda").view(torch.complex32).t()
    t = torch.empty((max(cols, 1), ld), dtype=api.torch_dtype(
        {np.float32: "s", np.float64: "d", np.complex64: "c", np.complex128: "z", np.float16: "h"}[X.dtype.type]),
        device="cuda").t()[:, :cols]
    t.copy_(torch.from_numpy(X))
    return t


def to_host(t):
    """A column-major device tensor back as a Fortran-ordered numpy array of
    its storage type (complex32 as inputs.HALF_COMPLEX)."""
    if t.dtype == torch.complex32:
        raw = t.t().contiguous().view(torch.float16).cpu().numpy()  # (cols, 2 ld)
        return raw.view(inputs.HALF_COMPLEX).T
    return t.cpu().numpy()


def run(tc, ta, tb, m, n, k, comp="d", transa="N", transb="N", alpha=1.5, beta=-0.5,
        dist="uniform", seed=7, pad_a=0, pad_b=0, pad_c=0, stream=None):
    """Run one product on the GPU.  Returns (gpu result (m,n) complex128,
    host C after, host inputs dict)."""
    ar, ac = (m, k) if transa.upper() in "NR" else (k, m)
    br, bc = (k, n) if transb.upper() in "NR" else (n, k)
    A = inputs.matrix(ar, ac, ta, seed * 3 + 1, ld=max(1, ar) + pad_a, dist=dist, pad=SENTINEL)
    B = inputs.matrix(br, bc, tb, seed * 3 + 2, ld=max(1, br) + pad_b, dist=dist, pad=SENTINEL)
    C = inputs.matrix(m, n, tc, seed * 3 + 3, ld=max(1, m) + pad_c, dist=dist, pad=SENTINEL)
    dA, dB, dC = to_device(A), to_device(B), to_device(C)
    st = _lib.mdgemm(transa, transb, m, n, k, alpha, dA.data_ptr(), ta, A.shape[0],
                     dB.data_ptr(), tb, B.shape[0], beta, dC.data_ptr(), tc, C.shape[0],
                     comp, stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    Cout = to_host(dC)
    return st, Cout, dict(A=A, B=B, C=C)


def strided_store(X, rows, cols, rs, cs, pad=SENTINEL):
    """A flat host buffer holding the rows x cols block of X at r*rs + c*cs;
    every other element holds `pad`."""
    size = (rows - 1) * rs + (cols - 1) * cs + 1 if rows and cols else 1
    buf = np.full(size, pad, dtype=X.dtype)
    if rows and cols:
        r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
        buf[r * rs + c * cs] = X[:rows, :cols]
    return buf


def strides_of(layout, rows, cols, pad):
    """(row stride, column stride) of a rows x cols operand stored by columns
    ("col") or by rows ("row") with `pad` spare elements per column/row, or in
    general storage with its columns ("gen", element stride 2) or its rows
    ("genr", element stride 3) apart."""
    if layout == "col":
        return 1, max(1, rows) + pad
    if layout == "row":
        return max(1, cols) + pad, 1
    if layout == "gen":
        return 2, 2 * max(1, rows) + pad
    return 3 * max(1, cols) + pad, 3


def run_strided(tc, ta, tb, m, n, k, layouts, comp="d", transa="N", transb="N", alpha=1.5, beta=-0.5,
                pads=(0, 0, 0), seed=7):
    """One product through mdgemm_strided with each operand stored by rows or
    by columns (layouts = (A, B, C) in "col"/"row").  Returns (status, gpu C
    (m, n), padding-intact flag, reference, bound factors)."""
    ar, ac = (m, k) if transa.upper() in "NR" else (k, m)
    br, bc = (k, n) if transb.upper() in "NR" else (n, k)
    shapes = ((ar, ac, ta), (br, bc, tb), (m, n, tc))
    host, dev, st_ = [], [], []
    for i, ((r, c, dt), lay, pad) in enumerate(zip(shapes, layouts, pads)):
        X = inputs.matrix(r, c, dt, seed * 3 + 1 + i)
        rs, cs = strides_of(lay, r, c, pad)
        buf = strided_store(X, r, c, rs, cs)
        host.append(buf)
        st_.append((rs, cs))
        dev.append(torch.from_numpy(buf).to("cuda"))
    (rsa, csa), (rsb, csb), (rsc, csc) = st_
    st = _lib.mdgemm_strided(transa, transb, m, n, k, alpha, dev[0].data_ptr(), ta, rsa, csa,
                             dev[1].data_ptr(), tb, rsb, csb, beta, dev[2].data_ptr(), tc, rsc, csc, comp,
                             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    cout = dev[2].cpu().numpy()
    got = np.zeros((m, n), dtype=np.complex128)
    mask = np.ones(cout.size, dtype=bool)
    if m and n:
        r, c = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
        got = cout[r * rsc + c * csc].astype(np.complex128)
        mask[(r * rsc + c * csc).ravel()] = False
    pad_ok = bool(np.all(cout[mask] == SENTINEL))
    o = oracle.get()
    sr, ref, g = o.gemm_gs(transa, transb, m, n, k, alpha, host[0], ta, rsa, csa, host[1], tb, rsb, csb,
                           beta, host[2], tc, rsc, csc)
    assert sr == 0, sr
    return st, got, pad_ok, ref, g


def reference(tc, ta, tb, m, n, k, ops, transa="N", transb="N", alpha=1.5, beta=-0.5, literal_alpha=False):
    A, B, C = ops["A"], ops["B"], ops["C"]
    st, ref, g = oracle.get().gemm(transa, transb, m, n, k, alpha, A, ta, A.shape[0],
                                   B, tb, B.shape[0], beta, C, tc, C.shape[0], literal_alpha=literal_alpha)
    assert st == 0, st
    return ref, g


def bound(tc, comp, k, ref, g, extra=0.0):
    comp = comp.split("+")[0] if isinstance(comp, str) else comp  # "+literal" does not change the precision
    comp = comp if comp is not None else PREC[tc]
    uc = U[PREC[tc]]
    if comp == "h":
        # operands rounded to binary16 (2 u_h per real product, u_h^2 absorbed),
        # exact binary16 products, FP32 accumulation
        return (4.0 * U["h"] + 4.0 * k * U["s"]) * g + 4.0 * uc * np.abs(ref) + extra
    ux = U["s" if comp == "bf16x3" else comp]
    split = BF16X3_SPLIT if comp == "bf16x3" else 0.0
    return (4.0 * k * ux + split) * g + 4.0 * uc * np.abs(ref) + extra


def check(tc, comp, k, Cout, m, n, ref, g, extra=0.0, what=""):
    got = inputs.to_complex128(np.asarray(Cout[:m, :n]))
    err = np.abs(got - ref)
    b = bound(tc, comp, k, ref, g, extra)
    bad = ~(err <= b)
    if bad.any():
        idx = np.argwhere(bad)[0]
        i, j = int(idx[0]), int(idx[1])
        raise AssertionError("%s: %d/%d entries outside the bound; first (%d,%d) got %r ref %r "
                             "err %.3g bound %.3g" % (what, int(bad.sum()), bad.size, i, j,
                                                      got[i, j], ref[i, j], err[i, j], b[i, j]))
    return float(np.max(err / np.maximum(b, 1e-300))) if err.size else 0.0


def check_padding(X, rows, what):
    """Rows beyond `rows` (the ld padding) still hold the sentinel."""
    if X.shape[0] > rows:
        pad = inputs.to_complex128(X[rows:, :])
        sentinel = float(np.float16(SENTINEL)) if X.dtype in (np.float16, inputs.HALF_COMPLEX) else SENTINEL
        want = sentinel * (1 + 1j) if X.dtype == inputs.HALF_COMPLEX else sentinel
        assert np.all(pad == want), "%s: ld padding was written" % what
