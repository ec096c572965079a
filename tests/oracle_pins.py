"""Pins of the CPU oracle to facts fixed outside the oracle itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` handle and returns a list of
failure strings (empty when the pin holds).  The same functions are run on the
real oracle (tests/test_oracle_pins.py) and on deliberately broken copies of
its source (tests/test_oracle_mutants.py), which must each fail at least one
pin.

What fixes what (the paper is Van Zee, Parikh, van de Geijn, FLAME WN #89):
  * pin_case_table / pin_flops      -- Figure "mixeddom" (golden fixture)
  * pin_same_type                   -- same-type combinations are an ordinary
                                       GEMM (Section 1): numpy.matmul
  * pin_domain_identities           -- each case's interpretation in Figure
                                       "mixeddom" / Section 4.2, written with
                                       real numpy products of the parts
  * pin_exact_integers              -- exact integer arithmetic (numpy int64)
  * pin_exact_rational              -- Python Fractions on tiny float inputs:
                                       the oracle's own error stays within the
                                       classical gamma_{2k} dot-product bound
  * pin_1m_equations                -- Eq. (1mc) and Eq. (1mr) of Section 4.1
  * pin_scalars                     -- Section 7 scalar policies (golden
                                       fixture) and BLAS quick-return rules
  * pin_transpose                   -- Section 1's op(A) = A^T / A^H variants
  * pin_bound_term                  -- the bound term sum_p |op(A)_ip||op(B)_pj|
                                       of the tolerance: numpy on the moduli
  * pin_gemm_at                     -- the sampled evaluator equals the full one
"""
import itertools
import os
from fractions import Fraction

import numpy as np

from paper_1901_06015_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
TAGS = ("s", "d", "c", "z")


def load_case_table():
    rows = []
    with open(os.path.join(HERE, "golden", "mixeddom_cases.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                case, dc, da, db, fl = line.split()
                rows.append((case, dc == "C", da == "C", db == "C", int(fl)))
    return rows


def load_alpha_policy():
    out = {}
    with open(os.path.join(HERE, "golden", "alpha_policy.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                case, ok = line.split()
                out[case] = ok == "yes"
    return out


def _dom_tags(is_cplx):
    return ("c", "z") if is_cplx else ("s", "d")


def _op(X, rows, cols, trans):
    """op(X) as a complex128 array of the promoted stored values; "R" is the
    conjugate without transposition of Section 3's hypothetical API."""
    M = inputs.to_complex128(X[:rows, :cols])
    if trans == "N":
        return M
    if trans == "R":
        return M.conj()
    if trans == "T":
        return M.T
    return M.conj().T


def _operands(dta, dtb, dtc, m, n, k, ta, tb, seed, dist="uniform"):
    ar, ac = (m, k) if ta in "NR" else (k, m)
    br, bc = (k, n) if tb in "NR" else (n, k)
    A = inputs.matrix(ar, ac, dta, seed + 1, dist=dist)
    B = inputs.matrix(br, bc, dtb, seed + 2, dist=dist)
    C = inputs.matrix(m, n, dtc, seed + 3, dist=dist)
    return A, B, C, ar, br


def _call(o, ta, tb, m, n, k, alpha, A, dta, B, dtb, beta, C, dtc):
    return o.gemm(ta, tb, m, n, k, alpha, A, dta, A.shape[0], B, dtb, B.shape[0],
                  beta, C, dtc, C.shape[0])


def pin_case_table(o):
    fails = []
    for case, dc, da, db, _ in load_case_table():
        for tc in _dom_tags(dc):
            for ta in _dom_tags(da):
                for tb in _dom_tags(db):
                    got = o.case(tc, ta, tb)
                    if got != case:
                        fails.append("case(%s%s%s)=%s expected %s" % (tc, ta, tb, got, case))
    return fails


def pin_flops(o):
    fails = []
    for case, dc, da, db, fl in load_case_table():
        tc, ta, tb = _dom_tags(dc)[0], _dom_tags(da)[1], _dom_tags(db)[0]
        got = o.flops(tc, ta, tb, 3, 5, 7)
        if got != fl * 3 * 5 * 7:
            fails.append("flops case %s = %r expected %d" % (case, got, fl * 105))
    return fails


def pin_same_type(o):
    """Homogeneous storage is an ordinary GEMM: compare with numpy.matmul, for
    the nine BLAS op() pairs and those with R (conjugate, not transposed)."""
    fails = []
    for dt in TAGS:
        for ta, tb in itertools.product("NTCR", "NTCR"):
            m, n, k = 5, 6, 7
            A, B, C, _, _ = _operands(dt, dt, dt, m, n, k, ta, tb, seed=11)
            alpha = 1.5 + (0.25j if dt in "cz" else 0)
            beta = -0.5 + (0.75j if dt in "cz" else 0)
            st, got, g = _call(o, ta, tb, m, n, k, alpha, A, dt, B, dt, beta, C, dt)
            if st != 0:
                fails.append("same-type %s %s%s status %d" % (dt, ta, tb, st))
                continue
            ref = alpha * (_op(A, A.shape[0], A.shape[1], ta) @ _op(B, B.shape[0], B.shape[1], tb))
            ref = ref + beta * np.asarray(C, dtype=np.complex128)
            if dt in "sd":
                ref = ref.real.astype(np.complex128)
            err = np.max(np.abs(got - ref) / (np.abs(g) + np.abs(ref) + 1e-300))
            if not err < 1e-13:
                fails.append("same-type %s %s%s rel err %.3g" % (dt, ta, tb, err))
    return fails


def _case_expect(case, Ar, Ai, Br, Bi, Cin, alpha, beta, c_complex):
    """Figure "mixeddom" interpretation of each case, via real products only."""
    if case == "0":
        ab = Ar @ Br + 0j
    elif case == "1b":
        ab = Ar @ Br + 0j                           # A Re(B)
    elif case == "1a":
        ab = Ar @ Br + 0j                           # Re(A) B
    elif case == "2ab":
        ab = (Ar @ Br - Ai @ Bi) + 0j               # Re(AB)
    elif case == "1c":
        ab = Ar @ Br + 0j                           # AB into Re(C)
    elif case == "2bc":
        ab = Ar @ Br + 1j * (Ar @ Bi)               # A Re(B) + i A Im(B)
    elif case == "2ac":
        ab = Ar @ Br + 1j * (Ai @ Br)               # Re(A) B + i Im(A) B
    else:
        ab = (Ar @ Br - Ai @ Bi) + 1j * (Ar @ Bi + Ai @ Br)
    if not c_complex:
        beta = beta.real
    r = alpha * ab + beta * Cin
    return r if c_complex else r.real + 0j


def pin_domain_identities(o):
    fails = []
    for tc, ta_, tb_ in itertools.product(TAGS, TAGS, TAGS):
        case = o.case(tc, ta_, tb_)
        for tra, trb in (("N", "N"), ("T", "C"), ("C", "N")):
            m, n, k = 4, 5, 6
            A, B, C, _, _ = _operands(ta_, tb_, tc, m, n, k, tra, trb, seed=23)
            alpha, beta = 1.5, -0.5 + (0.25j if tc in "cz" else 0.0)
            st, got, g = _call(o, tra, trb, m, n, k, alpha, A, ta_, B, tb_, beta, C, tc)
            if st != 0:
                fails.append("%s%s%s status %d" % (tc, ta_, tb_, st))
                continue
            opA = _op(A, A.shape[0], A.shape[1], tra)
            opB = _op(B, B.shape[0], B.shape[1], trb)
            exp = _case_expect(case, opA.real, opA.imag, opB.real, opB.imag,
                               np.asarray(C, dtype=np.complex128), alpha, beta, tc in "cz")
            err = np.max(np.abs(got - exp) / (g + np.abs(exp) + 1e-300))
            if not err < 1e-13:
                fails.append("identity %s%s%s (%s) %s%s rel err %.3g" % (tc, ta_, tb_, case, tra, trb, err))
    return fails


def _int_parts(X, rows, cols, trans):
    M = _op(X, rows, cols, trans)
    return np.rint(M.real).astype(np.int64), np.rint(M.imag).astype(np.int64)


def pin_exact_integers(o):
    """Integer entries in [-4, 4], alpha=1.5, beta=-0.5: every partial result is
    exact in FP64, so the oracle must equal exact integer arithmetic bitwise."""
    fails = []
    for tc, ta_, tb_ in itertools.product(TAGS, TAGS, TAGS):
        case = o.case(tc, ta_, tb_)
        tra, trb = ("N", "N") if (TAGS.index(tc) + TAGS.index(ta_)) % 2 == 0 else ("C", "T")
        m, n, k = 3, 4, 9
        A, B, C, _, _ = _operands(ta_, tb_, tc, m, n, k, tra, trb, seed=37, dist="int")
        st, got, _ = _call(o, tra, trb, m, n, k, 1.5, A, ta_, B, tb_, -0.5, C, tc)
        if st != 0:
            fails.append("exact %s%s%s status %d" % (tc, ta_, tb_, st))
            continue
        Ar, Ai = _int_parts(A, A.shape[0], A.shape[1], tra)
        Br, Bi = _int_parts(B, B.shape[0], B.shape[1], trb)
        Cr, Ci = _int_parts(C, m, n, "N")
        # twice the result, in integers: 3*AB - C
        if case in ("0", "1a", "1b", "1c"):
            pr, pi = Ar @ Br, np.zeros((m, n), np.int64)
        elif case == "2ab":
            pr, pi = Ar @ Br - Ai @ Bi, np.zeros((m, n), np.int64)
        elif case == "2bc":
            pr, pi = Ar @ Br, Ar @ Bi
        elif case == "2ac":
            pr, pi = Ar @ Br, Ai @ Br
        else:
            pr, pi = Ar @ Br - Ai @ Bi, Ar @ Bi + Ai @ Br
        twice_r = 3 * pr - Cr
        twice_i = (3 * pi - Ci) if tc in "cz" else np.zeros((m, n), np.int64)
        ok = np.array_equal(got.real * 2, twice_r.astype(np.float64)) and \
            np.array_equal(got.imag * 2, twice_i.astype(np.float64))
        if not ok:
            fails.append("exact %s%s%s (%s) mismatch" % (tc, ta_, tb_, case))
    return fails


def _frac(x):
    return Fraction(float(x))


def pin_exact_rational(o):
    """Exact rational evaluation of the definition on tiny float inputs.  A plain
    recursive FP64 sum of k complex products has error below gamma_{2k+2} * g
    (Higham, Accuracy and Stability, Section 4.1), so anything larger is a bug."""
    fails = []
    u = 2.0 ** -53
    for tc, ta_, tb_ in (("z", "c", "d"), ("d", "z", "z"), ("c", "s", "z"), ("z", "z", "z"),
                          ("s", "d", "c"), ("c", "d", "s")):
        m, n, k = 2, 3, 4
        A, B, C, _, _ = _operands(ta_, tb_, tc, m, n, k, "N", "T", seed=41)
        alpha = 0.75 + (0.5j if o.case(tc, ta_, tb_) == "3" else 0)
        beta = 0.5 - (0.25j if tc in "cz" else 0)
        st, got, g = _call(o, "N", "T", m, n, k, alpha, A, ta_, B, tb_, beta, C, tc)
        if st != 0:
            fails.append("rational %s%s%s status %d" % (tc, ta_, tb_, st))
            continue
        gam = (2 * k + 4) * u / (1 - (2 * k + 4) * u)
        for i in range(m):
            for j in range(n):
                sr = si = Fraction(0)
                for p in range(k):
                    a = complex(A[i, p])
                    b = complex(B[j, p])
                    sr += _frac(a.real) * _frac(b.real) - _frac(a.imag) * _frac(b.imag)
                    si += _frac(a.real) * _frac(b.imag) + _frac(a.imag) * _frac(b.real)
                ar_, ai_ = _frac(alpha.real), _frac(complex(alpha).imag)
                tr_ = ar_ * sr - ai_ * si
                ti_ = ar_ * si + ai_ * sr
                c = complex(C[i, j])
                br_ = _frac(beta.real)
                bi_ = _frac(complex(beta).imag) if tc in "cz" else Fraction(0)
                rr = br_ * _frac(c.real) - bi_ * _frac(c.imag) + tr_
                ri = br_ * _frac(c.imag) + bi_ * _frac(c.real) + ti_
                if tc in "sd":
                    ri = Fraction(0)
                bound = gam * (abs(alpha) * g[i, j] + abs(beta) * abs(c)) * 2 + 1e-300
                e = abs(complex(float(Fraction(got[i, j].real) - rr), float(Fraction(got[i, j].imag) - ri)))
                if not e <= bound:
                    fails.append("rational %s%s%s (%d,%d) err %.3g > %.3g" % (tc, ta_, tb_, i, j, e, bound))
                    break
    return fails


def pin_1m_equations(o):
    """Eq. (1mc): with C column-stored, a real product of A in the 1e format
    (2m x 2k) and B in the 1r format (2k x n) is C (2m x n, re/im rows
    interleaved).  Eq. (1mr): A in 1r (m x 2k) times B in 1e (2k x 2n) gives C
    with re/im columns interleaved.  Example size of Section 4.1: m=3, n=4, k=2,
    plus one larger size."""
    fails = []
    for m, n, k in ((3, 4, 2), (7, 5, 6)):
        A = inputs.matrix(m, k, "z", 51)
        B = inputs.matrix(k, n, "z", 52)
        C = inputs.matrix(m, n, "z", 53)
        st, got, _ = _call(o, "N", "N", m, n, k, 1.0, A, "z", B, "z", 0.0, C, "z")
        if st != 0:
            return ["1m status %d" % st]
        a, b = A[:m, :k], B[:k, :n]
        A1e = np.zeros((2 * m, 2 * k))
        A1e[0::2, 0::2] = a.real
        A1e[0::2, 1::2] = -a.imag
        A1e[1::2, 0::2] = a.imag
        A1e[1::2, 1::2] = a.real
        B1r = np.zeros((2 * k, n))
        B1r[0::2, :] = b.real
        B1r[1::2, :] = b.imag
        c_col = A1e @ B1r
        exp_c = c_col[0::2, :] + 1j * c_col[1::2, :]
        A1r = np.zeros((m, 2 * k))
        A1r[:, 0::2] = a.real
        A1r[:, 1::2] = a.imag
        B1e = np.zeros((2 * k, 2 * n))
        B1e[0::2, 0::2] = b.real
        B1e[0::2, 1::2] = b.imag
        B1e[1::2, 0::2] = -b.imag
        B1e[1::2, 1::2] = b.real
        c_row = A1r @ B1e
        exp_r = c_row[:, 0::2] + 1j * c_row[:, 1::2]
        for name, exp in (("1mc", exp_c), ("1mr", exp_r)):
            err = np.max(np.abs(got - exp)) / max(1e-300, np.max(np.abs(exp)))
            if not err < 1e-14:
                fails.append("%s m=%d rel err %.3g" % (name, m, err))
    return fails


def pin_scalars(o):
    fails = []
    policy = load_alpha_policy()
    m, n, k = 3, 4, 5
    for tc, ta_, tb_ in itertools.product(("s", "z"), ("d", "c"), ("s", "z")):
        case = o.case(tc, ta_, tb_)
        A, B, C, _, _ = _operands(ta_, tb_, tc, m, n, k, "N", "N", seed=61)
        # Section 7.2: complex alpha
        st, got, _ = _call(o, "N", "N", m, n, k, 1.5 + 0.5j, A, ta_, B, tb_, 1.0, C, tc)
        if policy[case] != (st == 0):
            fails.append("alpha policy case %s status %d" % (case, st))
        if case == "0" and st == 0:
            st2, ref, _ = _call(o, "N", "N", m, n, k, 1.5, A, ta_, B, tb_, 1.0, C, tc)
            if not np.array_equal(got, ref):
                fails.append("case 0 alpha not projected")
        # Section 7.2: Im(beta) cannot change a real C
        if tc == "s":
            st1, r1, _ = _call(o, "N", "N", m, n, k, 1.0, A, ta_, B, tb_, 0.5 + 7j, C, tc)
            st2, r2, _ = _call(o, "N", "N", m, n, k, 1.0, A, ta_, B, tb_, 0.5, C, tc)
            if not (st1 == 0 and np.array_equal(r1, r2)):
                fails.append("Im(beta) changed real C in case %s" % case)
        # a purely imaginary beta on a real C is beta == 0 after the projection
        if tc == "s":
            Cn = C.copy()
            Cn[:, :] = np.nan
            st1, r1, _ = _call(o, "N", "N", m, n, k, 1.0, A, ta_, B, tb_, 7j, Cn, tc)
            st2, r2, _ = _call(o, "N", "N", m, n, k, 1.0, A, ta_, B, tb_, 0.0, Cn, tc)
            if not (st1 == 0 and np.array_equal(r1, r2)):
                fails.append("Im(beta) on real C read C in case %s" % case)
        # beta == 0: C is not read (NaN in C does not propagate)
        Cn = C.copy()
        Cn[:, :] = np.nan
        st, r, _ = _call(o, "N", "N", m, n, k, 1.0, A, ta_, B, tb_, 0.0, Cn, tc)
        if st != 0 or not np.all(np.isfinite(r)):
            fails.append("beta=0 read C in case %s" % case)
        # alpha == 0 and k == 0: A and B are not read, C := beta*C
        An = A.copy()
        An[:, :] = np.nan
        st, r, _ = _call(o, "N", "N", m, n, k, 0.0, An, ta_, B, tb_, -0.5, C, tc)
        Cc = np.asarray(C[:m, :n], dtype=np.complex128)
        expect = -0.5 * (Cc if tc in "cz" else Cc.real + 0j)
        if st != 0 or not np.array_equal(r, expect):
            fails.append("alpha=0 case %s" % case)
        st, r, _ = o.gemm("N", "N", m, n, 0, 2.0, An, ta_, m, B, tb_, 1, -0.5, C, tc, m)
        if st != 0 or not np.array_equal(r, expect):
            fails.append("k=0 case %s" % case)
    # Section 4.2 case 1c: AB reaches only Re(C); Im(C) is beta*Im(C) exactly
    for tc in ("c", "z"):
        A, B, C, _, _ = _operands("d", "s", tc, m, n, k, "N", "N", seed=71)
        st, r, _ = _call(o, "N", "N", m, n, k, 1.5, A, "d", B, "s", -0.5, C, tc)
        if st != 0 or not np.array_equal(r.imag, -0.5 * np.asarray(C[:m, :n]).imag.astype(np.float64)):
            fails.append("1c Im(C) not beta*Im(C) for %s" % tc)
    return fails


def pin_transpose(o):
    """op(A) = A^T applied to a stored A^T equals op(A) = A applied to A (bitwise);
    likewise A^H of a stored conj(A)^T."""
    fails = []
    m, n, k = 4, 3, 5
    for dta, dtb in (("c", "z"), ("d", "c"), ("z", "s")):
        A = inputs.matrix(m, k, dta, 81)
        B = inputs.matrix(k, n, dtb, 82)
        C = inputs.matrix(m, n, "z", 83)
        st0, r0, _ = _call(o, "N", "N", m, n, k, 1.0, A, dta, B, dtb, 1.0, C, "z")
        At = np.asfortranarray(A.T)
        Bt = np.asfortranarray(B.T)
        st1, r1, _ = _call(o, "T", "T", m, n, k, 1.0, At, dta, Bt, dtb, 1.0, C, "z")
        Ah = np.asfortranarray(A.conj().T)
        Bh = np.asfortranarray(B.conj().T)
        st2, r2, _ = _call(o, "C", "C", m, n, k, 1.0, Ah, dta, Bh, dtb, 1.0, C, "z")
        if not (st0 == st1 == st2 == 0 and np.array_equal(r0, r1) and np.array_equal(r0, r2)):
            fails.append("transpose %s%s" % (dta, dtb))
    return fails


def _store(X, rows, cols, rs, cs, pad=777.25):
    """A flat buffer holding the rows x cols block of X at r*rs + c*cs; the
    other elements hold `pad`, so reading a wrong element changes the result."""
    size = (rows - 1) * rs + (cols - 1) * cs + 1 if rows and cols else 1
    buf = np.full(size, pad, dtype=X.dtype)
    for r in range(rows):
        for c in range(cols):
            buf[r * rs + c * cs] = X[r, c]
    return buf


def pin_strides(o):
    """Section 3's row and column strides: the same logical operands stored
    column-major, row-major and in general storage (neither stride 1) give
    numpy's product for homogeneous storage, and bitwise the column-major
    result for mixed storage."""
    fails = []
    m, n, k = 5, 4, 3
    layouts = {"col": lambda r, c: (1, r + 2), "row": lambda r, c: (c + 3, 1), "gen": lambda r, c: (2, 2 * r + 3)}
    for dta, dtb, dtc, ta, tb in (("z", "z", "z", "N", "R"), ("d", "d", "d", "T", "N"), ("c", "s", "z", "C", "T"),
                                   ("s", "z", "c", "R", "C"), ("z", "c", "d", "N", "N")):
        A, B, C, ar, br = _operands(dta, dtb, dtc, m, n, k, ta, tb, seed=61)
        ac, bc = A.shape[1], B.shape[1]
        st0, ref0, _ = _call(o, ta, tb, m, n, k, 1.5, A, dta, B, dtb, -0.5, C, dtc)
        same = dta == dtb == dtc
        ref = None
        if same:
            ref = 1.5 * (_op(A, ar, ac, ta) @ _op(B, br, bc, tb)) - 0.5 * np.asarray(C, dtype=np.complex128)
            if dtc in "sd":
                ref = ref.real.astype(np.complex128)
        for la, lb, lc in (("row", "row", "row"), ("gen", "col", "row"), ("col", "gen", "gen"), ("row", "gen", "col")):
            rsa, csa = layouts[la](ar, ac)
            rsb, csb = layouts[lb](br, bc)
            rsc, csc = layouts[lc](m, n)
            st, got, g = o.gemm_gs(ta, tb, m, n, k, 1.5, _store(A, ar, ac, rsa, csa), dta, rsa, csa,
                                   _store(B, br, bc, rsb, csb), dtb, rsb, csb, -0.5,
                                   _store(C, m, n, rsc, csc), dtc, rsc, csc)
            what = "strides %s%s%s %s%s %s/%s/%s" % (dtc, dta, dtb, ta, tb, la, lb, lc)
            if st != 0 or st0 != 0:
                fails.append(what + " status %d/%d" % (st, st0))
            elif same:
                err = np.max(np.abs(got - ref) / (np.abs(g) + np.abs(ref) + 1e-300))
                if not err < 1e-13:
                    fails.append(what + " rel err %.3g" % err)
            elif not np.array_equal(got, ref0):
                fails.append(what + " differs from the column-major result")
    return fails


def pin_literal_alpha(o):
    """Section 7.2's literal interpretation (all five operands in their own
    domains): with Im(alpha) != 0 every one of the 64 storage combinations
    equals the homogeneous complex product alpha*op(A)*op(B) + beta*C formed by
    numpy, projected to Re for a real C -- exactly for integer inputs; and for
    a real alpha it equals the paper's policy result bit for bit."""
    fails = []
    alpha, beta = 0.75 - 0.5j, -0.5 + 0.25j
    m, n, k = 5, 4, 6
    for i, (tc, ta_, tb_) in enumerate(itertools.product(("s", "d", "c", "z"), repeat=3)):
        trans = ("N", "T", "C", "R")
        ta, tb = trans[i % 4], trans[(i // 4) % 4]
        for dist in ("int", "uniform"):
            A, B, C, ar, br = _operands(ta_, tb_, tc, m, n, k, ta, tb, seed=300 + i, dist=dist)
            st, got, _ = o.gemm(ta, tb, m, n, k, alpha, A, ta_, A.shape[0], B, tb_, B.shape[0], beta, C, tc,
                                C.shape[0], literal_alpha=True)
            if st != 0:
                fails.append("literal %s%s%s status %d" % (tc, ta_, tb_, st))
                continue
            ac = (m, k) if ta in "NR" else (k, m)
            bc = (k, n) if tb in "NR" else (n, k)
            X = _op(A, ac[0], ac[1], ta) @ _op(B, bc[0], bc[1], tb)
            be = beta if tc in "cz" else beta.real
            want = alpha * X + be * np.asarray(C[:m, :n], dtype=np.complex128)
            if tc in "sd":
                want = want.real.astype(np.complex128)
            if dist == "int":
                ok = np.array_equal(got, want)
            else:
                ok = np.allclose(got, want, rtol=0, atol=1e-12)
            if not ok:
                fails.append("literal %s%s%s %s%s (%s) differs from numpy by %.3g" % (
                    tc, ta_, tb_, ta, tb, dist, float(np.max(np.abs(got - want)))))
            st1, r1, _ = o.gemm(ta, tb, m, n, k, 1.25, A, ta_, A.shape[0], B, tb_, B.shape[0], beta, C, tc,
                                C.shape[0], literal_alpha=True)
            st2, r2, _ = o.gemm(ta, tb, m, n, k, 1.25, A, ta_, A.shape[0], B, tb_, B.shape[0], beta, C, tc,
                                C.shape[0])
            if not (st1 == st2 == 0 and np.array_equal(r1, r2)):
                fails.append("literal %s%s%s with a real alpha differs from the policy result" % (tc, ta_, tb_))
    return fails


def pin_half_decoding(o):
    """IEEE binary16 storage: every finite bit pattern (zeros, subnormals,
    normals) decodes to numpy's float16 value, as the real type h and as
    either part of the complex type hc: the 63488 patterns fill a 256 x 256
    matrix multiplied by the identity (alpha = 1, beta = 0; square, so an
    index mistake stays inside the buffer).  NaN patterns give NaN (1 x 1
    products).  Infinities are left out: the product is formed in complex
    arithmetic, where inf * 0 in the imaginary part gives NaN."""
    fails = []
    n = 256
    bits = np.arange(65536, dtype=np.uint16)
    fin = bits[np.isfinite(bits.view(np.float16))]
    grid = np.zeros(n * n, dtype=np.uint16)
    grid[:fin.size] = fin
    A = np.asfortranarray(grid.view(np.float16).reshape(n, n, order="F"))
    eye = np.asfortranarray(np.eye(n))
    C = np.zeros((n, n), dtype=np.complex128, order="F")
    want = A.astype(np.float64)
    st, got, _ = o.gemm("N", "N", n, n, n, 1.0, A, "h", n, eye, "d", n, 0.0, C, "z", n)
    if st != 0 or not (np.array_equal(got.real, want) and np.all(got.imag == 0)):
        fails.append("h decoding differs from numpy's float16")
    Ac = np.zeros((n, n), dtype=inputs.HALF_COMPLEX, order="F")
    Ac["re"] = A
    Ac["im"] = np.asfortranarray(grid[::-1].copy().view(np.float16).reshape(n, n, order="F"))
    st, got, _ = o.gemm("N", "N", n, n, n, 1.0, Ac, "hc", n, eye, "d", n, 0.0, C, "z", n)
    if st != 0 or not (np.array_equal(got.real, want) and np.array_equal(got.imag, Ac["im"].astype(np.float64))):
        fails.append("hc decoding differs from numpy's float16")
    one = np.ones((1, 1), dtype=np.float64, order="F")
    c1 = np.zeros((1, 1), dtype=np.complex128, order="F")
    for nan_bits in (0x7C01, 0x7E00, 0xFE00, 0x7FFF):
        x = np.array([[nan_bits]], dtype=np.uint16).view(np.float16)
        st, got, _ = o.gemm("N", "N", 1, 1, 1, 1.0, np.asfortranarray(x), "h", 1, one, "d", 1, 0.0, c1, "z", 1)
        if st != 0 or not np.isnan(got[0, 0].real):
            fails.append("NaN pattern %#x did not decode to NaN" % nan_bits)
    return fails


def pin_half_products(o):
    """Half storage in every role: with h and hc among the operands, every
    storage combination of {h, hc, s, z} equals numpy's homogeneous complex
    product of the promoted values (Re kept for a real C) -- exactly for
    integer inputs -- and takes the case and flop count of its domains."""
    fails = []
    alpha, beta = 1.5, -0.5
    m, n, k = 4, 5, 6
    for i, (tc, ta_, tb_) in enumerate(itertools.product(("h", "hc", "s", "z"), repeat=3)):
        if "h" not in (tc, ta_, tb_) and "hc" not in (tc, ta_, tb_):
            continue
        doms = tuple(inputs.is_complex(t) for t in (tc, ta_, tb_))
        if o.case(tc, ta_, tb_) != o.case(*("z" if d else "d" for d in doms)):
            fails.append("case of %s/%s/%s" % (tc, ta_, tb_))
        ta, tb = ("N", "T", "C", "R")[i % 4], ("R", "C", "N", "T")[i % 4]
        for dist in ("int", "uniform"):
            A, B, C, _, _ = _operands(ta_, tb_, tc, m, n, k, ta, tb, seed=500 + i, dist=dist)
            st, got, _ = o.gemm(ta, tb, m, n, k, alpha, A, ta_, A.shape[0], B, tb_, B.shape[0], beta, C, tc,
                                C.shape[0])
            ac = (m, k) if ta in "NR" else (k, m)
            bc = (k, n) if tb in "NR" else (n, k)
            want = alpha * (_op(A, ac[0], ac[1], ta) @ _op(B, bc[0], bc[1], tb)) + \
                beta * inputs.to_complex128(C[:m, :n])
            if not inputs.is_complex(tc):
                want = want.real.astype(np.complex128)
            ok = np.array_equal(got, want) if dist == "int" else np.allclose(got, want, rtol=0, atol=1e-12)
            if st != 0 or not ok:
                fails.append("half %s/%s/%s %s%s (%s) status %d" % (tc, ta_, tb_, ta, tb, dist, st))
    return fails


def pin_bound_term(o):
    """The bound term g_ij = sum_p |op(A)_ip| |op(B)_pj| (complex modulus) that
    the error bound |C_gpu - C_ref| <= 4 k u_x g + 4 u_C |C_ref| scales by: for
    all 64 storage combinations and all 16 op pairs it must equal numpy's
    product of the elementwise moduli of op(A) and op(B) (the promoted stored
    values), to 1e-14 relative.  m != n, so a swapped index shows."""
    fails = []
    m, n, k = 5, 3, 7
    for i, (tc, ta_, tb_) in enumerate(itertools.product(TAGS, TAGS, TAGS)):
        for ta, tb in itertools.product("NTCR", "NTCR"):
            A, B, C, ar, br = _operands(ta_, tb_, tc, m, n, k, ta, tb, seed=900 + i)
            alpha = 1.5 + (0.25j if o.case(tc, ta_, tb_) in ("0", "3") else 0)
            st, _, g = _call(o, ta, tb, m, n, k, alpha, A, ta_, B, tb_, -0.5, C, tc)
            if st != 0:
                fails.append("bound term %s%s%s %s%s status %d" % (tc, ta_, tb_, ta, tb, st))
                continue
            want = np.abs(_op(A, A.shape[0], A.shape[1], ta)) @ np.abs(_op(B, B.shape[0], B.shape[1], tb))
            err = np.max(np.abs(g - want) / np.maximum(want, 1e-300))
            if not err < 1e-14:
                fails.append("bound term %s%s%s %s%s rel err %.3g" % (tc, ta_, tb_, ta, tb, err))
                break
    return fails


def pin_gemm_at(o):
    """The sampled evaluator (used where the full product is too large) is the
    same definition: at random (row, col) pairs of a non-square result it
    equals the full evaluator's value and bound term bit for bit.  Operands are
    allocated for max(m, n) rows and columns so that an index mix-up reads
    other stored values instead of leaving the buffers."""
    fails = []
    m, n, k = 9, 4, 6
    big = max(m, n)
    rng = np.random.Generator(np.random.PCG64(97))
    for i, (tc, ta_, tb_, ta, tb) in enumerate((("z", "c", "d", "N", "N"), ("d", "z", "z", "T", "C"),
                                                 ("c", "s", "z", "C", "R"), ("s", "d", "s", "N", "T"),
                                                 ("z", "z", "z", "R", "N"), ("c", "z", "c", "T", "T"))):
        A = inputs.matrix(big, big, ta_, 700 + i)
        B = inputs.matrix(big, big, tb_, 710 + i)
        C = inputs.matrix(big, big, tc, 720 + i)
        alpha = 0.75 + (0.5j if o.case(tc, ta_, tb_) == "3" else 0)
        st, full, gfull = o.gemm(ta, tb, m, n, k, alpha, A, ta_, big, B, tb_, big, -0.5, C, tc, big)
        rows = rng.integers(0, m, 40)
        cols = rng.integers(0, n, 40)
        st2, vals, g = o.gemm_at(ta, tb, m, n, k, alpha, A, ta_, big, B, tb_, big, -0.5, C, tc, big, rows, cols)
        if st != 0 or st2 != 0:
            fails.append("gemm_at %s%s%s status %d/%d" % (tc, ta_, tb_, st, st2))
            continue
        if not (np.array_equal(vals, full[rows, cols]) and np.array_equal(g, gfull[rows, cols])):
            fails.append("gemm_at %s%s%s %s%s differs from the full evaluation" % (tc, ta_, tb_, ta, tb))
    return fails


ALL_PINS = (pin_case_table, pin_flops, pin_same_type, pin_domain_identities,
            pin_exact_integers, pin_exact_rational, pin_1m_equations, pin_scalars,
            pin_transpose, pin_strides, pin_literal_alpha, pin_half_decoding, pin_half_products,
            pin_bound_term, pin_gemm_at)


def run_all(o):
    out = {}
    for p in ALL_PINS:
        try:
            out[p.__name__] = p(o)
        except Exception as e:  # a crash counts as a failed pin
            out[p.__name__] = ["raised %r" % (e,)]
    return out
