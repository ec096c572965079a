"""C ABI and host planner (not gpu): the library loads, exports every entry
point the public headers declare, and classifies/validates without a GPU."""
import glob
import itertools
import os
import re

import pytest

from paper_1901_06015_amd import _lib
import oracle_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TAGS = ("s", "d", "c", "z")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(md\w*)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert "mdgemm" in names and "mdgemm_plan" in names and "mdgemm_grouped" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_strerror():
    assert b"gfx950" in _lib.lib().mdgemm_version()
    for st in (0, 1, 2, 3, 4, 5, -1, -17):
        assert _lib.strerror(st)


def _plan(tc, ta, tb, comp=None, m=64, n=48, k=32, alpha=1.0, beta=0.0, transa="N", transb="N",
          lda=None, ldb=None, ldc=None, ptr=0x1000):
    lda = lda or max(1, m if transa == "N" else k)
    ldb = ldb or max(1, k if transb == "N" else n)
    ldc = ldc or max(1, m)
    return _lib.mdgemm_plan(transa, transb, m, n, k, alpha, ptr, ta, lda, ptr, tb, ldb, beta,
                            ptr, tc, ldc, comp)


GOLD = {r[0]: r for r in oracle_pins.load_case_table()}


@pytest.mark.parametrize("comp", [None, "s", "d"])
def test_plan_all_combinations(comp):
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        st, p = _plan(tc, ta, tb, comp)
        assert st == 0, (tc, ta, tb, st)
        case, dc, da, db, fl = GOLD[p["case"]]
        assert (dc, da, db) == (tc in "cz", ta in "cz", tb in "cz"), (tc, ta, tb, p["case"])
        assert p["flops"] == fl * 64 * 48 * 32
        want_comp = {None: (1 if tc in "dz" else 0), "s": 0, "d": 1}[comp]
        assert p["comp"] == want_comp
        # lowering: Re/Im of a complex operand that reaches a complex C (or the
        # other complex factor) doubles one dimension of the real product
        assert p["m_real"] == 64 * (2 if p["case"] in ("2ac", "3") else 1)
        assert p["n_real"] == 48 * (2 if p["case"] == "2bc" else 1)
        assert p["k_real"] == 32 * (2 if p["case"] in ("2ab", "3") else 1)
        # real-product flops equal the paper's minimum count: nothing wasted
        assert 2 * p["m_real"] * p["n_real"] * p["k_real"] == p["flops"]
        assert p["workgroups"] >= 1 and p["kernel"].startswith("md_gemm_")


def test_alpha_policy():
    policy = oracle_pins.load_alpha_policy()
    for tc, ta, tb in itertools.product(("s", "c"), ("d", "z"), ("s", "c")):
        st, p = _plan(tc, ta, tb, alpha=1.0 + 0.5j)
        assert (st == 0) == policy[p["case"]], (tc, ta, tb, st)
        if st != 0:
            assert st == _lib.MD_ERR_ALPHA_IMAG


def test_quick_returns():
    assert _plan("d", "d", "d", m=0)[1]["quick"] == 1
    assert _plan("d", "d", "d", n=0)[1]["quick"] == 1
    assert _plan("z", "c", "d", k=0)[1]["quick"] == 2
    assert _plan("z", "c", "d", alpha=0.0)[1]["quick"] == 2
    # case 0: a purely imaginary alpha projects to zero
    assert _plan("d", "s", "d", alpha=2j)[1]["quick"] == 2


def test_argument_errors():
    P = 0x1000
    ok = dict(transa="N", transb="N", m=4, n=3, k=2, alpha=1.0, A=P, dta="d", lda=4, B=P, dtb="d",
              ldb=2, beta=0.0, C=P, dtc="d", ldc=4, comp=None)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return _lib.mdgemm_plan(a["transa"], a["transb"], a["m"], a["n"], a["k"], a["alpha"],
                                a["A"], a["dta"], a["lda"], a["B"], a["dtb"], a["ldb"], a["beta"],
                                a["C"], a["dtc"], a["ldc"], a["comp"])[0]

    assert call() == 0
    assert call(transa="X") == -1
    assert call(transb="Q") == -2
    assert call(m=-1) == -3
    assert call(n=-1) == -4
    assert call(k=-1) == -5
    assert call(A=None) == -7
    assert call(dta=7) == -8
    assert call(lda=3) == -9
    assert call(transa="T", lda=1) == -9
    assert call(B=None) == -10
    assert call(dtb=-2) == -11
    assert call(ldb=1) == -12
    assert call(C=None) == -14
    assert call(dtc=4) == -15
    assert call(ldc=3) == -16
    assert call(comp=9) == -17
    # lower-case trans letters are accepted; 'C' on real operands equals 'T'
    assert call(transa="t", lda=2) == 0
    assert call(transa="c", transb="c", lda=2, ldb=3) == 0
    # A and B are not needed when alpha == 0 or k == 0
    assert call(A=None, B=None, alpha=0.0) == 0
    assert call(A=None, B=None, k=0) == 0


def test_grouped_empty_is_noop():
    assert _lib.mdgemm_grouped([], None) == 0


def test_server_create_without_device_fails_cleanly():
    """On a host without a GPU the serving loop refuses to start (no crash)."""
    import torch
    if torch.cuda.is_available():
        import pytest
        pytest.skip("a GPU is present")
    from paper_1901_06015_amd.serving import Server, ServerError
    try:
        Server(budget_bytes=1 << 30)
    except ServerError as e:
        assert e.status == _lib.MD_ERR_HIP
    else:
        raise AssertionError("server started without a device")


def test_server_config_is_validated_before_any_device_call():
    from paper_1901_06015_amd.serving import Server, ServerError
    for kw in (dict(budget_bytes=0), dict(budget_bytes=1 << 30, slots=0), dict(budget_bytes=1 << 30, max_batch=0),
               dict(budget_bytes=1 << 30, slots=2, big_lanes=3), dict(budget_bytes=1 << 30, big_lanes=0)):
        try:
            Server(**kw)
        except ServerError as e:
            assert e.status == _lib.MD_ERR_STATE, kw
        else:
            raise AssertionError("invalid configuration accepted: %r" % kw)
