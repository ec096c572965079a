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


@pytest.fixture(autouse=True)
def _tiled_planner(monkeypatch):
    """The planner tests below are about the tiled kernels: products with few
    tiles would otherwise take the small kernel (test_small_kernel_choice)."""
    monkeypatch.setenv("MDGEMM_SMALL", "0")


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
    lda = lda or max(1, m if transa in "NRnr" else k)
    ldb = ldb or max(1, k if transb in "NRnr" else n)
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


def test_half_storage_plans():
    """Binary16 storage (h, hc): the domain case follows the domains, the
    default computation precision of a half C is half (Section 5.1.1: C's
    precision); a half C takes the fast kernels, binary16 operands take them
    when both are binary16 and the precision is single or half, and the half
    computation precision keeps them for s/d/c/z storage."""
    half_tags = ("h", "hc", "s", "z")
    for tc, ta, tb in itertools.product(half_tags, half_tags, half_tags):
        st, p = _plan(tc, ta, tb)
        assert st == 0, (tc, ta, tb, st)
        want = GOLD[p["case"]]
        assert (want[1], want[2], want[3]) == (tc in ("hc", "z"), ta in ("hc", "z"), tb in ("hc", "z"))
        assert p["comp"] == {"h": 3, "hc": 3, "s": 0, "z": 1}[tc]
        a_h, b_h = ta in ("h", "hc"), tb in ("h", "hc")
        fast = (not a_h and not b_h) or (a_h and b_h and p["comp"] in (0, 3))
        assert ("_fast_" in p["kernel"]) == fast, (tc, ta, tb, p["kernel"])
    st, p = _plan("c", "z", "s", comp="h")
    assert st == 0 and p["comp"] == 3 and p["kernel"].startswith("md_gemm_f16_") and "_fast_" in p["kernel"]
    assert _plan("h", "d", "d", ldc=63)[0] == -16
    # an odd leading dimension of a real binary16 operand leaves columns off
    # 4-byte boundaries: component-wise loads
    assert "_generic_" in _plan("h", "h", "h", m=63, lda=63)[1]["kernel"]
    assert "_fast_" in _plan("h", "h", "h", m=64)[1]["kernel"]
    assert _plan("hc", "hc", "h", comp="h+literal", alpha=1j)[0] == 0


def test_literal_alpha_flag():
    """MD_COMP_LITERAL_ALPHA lifts Section 7.2's refusal of Im(alpha) in the
    six mixed cases; it needs an explicit precision and changes no flop count."""
    for tc, ta, tb in itertools.product(("s", "c"), ("d", "z"), ("s", "c")):
        st0, p0 = _plan(tc, ta, tb, comp="d", alpha=1.0 + 0.5j)
        st1, p1 = _plan(tc, ta, tb, comp="d+literal", alpha=1.0 + 0.5j)
        assert st1 == 0, (tc, ta, tb, st1)
        st2, p2 = _plan(tc, ta, tb, comp="d", alpha=1.0)
        assert p1["flops"] == p2["flops"] and p1["kernel"] == p2["kernel"] and p1["comp"] == 1
    assert _plan("s", "c", "s", comp="s+literal", alpha=2j)[1]["comp"] == 0
    assert _plan("s", "c", "s", comp=_lib.MD_COMP_LITERAL_ALPHA | 7, alpha=2j)[0] == -17
    assert _plan("s", "c", "s", comp=-2, alpha=1.0)[0] == -17
    with pytest.raises(ValueError):
        _lib.comp_tag("default+literal")


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
    assert call(dtc=6) == -15
    assert call(ldc=3) == -16
    assert call(comp=9) == -17
    # lower-case trans letters are accepted; 'C' on real operands equals 'T'
    assert call(transa="t", lda=2) == 0
    assert call(transa="c", transb="c", lda=2, ldb=3) == 0
    # A and B are not needed when alpha == 0 or k == 0
    assert call(A=None, B=None, alpha=0.0) == 0
    assert call(A=None, B=None, k=0) == 0


def test_conjugate_without_transpose_plans_like_n():
    """'R' (Section 3) reads A or B as stored, like 'N': same shapes, same
    leading-dimension rule, same kernel family."""
    for tc, ta, tb in (("z", "c", "z"), ("c", "z", "s"), ("d", "d", "d")):
        stn, pn = _plan(tc, ta, tb, transa="N", transb="N")
        str_, pr = _plan(tc, ta, tb, transa="R", transb="r")
        assert stn == str_ == 0
        assert (pn["case"], pn["flops"], pn["workgroups"]) == (pr["case"], pr["flops"], pr["workgroups"])
    # lda counts rows of A as stored: m for 'R'
    assert _plan("z", "c", "z", transa="R", lda=63)[0] == -9


def test_strided_argument_errors():
    """mdgemm_strided validates before touching the device: strides that make
    an operand's elements overlap name their position."""
    P = 0x1000
    ok = dict(transa="N", transb="N", m=4, n=3, k=2, alpha=1.0, A=P, dta="d", rsa=1, csa=4, B=P, dtb="z",
              rsb=1, csb=2, beta=0.0, C=P, dtc="c", rsc=1, csc=4, comp=None)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return _lib.mdgemm_strided(a["transa"], a["transb"], a["m"], a["n"], a["k"], a["alpha"],
                                   a["A"], a["dta"], a["rsa"], a["csa"], a["B"], a["dtb"], a["rsb"], a["csb"],
                                   a["beta"], a["C"], a["dtc"], a["rsc"], a["csc"], a["comp"], None)

    assert call(transa="X") == -1
    assert call(transb="?") == -2
    assert call(m=-1) == -3
    assert call(n=-1) == -4
    assert call(k=-1) == -5
    assert call(A=None) == -7
    assert call(dta=9) == -8
    assert call(rsa=0) == -9
    assert call(csa=0) == -10
    assert call(csa=3) == -10          # columns of a 4-row A overlap
    assert call(rsa=1, csa=1) == -10
    assert call(rsa=1, csa=-4) == -10
    assert call(rsa=1, csa=1, transa="T") == -10   # A stored 2 x 4: columns overlap
    assert call(rsa=3, csa=1, transa="T") == -9    # A stored 2 x 4 by rows: rows overlap below 4
    assert call(B=None) == -11
    assert call(dtb=6) == -12
    assert call(rsb=0) == -13
    assert call(csb=1) == -14
    assert call(rsb=2, csb=1) == -13   # B stored by rows: 3 columns need a row stride >= 3
    assert call(C=None) == -16
    assert call(dtc=-1) == -17
    assert call(rsc=0) == -18
    assert call(csc=2) == -19
    assert call(rsc=2, csc=1) == -18
    assert call(comp=7) == -20
    # general storage (neither stride 1): the elements must not overlap, so
    # either the columns (cs >= rs*rows) or the rows (rs >= cs*cols) lie apart
    assert call(rsa=2, csa=7) == -10   # 4 x 2: columns of span 8 overlap at 7
    assert call(rsa=3, csa=2) == -9    # rows of span 4 overlap at 3
    assert call(rsb=3, csb=5) == -14   # 2 x 3
    assert call(rsc=5, csc=19) == -19  # 4 x 3
    assert call(rsc=5, csc=20, C=None) == -16


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


@pytest.mark.parametrize("comp,tile_cols", [("h", 256), ("d", 128), ("s", 128), ("bf16x3", 128)])
def test_fast_path_leading_dimension_limit_follows_the_tile(comp, tile_cols):
    """The fast kernels address an operand tile with 32-bit byte offsets: the
    stored columns the tile spans, ld elements apart, must stay below 2 GiB.
    A z operand stored along k spans the tile's m (or n) extent: 256 columns
    under the half precision's 256 x 256 tiles, 128 otherwise.  Just below the
    limit the fast kernel runs; beyond it the component-wise kernel (64-bit
    addressing), whatever the tile."""
    limit = ((1 << 31) - 4096) // (tile_cols * 16)
    for ld, want_fast in ((limit - 1, True), (limit + 1, False), (600000, 600000 < limit)):
        # B z stored along k ('N'), case 2ab (C real, A and B complex)
        st, p = _plan("d", "z", "z", comp, m=300, n=300, k=64, ldb=ld)
        assert st == 0, st
        assert ("generic" not in p["kernel"]) == want_fast, (comp, ld, p["kernel"])
        # A z stored along k ('T')
        st, p = _plan("d", "z", "z", comp, m=300, n=300, k=64, transa="T", lda=ld)
        assert st == 0, st
        assert ("generic" not in p["kernel"]) == want_fast, (comp, ld, p["kernel"])
    # along m the tile spans only its k extent: a large ld stays fast
    st, p = _plan("d", "z", "z", comp, m=300, n=300, k=64, lda=limit + 1)
    assert st == 0 and "generic" not in p["kernel"], p["kernel"]


def test_grouped_noalloc_rejects_an_oversized_table():
    """mdgemm_grouped_noalloc keeps its work table in a fixed device array of
    MD_GROUPED_NOALLOC_BYTES; a table that does not fit (here 40000 one-tile
    products, about 270 bytes each) is refused with MD_ERR_SCRATCH before any
    device call, so this runs without a GPU."""
    count = 40000
    descs = [_lib.make_desc("N", "N", 8, 8, 8, 1.0, 0x1000, "s", 8, 0x1000, "s", 8, 0.0, 0x1000, "s", 8, "s")
             for _ in range(count)]
    st = _lib.mdgemm_grouped_noalloc(descs, None)
    assert st == _lib.MD_ERR_SCRATCH, st
    assert "scratch" in _lib.strerror(st)


def test_small_kernel_choice(monkeypatch):
    """The planner sends products with few tiles and a short inner dimension
    to the small kernel (32 x 32 tiles of the real product, eight waves
    sharing k) and the others to the tiled kernels; MDGEMM_SMALL=0 turns it
    off."""
    monkeypatch.delenv("MDGEMM_SMALL")

    def plan(m, n, k, ta="c", tb="d", tc="z", comp="d"):
        st, p = _lib.mdgemm_plan("N", "N", m, n, k, 1.0, 0x1000, ta, m, 0x1000, tb, k, 1.0, 0x1000, tc, m, comp)
        assert st == 0
        return p
    p = plan(256, 256, 256)  # the single-product configuration: case 2ac, real product 512 x 256
    assert "small" in p["kernel"] and p["workgroups"] == 16 * 8 and (p["tile_m"], p["tile_n"]) == (32, 32), p
    assert "small" not in plan(4096, 4096, 4096)["kernel"]
    assert "small" not in plan(256, 256, 4096)["kernel"]          # k' above the small kernel's limit
    assert "small" in plan(64, 64, 1024, "z", "z", "z")["kernel"]   # case 3: k' = 2048
    assert "small" not in plan(64, 64, 1025, "z", "z", "z")["kernel"]
    assert "small" not in plan(64, 64, 64, "h", "h", "h", "h")["kernel"]  # binary16 operands
    assert "small" not in plan(64, 64, 64, comp="bf16x3")["kernel"]
    monkeypatch.setenv("MDGEMM_SMALL", "0")
    assert "small" not in plan(256, 256, 256)["kernel"]


def test_tune_table_defaults_set_get_and_rejections():
    """Host-only tile table of the grouped kernel: the built-in rule, set/get
    round trips, and the entries it must refuse."""
    names = _lib.GTILE_NAMES
    assert _lib.tune_load(None) == 0
    try:
        for comp in ("s", "d"):
            for bm in range(_lib.TUNE_BUCKETS):
                for bn in range(_lib.TUNE_BUCKETS):
                    want = {(False, False): "64x64", (True, True): "128x128", (True, False): "128x64",
                            (False, True): "64x128"}[(bm > 2, bn > 2)]
                    assert names[_lib.tune_get(comp, "3", bm, bn)] == want
        assert _lib.tune_get("bf16x3", "0", 4, 4) == names.index("64x64")
        for cfg in names:
            assert _lib.tune_set("d", "2ac", 1, 3, cfg) == 0
            assert _lib.tune_get("d", "2ac", 1, 3) == names.index(cfg)
        bad = [("s", 8, 0, 0, 0), ("s", 0, _lib.TUNE_BUCKETS, 0, 0), ("s", 0, 0, -1, 0),
               ("d", 0, 0, 0, len(names)), ("bf16x3", 0, 0, 0, 1), ("h", 0, 0, 0, 0)]
        for comp, case, bm, bn, cfg in bad:
            assert _lib.tune_set(comp, case, bm, bn, cfg) == _lib.MD_ERR_STATE
        assert _lib.tune_get("s", 0, _lib.TUNE_BUCKETS, 0) == -1
        assert _lib.tune_get("h", 0, 0, 0) == -1
        # the bucket edges
        assert [_lib.tune_bucket(d) for d in (1, 64, 65, 128, 129, 256, 257, 512, 513, 10 ** 6)] == \
            [0, 0, 1, 1, 2, 2, 3, 3, 4, 4]
    finally:
        _lib.tune_load(None)


def test_tune_table_file_round_trip_and_malformed_files(tmp_path):
    good = tmp_path / "t.txt"
    good.write_text("# comment\ns 1c 0 4 128x64   # trailing comment\nd 3 4 4 64x64k\nbf16x3 2ab 2 2 64x64\n")
    try:
        assert _lib.tune_load(str(good)) == 0
        assert _lib.tune_get("s", "1c", 0, 4) == _lib.GTILE_NAMES.index("128x64")
        assert _lib.tune_get("d", "3", 4, 4) == _lib.GTILE_NAMES.index("64x64k")
        # entries not listed keep the built-in rule
        assert _lib.tune_get("d", "3", 0, 0) == _lib.GTILE_NAMES.index("64x64")
        for text in ("s 1c 0 4 96x96\n", "s 9z 0 0 64x64\n", "d 3 5 0 64x64\n", "bf16x3 0 0 0 128x128\n",
                     "s 0 0\n"):
            bad = tmp_path / "bad.txt"
            bad.write_text(text)
            assert _lib.tune_load(str(bad)) == _lib.MD_ERR_STATE, text
            # a failed load leaves the table as it was
            assert _lib.tune_get("s", "1c", 0, 4) == _lib.GTILE_NAMES.index("128x64")
        assert _lib.tune_load(str(tmp_path / "missing.txt")) == _lib.MD_ERR_STATE
        assert _lib.tune_get("d", "3", 4, 4) == _lib.GTILE_NAMES.index("64x64k")
    finally:
        _lib.tune_load(None)


def test_bf16x3_packed_path_choice(monkeypatch):
    """BF16x3 runs on packed operands from 128 tiles of 256 x 256 (and
    k' >= 256) on; MDGEMM_PACK=0 turns it off, 2 forces it for any size; never
    for general strides, binary16 operands or other precisions."""
    def plan(m, n, k, tc="s", ta="s", tb="s", comp="bf16x3", lda=None):
        st, pl = _lib.mdgemm_plan("N", "N", m, n, k, 1.0, 16, ta, lda or m, 16, tb, k, 1.0, 16, tc, m, comp)
        assert st == 0
        return pl
    monkeypatch.delenv("MDGEMM_PACK", raising=False)
    big = plan(4096, 2048, 512)                     # 16 x 8 = 128 tiles
    assert "packed" in big["kernel"] and big["tile_m"] == 256 and big["tile_n"] == 256
    assert big["workgroups"] == 16 * 8
    assert "packed" not in plan(4096, 1792, 512)["kernel"]    # 112 tiles
    assert "packed" not in plan(4096, 4096, 100)["kernel"]    # k' < 256
    ccs = plan(4096, 4096, 256, "c", "c", "s")                # case 2ac: m' = 8192
    assert "packed" in ccs["kernel"] and ccs["workgroups"] == 32 * 16
    assert "packed" not in plan(8192, 8192, 8192, comp="s")["kernel"]
    assert "packed" not in plan(8192, 8192, 8192, ta="h", tb="h", comp="bf16x3")["kernel"]
    monkeypatch.setenv("MDGEMM_PACK", "0")
    assert "packed" not in plan(8192, 8192, 8192)["kernel"]
    monkeypatch.setenv("MDGEMM_PACK", "2")
    small = plan(40, 30, 20)
    assert "packed" in small["kernel"] and small["workgroups"] == 1
