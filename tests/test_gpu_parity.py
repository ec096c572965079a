"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every test prints the case it is about to run (flushed) so that a failure on
the device names its combination, shape and entry point.
"""
import itertools
import sys

import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_1901_06015_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu
TAGS = ("s", "d", "c", "z")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _lib.lib()
    yield


# Products with few tiles run on the small kernel by default; "tiled" runs the
# same tests with MDGEMM_SMALL=0, on the tiled kernels (fast, ragged and
# component-wise loads, split k).
PATHS = ["small", "tiled"]


@pytest.fixture
def path(request, monkeypatch):
    if request.param == "tiled":
        monkeypatch.setenv("MDGEMM_SMALL", "0")
    else:
        monkeypatch.delenv("MDGEMM_SMALL", raising=False)
    return request.param


@pytest.fixture
def tiled(monkeypatch):
    monkeypatch.setenv("MDGEMM_SMALL", "0")


def one(tc, ta, tb, m, n, k, comp, transa="N", transb="N", alpha=1.5, beta=-0.5, **kw):
    say("mdgemm %s%s%s comp=%s %s%s m=%d n=%d k=%d %r" % (tc, ta, tb, comp, transa, transb, m, n, k, kw))
    st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, transa=transa, transb=transb,
                           alpha=alpha, beta=beta, **kw)
    assert st == 0, (st, _lib.strerror(st))
    ref, g = gu.reference(tc, ta, tb, m, n, k, ops, transa, transb, alpha, beta)
    r = gu.check(tc, comp, k, Cout, m, n, ref, g, what="%s%s%s/%s" % (tc, ta, tb, comp))
    gu.check_padding(Cout, m, "C")
    return r, Cout, ref, ops


@pytest.mark.parametrize("comp", ["s", "d"])
@pytest.mark.parametrize("tc", TAGS)
@pytest.mark.parametrize("path", PATHS, indirect=True)
def test_all_storage_combinations(tc, comp, path):
    """All 16 (A, B) storage pairs for this C and computation precision, at a
    size that spans several workgroup tiles and k tiles with ragged edges."""
    for ta, tb in itertools.product(TAGS, TAGS):
        one(tc, ta, tb, 150, 140, 70, comp)


@pytest.mark.parametrize("transa,transb", list(itertools.product("NTCR", "NTCR")))
@pytest.mark.parametrize("path", PATHS, indirect=True)
def test_transpose_variants(transa, transb, path):
    """The nine op(A), op(B) combinations of Section 1 plus conjugation
    without transposition (R, Section 3), on a combination of every domain
    case."""
    combos = ["ddd", "sdc", "dzs", "scz", "csd", "zdz", "czs", "zcz"]
    for i, cab in enumerate(combos):
        comp = "sd"[i % 2]
        one(cab[0], cab[1], cab[2], 77, 93, 41, comp, transa, transb)


@pytest.mark.parametrize("comp", ["s", "d"])
@pytest.mark.parametrize("path", PATHS, indirect=True)
def test_exact_inputs_bitwise(comp, path):
    """Integer entries in [-4, 4], alpha = 1.5, beta = -0.5: every rounding in
    either precision is exact, so the GPU must equal the oracle bit for bit,
    whatever its summation order."""
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        say("exact %s%s%s comp=%s" % (tc, ta, tb, comp))
        m, n, k = 70, 66, 45
        st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, dist="int", seed=11)
        assert st == 0
        ref, _ = gu.reference(tc, ta, tb, m, n, k, ops)
        got = np.asarray(Cout[:m, :n], dtype=np.complex128)
        assert np.array_equal(got, ref), "exact %s%s%s/%s: %d mismatches" % (
            tc, ta, tb, comp, int((got != ref).sum()))


@pytest.mark.parametrize("cab", ["zcd", "ccs", "zzz", "sdd", "dcz", "csz", "zss", "szc"])
@pytest.mark.parametrize("path", PATHS, indirect=True)
def test_edge_sizes(cab, path):
    """Tile edges and degenerate sizes (0 and 1 included), both precisions."""
    sizes = (0, 1, 2, 3, 5, 17, 33, 65, 129)
    rng = np.random.Generator(np.random.PCG64(5))
    for comp in ("s", "d"):
        for _ in range(10):
            m, n, k = (int(x) for x in rng.choice(sizes, 3))
            one(cab[0], cab[1], cab[2], m, n, k, comp)


@pytest.mark.parametrize("path", PATHS, indirect=True)
def test_unaligned_leading_dimensions(path):
    """Odd leading dimensions defeat 16-byte loads: the component-wise load
    path must give the same result; the padding rows are never written."""
    for cab, comp in (("zcd", "d"), ("sds", "s"), ("czz", "s"), ("dzc", "d")):
        one(cab[0], cab[1], cab[2], 131, 67, 53, comp, pad_a=1, pad_b=3, pad_c=5)
        one(cab[0], cab[1], cab[2], 131, 67, 53, comp, "T", "C", pad_a=2, pad_b=1, pad_c=2)


def test_complex_scalars_case3():
    """Case 3 uses a complex alpha and a complex beta (Section 7.2)."""
    for cab in ("zzz", "ccc", "zcz", "czc"):
        assert oracle.get().case(cab[0], cab[1], cab[2]) == "3"
        for comp in ("s", "d"):
            one(cab[0], cab[1], cab[2], 90, 70, 50, comp, alpha=0.75 - 0.5j, beta=0.5 + 0.25j)


def test_complex_beta_mixed_cases():
    """Complex beta is honoured whenever C is complex (cases 1c, 2ac, 2bc);
    a complex beta on a real C acts through Re(beta) only."""
    for cab in ("zdd", "czs", "zsz", "dcz", "sdc"):
        for comp in ("s", "d"):
            one(cab[0], cab[1], cab[2], 70, 50, 30, comp, alpha=1.25, beta=0.5 - 0.75j)


def test_case_1c_imaginary_part():
    """Case 1c: AB reaches only Re(C); Im(C) is beta*Im(C) exactly (beta real)."""
    for tc in ("c", "z"):
        for beta in (1.0, -0.5):
            _, Cout, ref, ops = one(tc, "d", "s", 100, 60, 40, "s", beta=beta)
            C0 = ops["C"][:100, :60]
            assert np.array_equal(Cout[:100, :60].imag, (beta * C0.imag).astype(C0.imag.dtype))


def test_beta_zero_does_not_read_c_and_alpha_zero_does_not_read_ab():
    import torch as T
    m, n, k = 40, 30, 20
    for cab in ("zcd", "sss", "dzz"):
        tc, ta, tb = cab
        A = gu.to_device(gu.inputs.matrix(m, k, ta, 1))
        B = gu.to_device(gu.inputs.matrix(k, n, tb, 2))
        C = gu.to_device(gu.inputs.matrix(m, n, tc, 3))
        C.fill_(float("nan"))
        say("beta=0 NaN C", cab)
        st = _lib.mdgemm("N", "N", m, n, k, 1.0, A.data_ptr(), ta, m, B.data_ptr(), tb, k, 0.0,
                         C.data_ptr(), tc, m, None, T.cuda.current_stream().cuda_stream)
        T.cuda.synchronize()
        assert st == 0 and bool(T.isfinite(C).all())
        A.fill_(float("nan"))
        C2h = gu.inputs.matrix(m, n, tc, 4)
        C2 = gu.to_device(C2h)
        say("alpha=0 NaN A", cab)
        st = _lib.mdgemm("N", "N", m, n, k, 0.0, A.data_ptr(), ta, m, B.data_ptr(), tb, k, -0.5,
                         C2.data_ptr(), tc, m, None, T.cuda.current_stream().cuda_stream)
        T.cuda.synchronize()
        assert st == 0
        assert np.array_equal(C2.cpu().numpy(), (-0.5 * C2h).astype(C2h.dtype))


def test_error_leaves_c_untouched():
    m, n, k = 16, 16, 16
    A = gu.to_device(gu.inputs.matrix(m, k, "c", 1))
    B = gu.to_device(gu.inputs.matrix(k, n, "s", 2))
    Ch = gu.inputs.matrix(m, n, "s", 3)
    C = gu.to_device(Ch)
    st = _lib.mdgemm("N", "N", m, n, k, 1.0 + 1.0j, A.data_ptr(), "c", m, B.data_ptr(), "s", k,
                     1.0, C.data_ptr(), "s", m, None, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == _lib.MD_ERR_ALPHA_IMAG
    assert np.array_equal(C.cpu().numpy(), Ch)


def test_paper_config_zcdd_256():
    """Single mixed GEMM: m=n=k=256, A single complex, B double real, C double
    complex, double computation, alpha = beta = 1, full oracle comparison."""
    one("z", "c", "d", 256, 256, 256, "d", alpha=1.0, beta=1.0, seed=2019)


def test_stream_argument():
    """Work is enqueued on the caller's stream."""
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        st, Cout, ops = gu.run("z", "z", "d", 64, 64, 64, comp="d", stream=s.cuda_stream)
    assert st == 0
    ref, g = gu.reference("z", "z", "d", 64, 64, 64, ops)
    gu.check("z", "d", 64, Cout, 64, 64, ref, g)


# ---------------------------------------------------------------------------
# BF16x3: single-precision semantics from three bf16 products per real product
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tc", TAGS)
def test_bf16x3_exact_inputs_bitwise(tc):
    """Integers in [-4, 4] are exact in bf16 (lo = 0) and every partial sum is
    exact in FP32, so the BF16x3 path must equal the oracle bit for bit."""
    for ta, tb in itertools.product(TAGS, TAGS):
        say("bf16x3 exact %s%s%s" % (tc, ta, tb))
        m, n, k = 70, 66, 45
        st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp="bf16x3", dist="int", seed=13)
        assert st == 0, st
        ref, _ = gu.reference(tc, ta, tb, m, n, k, ops)
        got = np.asarray(Cout[:m, :n], dtype=np.complex128)
        assert np.array_equal(got, ref), "bf16x3 exact %s%s%s: %d mismatches" % (
            tc, ta, tb, int((got != ref).sum()))


@pytest.mark.parametrize("tc", TAGS)
def test_bf16x3_within_single_precision_bound(tc):
    """Random inputs at k from 16 to 130: within 4 k u_s (|A||B|) plus the
    split's per-product term 3 * 2^-16 |a||b| (BF16X3_SPLIT), so the check
    holds worst-case at every k, below the k ~ 192 where 4 k u_s alone would
    cover the split."""
    for i, (ta, tb) in enumerate(itertools.product(TAGS, TAGS)):
        one(tc, ta, tb, 150, 140, (16, 47, 130)[i % 3], "bf16x3")


def test_bf16x3_transposes_and_loguniform():
    for transa, transb in (("T", "N"), ("N", "T"), ("C", "C")):
        for cab in ("sss", "css", "ccs", "ccc", "zdz"):
            one(cab[0], cab[1], cab[2], 131, 97, 160, "bf16x3", transa, transb)
    for cab in ("sss", "css", "ccs", "ccc"):
        one(cab[0], cab[1], cab[2], 128, 128, 256, "bf16x3", dist="loguniform", beta=0.0)


# BF16x3 on packed operands (cast, split and packed once, then multiplied from
# direct LDS copies): forced at every size with MDGEMM_PACK=2.
@pytest.fixture
def packed(monkeypatch):
    monkeypatch.setenv("MDGEMM_PACK", "2")


def _plan_kernel(tc, ta, tb, m, n, k, comp, transa="N", transb="N"):
    ar = m if transa in "NR" else k
    br = k if transb in "NR" else n
    st, pl = _lib.mdgemm_plan(transa, transb, m, n, k, 1.5, 1, ta, ar, 1, tb, br, -0.5, 1, tc, m, comp)
    assert st == 0
    return pl["kernel"]


@pytest.mark.parametrize("cab", ["sss", "css", "ccs", "ccc", "scs", "scc", "zdz", "dzd", "zzz", "czd", "sdc",
                                 "dcc"])
def test_bf16x3_packed_all_cases_and_ops(cab, packed):
    """Every case, double- and single-stored operands, the op pairs, ragged m,
    n and k (none a multiple of the 256 x 256 x 32 packed tile): within the
    BF16x3 bound; ld padding of C untouched."""
    tc, ta, tb = cab
    for i, (transa, transb) in enumerate((("N", "N"), ("T", "N"), ("N", "C"), ("C", "T"), ("R", "N"))):
        m, n, k = (300, 270, 77) if i % 2 == 0 else (97, 333, 130)
        assert "packed" in _plan_kernel(tc, ta, tb, m, n, k, "bf16x3", transa, transb)
        one(tc, ta, tb, m, n, k, "bf16x3", transa, transb, seed=31 + i)


def test_bf16x3_packed_exact_inputs_bitwise(packed):
    """Exact inputs: bitwise equal to the oracle.  m and n above 256 and k
    above 64, so both operands have packed blocks wholly inside the matrix
    (the pack's unchecked fast path) and blocks on the edges (the general
    path), each operand stored along m/n ('N' A, 'T' B) and along k."""
    for tc, ta, tb in itertools.product("sc", "sdcz", "sdcz"):
        for transa, transb in (("N", "N"), ("T", "C")):
            say("bf16x3 packed exact %s%s%s %s%s" % (tc, ta, tb, transa, transb))
            m, n, k = 260, 264, 70
            st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp="bf16x3", dist="int", seed=17,
                                   transa=transa, transb=transb)
            assert st == 0, st
            ref, _ = gu.reference(tc, ta, tb, m, n, k, ops, transa, transb)
            got = np.asarray(Cout[:m, :n], dtype=np.complex128)
            assert np.array_equal(got, ref), "packed exact %s%s%s %s%s: %d mismatches" % (
                tc, ta, tb, transa, transb, int((got != ref).sum()))


def test_bf16x3_packed_beta_zero_and_half_c(packed):
    """beta = 0 does not read C (NaN there stays out); a binary16 C takes the
    general epilogue of the packed kernel."""
    one("c", "c", "s", 270, 260, 64, "bf16x3", beta=0.0)
    for tc in ("h", "hc"):
        say("bf16x3 packed half C", tc)
        st, Cout, ops = gu.run(tc, "s", "c" if tc == "hc" else "s", 140, 300, 96, comp="bf16x3", seed=5)
        assert st == 0, st
        ref, g = gu.reference(tc, "s", "c" if tc == "hc" else "s", 140, 300, 96, ops)
        gu.check(tc, "bf16x3", 96, Cout, 140, 300, ref, g, what="packed half C %s" % tc)


@pytest.mark.parametrize("layouts", list(itertools.product(("col", "row", "gen", "genr"), repeat=3)))
def test_row_and_column_strides(layouts):
    """Section 3's row and column strides: every operand stored by columns, by
    rows (with spare elements between columns/rows) or in general storage
    (neither stride 1), on a combination of every domain case and all four
    ops; elements outside C's block are never written."""
    combos = ["ddd", "sdc", "dzs", "scz", "csd", "zdz", "czs", "zcz"]
    for i, cab in enumerate(combos):
        comp = "sd"[i % 2]
        transa, transb = "NTCR"[i % 4], "RCTN"[(i // 2) % 4]
        for m, n, k, pads in ((77, 93, 41, (0, 0, 0)), (130, 66, 35, (3, 1, 2))):
            say("strided %s%s%s comp=%s %s%s %s m=%d n=%d k=%d pads=%r" % (
                cab[0], cab[1], cab[2], comp, transa, transb, "/".join(layouts), m, n, k, pads))
            st, got, pad_ok, ref, g = gu.run_strided(cab[0], cab[1], cab[2], m, n, k, layouts, comp,
                                                     transa, transb, pads=pads, seed=31 + i)
            assert st == 0, (st, _lib.strerror(st))
            gu.check(cab[0], comp, k, got, m, n, ref, g, what="strided %s %s%s %s" % (
                cab, transa, transb, "/".join(layouts)))
            assert pad_ok, "elements outside C's block were written"


def test_row_major_torch_tensors():
    """api.gemm on torch's default (row-major) tensors, mixed with
    column-major ones, against the oracle given the same strides."""
    o = oracle.get()
    for i, (tc, ta, tb, transa, transb, comp) in enumerate((
            ("z", "c", "d", "N", "N", "d"), ("s", "d", "z", "T", "R", "s"),
            ("c", "z", "c", "R", "C", "s"), ("d", "d", "d", "N", "T", "d"))):
        m, n, k = 150, 70, 99
        say("api.gemm row-major %s%s%s %s%s comp=%s" % (tc, ta, tb, transa, transb, comp))
        ash = (m, k) if transa in "NR" else (k, m)
        bsh = (k, n) if transb in "NR" else (n, k)
        XA = np.ascontiguousarray(inputs.matrix(ash[0], ash[1], ta, 50 + 3 * i))
        XB = inputs.matrix(bsh[0], bsh[1], tb, 51 + 3 * i)
        XC = np.ascontiguousarray(inputs.matrix(m, n, tc, 52 + 3 * i))
        A = torch.from_numpy(XA).cuda()                            # stored by rows
        B = torch.from_numpy(np.ascontiguousarray(XB.T)).cuda().t()  # stored by columns
        C = torch.from_numpy(XC).cuda()                            # stored by rows
        assert A.stride() == (k if transa in "NR" else m, 1) and B.stride(0) == 1 and C.stride() == (n, 1)
        api.gemm(A, B, C, alpha=1.5, beta=-0.5, transa=transa, transb=transb, comp=comp)
        torch.cuda.synchronize()
        st, ref, g = o.gemm_gs(transa, transb, m, n, k, 1.5, XA.ravel(), ta, ash[1], 1,
                               np.ascontiguousarray(XB.T).ravel(), tb, 1, bsh[0],
                               -0.5, XC.ravel(), tc, n, 1)
        assert st == 0
        gu.check(tc, comp, k, C.cpu().numpy(), m, n, ref, g, what="api row-major %s%s%s" % (tc, ta, tb))


def test_sliced_torch_tensors():
    """api.gemm on strided slices (general storage: neither stride 1) of
    larger tensors, against the oracle on the same host buffers."""
    o = oracle.get()
    m, n, k = 90, 70, 50
    for i, (tc, ta, tb, transa, transb, comp) in enumerate((("z", "c", "d", "N", "T", "d"),
                                                            ("c", "s", "z", "R", "N", "s"))):
        say("api.gemm slices %s%s%s %s%s comp=%s" % (tc, ta, tb, transa, transb, comp))
        ash = (m, k) if transa in "NR" else (k, m)
        bsh = (k, n) if transb in "NR" else (n, k)
        bigs = [np.ascontiguousarray(inputs.matrix(2 * r + 1, 3 * c + 2, dt, 60 + 3 * i + j))
                for j, ((r, c), dt) in enumerate(((ash, ta), (bsh, tb), ((m, n), tc)))]
        dev = [torch.from_numpy(b).cuda() for b in bigs]
        A, B, C = (d[1::2, 2::3] for d in dev)
        assert A.shape == ash and B.shape == bsh and C.shape == (m, n)
        assert min(A.stride()) > 1 and min(C.stride()) > 1
        refs = []
        for t, b in zip((A, B, C), bigs):
            refs.append((b.ravel()[t.storage_offset():], t.stride(0), t.stride(1)))
        st, ref, g = o.gemm_gs(transa, transb, m, n, k, 1.5, refs[0][0], ta, refs[0][1], refs[0][2],
                               refs[1][0], tb, refs[1][1], refs[1][2], -0.5, refs[2][0], tc, refs[2][1], refs[2][2])
        assert st == 0
        api.gemm(A, B, C, alpha=1.5, beta=-0.5, transa=transa, transb=transb, comp=comp)
        torch.cuda.synchronize()
        gu.check(tc, comp, k, C.cpu().numpy(), m, n, ref, g, what="slices %s%s%s" % (tc, ta, tb))
        # the elements between the slices are untouched
        out = dev[2].cpu().numpy()
        keep = np.ones(out.shape, dtype=bool)
        keep[1::2, 2::3] = False
        assert np.array_equal(out[keep], bigs[2][keep])


MIXED = {"1a": ("scs", "dcd", "szs"), "1b": ("ssc", "dsz", "sdc"), "1c": ("css", "zdd", "zsd"),
         "2ab": ("scc", "dzc", "szz"), "2ac": ("ccs", "zcd", "czs"), "2bc": ("csc", "zdz", "cdc")}


@pytest.mark.parametrize("case", sorted(MIXED))
def test_literal_complex_alpha(case):
    """MD_COMP_LITERAL_ALPHA: Im(alpha) != 0 in the six mixed cases, applied as
    the literal interpretation of Section 7.2 (the oracle's literal variant),
    in both precisions and BF16x3, with every op on both operands, on the fast
    path, the ragged/unaligned path and the component-wise path."""
    alpha, beta = 0.75 - 0.5j, -0.5 + 0.25j
    for i, cab in enumerate(MIXED[case]):
        for comp in ("s+literal", "d+literal", "bf16x3+literal"):
            transa, transb = "NTCR"[i % 4], "CRNT"[(i + len(comp)) % 4]
            for m, n, k, pads in ((150, 140, 112, (0, 0, 0)), (77, 93, 97, (1, 3, 2))):
                say("literal alpha %s %s %s %s%s m=%d n=%d k=%d pads=%r" % (case, cab, comp, transa, transb,
                                                                         m, n, k, pads))
                st, Cout, ops = gu.run(cab[0], cab[1], cab[2], m, n, k, comp=comp, transa=transa, transb=transb,
                                       alpha=alpha, beta=beta, seed=40 + i, pad_a=pads[0], pad_b=pads[1],
                                       pad_c=pads[2])
                assert st == 0, (st, _lib.strerror(st))
                ref, g = gu.reference(cab[0], cab[1], cab[2], m, n, k, ops, transa, transb, alpha, beta,
                                      literal_alpha=True)
                gu.check(cab[0], comp, k, Cout, m, n, ref, g, what="literal %s %s %s" % (case, cab, comp))
                gu.check_padding(Cout, m, "C")
        # without the flag the paper's policy still refuses
        st, _, _ = gu.run(cab[0], cab[1], cab[2], 8, 8, 8, comp="d", alpha=alpha, beta=beta)
        assert st == _lib.MD_ERR_ALPHA_IMAG


def test_literal_complex_alpha_exact_inputs_bitwise():
    """Integer entries, alpha = 0.75 - 0.5i, beta = -0.5: the staged alpha*x and
    every sum are exact, so all 48 mixed-case combinations equal the oracle's
    literal result bit for bit."""
    o = oracle.get()
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        if o.case(tc, ta, tb) in ("0", "3"):
            continue
        for comp in ("s+literal", "d+literal"):
            say("literal exact %s%s%s %s" % (tc, ta, tb, comp))
            m, n, k = 70, 66, 45
            st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, dist="int", seed=13, alpha=0.75 - 0.5j,
                                   transa="C" if ta in "cz" else "N")
            assert st == 0
            ref, _ = gu.reference(tc, ta, tb, m, n, k, ops, "C" if ta in "cz" else "N", "N", 0.75 - 0.5j,
                                  literal_alpha=True)
            got = np.asarray(Cout[:m, :n], dtype=np.complex128)
            assert np.array_equal(got, ref), "literal exact %s%s%s/%s: %d mismatches" % (
                tc, ta, tb, comp, int((got != ref).sum()))


HALF_MIX = [("h", "h", "h"), ("hc", "hc", "hc"), ("s", "h", "h"), ("z", "hc", "d"), ("h", "z", "s"),
            ("hc", "c", "h"), ("h", "hc", "hc"), ("hc", "h", "z"), ("d", "hc", "h"), ("c", "s", "hc"),
            ("hc", "d", "s"), ("h", "hc", "z")]


@pytest.mark.parametrize("comp", ["s", "d", "h", "bf16x3"])
def test_half_storage(comp):
    """Binary16 storage (h, hc) for A, B and C in every domain case, each
    computation precision, all ops, unaligned leading dimensions; a half C
    rounds once to binary16 (u_C = 2^-11)."""
    for i, (tc, ta, tb) in enumerate(HALF_MIX):
        transa, transb = "NTCR"[i % 4], "RNTC"[(i // 2) % 4]
        m, n, k = (77, 93, 41) if comp != "bf16x3" else (77, 93, 112)
        say("half storage %s/%s/%s comp=%s %s%s" % (tc, ta, tb, comp, transa, transb))
        st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, transa=transa, transb=transb, seed=70 + i,
                               pad_a=i % 3, pad_b=(i + 1) % 3, pad_c=1)
        assert st == 0, (st, _lib.strerror(st))
        ref, g = gu.reference(tc, ta, tb, m, n, k, ops, transa, transb)
        gu.check(tc, comp, k, Cout, m, n, ref, g, what="half %s/%s/%s/%s" % (tc, ta, tb, comp))
        gu.check_padding(Cout, m, "C")


def test_half_storage_exact_inputs_bitwise():
    """Integer inputs with half storage anywhere (k = 30 keeps every result
    exact in binary16): all three computation precisions give the oracle's
    value bit for bit, through the plain path and a quick return."""
    for i, (tc, ta, tb) in enumerate(HALF_MIX):
        for comp in ("s", "d", "h"):
            say("half exact %s/%s/%s comp=%s" % (tc, ta, tb, comp))
            m, n, k = 70, 66, 30
            st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, dist="int", seed=90 + i,
                                   transa="C" if i % 2 else "N")
            assert st == 0
            ref, _ = gu.reference(tc, ta, tb, m, n, k, ops, "C" if i % 2 else "N")
            got = inputs.to_complex128(Cout[:m, :n])
            assert np.array_equal(got, ref), "half exact %s/%s/%s/%s: %d mismatches" % (
                tc, ta, tb, comp, int((got != ref).sum()))
        st, Cout, ops = gu.run(tc, ta, tb, 20, 10, 0, comp="s", dist="int", seed=3)
        assert st == 0
        ref, _ = gu.reference(tc, ta, tb, 20, 10, 0, ops)
        assert np.array_equal(inputs.to_complex128(Cout[:20, :10]), ref), "half quick return %s/%s/%s" % (tc, ta, tb)


@pytest.mark.parametrize("tc", TAGS)
def test_half_computation_precision(tc):
    """MD_COMP_H on s/d/c/z storage (the fp16 matrix-core kernels, fast path):
    every (A, B) pair within the half bound, tiles with ragged edges."""
    for ta, tb in itertools.product(TAGS, TAGS):
        for transa, transb, m, n, k in (("N", "N", 150, 140, 70), ("T", "C", 131, 67, 53)):
            one(tc, ta, tb, m, n, k, "h", transa, transb)


def test_half_computation_exact_inputs_bitwise():
    """Integer inputs are exact in binary16 and every sum is exact in FP32:
    MD_COMP_H equals the oracle bit for bit on all 64 combinations."""
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        say("half comp exact %s%s%s" % (tc, ta, tb))
        m, n, k = 70, 66, 45
        st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp="h", dist="int", seed=17)
        assert st == 0
        ref, _ = gu.reference(tc, ta, tb, m, n, k, ops)
        got = np.asarray(Cout[:m, :n], dtype=np.complex128)
        assert np.array_equal(got, ref), "half comp exact %s%s%s: %d mismatches" % (tc, ta, tb, int((got != ref).sum()))


@pytest.mark.parametrize("comp", ["s", "h"])
def test_half_fast_path(comp):
    """Binary16 A and B on the 16-byte fast loads (single and half precision):
    every op pair, ragged k (chunks of 8 binary16 components), tile edges,
    half and wider C; the plan confirms the fast or ragged kernel."""
    combos = [("h", "h", "h"), ("s", "h", "h"), ("hc", "hc", "hc"), ("z", "h", "hc"), ("c", "hc", "h"),
              ("h", "h", "hc"), ("hc", "hc", "h"), ("d", "hc", "hc")]
    for i, (tc, ta, tb) in enumerate(combos):
        for transa, transb in (("N", "N"), ("T", "C"), ("R", "T"), ("C", "R")):
            m, n, k = (150, 140, 70) if i % 2 == 0 else (98, 131, 41)
            ar = m if transa in "NR" else k
            br = k if transb in "NR" else n
            pad_a, pad_b = ar % 2, br % 2 + 2    # whole 4-byte words per stored column
            st, pl = _lib.mdgemm_plan(transa, transb, m, n, k, 1.5, 0x1000, ta, ar + pad_a, 0x1000, tb, br + pad_b,
                                      -0.5, 0x1000, tc, m + 1, comp)
            assert st == 0 and ("_fast_" in pl["kernel"] or "_ragged_" in pl["kernel"]), pl["kernel"]
            one(tc, ta, tb, m, n, k, comp, transa, transb, pad_a=pad_a, pad_b=pad_b, pad_c=1)


def test_half_fast_path_exact_inputs_bitwise():
    """Integer inputs through the binary16 fast loads: bit for bit."""
    for tc, ta, tb in (("h", "h", "h"), ("s", "h", "h"), ("hc", "hc", "hc"), ("z", "hc", "h")):
        for comp in ("s", "h"):
            say("half fast exact %s/%s/%s comp=%s" % (tc, ta, tb, comp))
            m, n, k = 70, 66, 30
            st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, dist="int", seed=29, transa="T", transb="C")
            assert st == 0
            ref, _ = gu.reference(tc, ta, tb, m, n, k, ops, "T", "C")
            got = inputs.to_complex128(Cout[:m, :n])
            assert np.array_equal(got, ref), "half fast exact %s/%s/%s/%s" % (tc, ta, tb, comp)


def test_half_torch_tensors():
    """api.gemm on torch.float16 / complex32 tensors (row-major and
    column-major), the default computation precision of a half C being half."""
    o = oracle.get()
    m, n, k = 90, 70, 64
    XA = inputs.matrix(m, k, "h", 1)
    XB = inputs.matrix(k, n, "hc", 2)
    XC = inputs.matrix(m, n, "hc", 3)
    A = torch.from_numpy(np.ascontiguousarray(XA)).cuda()          # float16, by rows
    B = gu.to_device(XB)                                            # complex32, by columns
    C = gu.to_device(XC)
    say("api.gemm half tensors")
    api.gemm(A, B, C, alpha=1.5, beta=-0.5)
    torch.cuda.synchronize()
    st, ref, g = o.gemm("N", "N", m, n, k, 1.5, XA, "h", m, XB, "hc", k, -0.5, XC, "hc", m)
    assert st == 0
    gu.check("hc", "h", k, gu.to_host(C), m, n, ref, g, what="api half tensors")


@pytest.mark.parametrize("comp", ["s", "d"])
def test_split_k_small_tiles(comp, tiled):
    """Products with few tiles and a deep k split k over several workgroups
    (partials in the computation type, summed in split order, one epilogue):
    every domain case, fast and component-wise loads, ragged k, a half C."""
    combos = ["ddd", "sdc", "dzs", "scz", "csd", "zdz", "czs", "zcz", "hss", "hcz"]
    for i, cab in enumerate(combos):
        tc, ta, tb = (cab[0], cab[1], cab[2]) if cab[0] != "h" else (("h", "s", "s") if i == 8 else ("hc", "c", "z"))
        m, n, k = (100, 90, 2000) if i % 2 == 0 else (70, 130, 1531)
        pad = 1 if i % 3 == 2 else 0
        st, pl = _lib.mdgemm_plan("T" if i % 4 == 1 else "N", "N", m, n, k, 1.5, 0x1000, ta,
                                  k if i % 4 == 1 else m + pad, 0x1000, tb, k, -0.5, 0x1000, tc, m, comp)
        assert st == 0 and pl["workgroups"] * 2 <= 256, pl
        one(tc, ta, tb, m, n, k, comp, "T" if i % 4 == 1 else "N", "N", pad_a=0 if i % 4 == 1 else pad)


def test_split_k_exact_and_strided(tiled):
    """Split k on integer inputs gives the oracle bit for bit; a general-stride
    and a row-major C through the split path stay within the bound."""
    for tc, ta, tb, comp in (("z", "c", "d", "d"), ("s", "s", "s", "s"), ("c", "z", "z", "s"), ("d", "d", "c", "d")):
        say("split exact %s%s%s/%s" % (tc, ta, tb, comp))
        m, n, k = 64, 96, 1024
        st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, dist="int", seed=5)
        assert st == 0
        ref, _ = gu.reference(tc, ta, tb, m, n, k, ops)
        got = np.asarray(Cout[:m, :n], dtype=np.complex128)
        assert np.array_equal(got, ref), "split exact %s%s%s/%s" % (tc, ta, tb, comp)
    for layouts in (("col", "col", "gen"), ("row", "col", "row")):
        say("split strided", layouts)
        st, got, pad_ok, ref, g = gu.run_strided("z", "c", "d", 60, 50, 1200, layouts, "d", "N", "T", seed=3)
        assert st == 0 and pad_ok
        gu.check("z", "d", 1200, got, 60, 50, ref, g, what="split strided %s" % (layouts,))


def test_huge_leading_dimension_generic_path():
    """A stored along m with a leading dimension above 2^20: its fast tile
    spans only its k extent of columns, so the 32-bit tile offsets still fit
    and the result is the same as at any other ld."""
    for cab, comp in (("zcd", "d"), ("sds", "s")):
        one(cab[0], cab[1], cab[2], 40, 24, 8, comp, pad_a=(1 << 20) - 40 + 8)


@pytest.mark.parametrize("comp", ["h", "d"])
def test_large_ld_operand_stored_along_k(comp):
    """B (z, 'N') stored along k with ld = 600000 spans one column per n of
    its tile: under the half precision's 256-wide tiles, 240 columns of
    600000 x 16 bytes pass 2 GiB, so the planner must leave the 32-bit fast
    kernels (Section 2.2.1 storage: any ld >= rows is valid and must not change
    the result).  Under the double precision (128-wide tiles) the fast kernel
    still fits and runs.  Case 1b: C and A single real, B double complex."""
    m, n, k, ldb = 64, 240, 40, 600000
    st, p = _lib.mdgemm_plan("N", "N", m, n, k, 1.5, 0x1000, "s", m, 0x1000, "z", ldb, -0.5, 0x1000, "s", m, comp)
    assert st == 0
    assert ("generic" in p["kernel"]) == (comp == "h"), p["kernel"]
    say("large ld along k:", p["kernel"])
    one("s", "s", "z", m, n, k, comp, pad_b=ldb - k)


@pytest.mark.parametrize("comp", ["s", "d"])
def test_small_kernel_k_edges(comp):
    """The small kernel at inner dimensions around its wave split and step
    size (k' = 1 .. 9, odd, at its limit) and tile edges, every case."""
    combos = ["ddd", "sdc", "dzs", "scz", "csd", "zdz", "czs", "zcz"]
    for i, cab in enumerate(combos):
        for k in (1, 2, 3, 5, 9, 31, 33):
            one(cab[0], cab[1], cab[2], 33 + i, 47 - i, k, comp, "NTCR"[i % 4], "NTCR"[(i + k) % 4])
        kmax = 2048 // (2 if cab[1] in "cz" and cab[2] in "cz" else 1)
        one(cab[0], cab[1], cab[2], 65, 31, kmax, comp)


def test_small_kernel_exact_inputs_bitwise():
    """Integer inputs on the small kernel: bitwise equal to the oracle."""
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        for comp in ("s", "d"):
            st, Cout, ops = gu.run(tc, ta, tb, 70, 66, 300, comp=comp, dist="int", seed=21)
            assert st == 0
            ref, _ = gu.reference(tc, ta, tb, 70, 66, 300, ops)
            got = np.asarray(Cout[:70, :66], dtype=np.complex128)
            assert np.array_equal(got, ref), "small exact %s%s%s/%s" % (tc, ta, tb, comp)


def test_two_threads_share_a_stream_split_and_packed(monkeypatch):
    """Two host threads enqueue products on the same stream at once: split-k
    products (few tiles, deep k) and packed BF16x3 products, shapes growing
    so that the per-stream workspaces are reallocated while the other thread
    is using them.  Every result must match the oracle."""
    import threading
    monkeypatch.setenv("MDGEMM_SMALL", "0")
    monkeypatch.setenv("MDGEMM_PACK", "2")
    stream = torch.cuda.current_stream().cuda_stream
    jobs = [[], []]
    for t in range(2):
        for i in range(4):
            if (i + t) % 2 == 0:
                cab, comp, (m, n, k) = ("zcd" if t == 0 else "dzz"), "d", (130 + 40 * i, 120 + 30 * t, 2000 + 500 * i)
            else:
                cab, comp, (m, n, k) = ("ccs" if t == 0 else "sdc"), "bf16x3", (90 + 70 * i, 260 + 50 * t, 300 + 200 * i)
            tc, ta, tb = cab
            A = inputs.matrix(m, k, ta, 900 + 10 * i + t)
            B = inputs.matrix(k, n, tb, 950 + 10 * i + t)
            C = inputs.matrix(m, n, tc, 990 + 10 * i + t)
            jobs[t].append(dict(cab=cab, comp=comp, m=m, n=n, k=k, A=A, B=B, C=C,
                                dA=gu.to_device(A), dB=gu.to_device(B), dC=gu.to_device(C)))
    torch.cuda.synchronize()
    status = [[], []]

    def worker(t):
        for j in jobs[t]:
            tc, ta, tb = j["cab"]
            st = _lib.mdgemm("N", "N", j["m"], j["n"], j["k"], 1.5, j["dA"].data_ptr(), ta, j["A"].shape[0],
                             j["dB"].data_ptr(), tb, j["B"].shape[0], -0.5, j["dC"].data_ptr(), tc, j["C"].shape[0],
                             j["comp"], stream)
            status[t].append(st)

    say("two threads on one stream: split-k and packed products")
    threads = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert status == [[0] * 4, [0] * 4], status
    for t in range(2):
        for j in jobs[t]:
            tc, ta, tb = j["cab"]
            say("check %s comp=%s %dx%dx%d (thread %d)" % (j["cab"], j["comp"], j["m"], j["n"], j["k"], t))
            plan = _plan_kernel(tc, ta, tb, j["m"], j["n"], j["k"], j["comp"])
            assert ("packed" in plan) == (j["comp"] == "bf16x3"), plan
            ref, g = gu.reference(tc, ta, tb, j["m"], j["n"], j["k"], dict(A=j["A"], B=j["B"], C=j["C"]))
            gu.check(tc, j["comp"], j["k"], gu.to_host(j["dC"]), j["m"], j["n"], ref, g,
                     what="threaded %s/%s" % (j["cab"], j["comp"]))
