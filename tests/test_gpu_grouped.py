"""GPU parity of the grouped form: many products of uneven shapes, mixed storage
types and computation precisions in one persistent launch, each checked against
the CPU oracle (elementwise bound), plus exact-input bitwise checks, the
quick-return entries (alpha = 0, k = 0, m = 0) and the tile-shape table."""
import itertools
import sys

import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_1901_06015_amd import _lib, inputs

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
    _lib.tune_load(None)
    yield
    _lib.tune_load(None)


def make_entries(count, seed, lo=1, hi=300, dist="uniform", comps=("s", "d", "bf16x3")):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        tc, ta, tb = (TAGS[j] for j in rng.integers(0, 4, 3))
        comp = comps[int(rng.integers(0, len(comps)))]
        m, n, k = (int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1))))) for _ in range(3))
        transa, transb = "NTCR"[int(rng.integers(0, 4))], "NTCR"[int(rng.integers(0, 4))]
        case = oracle.get().case(tc, ta, tb)
        alpha = 0.75 - 0.5j if case == "3" else 1.5
        beta = (-0.5, 1.0, 0.0)[int(rng.integers(0, 3))]
        out.append(dict(tc=tc, ta=ta, tb=tb, comp=comp, m=m, n=n, k=k, transa=transa, transb=transb,
                        alpha=alpha, beta=beta, seed=seed * 1000 + i))
    return out


def run_grouped(entries, dist="uniform"):
    descs, keep = [], []
    for e in entries:
        ar, ac = (e["m"], e["k"]) if e["transa"] in "NR" else (e["k"], e["m"])
        br, bc = (e["k"], e["n"]) if e["transb"] in "NR" else (e["n"], e["k"])
        A = inputs.matrix(ar, ac, e["ta"], e["seed"] * 3 + 1, dist=dist)
        B = inputs.matrix(br, bc, e["tb"], e["seed"] * 3 + 2, dist=dist)
        C = inputs.matrix(e["m"], e["n"], e["tc"], e["seed"] * 3 + 3, ld=max(1, e["m"]) + 2, dist=dist,
                          pad=gu.SENTINEL)
        dA, dB, dC = gu.to_device(A), gu.to_device(B), gu.to_device(C)
        descs.append(_lib.make_desc(e["transa"], e["transb"], e["m"], e["n"], e["k"], e["alpha"],
                                    dA.data_ptr(), e["ta"], A.shape[0], dB.data_ptr(), e["tb"], B.shape[0],
                                    e["beta"], dC.data_ptr(), e["tc"], C.shape[0], e["comp"]))
        keep.append((A, B, C, dA, dB, dC))
    st = _lib.mdgemm_grouped(descs, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return st, keep


def check_all(entries, keep, exact=False):
    o = oracle.get()
    for e, (A, B, C, dA, dB, dC) in zip(entries, keep):
        st, ref, g = o.gemm(e["transa"], e["transb"], e["m"], e["n"], e["k"], e["alpha"], A, e["ta"],
                            A.shape[0], B, e["tb"], B.shape[0], e["beta"], C, e["tc"], C.shape[0],
                            literal_alpha="+literal" in str(e["comp"]))
        assert st == 0
        Cout = gu.to_host(dC)
        what = "%s%s%s/%s %s%s %dx%dx%d" % (e["tc"], e["ta"], e["tb"], e["comp"], e["transa"], e["transb"],
                                            e["m"], e["n"], e["k"])
        if exact:
            got = inputs.to_complex128(Cout[:e["m"], :e["n"]])
            assert np.array_equal(got, ref), what
        else:
            gu.check(e["tc"], e["comp"], e["k"], Cout, e["m"], e["n"], ref, g, what=what)
        gu.check_padding(Cout, e["m"], what)


def test_grouped_mixed_batch():
    entries = make_entries(96, seed=3)
    say("grouped batch of", len(entries))
    st, keep = run_grouped(entries)
    assert st == 0, (st, _lib.strerror(st))
    check_all(entries, keep)


def test_grouped_exact_inputs_bitwise():
    entries = make_entries(64, seed=5, hi=200, dist="int")
    say("grouped exact batch of", len(entries))
    st, keep = run_grouped(entries, dist="int")
    assert st == 0
    check_all(entries, keep, exact=True)


def test_grouped_literal_complex_alpha():
    """A grouped call mixing literal complex alphas in all six mixed cases
    (real-C cases run on the plain kernels inside the call, complex-C cases in
    the grouped kernel) with ordinary products: each matches the oracle."""
    entries = make_entries(40, seed=17)
    o = oracle.get()
    for i, e in enumerate(entries):
        if o.case(e["tc"], e["ta"], e["tb"]) not in ("0", "3") and e["comp"] != "bf16x3" and i % 2 == 0:
            e["alpha"] = 0.75 - 0.5j
            e["comp"] = e["comp"] + "+literal"
    assert sum("+literal" in e["comp"] for e in entries) >= 8
    say("grouped literal alpha batch of", len(entries))
    st, keep = run_grouped(entries)
    assert st == 0, (st, _lib.strerror(st))
    check_all(entries, keep)


def test_grouped_half_precision():
    """Binary16 storage and the half computation precision inside a grouped
    call (run on the plain kernels) next to ordinary products, one of them a
    quick return on a half C."""
    entries = make_entries(24, seed=23, comps=("s", "d"))
    halves = (("h", "h", "h", "h"), ("hc", "c", "h", "s"), ("z", "hc", "d", "d"), ("s", "d", "z", "h"),
              ("hc", "hc", "hc", "h"), ("h", "s", "hc", "s"))
    for i, (tc, ta, tb, comp) in enumerate(halves):
        e = entries[3 * i]
        e.update(tc=tc, ta=ta, tb=tb, comp=comp, alpha=1.5)
    entries[15]["alpha"] = 0.0
    say("grouped half batch of", len(entries))
    st, keep = run_grouped(entries)
    assert st == 0, (st, _lib.strerror(st))
    check_all(entries, keep)


def test_grouped_every_combination_once():
    entries = []
    for i, (tc, ta, tb) in enumerate(itertools.product(TAGS, TAGS, TAGS)):
        for comp in ("s", "d"):
            case = oracle.get().case(tc, ta, tb)
            entries.append(dict(tc=tc, ta=ta, tb=tb, comp=comp, m=40 + i, n=90 - i // 2, k=33 + i % 7,
                                transa="N", transb="N", alpha=1.5, beta=-0.5, seed=700 + 2 * i + (comp == "d")))
    say("grouped all combinations", len(entries))
    st, keep = run_grouped(entries)
    assert st == 0
    check_all(entries, keep)


def test_grouped_quick_returns_and_every_tile_configuration():
    """Every grouped tile configuration, forced for every entry, against the
    oracle (ragged tiles along m', n' and k in every configuration)."""
    entries = make_entries(24, seed=9, lo=16, hi=700)
    entries[0]["alpha"] = 0.0
    entries[1]["k"] = 0
    entries[2]["m"] = 0
    entries[3]["n"] = 0
    for cfg in _lib.GTILE_NAMES:
        for comp in ("s", "d"):
            for case in range(8):
                for bm in range(_lib.TUNE_BUCKETS):
                    for bn in range(_lib.TUNE_BUCKETS):
                        assert _lib.tune_set(comp, case, bm, bn, cfg) == 0
        say("grouped with tile configuration", cfg)
        st, keep = run_grouped(entries)
        assert st == 0
        check_all(entries, keep)
    _lib.tune_load(None)


def test_grouped_invalid_descriptor_enqueues_nothing():
    entries = make_entries(4, seed=11)
    entries[2]["transa"] = "X"
    descs = []
    keep = []
    for e in entries:
        A = gu.to_device(inputs.matrix(200, 200, "z", 1))
        C = gu.to_device(inputs.matrix(200, 200, "z", 2))
        keep += [A, C]
        descs.append(_lib.make_desc(e["transa"], "N", 10, 10, 10, 1.0, A.data_ptr(), "z", 200,
                                    A.data_ptr(), "z", 200, 0.0, C.data_ptr(), "z", 200, "d"))
    before = [t.clone() for t in keep[1::2]]
    st = _lib.mdgemm_grouped(descs, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == -(1000 * 2 + 1)
    for a, b in zip(before, keep[1::2]):
        assert torch.equal(a, b)


def test_grouped_huge_leading_dimension_runs_alongside():
    """A product whose leading dimension is too large for the grouped kernel's
    32-bit tile offsets (lda >= 2^20) runs on the plain kernels in the same
    call; it and the products around it still match the oracle."""
    entries = make_entries(6, seed=13, lo=8, hi=96, comps=("s", "d"))
    entries[2]["k"], entries[2]["transa"] = 8, "N"  # A is m x 8 inside a 2^20-row buffer
    say("grouped with one huge-lda product")
    o = oracle.get()
    descs, keep = [], []
    for idx, e in enumerate(entries):
        ar, ac = (e["m"], e["k"]) if e["transa"] in "NR" else (e["k"], e["m"])
        br, bc = (e["k"], e["n"]) if e["transb"] in "NR" else (e["n"], e["k"])
        lda = (1 << 20) + 8 if idx == 2 else ar
        A = inputs.matrix(ar, ac, e["ta"], e["seed"] * 3 + 1, ld=lda)
        B = inputs.matrix(br, bc, e["tb"], e["seed"] * 3 + 2)
        C = inputs.matrix(e["m"], e["n"], e["tc"], e["seed"] * 3 + 3, ld=max(1, e["m"]) + 2, pad=gu.SENTINEL)
        dA, dB, dC = gu.to_device(A), gu.to_device(B), gu.to_device(C)
        descs.append(_lib.make_desc(e["transa"], e["transb"], e["m"], e["n"], e["k"], e["alpha"],
                                    dA.data_ptr(), e["ta"], A.shape[0], dB.data_ptr(), e["tb"], B.shape[0],
                                    e["beta"], dC.data_ptr(), e["tc"], C.shape[0], e["comp"]))
        keep.append((A, B, C, dA, dB, dC))
    st = _lib.mdgemm_grouped(descs, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == 0
    assert keep[2][0].shape[0] >= 1 << 20
    check_all(entries, keep)
