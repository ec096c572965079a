"""mdgemm_grouped_noalloc against mdgemm_grouped on the same products: two
calls in a row, the second with fewer and smaller products (the fixed table
keeps the first call's contents, which must not matter).  Products the
grouped kernel runs must match bit for bit (same tiles, same kernel); the
ones both entry points hand to the plain kernels (binary16 C here, where
mdgemm_grouped may split k and mdgemm_grouped_noalloc never does) must both
lie within the oracle's bound, like every other product."""
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


def entries_for(count, seed, hi):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        tc, ta, tb = (TAGS[j] for j in rng.integers(0, 4, 3))
        comp = ("s", "d", "bf16x3")[int(rng.integers(0, 3))]
        m, n, k = (int(np.floor(np.exp(rng.uniform(np.log(8), np.log(hi + 1))))) for _ in range(3))
        transa, transb = "NTCR"[int(rng.integers(0, 4))], "NTCR"[int(rng.integers(0, 4))]
        alpha = 0.75 - 0.5j if oracle.get().case(tc, ta, tb) == "3" else 1.5
        out.append(dict(tc=tc, ta=ta, tb=tb, comp=comp, m=m, n=n, k=k, transa=transa, transb=transb,
                        alpha=alpha, beta=-0.5, seed=seed * 1000 + i, alone=False))
    # a binary16 C: handed to the plain kernels; few tiles and a deep k, so
    # mdgemm_grouped splits k while mdgemm_grouped_noalloc must not
    out.append(dict(tc="h", ta="s", tb="d", comp="s", m=min(hi, 100), n=min(hi, 90), k=1500, transa="N",
                    transb="N", alpha=1.5, beta=-0.5, seed=seed * 1000 + count, alone=True))
    return out


def operands(entries):
    host = []
    for e in entries:
        ar, ac = (e["m"], e["k"]) if e["transa"] in "NR" else (e["k"], e["m"])
        br, bc = (e["k"], e["n"]) if e["transb"] in "NR" else (e["n"], e["k"])
        A = inputs.matrix(ar, ac, e["ta"], e["seed"] * 3 + 1)
        B = inputs.matrix(br, bc, e["tb"], e["seed"] * 3 + 2)
        C = inputs.matrix(e["m"], e["n"], e["tc"], e["seed"] * 3 + 3, ld=e["m"] + 2, pad=gu.SENTINEL)
        host.append((A, B, C))
    return host


def launch(entries, host, fn):
    dev, descs = [], []
    for e, (A, B, C) in zip(entries, host):
        dA, dB, dC = gu.to_device(A), gu.to_device(B), gu.to_device(C)
        descs.append(_lib.make_desc(e["transa"], e["transb"], e["m"], e["n"], e["k"], e["alpha"],
                                    dA.data_ptr(), e["ta"], A.shape[0], dB.data_ptr(), e["tb"], B.shape[0],
                                    e["beta"], dC.data_ptr(), e["tc"], C.shape[0], e["comp"]))
        dev.append((dA, dB, dC))
    st = fn(descs, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == 0, (st, _lib.strerror(st))
    return [gu.to_host(d[2]) for d in dev]


def test_noalloc_matches_grouped_on_two_calls():
    o = oracle.get()
    for call, (count, seed, hi) in enumerate(((48, 71, 300), (10, 72, 60))):
        entries = entries_for(count, seed, hi)
        host = operands(entries)
        say("call %d: %d products through mdgemm_grouped" % (call, len(entries)))
        ref_out = launch(entries, host, _lib.mdgemm_grouped)
        say("call %d: the same through mdgemm_grouped_noalloc" % call)
        out = launch(entries, host, _lib.mdgemm_grouped_noalloc)
        for e, (A, B, C), a, b in zip(entries, host, ref_out, out):
            what = "call %d %s%s%s/%s %s%s %dx%dx%d" % (call, e["tc"], e["ta"], e["tb"], e["comp"], e["transa"],
                                                       e["transb"], e["m"], e["n"], e["k"])
            if not e["alone"]:
                ga = inputs.to_complex128(np.asarray(a))
                gb = inputs.to_complex128(np.asarray(b))
                assert np.array_equal(ga, gb), what + ": differs from mdgemm_grouped"
            st, ref, g = o.gemm(e["transa"], e["transb"], e["m"], e["n"], e["k"], e["alpha"], A, e["ta"],
                                A.shape[0], B, e["tb"], B.shape[0], e["beta"], C, e["tc"], C.shape[0])
            assert st == 0
            gu.check(e["tc"], e["comp"], e["k"], a, e["m"], e["n"], ref, g, what=what + " (grouped)")
            gu.check(e["tc"], e["comp"], e["k"], b, e["m"], e["n"], ref, g, what=what + " (noalloc)")
            gu.check_padding(b, e["m"], what)
