"""Breadth: every storage combination of C, A and B (4 x 4 x 4), both
computation precisions, every pair of the operations N, T and C on A and B,
at the tile-edge sizes {0, 1, 2, 3, 5, 17, 33, 65}, with tight, padded and odd
leading dimensions, through the C ABI against the CPU oracle (brute force on
tiny inputs, within the elementwise bound of gpu_util).

Each (combination, precision, operation pair) runs 8 products whose m, n and k
each take every size once (three different orders of the size list, shifted
by the operation pair so that the triples differ between pairs); the leading
dimensions cycle through tight (ld = rows), padded (ld = rows + 8) and odd
(the next odd ld above rows).  Padding rows of C must keep their sentinel.
"""
import itertools
import sys

import numpy as np
import pytest
import torch

import gpu_util as gu
from paper_1901_06015_amd import _lib

pytestmark = pytest.mark.gpu
TAGS = ("s", "d", "c", "z")
SIZES = (0, 1, 2, 3, 5, 17, 33, 65)
OPS = list(itertools.product("NTC", "NTC"))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _lib.lib()
    yield


@pytest.fixture(params=["small", "tiled"])
def path(request, monkeypatch):
    if request.param == "tiled":
        monkeypatch.setenv("MDGEMM_SMALL", "0")
    else:
        monkeypatch.delenv("MDGEMM_SMALL", raising=False)
    return request.param


def pad_for(rows, style):
    """Spare elements per column for a tight, padded or odd leading dimension."""
    if style == 0:
        return 0
    if style == 1:
        return 8
    return 1 if max(1, rows) % 2 == 0 else 2


def triples(op_index):
    """8 (m, n, k) triples in which each dimension takes every size once."""
    n_s = len(SIZES)
    out = []
    for i in range(n_s):
        m = SIZES[(i + op_index) % n_s]
        n = SIZES[(3 * i + 1 + op_index) % n_s]
        k = SIZES[(5 * i + 2 + 2 * op_index) % n_s]
        out.append((m, n, k))
    return out


def test_triples_cover_every_size():
    for o in range(len(OPS)):
        t = triples(o)
        for d in range(3):
            assert sorted(x[d] for x in t) == sorted(SIZES)


@pytest.mark.parametrize("cab", ["".join(p) for p in itertools.product(TAGS, repeat=3)])
def test_all_combinations_ops_and_edge_sizes(cab, path):
    tc, ta, tb = cab
    worst = 0.0
    for comp in ("s", "d"):
        for o, (transa, transb) in enumerate(OPS):
            for i, (m, n, k) in enumerate(triples(o)):
                style = (i + o) % 3
                ar = m if transa == "N" else k
                br = k if transb == "N" else n
                pads = dict(pad_a=pad_for(ar, style), pad_b=pad_for(br, (style + 1) % 3),
                            pad_c=pad_for(m, (style + 2) % 3))
                seed = 1000 + 97 * o + i
                say("mdgemm %s comp=%s %s%s m=%d n=%d k=%d %r seed=%d [%s]" % (
                    cab, comp, transa, transb, m, n, k, pads, seed, path))
                st, Cout, ops = gu.run(tc, ta, tb, m, n, k, comp=comp, transa=transa, transb=transb,
                                       seed=seed, **pads)
                assert st == 0, (st, _lib.strerror(st))
                ref, g = gu.reference(tc, ta, tb, m, n, k, ops, transa, transb)
                r = gu.check(tc, comp, k, Cout, m, n, ref, g,
                             what="%s/%s %s%s %dx%dx%d" % (cab, comp, transa, transb, m, n, k))
                gu.check_padding(Cout, m, "C")
                worst = max(worst, r)
    say("%s [%s]: worst err/bound %.3g" % (cab, path, worst))
