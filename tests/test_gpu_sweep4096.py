"""GPU parity at the full size of the plain method's sweep: all 64 storage
combinations of (C, A, B) in {s, d, c, z}^3 x computation precision {s, d},
m = n = k = 4096, column-major, alpha = 1.5, beta = -0.5, no transpose, each
product on a fresh copy of C, launched exactly as the benchmark launches it.

Two checks per combination, both elementwise within
    |C_gpu - C_ref| <= 4 k u_x (|A||B|)_ij + 4 u_C |C_ref,ij|:
  * sampled entries against the CPU oracle (evaluated one by one): the four
    corners, every row and column on a 64-boundary (the edges of every
    workgroup tile, whose real-product tiles span 64 or 128 rows and columns
    of C), each at 8 random positions along it, and 2048 random entries --
    4100 entries per combination;
  * the whole matrix against an FP64 library reference on the device
    (torch.matmul in complex128 of the exactly promoted operands, |A||B| in
    float64), whose own rounding (at most about 2k u_d |alpha| (|A||B|)) is
    added to the tolerance of this comparison only.
A second pass with integer entries in [-4, 4] requires the sampled entries
to equal the oracle bit for bit (every partial sum is exact in FP32 and FP64).
"""
import concurrent.futures
import itertools
import os
import sys

import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_1901_06015_amd import _lib, inputs

pytestmark = pytest.mark.gpu
TAGS = ("s", "d", "c", "z")
N = 4096
ALPHA, BETA = 1.5, -0.5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _lib.lib()
    yield


def sample_positions(n, seed=4096):
    """(rows, cols) of the sampled entries: corners, every 64-boundary row and
    column at 8 random places each, 2048 random entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = np.unique(np.concatenate([np.arange(0, n, 64), np.arange(63, n, 64)]))
    rows = [np.array([0, 0, n - 1, n - 1])]
    cols = [np.array([0, n - 1, 0, n - 1])]
    rows.append(np.repeat(edges, 8))
    cols.append(rng.integers(0, n, size=edges.size * 8))
    rows.append(rng.integers(0, n, size=edges.size * 8))
    cols.append(np.repeat(edges, 8))
    rows.append(rng.integers(0, n, size=2048))
    cols.append(rng.integers(0, n, size=2048))
    return np.concatenate(rows).astype(np.int64), np.concatenate(cols).astype(np.int64)


def operands(dist):
    """Host and device copies of one A, B and C per storage type."""
    host, dev = {}, {}
    for role, off in (("A", 0), ("B", 100), ("C", 200)):
        for i, dt in enumerate(TAGS):
            X = inputs.matrix(N, N, dt, 4096 + off + i, dist=dist)
            host[role + dt] = X
            dev[role + dt] = torch.from_numpy(X).cuda()
    return host, dev


def oracle_samples(host, rows, cols):
    """Oracle values and bound terms at the sampled entries for every storage
    combination, on a pool of host threads (the oracle releases the GIL)."""
    o = oracle.get()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))

    def one(cab):
        tc, ta, tb = cab
        st, ref, g = o.gemm_at("N", "N", N, N, N, ALPHA, host["A" + ta], ta, N, host["B" + tb], tb, N,
                               BETA, host["C" + tc], tc, N, rows, cols)
        assert st == 0, (cab, st)
        return cab, ref, g

    cabs = ["".join(t) for t in itertools.product(TAGS, TAGS, TAGS)]
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        return {cab: (ref, g) for cab, ref, g in ex.map(one, cabs)}


def run_product(dev, tc, ta, tb, x):
    """mdgemm on a fresh copy of C; returns the result tensor."""
    Cw = dev["C" + tc].clone()
    stream = torch.cuda.current_stream().cuda_stream
    st = _lib.mdgemm("N", "N", N, N, N, ALPHA, dev["A" + ta].data_ptr(), ta, N, dev["B" + tb].data_ptr(), tb, N,
                     BETA, Cw.data_ptr(), tc, N, x, stream)
    assert st == 0, (tc + ta + tb + x, st, _lib.strerror(st))
    return Cw


def test_sweep4096_sampled_and_full_matrix():
    rows, cols = sample_positions(N)
    say("sweep4096: generating operands")
    host, dev = operands("uniform")
    say("sweep4096: oracle at %d sampled entries per combination" % rows.size)
    samples = oracle_samples(host, rows, cols)
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    worst = {}
    for ta, tb in itertools.product(TAGS, TAGS):
        Ap = dev["A" + ta].to(torch.complex128)
        Bp = dev["B" + tb].to(torch.complex128)
        prod = torch.matmul(Ap, Bp)
        g = torch.matmul(Ap.abs(), Bp.abs())
        del Ap, Bp
        for tc, x in itertools.product(TAGS, ("s", "d")):
            cabx = tc + ta + tb + x
            say("sweep4096 %s" % cabx)
            Cw = run_product(dev, tc, ta, tb, x)
            torch.cuda.synchronize()
            # sampled entries against the CPU oracle
            ref, gs = samples[tc + ta + tb]
            got = Cw[ri, ci].cpu().numpy().astype(np.complex128)
            err = np.abs(got - ref)
            b = gu.bound(tc, x, N, ref, gs)
            bad = ~(err <= b)
            assert not bad.any(), "%s: %d sampled entries outside the bound; first (%d,%d) err %.3g bound %.3g" % (
                cabx, int(bad.sum()), rows[bad][0], cols[bad][0], err[bad][0], b[bad][0])
            # the whole matrix against the device FP64 library reference
            Cp = dev["C" + tc].to(torch.complex128)
            full = ALPHA * prod + BETA * Cp
            if tc in "sd":
                full = full.real.to(torch.complex128)
            gotf = Cw.to(torch.complex128)
            errf = (gotf - full).abs()
            ux = gu.U[x]
            uc = gu.U[gu.PREC[tc]]
            tol = (4.0 * N * ux + 2.0 * N * gu.U["d"] * abs(ALPHA)) * g + 4.0 * uc * full.abs()
            nbad = int((errf > tol).sum().item())
            assert nbad == 0, "%s: %d entries outside the bound against the FP64 library reference" % (cabx, nbad)
            worst[cabx] = max(float(np.max(err / np.maximum(b, 1e-300))), float((errf / tol).max().item()))
            del Cw, Cp, full, gotf, errf, tol
        del prod, g
        torch.cuda.empty_cache()
    say("sweep4096: max err/bound over combinations %.3g (%s)" % (max(worst.values()), max(worst, key=worst.get)))


def test_sweep4096_exact_inputs_bitwise():
    rows, cols = sample_positions(N, seed=99)
    say("sweep4096 exact: generating operands")
    host, dev = operands("int")
    samples = oracle_samples(host, rows, cols)
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        ref, _ = samples[tc + ta + tb]
        for x in ("s", "d"):
            say("sweep4096 exact %s%s%s%s" % (tc, ta, tb, x))
            Cw = run_product(dev, tc, ta, tb, x)
            got = Cw[ri, ci].cpu().numpy().astype(np.complex128)
            nbad = int((got != ref).sum())
            assert nbad == 0, "%s%s%s%s: %d sampled entries differ from the oracle" % (tc, ta, tb, x, nbad)
            del Cw
