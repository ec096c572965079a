"""GPU tests of the serving loop: continuous batching under an HBM budget.
Each result is checked against the CPU oracle and is bitwise the same whether
the request ran alone or in a mix; admission respects the budget; invalid
requests are refused while the server keeps serving."""
import sys

import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_1901_06015_amd import _lib, inputs
from paper_1901_06015_amd.serving import Server

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


def make_requests(srv, count, seed, hi=400, big_every=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(count):
        tc, ta, tb = (TAGS[j] for j in rng.integers(0, 4, 3))
        comp = ("s", "d", "bf16x3")[int(rng.integers(0, 3))]
        if i % big_every == 0:
            m, n, k = 512, 384, 640
        else:
            m, n, k = (int(np.floor(np.exp(rng.uniform(np.log(8), np.log(hi))))) for _ in range(3))
        transa, transb = "NTR"[int(rng.integers(0, 3))], "NCR"[int(rng.integers(0, 3))]
        ar, ac = (m, k) if transa in "NR" else (k, m)
        br, bc = (k, n) if transb in "NR" else (n, k)
        A = inputs.matrix(ar, ac, ta, 9 * i + seed)
        B = inputs.matrix(br, bc, tb, 9 * i + seed + 1)
        C = inputs.matrix(m, n, tc, 9 * i + seed + 2)
        case = oracle.get().case(tc, ta, tb)
        alpha = 0.75 - 0.5j if case == "3" else 1.5
        beta = (-0.5, 0.0)[i % 2]
        ha, hb, hc = srv.put(A), srv.put(B), srv.put(C)
        reqs.append(dict(tc=tc, ta=ta, tb=tb, comp=comp, m=m, n=n, k=k, transa=transa, transb=transb,
                         alpha=alpha, beta=beta, A=A, B=B, C=C, ha=ha, hb=hb, hc=hc))
    return reqs


def submit(srv, r):
    st, t = srv.submit(r["transa"], r["transb"], r["m"], r["n"], r["k"], r["alpha"], r["ha"], r["hb"],
                       r["beta"], r["hc"], r["tc"], r["comp"], keep_output=True)
    assert st == 0, st
    return t


def collect(srv, r, t):
    st, res = srv.wait(t, 120.0)
    assert st == 0 and res.done and res.status == 0, (st, res.done, res.status)
    out = srv.fetch(res.output, r["m"], r["n"], r["tc"])
    srv.drop(res.output)
    srv.forget(t)
    return out, res


def test_alone_equals_in_mix_and_oracle():
    with Server(budget_bytes=8 << 30, slots=4, max_batch=16, big_flops=2e8) as srv:
        reqs = make_requests(srv, 40, seed=21)
        say("serving: submitting", len(reqs), "requests as one burst")
        tickets = [submit(srv, r) for r in reqs]
        mix = [collect(srv, r, t) for r, t in zip(reqs, tickets)]
        stats = srv.stats()
        say("serving stats", stats)
        assert stats["completed"] >= len(reqs)
        assert stats["max_concurrent_batches"] >= 2, "device work of different batches never overlapped"
        assert stats["grouped_launches"] >= 1 and stats["plain_launches"] >= 1
        o = oracle.get()
        for r, (out_mix, res) in zip(reqs, mix):
            t = submit(srv, r)
            out_alone, _ = collect(srv, r, t)
            what = "%s%s%s/%s %s%s %dx%dx%d" % (r["tc"], r["ta"], r["tb"], r["comp"], r["transa"], r["transb"],
                                                r["m"], r["n"], r["k"])
            assert np.array_equal(out_mix, out_alone), "alone != in mix: " + what
            st, ref, g = o.gemm(r["transa"], r["transb"], r["m"], r["n"], r["k"], r["alpha"], r["A"], r["ta"],
                                r["A"].shape[0], r["B"], r["tb"], r["B"].shape[0], r["beta"], r["C"], r["tc"],
                                r["C"].shape[0])
            assert st == 0
            gu.check(r["tc"], r["comp"], r["k"], out_mix, r["m"], r["n"], ref, g, what=what)


def test_budget_caps_inflight_working_set():
    with Server(budget_bytes=8 << 30, slots=4, max_batch=8, big_flops=1e12) as probe:
        reqs = make_requests(probe, 24, seed=33, hi=300, big_every=1000)
    ws = []
    for r in reqs:
        cb = r["m"] * r["n"] * r["C"].itemsize
        ws.append(r["A"].nbytes + r["B"].nbytes + cb + (cb if r["beta"] != 0 else 0))
    budget = int(max(ws) * 1.5)
    with Server(budget_bytes=budget, slots=4, max_batch=8, big_flops=1e12) as srv:
        reqs = make_requests(srv, 24, seed=33, hi=300, big_every=1000)
        tickets = [submit(srv, r) for r in reqs]
        for r, t in zip(reqs, tickets):
            collect(srv, r, t)
        s = srv.stats()
        say("budget", budget, "stats", s)
        assert s["peak_inflight_bytes"] <= budget
        assert s["completed"] == len(reqs)
        # a request whose working set exceeds the whole budget is refused
        big = np.zeros((2048, 2048), dtype=np.complex128, order="F")
        h = srv.put(big)
        st, _ = srv.submit("N", "N", 2048, 2048, 2048, 1.0, h, h, 0.0, None, "z", "d")
        assert st == _lib.MD_ERR_BUDGET


def test_invalid_requests_refused_server_keeps_serving():
    with Server(budget_bytes=4 << 30, slots=2, max_batch=8, big_flops=1e12) as srv:
        reqs = make_requests(srv, 6, seed=44, hi=120, big_every=1000)
        r = reqs[0]
        st, _ = srv.submit("X", "N", r["m"], r["n"], r["k"], 1.0, r["ha"], r["hb"], 0.0, None, r["tc"], "s")
        assert st != 0
        st, _ = srv.submit("N", "N", r["m"], r["n"], r["k"], 1.0, 987654, r["hb"], 0.0, None, r["tc"], "s")
        assert st == _lib.MD_ERR_STATE
        # Im(alpha) != 0 in a mixed case (Section 7.2)
        A = srv.put(inputs.matrix(16, 16, "c", 1))
        Bh = srv.put(inputs.matrix(16, 16, "s", 2))
        st, _ = srv.submit("N", "N", 16, 16, 16, 1.0 + 1.0j, A, Bh, 0.0, None, "s", "s")
        assert st == _lib.MD_ERR_ALPHA_IMAG
        # an operand in use cannot be dropped
        t = submit(srv, reqs[1])
        tickets = [t] + [submit(srv, q) for q in reqs[2:]]
        for q, tt in zip(reqs[1:], tickets):
            collect(srv, q, tt)
        s = srv.stats()
        assert s["refused"] == 3 and s["completed"] == len(reqs) - 1


def test_input_c_is_read_not_written_and_blocks_are_reused():
    """The output goes to fresh memory (C_in stays bitwise unchanged, so one
    resident C serves many requests), and a repeated burst is served from the
    allocator's recycled blocks."""
    with Server(budget_bytes=8 << 30, slots=4, max_batch=16, big_flops=2e8) as srv:
        reqs = make_requests(srv, 24, seed=55, hi=300)
        for r in reqs:
            r["beta"] = -0.5
        tickets = [submit(srv, r) for r in reqs]
        first = [collect(srv, r, t)[0] for r, t in zip(reqs, tickets)]
        mallocs = srv.stats()["device_mallocs"]
        tickets = [submit(srv, r) for r in reqs]
        second = [collect(srv, r, t)[0] for r, t in zip(reqs, tickets)]
        s = srv.stats()
        say("reuse stats", s)
        for r, a, b in zip(reqs, first, second):
            assert np.array_equal(a, b)
            cin = srv.fetch(r["hc"], r["m"], r["n"], r["tc"])
            assert np.array_equal(cin, r["C"][:r["m"], :r["n"]]), "input C was modified"
        # outputs of the second burst come from recycled blocks (a kept output
        # is handed to the caller, so only a few classes may need new blocks)
        assert s["device_mallocs"] - mallocs <= len(reqs) // 2, (mallocs, s["device_mallocs"])


def test_large_requests_take_one_lane_small_ones_pass():
    """With one large-request lane, large requests never run at the same time,
    and small requests submitted behind them finish before the last of them."""
    with Server(budget_bytes=16 << 30, slots=4, max_batch=16, big_flops=1e10, big_lanes=1) as srv:
        big = []
        for i in range(3):
            A = inputs.matrix(2048, 2048, "z", 600 + 2 * i)
            B = inputs.matrix(2048, 2048, "z", 601 + 2 * i)
            big.append((srv.put(A), srv.put(B)))
        smalls = make_requests(srv, 16, seed=66, hi=96, big_every=1000)
        tb = []
        for ha, hb in big:
            st, t = srv.submit("N", "N", 2048, 2048, 2048, 1.0, ha, hb, 0.0, None, "z", "d")
            assert st == 0
            tb.append(t)
        ts = [submit(srv, r) for r in smalls]
        rb = []
        for t in tb:
            st, res = srv.wait(t, 120.0)
            assert st == 0 and res.status == 0
            rb.append((res.t_admit_us, res.t_done_us))
        rs = [collect(srv, r, t)[1] for r, t in zip(smalls, ts)]
        say("big intervals", rb, "last small done", max(x.t_done_us for x in rs))
        for (a0, d0), (a1, d1) in zip(rb, rb[1:]):
            assert a1 >= d0, "two large requests ran at once"
        assert max(x.t_done_us for x in rs) < rb[-1][1], "small requests waited for every large one"
        assert srv.stats()["completed"] == len(tb) + len(smalls)


def test_half_precision_requests():
    """Binary16 operands, outputs and the half computation precision through
    the server (small requests batched with ordinary ones): each output
    matches the oracle."""
    with Server(budget_bytes=4 << 30, slots=2, max_batch=8, big_flops=2e9) as srv:
        o = oracle.get()
        spec = (("h", "h", "h", "h"), ("hc", "c", "hc", "s"), ("z", "hc", "d", "d"), ("s", "s", "s", "h"),
                ("hc", "hc", "hc", None), ("d", "d", "z", "d"))
        reqs = []
        for i, (tc, ta, tb, comp) in enumerate(spec):
            m, n, k = 40 + 7 * i, 33 + 5 * i, 64
            A = inputs.matrix(m, k, ta, 300 + 3 * i)
            B = inputs.matrix(k, n, tb, 301 + 3 * i)
            C = inputs.matrix(m, n, tc, 302 + 3 * i)
            r = dict(tc=tc, ta=ta, tb=tb, comp=comp, m=m, n=n, k=k, transa="N", transb="N", alpha=1.5,
                     beta=-0.5, A=A, B=B, C=C, ha=srv.put(A), hb=srv.put(B), hc=srv.put(C))
            reqs.append(r)
        say("serving: half-precision burst of", len(reqs))
        tickets = [submit(srv, r) for r in reqs]
        for r, t in zip(reqs, tickets):
            out, _ = collect(srv, r, t)
            st, ref, g = o.gemm("N", "N", r["m"], r["n"], r["k"], 1.5, r["A"], r["ta"], r["m"], r["B"], r["tb"],
                                r["k"], -0.5, r["C"], r["tc"], r["m"])
            assert st == 0
            gu.check(r["tc"], r["comp"], r["k"], out, r["m"], r["n"], ref, g,
                     what="serving half %s/%s/%s/%s" % (r["tc"], r["ta"], r["tb"], r["comp"]))
