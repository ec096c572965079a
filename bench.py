"""Benchmark: mixed-datatype GEMM on one MI355X.

Workload (one "step"): the full sweep of the plain method -- all 64 storage
combinations of (C, A, B) in {s, d, c, z}^3 times computation precision
{single, double} = 128 products, each m = n = k = 4096, column-major, entries
U[-1, 1] per real/imaginary part (seeded), alpha = 1.5, beta = -0.5, no
transpose.  Inputs are resident in HBM before timing starts.

Reported: one compact JSON line on stdout (the last line), with
  value        aggregate GFLOP/s of the sweep: sum of the paper's minimum flop
               counts (2/4/8 mnk per case) / time of the step
  vs_native    ratio of each combination's p50 GFLOP/s to the same-GPU native
               kernel the paper uses as its reference (sgemm/dgemm for cases
               0-2, cgemm/zgemm for case 3, at the computation precision;
               torch.matmul -> hipBLASLt/rocBLAS), timed once per step between
               the sweep's steps: min, median, count >= 0.9, worst five
  roofline     dominant kernel's achieved TFLOP/s (algorithmic flops / its
               measured duration, HIP events on its stream) vs the MFMA peak
  vs_adhoc     time of the ad-hoc alternative (cast and copy every operand to
               the domain's computation type with torch, vendor GEMM, update,
               cast back) over mdgemm's: median and minimum
  cpu_baseline the FP64 oracle timed on this host's cores on a bounded sample
and, before it, the per-combination and per-kernel record (p50/p99 latency,
GFLOP/s, ratios) as one '# detail' line on stderr or in the --detail file.

    python bench.py [--steps K] [--warmup W] [--size N] [--combos zcd,sss] [--no-cpu] [--no-adhoc]
"""
import argparse
import hashlib
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
TAGS = ("s", "d", "c", "z")
CASE_FACTOR = {"0": 2, "1a": 2, "1b": 2, "1c": 2, "2ab": 4, "2ac": 4, "2bc": 4, "3": 8}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--size", type=int, default=4096)
    p.add_argument("--combos", type=str, default="", help="comma list like zcdd,ssss (cabx)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-native", action="store_true")
    p.add_argument("--no-adhoc", action="store_true", help="skip the ad-hoc (cast, copy, vendor GEMM) baseline")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--detail", type=str, default="",
                   help="sweep: write the per-combination and per-kernel record to this file "
                        "(default: one '# detail' line on stderr)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain copy kernel of known size (HBM counter calibration)")
    p.add_argument("--check", action="store_true", help="grouped: check every product against the oracle")
    p.add_argument("--duration", type=float, default=60.0, help="serving: seconds of Poisson arrivals per stream")
    p.add_argument("--qps", type=float, default=0.0,
                   help="serving: offered requests/s (0: --load times the measured served capacity)")
    p.add_argument("--load", type=float, default=0.7, help="serving: offered load as a fraction of capacity")
    p.add_argument("--slots", type=int, default=4, help="serving: concurrent batches (streams)")
    p.add_argument("--max-batch", type=int, default=64, help="serving: requests per grouped launch")
    p.add_argument("--big-gflop", type=float, default=2.0, help="serving: requests above this run alone")
    p.add_argument("--big-lanes", type=int, default=2, help="serving: large requests running at once")
    p.add_argument("--no-plain-stream", action="store_true",
                   help="serving: skip the plain-form run of the same arrival stream")
    p.add_argument("--workload", default="sweep", choices=["sweep", "precision", "grouped", "serving", "single"],
                   help="sweep: the 128-combination plain method at 4096 (default); precision: "
                        "FP32 vs BF16x3 at 8192; grouped: 512 mixed GEMMs in one launch; serving: "
                        "Poisson request stream; single: one zcdd product at 256 (latency)")
    return p.parse_args()


def combos(filter_str):
    out = []
    for tc, ta, tb in itertools.product(TAGS, TAGS, TAGS):
        for x in ("s", "d"):
            out.append(tc + ta + tb + x)
    if filter_str:
        keep = set(filter_str.split(","))
        out = [c for c in out if c in keep]
    return out


def make_operands(n, seed=1901):
    """One A, B and C per storage type, resident on the device."""
    import torch
    from paper_1901_06015_amd import inputs
    ops = {}
    for role, off in (("A", 0), ("B", 100), ("C", 200)):
        for dt in TAGS:
            h = inputs.matrix(n, n, dt, seed + off + TAGS.index(dt))
            t = torch.from_numpy(h).cuda()
            assert t.stride(0) == 1
            ops[role + dt] = t
            del h
    return ops


NATIVE = (("sgemm", "float32", 2), ("dgemm", "float64", 2), ("cgemm", "complex64", 8), ("zgemm", "complex128", 8))


def native_operands(n):
    """Operands of the native same-type GEMMs (torch.matmul), one set per dtype."""
    import torch
    res = {}
    for name, dtn, fl in NATIVE:
        dt = getattr(torch, dtn)
        g = torch.Generator(device="cuda").manual_seed(5)
        if dt.is_complex:
            rdt = torch.float32 if dt == torch.complex64 else torch.float64
            a = torch.complex(torch.rand(n, n, device="cuda", dtype=rdt, generator=g) * 2 - 1,
                              torch.rand(n, n, device="cuda", dtype=rdt, generator=g) * 2 - 1)
            b = torch.complex(torch.rand(n, n, device="cuda", dtype=rdt, generator=g) * 2 - 1,
                              torch.rand(n, n, device="cuda", dtype=rdt, generator=g) * 2 - 1)
        else:
            a = torch.rand(n, n, device="cuda", dtype=dt, generator=g) * 2 - 1
            b = torch.rand(n, n, device="cuda", dtype=dt, generator=g) * 2 - 1
        c = torch.empty(n, n, device="cuda", dtype=dt)
        for _ in range(2):
            torch.matmul(a, b, out=c)
        res[name] = (a, b, c, fl)
    torch.cuda.synchronize()
    return res


def native_once(nops, stream):
    """One timed call of each native GEMM on `stream` (HIP events); seconds."""
    import torch
    evs = []
    for name, (a, b, c, fl) in nops.items():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        torch.matmul(a, b, out=c)
        e1.record(stream)
        evs.append((name, e0, e1))
    torch.cuda.synchronize()
    return {name: e0.elapsed_time(e1) / 1e3 for name, e0, e1 in evs}


def native_times(n, reps=20):
    """p50 seconds of torch.matmul per dtype (the native same-type GEMM)."""
    import torch
    nops = native_operands(n)
    ts = {name: [] for name in nops}
    for _ in range(reps):
        for name, t in native_once(nops, torch.cuda.current_stream()).items():
            ts[name].append(t)
    res = {}
    for name, (a, b, c, fl) in nops.items():
        p50 = float(np.median(ts[name]))
        res[name] = {"p50_s": p50, "gflops": fl * n ** 3 / p50 / 1e9}
    del nops
    torch.cuda.empty_cache()
    return res


def adhoc_times(ops, todo, reps=3):
    """p50 seconds of the ad-hoc alternative for each combination: cast and
    copy A, B and C to the computation type of the product's domain (complex
    when any operand is complex), one vendor GEMM (torch.matmul), then
    beta*C + alpha*AB and the cast back to C's storage type (Re for a real
    C), all with torch on the device.  A timing baseline only: it spends the
    flops of the common domain and the traffic of the casts and copies that
    the in-kernel cast avoids (and rounds beta*C in the computation precision,
    not C's).  It works on a copy of C."""
    import torch
    res = {}
    for cabx in todo:
        tc, ta, tb, x = cabx
        cplx = any(t in "cz" for t in (tc, ta, tb))
        T = {(False, "s"): torch.float32, (False, "d"): torch.float64,
             (True, "s"): torch.complex64, (True, "d"): torch.complex128}[(cplx, x)]
        A, B, C = ops["A" + ta], ops["B" + tb], ops["C" + tc].clone()

        def run():
            R = (-0.5) * C.to(T) + 1.5 * torch.matmul(A.to(T), B.to(T))
            C.copy_(R.real if (R.is_complex() and not C.is_complex()) else R)

        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        res[cabx] = float(np.median(ts))
        del C
    torch.cuda.empty_cache()
    return res


ELEM_BYTES = {"s": 4, "d": 8, "c": 8, "z": 16}


def algorithmic_bytes(cabx, n):
    """Bytes one product must move at least: A and B read once, C read once
    (beta != 0) and written once."""
    tc, ta, tb = cabx[0], cabx[1], cabx[2]
    return n * n * (ELEM_BYTES[ta] + ELEM_BYTES[tb] + 2 * ELEM_BYTES[tc])


def native_for(case, x):
    if case == "3":
        return "cgemm" if x == "s" else "zgemm"
    return "sgemm" if x == "s" else "dgemm"


def kernel_source_sha():
    """Hash of the sources that define the product kernels."""
    h = hashlib.sha256()
    for f in ("md_tile.h", "mdgemm_kernels.hip", "md_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1901_06015_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def kernel_symbol(plan, transa="N", transb="N"):
    """The demangled symbol rocprofv3 reports for the kernel a plan launches
    (plan kernel names read md_gemm_<prec>_case<c>_<path>_<A><B>_<tile>)."""
    parts = plan["kernel"].split("_")
    t = "double" if parts[2] == "f64" else "float"
    fast, rag = parts[4] in ("fast", "ragged"), parts[4] == "ragged"
    ad, bd = parts[5][0] == "d", parts[5][1] == "d"
    cfg = {"t128x128w4": "TileCfg", "t128x256w8": "WideN", "t256x128w8": "WideM",
           "t128x128w8": "Deep", "t256x256w8": "Big"}[parts[6]]
    amnc = (transa in "NR") if fast else True
    bmnc = (transb in "TC") if fast else True
    b = lambda v: "true" if v else "false"
    # the last two template arguments: alpha staged into an operand, binary16
    # operands (never in the sweep)
    return "void md::md_gemm_kernel<%s, %d, %s, %s, %s, %s, %s, md::%s<%s>, %s, false, false>(md::GemmArgs)" % (
        t, plan["domain_case"], b(fast), b(ad), b(bd), b(amnc), b(bmnc), cfg, t, b(rag))


def traffic_record(symbol):
    """HBM bytes per launch of `symbol` (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy kernel's counters) from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha()
    for line in open(path):
        parts = line.rstrip("\n").split("\t")
        if len(parts) == 5 and parts[0] == symbol and parts[1] == sha:
            return {"fetch_bytes": float(parts[2]), "write_bytes": float(parts[3]),
                    "bytes": float(parts[4]), "source": "profiles/hbm_traffic.txt"}
    return None


def copy_calibration(nbytes=256 << 20, reps=3):
    """A plain elementwise copy of known size (read n bytes, write n bytes)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


# The paper's CPU figures are theoretical peaks per core (Section 8.1); it
# prints no measured GFLOP/s.
PAPER_CPU_PEAKS = {"ThunderX2 CN9975 2.2GHz": {"dp": 17.6, "sp": 35.2},
                   "Xeon Platinum 8167M 2.0GHz": {"dp": 64.0, "sp": 128.0}}


def host_cpu():
    """(model name, logical CPUs this process may run on)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(budget_s, threads=0):
    """The oracle, as it is, timed on this host's cores: whole columns of C
    for dddd, zcdd and zzzd at 4096 (the sample), the columns of each
    combination dealt to `threads` host threads (ctypes releases the GIL) for
    about a third of the time budget; GFLOP/s counted with the same
    algorithmic flops as the GPU."""
    import concurrent.futures
    import threading
    import oracle
    from paper_1901_06015_amd import inputs
    o = oracle.get()
    model, nproc = host_cpu()
    if threads <= 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or nproc
    threads = max(1, min(threads, nproc))
    n = 4096
    total_fl, total_t, cols_done = 0.0, 0.0, {}
    per = budget_s / 3.0
    rows = np.arange(n, dtype=np.int64)
    for cab in ("ddd", "zcd", "zzz"):
        tc, ta, tb = cab
        A = inputs.matrix(n, n, ta, 11)
        B = inputs.matrix(n, n, tb, 12)
        C = inputs.matrix(n, n, tc, 13)
        fac = CASE_FACTOR[o.case(tc, ta, tb)]
        lock = threading.Lock()
        nxt = [0]
        t0 = time.perf_counter()

        def worker():
            done = 0
            while time.perf_counter() - t0 < per:
                with lock:
                    j = nxt[0]
                    nxt[0] += 1
                if j >= n:
                    break
                cols = np.full(n, j, dtype=np.int64)
                st, _, _ = o.gemm_at("N", "N", n, n, n, 1.5, A, ta, n, B, tb, n, -0.5, C, tc, n, rows, cols)
                assert st == 0
                done += 1
            return done

        with concurrent.futures.ThreadPoolExecutor(threads) as ex:
            done = sum(ex.map(lambda _: worker(), range(threads)))
        dt = time.perf_counter() - t0
        total_fl += fac * n * n * done
        total_t += dt
        cols_done[cab + "d"] = done
    value = total_fl / total_t / 1e9
    return {"value": round(value, 2), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "per_core": round(value / threads, 3), "cpu": model, "nproc": nproc,
            "sample": "whole columns of C at m=n=k=4096 (%s), FP64 triple loop, %d threads, %.1f s"
                      % (", ".join("%s:%d" % kv for kv in cols_done.items()), threads, total_t),
            "paper_peak_per_core": PAPER_CPU_PEAKS}


def precision_workload(args):
    """FP32 MFMA vs BF16x3 (and, beside them, the half computation precision
    on the fp16 matrix cores) at m=n=k=size (8192 by default) for ssss, csss,
    ccss, cccs (the cab(x) reading of the combinations) and scss, sccs (the
    other reading), each with U[-1,1] and log-uniform 10^U(-3,3) entries,
    alpha = 1, beta = 0.  Errors: against the CPU oracle on 512 sampled
    entries (the bound ratio and |dC|/(|A||B|)), and normwise against a full
    FP64 reference product (torch.matmul in complex128 on the promoted
    operands, checked against the same oracle samples)."""
    import torch
    import oracle
    from paper_1901_06015_amd import _lib, inputs
    n = args.size if args.size != 4096 else 8192
    o = oracle.get()
    sp = torch.cuda.current_stream().cuda_stream
    rng = np.random.Generator(np.random.PCG64(77))
    rows = np.concatenate([[0, n - 1, 0, n - 1, 127, 128], rng.integers(0, n, 506)]).astype(np.int64)
    cols = np.concatenate([[0, 0, n - 1, n - 1, 128, 127], rng.integers(0, n, 506)]).astype(np.int64)
    out = {}
    total = {"s": [0.0, 0.0], "bf16x3": [0.0, 0.0], "h": [0.0, 0.0]}
    for cab in ("sss", "css", "ccs", "ccc", "scs", "scc"):
        for dist in ("uniform", "loguniform"):
            tc, ta, tb = cab
            key = cab + "s/" + dist
            print("# precision %s" % key, file=sys.stderr, flush=True)
            A = inputs.matrix(n, n, ta, 301, dist=dist)
            B = inputs.matrix(n, n, tb, 302, dist=dist)
            C0 = inputs.matrix(n, n, tc, 303, dist=dist)
            dA = torch.from_numpy(A).cuda()
            dB = torch.from_numpy(B).cuda()
            st, ref_s, g_s = o.gemm_at("N", "N", n, n, n, 1.0, A, ta, n, B, tb, n, 0.0, C0, tc, n, rows, cols)
            assert st == 0
            # FP64 reference product of the promoted operands
            Ar = dA.to(torch.complex128)
            Br = dB.to(torch.complex128)
            Cref = torch.matmul(Ar, Br)
            del Ar, Br
            if tc in "sd":
                Cref = Cref.real.to(torch.complex128)
            lib_ref = Cref[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
            ref_check = float(np.max(np.abs(lib_ref - ref_s) / np.maximum(g_s, 1e-300)))
            res = {"fp64_reference_vs_oracle_max_rel": ref_check}
            for comp in ("s", "bf16x3", "h"):
                dC = torch.from_numpy(C0).cuda()
                ts = []
                for r in range(1 + args.steps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    stx = _lib.mdgemm("N", "N", n, n, n, 1.0, dA.data_ptr(), ta, n, dB.data_ptr(), tb, n,
                                      0.0, dC.data_ptr(), tc, n, comp, sp)
                    e1.record()
                    torch.cuda.synchronize()
                    assert stx == 0
                    if r > 0:
                        ts.append(e0.elapsed_time(e1) / 1e3)
                p50 = float(np.median(ts))
                st, pl = _lib.mdgemm_plan("N", "N", n, n, n, 1.0, 1, ta, n, 1, tb, n, 0.0, 1, tc, n, comp)
                gf = pl["flops"] / p50 / 1e9
                got = dC[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.complex128)
                err = np.abs(got - ref_s)
                # single-precision bound; for half, operands rounded to binary16
                # and FP32 accumulation
                ux_term = (4 * 2.0 ** -11 + 4 * n * 2.0 ** -24) if comp == "h" else 4 * n * 2.0 ** -24
                bound = ux_term * g_s + 4 * (2.0 ** -24 if tc in "sc" else 2.0 ** -53) * np.abs(ref_s)
                full = dC.to(torch.complex128)
                nf = float(torch.linalg.norm(full - Cref) / torch.linalg.norm(Cref))
                del full, dC
                res[comp] = {"p50_ms": round(p50 * 1e3, 3), "gflops": round(gf, 1),
                             "max_err_over_bound": float(np.max(err / bound)),
                             "median_err_over_AB": float(np.median(err / g_s)),
                             "max_err_over_AB": float(np.max(err / g_s)),
                             "normwise_rel_err": nf}
                total[comp][0] += pl["flops"]
                total[comp][1] += p50
            res["bf16x3_speedup"] = round(res["s"]["p50_ms"] / res["bf16x3"]["p50_ms"], 3)
            out[key] = res
            del dA, dB, Cref
            torch.cuda.empty_cache()
    agg = {c: v[0] / v[1] / 1e9 for c, v in total.items()}
    line = {"metric": "GFLOP/s FP32-MFMA vs BF16x3 at m=n=k=%d, error vs FP64 oracle" % n,
            "value": round(agg["bf16x3"], 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
            "higher_is_better": True, "dtype": "bf16x3 (f32 semantics)", "data": "synthetic",
            "config": {"workload": "precision form: m=n=k=%d, combos ssss csss ccss cccs scss sccs, "
                                   "U[-1,1] and 10^U(-3,3), alpha=1, beta=0" % n},
            "fp32_gflops": round(agg["s"], 1),
            "speedup_bf16x3_over_fp32": round(agg["bf16x3"] / agg["s"], 3),
            "half_gflops": round(agg["h"], 1),
            "speedup_half_over_fp32": round(agg["h"] / agg["s"], 3),
            "roofline": {"bf16x3_vs_fp32_peak": round(agg["bf16x3"] / 157.3e3, 4),
                         "bf16_mfma_utilisation": round(3 * agg["bf16x3"] / 2.5e6, 4),
                         "f16_mfma_utilisation": round(agg["h"] / 2.5e6, 4)},
            "per_combo": out}
    print(json.dumps(line), flush=True)


def single_workload(args):
    """One mixed product, zcdd (case 2ac) at m=n=k=256, alpha = beta = 1,
    double precision: a latency-bound call.  Device time per call (HIP events
    on the call's stream) and host wall time per call (enqueue to
    completion), p50/p99 over 2000 calls; beside them the vendor dgemm at the
    lowered real shape 512 x 256 x 256 and at 256^3; the result checked in
    full against the oracle."""
    import torch
    import oracle
    from paper_1901_06015_amd import _lib, inputs
    n, reps = 256, 2000
    A = inputs.matrix(n, n, "c", 11)
    B = inputs.matrix(n, n, "d", 12)
    C0 = inputs.matrix(n, n, "z", 13)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.from_numpy(C0).cuda()
    s = torch.cuda.current_stream()
    sp = s.cuda_stream
    call = lambda: _lib.mdgemm("N", "N", n, n, n, 1.0, dA.data_ptr(), "c", n, dB.data_ptr(), "d", n, 1.0,
                               dC.data_ptr(), "z", n, "d", sp)
    assert call() == 0
    torch.cuda.synchronize()
    dC.copy_(torch.from_numpy(C0))
    assert call() == 0
    torch.cuda.synchronize()
    st, ref, g = oracle.get().gemm("N", "N", n, n, n, 1.0, A, "c", n, B, "d", n, 1.0, C0, "z", n)
    assert st == 0
    got = dC.cpu().numpy()
    bound = 4 * n * 2.0 ** -53 * g + 4 * 2.0 ** -53 * np.abs(ref)
    ratio = float(np.max(np.abs(got - ref) / bound))
    assert ratio <= 1.0, "single: outside the bound (%.3g)" % ratio
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(s)
        call()
        e1.record(s)
    torch.cuda.synchronize()
    dev = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev])  # us
    wall = []
    for _ in range(reps):
        t0 = time.perf_counter()
        call()
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e6)
    wall = np.array(wall)

    def native(m_, n_, k_):
        a = torch.rand(m_, k_, dtype=torch.float64, device="cuda")
        b = torch.rand(k_, n_, dtype=torch.float64, device="cuda")
        c = torch.empty(m_, n_, dtype=torch.float64, device="cuda")
        for _ in range(20):
            torch.matmul(a, b, out=c)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record()
            torch.matmul(a, b, out=c)
            e1.record()
        torch.cuda.synchronize()
        t = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in evs])
        return {"p50_us": round(float(np.median(t)), 2), "p99_us": round(float(np.percentile(t, 99)), 2),
                "gflops": round(2.0 * m_ * n_ * k_ / (np.median(t) * 1e-6) / 1e9, 1)}

    # the same product as a one-descriptor grouped launch (64-wide tiles: more
    # workgroups for a small product)
    desc = [_lib.make_desc("N", "N", n, n, n, 1.0, dA.data_ptr(), "c", n, dB.data_ptr(), "d", n, 1.0,
                           dC.data_ptr(), "z", n, "d")]
    for _ in range(20):
        assert _lib.mdgemm_grouped(desc, sp) == 0
    torch.cuda.synchronize()
    evg = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evg:
        e0.record(s)
        _lib.mdgemm_grouped(desc, sp)
        e1.record(s)
    torch.cuda.synchronize()
    grp = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in evg])
    dC.copy_(torch.from_numpy(C0))
    assert _lib.mdgemm_grouped(desc, sp) == 0
    torch.cuda.synchronize()
    gratio = float(np.max(np.abs(dC.cpu().numpy() - ref) / bound))
    assert gratio <= 1.0, "single (grouped): outside the bound (%.3g)" % gratio

    flops = 4.0 * n ** 3
    nbytes = n * n * (8 + 8 + 16 + 16)  # A (c), B (d), C read and written (z)
    p50 = float(np.median(dev))
    t_floor = max(flops / 78.6e12, nbytes / 8e12) * 1e6
    line = {"metric": "latency of one mixed GEMM (zcdd, m=n=k=256, double)", "value": round(p50, 2),
            "unit": "us", "n_gpus": 1, "steps": reps, "higher_is_better": False, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "single product zcdd (case 2ac) m=n=k=256 column-major, alpha=1, beta=1, "
                                   "computation precision double, U[-1,1]"},
            "device_us": {"p50": round(p50, 2), "p99": round(float(np.percentile(dev, 99)), 2)},
            "host_wall_us": {"p50": round(float(np.median(wall)), 2), "p99": round(float(np.percentile(wall, 99)), 2)},
            "gflops": round(flops / (p50 * 1e-6) / 1e9, 1),
            "roofline": {"bound": "latency", "floor_us": round(t_floor, 3),
                         "note": "max(4mnk / FP64 MFMA peak, algorithmic bytes / 8 TB/s)",
                         "frac": round(t_floor / p50, 4)},
            "grouped_one_descriptor_us": {"p50": round(float(np.median(grp)), 2),
                                          "p99": round(float(np.percentile(grp, 99)), 2)},
            "native_dgemm": {"512x256x256": native(2 * n, n, n), "256x256x256": native(n, n, n)},
            "oracle_max_err_over_bound": ratio}
    print(json.dumps(line), flush=True)


def grouped_workload(args):
    """Batching form: 512 products, m, n, k each log-uniform integers in
    [16, 1024], (storage combination, computation precision) uniform over the
    128 cases, U[-1,1], alpha = beta = 1, fixed seed.  One grouped launch (tile
    shapes from the autotuned table when present) against the same 512
    products as back-to-back mdgemm calls on one stream."""
    import torch
    import oracle
    from paper_1901_06015_amd import _lib, inputs
    count = 512
    dims = inputs.loguniform_dims(3 * count, 4242, 16, 1024).reshape(count, 3)
    rng = np.random.Generator(np.random.PCG64(4243))
    table = os.path.join(ROOT, "paper_1901_06015_amd", "tune_table.txt")
    tuned = os.path.exists(table) and _lib.tune_load(table) == 0
    if not tuned:
        _lib.tune_load(None)
    allc = combos("")
    ents, keep, host = [], [], []
    sp = torch.cuda.current_stream().cuda_stream
    for i in range(count):
        cabx = allc[int(rng.integers(0, len(allc)))]
        m, n, k = (int(x) for x in dims[i])
        tc, ta, tb, x = cabx
        A = inputs.matrix(m, k, ta, 10 * i + 1)
        B = inputs.matrix(k, n, tb, 10 * i + 2)
        C = inputs.matrix(m, n, tc, 10 * i + 3)
        dA, dB, dC = (torch.from_numpy(t).cuda() for t in (A, B, C))
        ents.append((cabx, m, n, k))
        keep.append((dA, dB, dC))
        host.append((A, B, C))
    def descs():
        return [_lib.make_desc("N", "N", m, n, k, 1.0, dA.data_ptr(), c[1], m, dB.data_ptr(), c[2], k, 1.0,
                               dC.data_ptr(), c[0], m, c[3]) for (c, m, n, k), (dA, dB, dC) in zip(ents, keep)]
    D = descs()
    flops = 0.0
    roof = 0.0
    for c, m, n, k in ents:
        st, pl = _lib.mdgemm_plan("N", "N", m, n, k, 1.0, 1, c[1], m, 1, c[2], k, 1.0, 1, c[0], m, c[3])
        flops += pl["flops"]
        peak = (78.6 if c[3] == "d" else 157.3) * 1e12
        byts = ELEM_BYTES[c[1]] * m * k + ELEM_BYTES[c[2]] * k * n + 2 * ELEM_BYTES[c[0]] * m * n
        roof += max(pl["flops"] / peak, byts / 8e12)

    def plain():
        for (c, m, n, k), (dA, dB, dC) in zip(ents, keep):
            st = _lib.mdgemm("N", "N", m, n, k, 1.0, dA.data_ptr(), c[1], m, dB.data_ptr(), c[2], k, 1.0,
                             dC.data_ptr(), c[0], m, c[3], sp)
            assert st == 0

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        return float(np.median(ts)), ts

    print("# grouped: %d products, %.2f GFLOP" % (count, flops / 1e9), file=sys.stderr, flush=True)
    tg, tgs = timed(lambda: _lib.mdgemm_grouped(D, sp), args.steps)
    tp, tps = timed(plain, args.steps)
    # correctness of one grouped launch on fresh C, every product against the oracle
    for (dA, dB, dC), (A, B, C) in zip(keep, host):
        dC.copy_(torch.from_numpy(C))
    st = _lib.mdgemm_grouped(D, sp)
    torch.cuda.synchronize()
    o = oracle.get()
    worst = 0.0
    nchk = count if args.check else 16
    for idx in range(nchk):
        (c, m, n, k), (dA, dB, dC), (A, B, C) = ents[idx], keep[idx], host[idx]
        st2, ref, g = o.gemm("N", "N", m, n, k, 1.0, A, c[1], m, B, c[2], k, 1.0, C, c[0], m)
        got = dC.cpu().numpy().astype(np.complex128)
        ux = 2.0 ** -24 if c[3] == "s" else 2.0 ** -53
        uc = 2.0 ** -24 if c[0] in "sc" else 2.0 ** -53
        bound = 4 * k * ux * g + 4 * uc * np.abs(ref)
        worst = max(worst, float(np.max(np.abs(got - ref) / np.maximum(bound, 1e-300))))
    line = {"metric": "GFLOP/s of 512 mixed GEMMs: one grouped launch vs one launch per GEMM",
            "value": round(flops / tg / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
            "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "batching form: 512 GEMMs, m,n,k log-uniform in [16,1024], 128 cases "
                                   "uniform, U[-1,1], alpha=beta=1", "count": count,
                       "tile_table": "autotuned" if tuned else "defaults"},
            "total_gflop": round(flops / 1e9, 3),
            "grouped_ms": round(tg * 1e3, 3), "plain_ms": round(tp * 1e3, 3),
            "plain_gflops": round(flops / tp / 1e9, 1),
            "speedup_grouped_over_plain": round(tp / tg, 2),
            "roofline": {"sum_of_per_gemm_roofline_ms": round(roof * 1e3, 3),
                         "grouped_frac": round(roof / tg, 4), "plain_frac": round(roof / tp, 4)},
            "max_err_over_bound": worst, "checked_products": nchk}
    print(json.dumps(line), flush=True)


class _ServingPool:
    """Device-resident request templates for the serving form.

    Small requests follow the batching form's distribution (m, n, k each a
    log-uniform integer in [16, 1024], storage combination and computation
    precision uniform over the 128 cases, U[-1,1], alpha = beta = 1), one
    template per shape with its own A, B and input C.  Large requests are
    m = n = k = 4096 in a uniformly drawn case; since they all share one
    shape, one 4096 x 4096 operand per storage type serves as A, B or C of
    every combination.  Templates are uploaded once (md_server_put) and every
    request names them by handle."""

    def __init__(self, srv, nsmall=1024, seed=5150, big=4096, host_cache=None):
        import ctypes
        from paper_1901_06015_amd import _lib, inputs, serving
        self.srv, self.L = srv, srv.L
        self.allc = combos("")
        dims = inputs.loguniform_dims(3 * nsmall, seed, 16, 1024).reshape(nsmall, 3)
        rng = np.random.Generator(np.random.PCG64(seed + 1))
        self.small, self.small_flops = [], []
        for i in range(nsmall):
            cabx = self.allc[int(rng.integers(0, len(self.allc)))]
            m, n, k = (int(x) for x in dims[i])
            tc, ta, tb, x = cabx
            ha = srv.put(inputs.matrix(m, k, ta, 10 * i + seed + 1))
            hb = srv.put(inputs.matrix(k, n, tb, 10 * i + seed + 2))
            hc = srv.put(inputs.matrix(m, n, tc, 10 * i + seed + 3))
            self.small.append(dict(cabx=cabx, m=m, n=n, k=k, a=ha, b=hb, c=hc, seed=10 * i + seed))
            st, pl = _lib.mdgemm_plan("N", "N", m, n, k, 1.0, 1, ta, m, 1, tb, k, 1.0, 1, tc, m, x)
            self.small_flops.append(pl["flops"])
        self.big_ops = {}
        for j, t in enumerate("sdcz"):
            for role in "abc":
                key = (role, t, big, seed)
                X = host_cache.get(key) if host_cache is not None else None
                if X is None:
                    X = inputs.matrix(big, big, t, seed + 100 + 3 * j + "abc".index(role))
                    if host_cache is not None:
                        host_cache[key] = X
                self.big_ops[role + t] = srv.put(X)
        self.big = big
        self.big_tpl = [dict(cabx=c, m=big, n=big, k=big, a=self.big_ops["a" + c[1]], b=self.big_ops["b" + c[2]],
                             c=self.big_ops["c" + c[0]]) for c in self.allc]
        self.big_flops = []
        for c in self.allc:
            st, pl = _lib.mdgemm_plan("N", "N", big, big, big, 1.0, 1, c[1], big, 1, c[2], big, 1.0, 1, c[0],
                                      big, c[3])
            self.big_flops.append(pl["flops"])

        def req(t, keep):
            return serving.MdRequest(b"N", b"N", t["m"], t["n"], t["k"], _lib.scalar(1.0), t["a"], t["b"],
                                     _lib.scalar(1.0), t["c"], _lib.tag(t["cabx"][0]), _lib.comp_tag(t["cabx"][3]),
                                     1 if keep else 0)
        self.small_req = [req(t, False) for t in self.small]
        self.small_req_keep = [req(t, True) for t in self.small]
        self.big_req = [req(t, False) for t in self.big_tpl]
        self.ticket = ctypes.c_int64()

    def draw(self, count, seed, big_frac=0.05):
        """A seeded request sequence: (is_big, template index) per request."""
        rng = np.random.Generator(np.random.PCG64(seed))
        big = rng.random(count) < big_frac
        si = rng.integers(0, len(self.small), count)
        bi = rng.integers(0, len(self.big_tpl), count)
        return [(bool(b), int(bb if b else s)) for b, s, bb in zip(big, si, bi)]

    def flops_of(self, r):
        return self.big_flops[r[1]] if r[0] else self.small_flops[r[1]]

    def submit(self, srv, r, keep=False):
        import ctypes
        q = self.big_req[r[1]] if r[0] else (self.small_req_keep if keep else self.small_req)[r[1]]
        st = self.L.md_server_submit(srv.h, ctypes.byref(q), ctypes.byref(self.ticket))
        if st != 0:
            raise RuntimeError("md_server_submit refused a benchmark request: %d" % st)
        return self.ticket.value


def _collect(srv, tickets, timeout):
    """Wait for every ticket; returns arrays of (submit, admit, done) times in
    microseconds and the batch sizes, then forgets the records."""
    out = np.zeros((len(tickets), 4))
    deadline = time.time() + timeout
    for i, t in enumerate(tickets):
        st, r = srv.wait(t, max(0.001, deadline - time.time()))
        if st != 0 or r.status != 0:
            raise RuntimeError("request %d did not complete (wait %d, status %d)" % (t, st, r.status))
        out[i] = (r.t_submit_us, r.t_admit_us, r.t_done_us, r.batch_size)
        srv.forget(t)
    return out


def _latency_stats(times, is_big, flops):
    lat = (times[:, 2] - times[:, 0]) / 1e3
    span = (times[:, 2].max() - times[:, 0].min()) / 1e6

    def pct(x):
        if len(x) == 0:
            return None
        return {"p50_ms": round(float(np.percentile(x, 50)), 3), "p99_ms": round(float(np.percentile(x, 99)), 3),
                "mean_ms": round(float(np.mean(x)), 3), "count": int(len(x))}
    return {"all": pct(lat), "small": pct(lat[~is_big]), "big_4096": pct(lat[is_big]),
            "queue_wait_p99_ms": round(float(np.percentile((times[:, 1] - times[:, 0]) / 1e3, 99)), 3),
            "mean_batch": round(float(np.mean(times[:, 3])), 2),
            "sustained_gflops": round(float(np.sum(flops)) / span / 1e9, 1), "span_s": round(span, 3)}


def _closed_loop(pool, srv, reqs):
    tickets = [pool.submit(srv, r) for r in reqs]
    times = _collect(srv, tickets, 600)
    span = (times[:, 2].max() - times[:, 0].min()) / 1e6
    fl = sum(pool.flops_of(r) for r in reqs)
    return len(reqs) / span, fl / span / 1e9, span


def _open_loop(pool, srv, reqs, arrivals, label, keep_first=0):
    """Submit each request at its arrival time (busy-wait for the last
    fraction of a millisecond), then wait for all of them."""
    tickets, kept = [], []
    t0 = time.perf_counter()
    next_report = 10.0
    late = 0.0
    for i, (r, ta) in enumerate(zip(reqs, arrivals)):
        target = t0 + ta
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            if target - now > 1e-3:
                time.sleep(target - now - 5e-4)
        late = max(late, now - target)
        keep = (not r[0]) and len(kept) < keep_first
        t = pool.submit(srv, r, keep=keep)
        tickets.append(t)
        if keep:
            kept.append((i, t))
        if ta >= next_report:
            print("# %s: %.0f s, %d requests submitted" % (label, ta, i + 1), file=sys.stderr, flush=True)
            next_report += 10.0
    submit_s = time.perf_counter() - t0
    outputs = []
    for i, t in kept:
        st, res = srv.wait(t, 600)
        outputs.append((i, res.output))
    times = _collect(srv, tickets, 3 * max(60.0, arrivals[-1]))
    return times, submit_s, late, outputs


def serving_workload(args):
    """Serving form: a Poisson stream of requests at a fixed rate (by default
    70 % of the measured served capacity) for --duration seconds; each request
    is drawn from the batching form's distribution, or with probability 0.05
    is an m = n = k = 4096 product of a uniformly drawn case.  Admission is
    capped by a 64 GB in-flight working-set budget.  The plain form is the
    same server with batching and overlap off (one stream slot, every request
    its own mdgemm, in arrival order).  Reported: both forms' closed-loop
    capacity, the served form's latency at --load of its capacity, and both
    forms' latency on one stream at --load of the plain form's capacity, the
    plain form on the headline trace, and a sample of requests re-run alone
    (bitwise equal to their in-mix results).
    Latency = completion observed by the server minus submission."""
    import torch
    import oracle
    from paper_1901_06015_amd import _lib, inputs, serving
    _lib.lib()
    torch.cuda.set_device(0)
    torch.cuda.init()
    table = os.path.join(ROOT, "paper_1901_06015_amd", "tune_table.txt")
    tuned = os.path.exists(table) and _lib.tune_load(table) == 0
    budget = 64 << 30
    big_flops = args.big_gflop * 1e9
    srv = serving.Server(budget, slots=args.slots, max_batch=args.max_batch, big_flops=big_flops,
                         big_lanes=args.big_lanes)
    plain = None if args.no_plain_stream else serving.Server(budget, slots=1, max_batch=1, big_flops=0.0)
    t0 = time.time()
    cache = {}
    pool = _ServingPool(srv, host_cache=cache)
    # the plain-form server holds its own copies of the same templates
    ppool = _ServingPool(plain, host_cache=cache) if not args.no_plain_stream else None
    cache.clear()
    print("# serving: templates resident in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    # closed-loop capacity of both forms on one seeded sample (after a warm-up)
    sample = pool.draw(2000, 6001)
    _closed_loop(pool, srv, pool.draw(300, 6000))
    cap_rps, cap_gf, cap_span = _closed_loop(pool, srv, sample)
    print("# serving capacity: %.0f req/s, %.0f GFLOP/s" % (cap_rps, cap_gf), file=sys.stderr, flush=True)
    pcap = None
    if ppool is not None:
        _closed_loop(ppool, plain, ppool.draw(300, 6000))
        p_rps, p_gf, p_span = _closed_loop(ppool, plain, sample)
        pcap = {"req_per_s": round(p_rps, 1), "gflops": round(p_gf, 1)}
        print("# plain capacity: %.0f req/s, %.0f GFLOP/s" % (p_rps, p_gf), file=sys.stderr, flush=True)

    def stream(qps, seed):
        rng = np.random.Generator(np.random.PCG64(seed))
        nreq = int(np.ceil(qps * args.duration * 1.2)) + 16
        arr = np.cumsum(rng.exponential(1.0 / qps, nreq))
        arr = arr[arr < args.duration]
        rq = pool.draw(len(arr), seed + 1)
        return arr, rq, np.array([r[0] for r in rq]), np.array([pool.flops_of(r) for r in rq])

    # headline: the served form at --load of its own capacity
    qps = args.qps if args.qps > 0 else args.load * cap_rps
    arrivals, reqs, is_big, flops = stream(qps, 6002)
    print("# serving stream: %d requests over %.0f s at %.0f req/s" % (len(reqs), args.duration, qps),
          file=sys.stderr, flush=True)
    times, submit_s, late, outputs = _open_loop(pool, srv, reqs, arrivals, "served", keep_first=8)
    served = _latency_stats(times, is_big, flops)
    served["offered_req_per_s"] = round(qps, 1)
    served["submit_lag_max_ms"] = round(late * 1e3, 3)
    counters = srv.stats()

    # the kept outputs against the oracle (elementwise bound)
    o = oracle.get()
    worst = 0.0
    mixed_out = {}
    for i, h in outputs:
        t = pool.small[reqs[i][1]]
        tc, ta, tb, x = t["cabx"]
        m, n, k, sd = t["m"], t["n"], t["k"], t["seed"]
        A, B, C = inputs.matrix(m, k, ta, sd + 1), inputs.matrix(k, n, tb, sd + 2), inputs.matrix(m, n, tc, sd + 3)
        st, ref, g = o.gemm("N", "N", m, n, k, 1.0, A, ta, m, B, tb, k, 1.0, C, tc, m)
        got_raw = srv.fetch(h, m, n, tc)
        mixed_out[i] = got_raw
        got = got_raw.astype(np.complex128)
        srv.drop(h)
        ux = 2.0 ** -24 if x == "s" else 2.0 ** -53
        uc = 2.0 ** -24 if tc in "sc" else 2.0 ** -53
        bound = 4 * k * ux * g + 4 * uc * np.abs(ref)
        worst = max(worst, float(np.max(np.abs(got - ref) / np.maximum(bound, 1e-300))))

    # alone vs in the mix: each kept request again, by itself, bitwise
    alone_equal = 0
    for i, h in outputs:
        t = pool.small[reqs[i][1]]
        tk = pool.submit(srv, reqs[i], keep=True)
        st, res = srv.wait(tk, 600)
        a = srv.fetch(res.output, t["m"], t["n"], t["cabx"][0])
        srv.drop(res.output)
        srv.forget(tk)
        alone_equal += int(np.array_equal(a, mixed_out[i]))

    # the plain form on the same trace (it may be over capacity at this rate)
    same_trace = None
    if ppool is not None:
        t_p, _, lag_p, _ = _open_loop(ppool, plain, reqs, arrivals, "plain@same")
        same_trace = _latency_stats(t_p, is_big, flops)

    # both forms at one rate the plain form can sustain (--load of its capacity)
    equal = None
    if ppool is not None:
        q2 = args.load * pcap["req_per_s"]
        arr2, req2, big2, fl2 = stream(q2, 6004)
        print("# equal-rate streams: %d requests at %.0f req/s" % (len(req2), q2), file=sys.stderr, flush=True)
        t_s, _, lag_s, _ = _open_loop(pool, srv, req2, arr2, "served@equal")
        t_p, _, lag_p, _ = _open_loop(ppool, plain, req2, arr2, "plain@equal")
        equal = {"offered_req_per_s": round(q2, 1), "requests": len(req2),
                 "served": _latency_stats(t_s, big2, fl2), "plain": _latency_stats(t_p, big2, fl2)}
        plain.close()
    srv.close()

    line = {"metric": "served mixed GEMM: sustained GFLOP/s and p50/p99 latency under a Poisson stream",
            "value": served["sustained_gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
            "data": "synthetic",
            "config": {"workload": "serving form: Poisson arrivals for %.0f s; 95%% batching-form requests "
                                   "(m,n,k log-uniform in [16,1024], 128 cases uniform), 5%% m=n=k=4096 of a "
                                   "uniform case; U[-1,1], alpha=beta=1; 64 GB working-set budget"
                                   % args.duration,
                       "offered_req_per_s": round(qps, 1), "requests": len(reqs),
                       "big_fraction": round(float(is_big.mean()), 4), "slots": args.slots,
                       "max_batch": args.max_batch, "big_gflop": args.big_gflop, "big_lanes": args.big_lanes,
                       "tile_table": "autotuned" if tuned else "defaults", "budget_bytes": budget},
            "latency": served, "plain_same_trace": same_trace, "equal_rate": equal,
            "capacity": {"served": {"req_per_s": round(cap_rps, 1), "gflops": round(cap_gf, 1)}, "plain": pcap},
            "counters": {k: counters[k] for k in ("batches", "grouped_launches", "plain_launches",
                                                  "peak_inflight_bytes", "max_concurrent_batches",
                                                  "resident_bytes", "pool_bytes", "device_mallocs")},
            "max_err_over_bound": worst, "checked_outputs": len(outputs),
            "alone_equals_in_mix": "%d of %d bitwise" % (alone_equal, len(outputs))}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "precision":
        return precision_workload(args)
    if args.workload == "grouped":
        return grouped_workload(args)
    if args.workload == "serving":
        return serving_workload(args)
    if args.workload == "single":
        return single_workload(args)
    import torch
    from paper_1901_06015_amd import _lib, api
    _lib.lib()
    n = args.size
    todo = combos(args.combos)
    print("# bench: %d combinations at %d^3" % (len(todo), n), file=sys.stderr, flush=True)
    ops = make_operands(n)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    plans = {}
    for cabx in todo:
        tc, ta, tb, x = cabx
        st, p = _lib.mdgemm_plan("N", "N", n, n, n, 1.5, ops["A" + ta].data_ptr(), ta, n,
                                 ops["B" + tb].data_ptr(), tb, n, -0.5, ops["C" + tc].data_ptr(), tc, n, x)
        assert st == 0, (cabx, st)
        plans[cabx] = p

    def launch(cabx):
        tc, ta, tb, x = cabx
        st = _lib.mdgemm("N", "N", n, n, n, 1.5, ops["A" + ta].data_ptr(), ta, n,
                         ops["B" + tb].data_ptr(), tb, n, -0.5, ops["C" + tc].data_ptr(), tc, n, x, sp)
        if st != 0:
            raise RuntimeError("mdgemm %s failed: %d" % (cabx, st))

    for w in range(args.warmup):
        for cabx in todo:
            launch(cabx)
        torch.cuda.synchronize()
        print("# warmup %d done" % w, file=sys.stderr, flush=True)

    # the native same-type GEMMs are timed once per step, after the sweep's
    # closing event, so that they see the same clocks and thermal state
    nops = native_operands(n) if not args.no_native else {}
    nat_ts = {name: [] for name in nops}
    times = {c: [] for c in todo}
    step_ms = []
    for s in range(args.steps):
        evs = []
        torch.cuda.synchronize()
        e_start = torch.cuda.Event(enable_timing=True)
        e_start.record(stream)
        prev = e_start
        for cabx in todo:
            launch(cabx)
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            evs.append((cabx, prev, e))
            prev = e
        torch.cuda.synchronize()
        for cabx, a, b in evs:
            times[cabx].append(a.elapsed_time(b) / 1e3)
        step_ms.append(e_start.elapsed_time(prev))
        if nops:
            for name, t in native_once(nops, stream).items():
                nat_ts[name].append(t)
        print("# step %d: %.1f ms" % (s, step_ms[-1]), file=sys.stderr, flush=True)

    flops = {c: plans[c]["flops"] for c in todo}
    step_flops = sum(flops.values())
    ms = float(np.median(step_ms))
    value = step_flops / (ms / 1e3) / 1e9

    native = {}
    for name, (a, b, c, fl) in nops.items():
        p50 = float(np.median(nat_ts[name]))
        native[name] = {"p50_s": p50, "gflops": fl * n ** 3 / p50 / 1e9}
    del nops
    torch.cuda.empty_cache()
    adhoc = adhoc_times(ops, todo) if not args.no_adhoc else {}
    if args.calibrate_copy:
        copy_calibration()
    per = {}
    by_kernel = {}
    short = {}
    for c in todo:
        ts = np.array(times[c])
        p50 = float(np.median(ts))
        gf = flops[c] / p50 / 1e9
        nat = native.get(native_for(plans[c]["case"], c[3]))
        per[c] = {"case": plans[c]["case"], "gflops": round(gf, 1),
                  "vs_native": round(gf / nat["gflops"], 3) if nat else None,
                  "p50_ms": round(p50 * 1e3, 4), "p99_ms": round(float(np.percentile(ts, 99)) * 1e3, 4),
                  "kernel": plans[c]["kernel"]}
        if c in adhoc:
            per[c]["adhoc_ms"] = round(adhoc[c] * 1e3, 4)
            per[c]["speedup_vs_adhoc"] = round(adhoc[c] / p50, 3)
        k = kernel_symbol(plans[c])
        short[k] = plans[c]["kernel"]
        bk = by_kernel.setdefault(k, {"flops": 0.0, "time": 0.0, "launches": 0, "bytes": 0.0})
        bk["flops"] += flops[c] * len(ts)
        bk["bytes"] += algorithmic_bytes(c, n) * len(ts)
        bk["time"] += float(ts.sum())
        bk["launches"] += len(ts)
    dom = max(by_kernel, key=lambda k: by_kernel[k]["time"])
    dk = by_kernel[dom]
    prec = "f64" if "<double" in dom else "f32"
    achieved = dk["flops"] / dk["time"] / 1e12
    ratios = {c: v["vs_native"] for c, v in per.items() if v["vs_native"] is not None}
    rv = list(ratios.values())
    worst = sorted(ratios, key=lambda c: ratios[c])[:5]
    traffic = traffic_record(dom)
    # everything per combination and per kernel goes to the detail record
    detail = {"per_combo": per,
              "per_kernel": {k: {"short": short[k], "tflops": round(v["flops"] / v["time"] / 1e12, 2),
                                 "avg_ms": round(v["time"] / v["launches"] * 1e3, 4),
                                 "launches": v["launches"]} for k, v in sorted(by_kernel.items())},
              "native_p50_ms": {k: round(v["p50_s"] * 1e3, 4) for k, v in native.items()},
              "dominant_kernel_symbol": dom, "traffic": traffic}
    if args.detail:
        with open(args.detail, "w") as f:
            json.dump(detail, f, indent=1)
    else:
        print("# detail " + json.dumps(detail), file=sys.stderr, flush=True)
    out = {
        "metric": "GFLOP/s per type combo at m=n=k=4096 vs native same-type; p50/p99 latency",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "plain method full sweep: %d of the 128 storage x computation-precision "
                               "combinations, m=n=k=%d column-major, U[-1,1], alpha=1.5, beta=-0.5, "
                               "no transpose" % (len(todo), n),
                   "m": n, "n": n, "k": n, "combos": len(todo)},
        "latency_ms": {"p50_of_p50": round(float(np.median([v["p50_ms"] for v in per.values()])), 4),
                       "max_p99": round(max(v["p99_ms"] for v in per.values()), 4)},
        "vs_native": ({"min": min(rv), "median": round(float(np.median(rv)), 3),
                       "ge_0.9": sum(1 for r in rv if r >= 0.9), "of": len(rv),
                       "worst": {c: ratios[c] for c in worst},
                       "native_gflops": {k: round(v["gflops"], 1) for k, v in native.items()},
                       "timing": "vendor GEMMs timed once per step, interleaved with the sweep; medians"}
                      if rv else None),
        "vs_adhoc": ({"median": round(float(np.median([v["speedup_vs_adhoc"] for v in per.values()])), 3),
                      "min": min(v["speedup_vs_adhoc"] for v in per.values())}
                     if adhoc else None),
        "roofline": {"bound": "mfma", "kernel": short[dom], "achieved": round(achieved, 2),
                     "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS[prec], 4),
                     "traffic": round(traffic["bytes"]) if traffic else None,
                     "algorithmic_bytes": round(dk["bytes"] / dk["launches"]),
                     "algorithmic_flops": round(dk["flops"] / dk["launches"]),
                     "avg_launch_ms": round(dk["time"] / dk["launches"] * 1e3, 4),
                     "launches": dk["launches"], "kernel_src": kernel_source_sha()},
    }
    if not args.no_cpu:
        print("# cpu baseline (%.0f s)" % args.cpu_seconds, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
