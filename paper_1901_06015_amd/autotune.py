"""Autotuner for the grouped kernel's tile-shape table.

The table maps (computation precision s/d, domain case, size bucket of the
larger real-product dimension: <=64, <=128, <=256, <=512, <=1024, larger) to
a tile edge (64 or 128).  Tiles of one grouped launch share the GPU, so the
best shape for a product depends on the mix it runs in.  The tuner therefore
works in context: it draws a representative training batch (by default the
batching workload's distribution -- 512 products, m, n, k log-uniform in
[16, 1024], combination and precision uniform over the 128 cases -- with its
own seed), then does coordinate descent over the table entries that the batch
touches, flipping one entry at a time and keeping a flip only if the measured
time of the whole grouped launch improves by more than 1 %.  Entries the batch
does not touch keep their defaults.  The result is a text table for
mdgemm_tune_load():

    python -m paper_1901_06015_amd.autotune --out paper_1901_06015_amd/tune_table.txt

Every measurement is a real launch on the GPU (HIP events, best of a few
repetitions); nothing is modelled.
"""
import argparse
import itertools
import sys
import time

import numpy as np

from . import _lib, inputs

CASES = ("0", "1a", "1b", "1c", "2ab", "2ac", "2bc", "3")
BUCKET_EDGES = (64, 128, 256, 512, 1024, 2048)


def combos_of_case(case):
    """Storage combinations (C, A, B) that fall in a domain case."""
    out = []
    for tc, ta, tb in itertools.product("sdcz", repeat=3):
        c, a, b = tc in "cz", ta in "cz", tb in "cz"
        name = {(0, 0, 0): "0", (0, 1, 0): "1a", (0, 0, 1): "1b", (1, 0, 0): "1c", (0, 1, 1): "2ab",
                (1, 1, 0): "2ac", (1, 0, 1): "2bc", (1, 1, 1): "3"}[(c, a, b)]
        if name == case:
            out.append((tc, ta, tb))
    return out


def training_batch(count=512, seed=777, lo=16, hi=1024):
    """The in-context training batch (seeded, distinct from the benchmark's)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = inputs.loguniform_dims(3 * count, seed + 1, lo, hi).reshape(count, 3)
    keep, descs, touched = [], [], set()
    for i in range(count):
        tc, ta, tb = ("sdcz"[j] for j in rng.integers(0, 4, 3))
        comp = "sd"[int(rng.integers(0, 2))]
        m, n, k = (int(x) for x in dims[i])
        A = torch.from_numpy(inputs.matrix(m, k, ta, 3 * i + seed)).cuda()
        B = torch.from_numpy(inputs.matrix(k, n, tb, 3 * i + seed + 1)).cuda()
        C = torch.from_numpy(inputs.matrix(m, n, tc, 3 * i + seed + 2)).cuda()
        keep += [A, B, C]
        descs.append(_lib.make_desc("N", "N", m, n, k, 1.0, A.data_ptr(), ta, m, B.data_ptr(), tb, k, 1.0,
                                    C.data_ptr(), tc, m, comp))
        st, pl = _lib.mdgemm_plan("N", "N", m, n, k, 1.0, 1, ta, m, 1, tb, k, 1.0, 1, tc, m, comp)
        big = max(pl["m_real"], pl["n_real"])
        bucket = next((b for b, e in enumerate(BUCKET_EDGES[:-1]) if big <= e), len(BUCKET_EDGES) - 1)
        touched.add((comp, pl["case"], bucket))
    return keep, descs, touched


def time_grouped_median(descs, reps=7):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    if _lib.mdgemm_grouped(descs, stream) != 0:
        raise RuntimeError("grouped launch failed")
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.mdgemm_grouped(descs, stream)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    return float(np.median(ts))


def tune(out_path, seed=777, passes=2, verbose=True):
    _lib.lib()
    _lib.tune_load(None)
    keep, descs, touched = training_batch(seed=seed)
    best = time_grouped_median(descs)
    if verbose:
        print("# start (defaults): %.4f ms, %d entries touched" % (best * 1e3, len(touched)), flush=True)
    for p in range(passes):
        changed = False
        for comp, case, bucket in sorted(touched):
            cur = _lib.tune_get(comp, case, bucket)
            alt = 64 if cur == 128 else 128
            _lib.tune_set(comp, case, bucket, alt)
            t = time_grouped_median(descs)
            if t < best * 0.99:
                best = t
                changed = True
                if verbose:
                    print("# pass %d: %s %s %d -> %d: %.4f ms" % (p, comp, case, bucket, alt, t * 1e3), flush=True)
            else:
                _lib.tune_set(comp, case, bucket, cur)
        if not changed:
            break
    lines = ["# grouped-kernel tile-shape table written by paper_1901_06015_amd.autotune",
             "# tuned in context on a seeded training batch (seed %d): %.4f ms per grouped launch" % (seed, best * 1e3),
             "# comp case bucket tile"]
    for comp in ("s", "d"):
        for case in CASES:
            for b in range(len(BUCKET_EDGES)):
                lines.append("%s %s %d %d" % (comp, case, b, _lib.tune_get(comp, case, b)))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    del keep
    return out_path


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--out", required=True)
    p.add_argument("--seed", type=int, default=777)
    a = p.parse_args(argv)
    t0 = time.time()
    tune(a.out, seed=a.seed)
    print("wrote %s in %.1f s" % (a.out, time.time() - t0))
    return 0


if __name__ == "__main__":
    sys.exit(main())
