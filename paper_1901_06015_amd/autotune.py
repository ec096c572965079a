"""Autotuner for the grouped kernel's tile table.

The table maps (computation precision s/d, domain case, size bucket of the
real product's m', size bucket of its n' -- each <=64, <=128, <=256, <=512,
larger) to one of the grouped kernel's tile configurations: the workgroup
tile (64x64, 128x128, 128x64, 64x128), its wave arrangement (2x2 waves in two
k-groups, or 2x4 / 4x2 waves) and its k-tile depth (the 64x64 tile also
comes with a doubled k-tile, "64x64k").  Tiles of one grouped launch share
the GPU, so the best configuration for a product depends on the mix it runs
in.  The tuner therefore works in context: it draws a representative
training batch (by default the batching workload's distribution -- 512
products, m, n, k log-uniform in [16, 1024], combination and precision
uniform over the 128 cases -- with its own seed), then does coordinate
descent over the table entries that the batch touches: for one entry at a
time it times the whole grouped launch with each configuration (interleaved
repetitions, medians) and keeps the best only if it beats the entry's
current configuration by more than 1 %.
Entries the batch does not touch keep their defaults.  The result is a text
table for mdgemm_tune_load():

    python -m paper_1901_06015_amd.autotune --out paper_1901_06015_amd/tune_table.txt

Every measurement is a real launch on the GPU (HIP events, median of a few
repetitions); nothing is modelled.  Not searched: the MFMA instruction shape
(FP64 has one dense 16x16 shape; the FP32 32x32 shape has the same rate) and
split k (a grouped tile is one workgroup's; products long in k keep whole
k ranges, the plain path splits them).
"""
import argparse
import itertools
import sys
import time

import numpy as np

from . import _lib, inputs

CASES = ("0", "1a", "1b", "1c", "2ab", "2ac", "2bc", "3")
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
        touched.add((comp, pl["case"], _lib.tune_bucket(pl["m_real"]), _lib.tune_bucket(pl["n_real"])))
    return keep, descs, touched


def _timed_launch(descs, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    if _lib.mdgemm_grouped(descs, stream) != 0:
        raise RuntimeError("grouped launch failed")
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def time_grouped_median(descs, reps=7):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    _timed_launch(descs, stream)
    return float(np.median([_timed_launch(descs, stream) for _ in range(reps)]))


def compare_configs(descs, entry, configs, reps=7):
    """Median launch time of the whole batch with `entry` set to each of
    `configs`, measured interleaved (one launch per configuration in turn,
    `reps` rounds) so that clock and thermal drift hit every candidate alike."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    comp, case, bm, bn = entry
    times = {c: [] for c in configs}
    for _ in range(reps):
        for c in configs:
            _lib.tune_set(comp, case, bm, bn, c)
            times[c].append(_timed_launch(descs, stream))
    return {c: float(np.median(t)) for c, t in times.items()}


def tune(out_path, seed=777, passes=2, verbose=True):
    _lib.lib()
    _lib.tune_load(None)
    keep, descs, touched = training_batch(seed=seed)
    for _ in range(20):  # warm up clocks, caches and the upload staging
        time_grouped_median(descs, reps=1)
    start = time_grouped_median(descs, reps=15)
    if verbose:
        print("# start (defaults): %.4f ms, %d entries touched" % (start * 1e3, len(touched)), flush=True)
    configs = list(range(len(_lib.GTILE_NAMES)))
    for p in range(passes):
        changed = False
        for entry in sorted(touched):
            comp, case, bm, bn = entry
            cur = _lib.tune_get(comp, case, bm, bn)
            med = compare_configs(descs, entry, configs)
            best_cfg = min(configs, key=lambda c: med[c])
            if med[best_cfg] >= med[cur] * 0.99:
                best_cfg = cur
            _lib.tune_set(comp, case, bm, bn, best_cfg)
            if best_cfg != cur:
                changed = True
                if verbose:
                    print("# pass %d: %s %s %d %d: %s -> %s (%.4f -> %.4f ms)" % (
                        p, comp, case, bm, bn, _lib.GTILE_NAMES[cur], _lib.GTILE_NAMES[best_cfg],
                        med[cur] * 1e3, med[best_cfg] * 1e3), flush=True)
        if not changed:
            break
    best = time_grouped_median(descs, reps=15)
    if verbose:
        print("# tuned: %.4f ms (defaults %.4f ms)" % (best * 1e3, start * 1e3), flush=True)
    lines = ["# grouped-kernel tile table written by paper_1901_06015_amd.autotune",
             "# tuned in context on a seeded training batch (seed %d): %.4f ms per grouped launch "
             "(built-in rule %.4f ms)" % (seed, best * 1e3, start * 1e3),
             "# comp case bucket_m bucket_n config"]
    for comp in ("s", "d"):
        for case in CASES:
            for bm in range(_lib.TUNE_BUCKETS):
                for bn in range(_lib.TUNE_BUCKETS):
                    lines.append("%s %s %d %d %s" % (comp, case, bm, bn,
                                                     _lib.GTILE_NAMES[_lib.tune_get(comp, case, bm, bn)]))
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
