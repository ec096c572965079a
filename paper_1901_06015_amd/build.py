"""Build libmdgemm.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1901_06015_amd.build [--incremental]

Every HIP source is compiled with packed-FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host planner is
plain C++.  Objects go to ``_build/``; the shared library is written next to
this file.

The compiler's resource report of every kernel (registers, spills, scratch,
occupancy, LDS) is collected into ``_build/kernel_resources.txt``; a kernel
whose scratch is more than its register spills account for (an array the
compiler could not keep in registers, e.g. accumulators indexed at run time)
fails the build.
"""
import json
import re
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmdgemm.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = os.environ.get("MDGEMM_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-Rpass-analysis=kernel-resource-usage"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "--offload-arch=" + ARCH, "-I" + os.path.join(ROOT, "include")]

# (source, extra defines, object name)
SOURCES = [("mdgemm_grouped_kernel.hip", [], "grouped_kernel.o")] + [("mdgemm_kernels.hip", ["-DMD_KT=%d" % t, "-DMD_KCASE=%d" % c], "k_%d_%d.o" % (t, c))
           for t in (1, 0, 2, 3) for c in (7, 4, 5, 6, 0, 1, 2, 3)] + [
    ("mdgemm_launch.hip", [], "launch.o"),
    ("mdgemm_packed.hip", [], "packed.o"),
    ("mdgemm_grouped.hip", [], "grouped.o"),
    ("mdgemm_api.cpp", [], "api.o"),
    ("md_server.cpp", [], "server.o"),
]


def _newest_input(src, depfile):
    """Modification time of the newest file an object of `src` depends on:
    the files its compiler depfile lists, else the source and every header
    under csrc/ and include/."""
    paths = []
    if os.path.exists(depfile):
        text = open(depfile).read().replace("\\\n", " ")
        for tok in text.split(":", 1)[-1].split():
            if tok.startswith(ROOT) or not tok.startswith("/"):
                paths.append(tok if tok.startswith("/") else os.path.join(ROOT, tok))
    if not paths:
        paths = [os.path.join(CSRC, src)]
        for d in (CSRC, os.path.join(ROOT, "include")):
            paths += [os.path.join(d, f) for f in os.listdir(d) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in paths if os.path.exists(p))


_REMARK = re.compile(r"remark:\s+(Function Name|TotalSGPRs|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|SGPRs Spill|VGPRs Spill|LDS Size \[bytes/block\]): (\S+)")
_KEYS = {"TotalSGPRs": "sgpr", "VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
         "Occupancy [waves/SIMD]": "occupancy", "SGPRs Spill": "sgpr_spill", "VGPRs Spill": "vgpr_spill",
         "LDS Size [bytes/block]": "lds"}


def _resources(stderr):
    """Per-kernel resource usage from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in stderr.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val) if val.isdigit() else val
    return out


def _unexplained_scratch(r):
    """Scratch bytes per lane beyond what the VGPR spills occupy."""
    return r.get("scratch", 0) - 4 * r.get("vgpr_spill", 0)


def _compile(entry, extra=(), build_dir=BUILD, incremental=False):
    src, defs, objname = entry
    defs = list(defs) + list(extra)
    path = os.path.join(CSRC, src)
    obj = os.path.join(build_dir, objname)
    stamp = obj + ".flags"
    dep = obj + ".d"
    resf = obj + ".res"
    key = " ".join(defs)
    if (incremental and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == key
            and os.path.exists(resf) and os.path.getmtime(obj) > _newest_input(src, dep)):
        return obj, json.load(open(resf))
    flags = HIP_FLAGS if src.endswith(".hip") else CXX_FLAGS
    # the host pass writes the depfile (every header either pass includes)
    cmd = [HIPCC] + flags + defs + ["-MD", "-MF", dep, "-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), res.stderr))
    resources = _resources(res.stderr)
    with open(resf, "w") as f:
        json.dump(resources, f)
    with open(stamp, "w") as f:
        f.write(key)
    return obj, resources


def build(verbose=True, defines=(), out=OUT, build_dir=BUILD, incremental=False):
    """Compile and link.  `defines` (e.g. ["-DMD_OCC=1"]) set the tuning knobs
    of md_tile.h; `out` and `build_dir` place a variant build elsewhere.
    `incremental` keeps objects newer than their source and every header
    (compiled with the same defines); the default recompiles everything."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = [e for e in SOURCES if os.path.exists(os.path.join(CSRC, e[0]))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(int(os.environ.get('MAX_JOBS', '8')), len(srcs))) as ex:
        done = list(ex.map(lambda e: _compile(e, defines, build_dir, incremental), srcs))
    objs = [o for o, _ in done]
    resources = {}
    for _, r in done:
        resources.update(r)
    with open(os.path.join(build_dir, "kernel_resources.txt"), "w") as f:
        f.write("# kernel  vgpr agpr sgpr occupancy scratch vgpr_spill lds\n")
        for name in sorted(resources):
            r = resources[name]
            f.write("%s  %s\n" % (name, " ".join(str(r.get(k, "?")) for k in
                                               ("vgpr", "agpr", "sgpr", "occupancy", "scratch", "vgpr_spill", "lds"))))
    bad = sorted(n for n, r in resources.items() if _unexplained_scratch(r) > 64)
    if bad:
        raise RuntimeError("kernels with scratch beyond their spills (an array left in memory):\n" +
                           "\n".join("%s: %s" % (n, resources[n]) for n in bad))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr))
    # a shared library links with undefined symbols; refuse one that would
    # fail only when the GPU path first calls into the missing piece
    und = subprocess.run(["nm", "-C", "-u", tmp], capture_output=True, text=True).stdout
    missing = [l.strip() for l in und.splitlines() if " md::" in l or "mdgemm" in l or " md_" in l]
    if missing:
        os.remove(tmp)
        raise RuntimeError("link left library symbols undefined:\n" + "\n".join(missing))
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
