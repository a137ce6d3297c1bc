"""Build the gfx950 library ``libwost.so`` in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwost.so")
SOURCES = ["geom_build.cpp", "geom_gpu.hip", "walk.hip", "wavefront.hip", "lbvh.hip", "guide.hip", "train.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed-FP32 VALU forms are kept out of every device object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware fp32 atomics for the grid-gradient scatter
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]


# per-source extra flags: the walk kernel keeps machine-level loop-invariant
# code motion off, which otherwise hoists per-phase values across all phases
# of a walk round and costs resident waves (measured 4-6% faster)
EXTRA = {"walk.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False) -> str:
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    inc = ["-I", os.path.join(HERE, "..", "include")]
    objs = []
    tag = "%d" % os.getpid()

    def compile_one(src):
        obj = os.path.join(CSRC, src + ".o" + tag)
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], *EXTRA.get(src, []), *inc, "-c",
               os.path.join(CSRC, src), "-o", obj]
        return src, obj, subprocess.run(cmd, capture_output=True, text=True)

    try:
        # the sources compile independently: one hipcc process each
        jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(compile_one, srcs))
        for src, obj, res in results:
            if res.returncode == 0:
                objs.append(obj)
        for src, obj, res in results:
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError("hipcc failed compiling %s" % src)
            if verbose:
                sys.stderr.write(res.stderr)
        tmp = LIB + ".tmp" + tag
        res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                             capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libwost.so")
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
