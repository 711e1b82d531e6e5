"""Build libmegapf.so (all HIP sources, gfx950) next to this file.

    python -m paper_2404_16370_amd.build

Every translation unit is compiled with -ffp-contract=off: the deterministic
FP32 programs that take the filter's discrete decisions must not be fused,
and the floating-point paths use explicit fma where they want one.  Packed
FP32 instructions are disabled for the whole library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmegapf.so")
SOURCES = ["api.hip", "map_build.hip", "scan.hip", "sort.hip", "neighbors.hip", "likelihood.hip",
           "filter_kernels.hip", "surrogate.hip", "batch.hip", "odometry.hip", "smoother.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fvisibility=hidden", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(jobs: int = 8, verbose: bool = False) -> str:
    objs = []
    procs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared",)], "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(tmp, LIB)
    return LIB


def _wait(procs):
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode()
        if p.returncode != 0:
            failed.append((src, out))
        elif out.strip():
            sys.stderr.write(out)
    if failed:
        raise RuntimeError("\n".join("%s:\n%s" % f for f in failed))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
