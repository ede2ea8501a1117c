"""Build liblma.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1411_4510_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblma.so")
SOURCES = ["engine.hip", "kernels_misc.hip", "vecsolve.hip", "grad.hip", "kvec.hip", "lma.hip", "lma_grad.hip", "ds.hip",
           "kmeans.hip", "partition.hip"]
ARCH = os.environ.get("LMA_OFFLOAD_ARCH", "gfx950")
# Per-source flags.  kvec.hip: its MFMA accumulators feed vector arithmetic
# right after every short k loop; in the accumulator-register form the compiler
# copies them between register files on every iteration, the VGPR form does not.
SOURCE_FLAGS = {"kvec.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=3):
    """Compile every HIP source for gfx950 and link liblma.so next to this file."""
    cc = hipcc()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    flags = [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result", "-I", CSRC, "-I", INCLUDE,
    ]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc] + flags + SOURCE_FLAGS.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    lines = [l for l in text.splitlines()
             if "packed-fp32-ops" not in l and "warnings generated" not in l and l.strip()]
    if p.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n" + text)
    if lines and os.environ.get("LMA_BUILD_VERBOSE"):
        print("\n".join(lines))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
