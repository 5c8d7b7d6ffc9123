"""Compile libldpc.so (HIP, gfx950) in-tree.

hipcc flags that matter for results:
  -ffp-contract=off                  no fused multiply-add where the code has
                                     a separate multiply and add
  -fno-gpu-flush-denormals-to-zero   IEEE binary32 subnormals
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                     no packed FP32 instructions

The target-feature flag can only reach the device compile through -Xclang,
which the driver hands to the host compile as well (hipcc's -Xarch_device
does not forward options that take an argument).  The host (x86) pass then
prints, once per source file, a notice that it does not know the feature and
ignores it; the build drops exactly that notice from its output and passes
every other diagnostic through.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libldpc.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # No wavefront-level combining of atomics: it makes the wavefront wait for
    # an atomic's return at once, where the on-chip decoder's frame counter
    # result is only needed a round later.
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function",
]


# what the host pass prints for the device-only target feature (see above)
HOST_FEATURE_NOTICE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
    for line in res.stderr.splitlines():
        if line.strip() != HOST_FEATURE_NOTICE:
            print(line, file=sys.stderr)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object (in parallel, one hipcc per file),
    then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(objdir, os.path.splitext(os.path.basename(f))[0] + ".o") for f in srcs]
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    cmds = [[hipcc, *compile_flags, "-I", INCLUDE, "-I", CSRC, "-c", f, "-o", o] for f, o in zip(srcs, objs)]
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for fut in [ex.submit(_run, c, verbose) for c in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
