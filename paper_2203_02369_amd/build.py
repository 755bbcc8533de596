"""Builds libhamlet.so (HIP, gfx950) in the package directory.

    python -m paper_2203_02369_amd.build
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libhamlet.so")
SOURCES = [os.path.join(PKG, "csrc", "hamlet.hip")]
HEADERS = ["common.hpp", "schedule.hpp", "tuned.hpp", "fft.hpp", "workspace.hpp", "random.hpp", "flat.hpp", "passes.hpp",
           "galaxies.hpp", "hmc.hpp", "nuts.hpp", "analysis.hpp"]

ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions on this target (some forms misbehave)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, out=None, defines=(), quiet=False):
    """Compile every HIP source into libhamlet.so (or `out`, with extra -D
    `defines`: the autotuner's candidate libraries); always recompiles.
    quiet: the compiler's messages go into the exception, not stderr."""
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [hipcc()] + FLAGS + ["-D" + d for d in defines] + ["-I", os.path.join(ROOT, "include"), "-I",
                                                             os.path.join(PKG, "csrc"), "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        if quiet:
            raise RuntimeError("hipcc failed building %s:\n%s" % (os.path.basename(lib), (res.stdout + res.stderr)[-4000:]))
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libhamlet.so")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
