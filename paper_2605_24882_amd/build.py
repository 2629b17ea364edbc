"""Build libgfield.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2605_24882_amd.build   (or call build()).
Objects go to paper_2605_24882_amd/_build/, the library to paper_2605_24882_amd/libgfield.so, and the
operator-kernel timing tool (csrc/kbench.hip, linked against the library) to paper_2605_24882_amd/kbench.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgfield.so")
KBENCH = os.path.join(HERE, "kbench")  # operator-kernel timing tool (measurement support)
SOURCES = ["gfield.cpp", "host_spline.cpp", "k_setup.hip", "k_solve.hip", "k_fused.hip", "k_adjoint.hip",
           "k_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wno-unused-command-line-argument",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=5) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    cmd = [HIPCC] + COMMON + [os.path.join(CSRC, "kbench.hip"), "-o", KBENCH + ".tmp", "-L" + HERE, "-lgfield",
                              "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"kbench build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(KBENCH + ".tmp", KBENCH)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
