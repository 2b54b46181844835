"""Build libcrsolve.so (HIP, gfx950) in-tree.

    python paper_1710_00621_amd/csrc/build.py [--jobs N] [--save-temps DIR]

Compiles every .hip file in this directory with hipcc for gfx950 and links
them into paper_1710_00621_amd/libcrsolve.so.  Object files go to
paper_1710_00621_amd/csrc/_build/ (not tracked).
"""
import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libcrsolve.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA operands and accumulators in ordinary VGPRs (no AGPR copies around
    # every matrix instruction inside loops)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_one(src, objdir, extra):
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=8, save_temps=None, verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "*.hip")))
    extra = []
    if save_temps:
        os.makedirs(save_temps, exist_ok=True)
        extra = ["-save-temps=obj"]
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, objdir, extra), srcs))
    tmp = OUT + ".tmp"
    # rocSOLVER / rocBLAS: the eigendecomposition of the mask preconditioner's
    # bottom level (setup only)
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--save-temps", default=None)
    a = ap.parse_args()
    build(a.jobs, a.save_temps, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
