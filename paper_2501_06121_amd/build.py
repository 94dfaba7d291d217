"""Compile libann.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libann.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -ffp-contract=off: every multiply and add stays as written (the fixed FP32
# order relies on it); packed FP32 instructions are disabled.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-value", f"-I{INCLUDE}", f"-I{CSRC}"]


def hip_runtime_dir():
    """Directory of the HIP runtime PyTorch loads.

    The library links that same libamdhip64 so that a process holding both
    torch tensors and this library has one HIP runtime (two runtimes in one
    process cannot share the GPU).
    """
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec and spec.origin:
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    return "/opt/rocm/lib"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


DEBUG_LIB = os.path.join(PKG, "libann_debug.so")


def build(verbose: bool = False, jobs: int | None = None, defines=(), out: str | None = None) -> str:
    """Compile every source to an object, then link libann.so (or `out`)."""
    srcs = sources()
    extra = [f"-D{d}" for d in defines]
    tmpdir = tempfile.mkdtemp(prefix="annbuild_")
    objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]

    def compile_one(pair):
        src, obj = pair
        cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(jobs or min(len(srcs), os.cpu_count() or 1)) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    target = out or LIB
    tmp_lib = target + ".tmp"
    rt = hip_runtime_dir()
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp_lib, *objs, f"-L{rt}", "-l:libamdhip64.so",
           f"-Wl,-rpath,{rt}", "-Wl,--no-undefined", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp_lib, target)
    for o in objs:
        os.remove(o)
    os.rmdir(tmpdir)
    return target


def build_debug(verbose: bool = False, jobs: int | None = None) -> str:
    """libann_debug.so: the same library with the kernels' invariant checks."""
    return build(verbose, jobs, defines=("ANN_DEBUG_CHECKS",), out=DEBUG_LIB)


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_debug(verbose=True))
