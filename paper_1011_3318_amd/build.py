"""Builds the HIP library libwcl.so for gfx950 in-tree.

Every .hip source under csrc/ is compiled with hipcc to an object, then the
objects are linked into one shared library.  The library is linked against
the HIP runtime that PyTorch-ROCm loads (torch/lib/libamdhip64.so) so that a
process using both shares one runtime, with an rpath to it.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.environ.get("WCL_BUILD_DIR", os.path.join(HERE, "_build"))
LIB = os.environ.get("WCL_LIB_OUT", os.path.join(HERE, "libwcl.so"))
ARCH = os.environ.get("WCL_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no two-address v_dot2c_f32_f16: the three-address v_dot2_f32_f16 starts
    # each product chain from a shared zero without copying it first
    "-Xclang", "-target-feature", "-Xclang", "-dot5-insts",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}", f"-I{CSRC}",
] + os.environ.get("WCL_HIPCC_EXTRA", "").split()


def _torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("PyTorch-ROCm is required to build libwcl (its HIP runtime is linked)")
    return os.path.join(os.path.dirname(spec.origin), "lib")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", src, "-o", obj] + HIPCC_FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    if r.stderr.strip():
        # host-pass warning about the packed-fp32 feature is expected
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    cpp = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs + cpp))
    tlib = _torch_lib_dir()
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-nohipwrapperinc", f"-L{tlib}", f"-Wl,-rpath,{tlib}", os.path.join(tlib, "libamdhip64.so"), "-lpthread", "-Wl,--no-undefined",
    ]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libwcl.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
