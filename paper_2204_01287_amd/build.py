"""Compile libptraster.so (HIP, gfx950 only) in-tree.

Flags: -ffp-contract=off keeps every binary64 / binary32 operation separately
rounded as the arithmetic contract requires (fmaf is always explicit);
packed fp32 instructions are disabled; no fast-math.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libptraster.so")
SOURCES = ["ptraster.cpp", "kern_render.hip", "kern_build.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _obj(src):
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def _compile(src):
    path = os.path.join(CSRC, src)
    lang = ["-x", "hip"] + DEVICE
    cmd = [HIPCC, *lang, *COMMON, "-c", path, "-o", _obj(src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose=False):
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        logs = list(ex.map(_compile, SOURCES))
    if verbose:
        for l in logs:
            if l.strip():
                print(l, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [_obj(s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
