"""Compile libptraster.so (HIP, gfx950 only) in-tree.

Flags: -ffp-contract=off keeps every binary64 / binary32 operation separately
rounded as the arithmetic contract requires (fmaf is always explicit);
packed fp32 instructions are disabled; no fast-math.
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libptraster.so")
SOURCES = ["ptraster.cpp", "kern_render.hip", "kern_accum.hip", "kern_build.hip", "kern_stream.hip",
           "render_static.hip"]
SHAPE_SOURCE = "kern_raster.hip"  # compiled once per workgroup shape
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def shapes():
    """The workgroup shapes (waves, depth, tile) listed in PR_RASTER_SHAPES of internal.h, in order."""
    with open(os.path.join(CSRC, "internal.h")) as f:
        text = f.read()
    m = re.search(r"#define PR_RASTER_SHAPES\(X\)((?:[^\n]*\\\n)*[^\n]*)", text)
    if not m:
        raise RuntimeError("PR_RASTER_SHAPES not found in internal.h")
    found = [tuple(int(v) for v in t) for t in re.findall(r"X\((\d+),\s*(\d+),\s*(\d+)\)", m.group(1))]
    if not found:
        raise RuntimeError("PR_RASTER_SHAPES is empty")
    return found


def _units():
    """(source, object, extra flags) of every translation unit."""
    units = [(s, os.path.join(CSRC, "_build", os.path.splitext(s)[0] + ".o"), []) for s in SOURCES]
    for w, d, t in shapes():
        obj = os.path.join(CSRC, "_build", f"kern_raster_w{w}_d{d}_t{t}.o")
        units.append((SHAPE_SOURCE, obj, [f"-DPR_WAVES={w}", f"-DPR_DEPTH={d}", f"-DPR_TILE={t}"]))
    return units


def _compile(unit):
    src, obj, extra = unit
    path = os.path.join(CSRC, src)
    lang = ["-x", "hip"] + DEVICE
    cmd = [HIPCC, *lang, *COMMON, *extra, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {' '.join(extra)}:\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose=False):
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    units = _units()
    with ThreadPoolExecutor(min(len(units), max(1, min(16, os.cpu_count() or 1)))) as ex:
        logs = list(ex.map(_compile, units))
    if verbose:
        for l in logs:
            if l.strip():
                print(l, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [u[1] for u in units]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
