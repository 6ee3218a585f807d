"""The C ABI on a machine without a GPU: symbols, sizes, argument checks, PR_EDEVICE."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptraster.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def pr():
    import paper_2204_01287_amd as pr

    return pr


def test_header_declares_the_four_verbs():
    names = _declared()
    for verb in ("pr_load_points", "pr_build_batches", "pr_render", "pr_resolve"):
        assert verb in names


def test_library_exports_every_declared_symbol(pr):
    names = _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", pr.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pr_[a-z_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(pr.lib, n)
    assert sorted(pr.EXPORTED) == names  # the binding covers the whole ABI


def test_cloud_sizes(pr):
    s = pr.pr_cloud_sizes(1_000_000, 10240, False)
    assert s.xyz == 12_000_000 and s.rgba == 4_000_000
    assert s.low == s.med == s.high == s.colors == s.perm == 4_000_000
    assert s.batches == 98 * 32 + (256 - (98 * 32) % 256)  # 98 batches, rounded to 256 bytes
    sm = pr.pr_cloud_sizes(1_000_000, 10240, True)
    assert sm.scratch > 20_000_000  # keys x2 (then the gather's 16-byte records), second value buffer
    z = pr.pr_cloud_sizes(0, 64, True)
    assert z.xyz == 0 and z.batches == 0


@pytest.mark.parametrize("n,bs,code", [(1000, 0, "PR_EINVAL"), (1000, 6, "PR_EINVAL"), (2 ** 32, 64, "PR_ERANGE"),
                                       (2 ** 40, 64, "PR_ERANGE")])
def test_cloud_sizes_rejects(pr, n, bs, code):
    with pytest.raises(pr.PrError) as e:
        pr.pr_cloud_sizes(n, bs, False)
    assert e.value.name == code
    assert pr.pr_last_error()


def test_null_arguments_are_einval(pr):
    lib = pr.lib
    assert lib.pr_create(0, None, None) == -1
    assert lib.pr_cloud_sizes(10, 64, 0, None) == -1
    assert lib.pr_build_batches(None, None, 64, 0) == -1
    assert lib.pr_render(None, None, None, None, 8, 8, None, None) == -1
    assert lib.pr_resolve(None, None, None, 8, 8, 0, None) == -1
    assert lib.pr_get_stats(None, None) == -1
    assert lib.pr_sync(None) == -1
    assert lib.pr_cloud_info(None, None, None, None) == -1
    lib.pr_destroy(None)
    lib.pr_cloud_free(None)


def test_no_gpu_is_edevice(pr):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pr.PrError) as e:
        pr.pr_create(0, None)
    assert e.value.name == "PR_EDEVICE"


def test_binding_has_no_fallback_path():
    """The product package must not import the oracle or any CPU implementation."""
    pkg = os.path.join(ROOT, "paper_2204_01287_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "oracle" not in src and "synth" not in src, f


def test_tuning_abi(pr):
    lib = pr.lib
    assert ctypes.sizeof(pr.Tuning) == 16 and ctypes.sizeof(pr.TuneTrial) == 24
    assert ctypes.sizeof(pr.RasterShape) == 16
    n = ctypes.c_uint32()
    assert lib.pr_raster_shapes(None, None, 0, ctypes.byref(n)) == -1
    assert lib.pr_set_tuning(None, None) == -1
    assert lib.pr_get_tuning(None, None) == -1
    assert lib.pr_autotune(None, None, None, 0, None, None, 0, 0, None, 0, None, None) == -1


def test_every_listed_shape_is_compiled_in(pr):
    """Each workgroup shape of the build's list is a translation unit of its own in the library."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("_b", os.path.join(ROOT, "paper_2204_01287_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    shapes = b.shapes()
    assert shapes[0] == (4, 5, 4992) and len(set(shapes)) == len(shapes)
    out = subprocess.run(["nm", "-C", "--defined-only", pr.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    for w, d, t in shapes:
        assert f"ptr::raster_shape_w{w}_d{d}_t{t}()" in out, (w, d, t)


def test_binding_shares_torchs_hip_runtime():
    """Importing the binding (here through the served-mode module, as test collection does) maps one HIP runtime:
    the one PyTorch ships, which then also serves the library.  A second runtime would find no device."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2204_01287_amd.serve\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n") % ROOT
    r = subprocess.run(["python", "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    mapped = eval(r.stdout.strip().splitlines()[-1])
    assert len(mapped) == 1, mapped
