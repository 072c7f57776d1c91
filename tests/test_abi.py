"""The C-ABI library builds, loads and exports every function include/vr.h
declares; without a GPU it refuses to create a context (no CPU fallback)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vr.h")
LIB = os.path.join(ROOT, "paper_2512_18646_amd", "libvr.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z0-9_]+)\s*\(", src)) - {"vr_params"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2512_18646_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["vr_context_create", "vr_keygen", "vr_encode", "vr_encrypt", "vr_encrypt_columns",
                 "vr_encrypt_matrix_columns", "vr_decrypt", "vr_decode", "vr_add", "vr_mul_plain",
                 "vr_mul_const", "vr_mul", "vr_rescale", "vr_rotate", "vr_rotate_many", "vr_matmul",
                 "vr_conv2d", "vr_square", "vr_fc", "vr_ct_export", "vr_ct_import", "vr_ntt"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (vr_[a-z0-9_]+)", out))
    assert set(declared_functions()) <= exported


def test_binding_covers_the_header():
    from paper_2512_18646_amd import vr
    assert set(declared_functions()) == set(vr.exported_symbols())


def test_library_carries_gfx950_code():
    assert b"amdgcn-amd-amdhsa--gfx950" in open(LIB, "rb").read()


def test_no_gpu_means_no_context():
    """Without a device the product path fails loudly instead of computing on the CPU."""
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    from paper_2512_18646_amd import vr
    with pytest.raises(vr.VRError) as e:
        vr.Context(13, [49, 40, 40, 40], [49], 4, 40.0)
    assert e.value.code == vr.VR_EDEVICE


def test_security_check_runs_before_device_use():
    from paper_2512_18646_amd import vr
    with pytest.raises(vr.VRError) as e:
        vr.Context(13, [60, 40, 40, 40], [60], 4, 40.0)   # 240 bits > 218
    assert e.value.code == vr.VR_ESECURITY
    with pytest.raises(vr.VRError) as e:
        vr.Context(13, [49, 40, 40, 40], [49], 4, 40.0, sigma=3.0)
    assert e.value.code == vr.VR_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 (or a WORLD_SIZE above 1) exits
    with status 2 and says so, before touching the library or a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py")] + args, cwd=root,
                           env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""
