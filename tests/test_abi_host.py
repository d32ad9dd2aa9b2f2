"""The C ABI's host code built without device code at -O0 under
AddressSanitizer and UndefinedBehaviorSanitizer (host side only), driven by a
small C++ program that makes only calls the host validation rejects before
any launch. Also checks, through the shipped -O3 library, that a successful
call clears the message of an earlier failure."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2504_05562_amd as stf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_05562_amd", "csrc")
SOURCES = ["stf.hip", "footprints.hip", "stf_forward_bicubic.hip", "stf_forward_bilinear.hip"]


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_success_clears_last_error():
    lib = stf.library()
    scr = stf.Screen(None, 16, 16)
    prm = stf.Params(1, 0, 0, 0)
    tex = (stf.Texture * 1)()
    out = (ctypes.c_void_p * 1)(4096)
    assert lib.stf_filter(tex, 1, ctypes.byref(scr), ctypes.byref(prm), out, None, None) == -1
    assert lib.stf_last_error() != b""
    good = stf.FootprintParams(9, 32, 1.4, 10000, 30, 0, 0)
    assert lib.stf_footprint_workspace_bytes(ctypes.byref(good)) > 0
    assert lib.stf_last_error() == b""


@pytest.mark.skipif(not os.path.exists(_hipcc()), reason="hipcc not available")
def test_host_validation_under_sanitizers(tmp_path):
    objs = []
    # relocatable device code: the host objects then name no per-file device
    # binary, and the device link of an empty device program is trivial
    common = [_hipcc(), "--offload-arch=gfx950", "-fgpu-rdc", "--offload-host-only", "-O0", "-g", "-std=c++17",
              "-fno-omit-frame-pointer",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for name in SOURCES:
        obj = str(tmp_path / (name + ".o"))
        subprocess.run(common + ["-c", os.path.join(CSRC, name), "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    drv = str(tmp_path / "abi_host_check.o")
    subprocess.run(common + ["-x", "c++", "-c", os.path.join(ROOT, "tests", "abi_host_check.cpp"), "-o", drv],
                   check=True, capture_output=True)
    exe = str(tmp_path / "abi_host_check")
    subprocess.run([_hipcc(), "--offload-arch=gfx950", "-fgpu-rdc", "--hip-link", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", exe, drv, *objs], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "abi host checks passed" in res.stdout
