"""The C-ABI's host-side validation and workspace-size paths under
AddressSanitizer and UndefinedBehaviorSanitizer: tk_api.cpp is rebuilt with
host-only sanitizer instrumentation (device code is built as usual), linked
with the library's other objects and a C driver (sanitize_driver.c) that
makes only calls the library answers or refuses without a device.  Any
invalid host access or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_21379_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="ROCm toolchain missing")
def test_validation_paths_under_asan_ubsan(tmp_path):
    objs = sorted(os.path.join(BUILD, f) for f in os.listdir(BUILD) if f.endswith(".hip.o")) \
        if os.path.isdir(BUILD) else []
    if not objs:
        pytest.skip("library objects not built (run the package build first)")
    api = str(tmp_path / "tk_api_san.o")
    # host side instrumented, device side untouched (each flag passed to the host compile only)
    host_san = [a for f in SAN for a in ("-Xarch_host", f)]
    _run([HIPCC, "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san +
         ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, "tk_api.cpp"), "-o", api])
    drv = str(tmp_path / "driver.o")
    _run([CLANG, "-O1", "-g", "-std=c11", "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "tests", "sanitize_driver.c"), "-o", drv] + SAN)
    exe = str(tmp_path / "driver")
    _run([CLANGXX, "-o", exe, drv, api] + objs + SAN +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lrocprofiler-sdk-roctx",
          "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    env = dict(os.environ)
    # the HIP runtime keeps process-lifetime allocations; leaks are not what is checked here
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ok" in res.stdout
