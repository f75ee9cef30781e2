"""The library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host side only; the kernels are the regular
build's objects) and driven through every query and validation path of the
C ABI by tests/sanitize/abi_checks.cpp.  Nothing reaches the device, so this
runs on the CPU."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_00626_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2109_00626_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def test_host_code_under_asan_ubsan(tmp_path):
    kernels = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or not kernels:
        pytest.skip("needs hipcc, clang++ and the regular build's kernel objects")
    hosts = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))

    def compile_host(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"] + SAN + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(min(8, len(hosts))) as ex:
        objs = list(ex.map(compile_host, hosts))
    drv = str(tmp_path / "abi_checks.o")
    r = subprocess.run([CLANG, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-c",
                        os.path.join(ROOT, "tests", "sanitize", "abi_checks.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "abi_checks")
    r = subprocess.run([CLANG, "-fsanitize=address,undefined", drv] + objs + kernels +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ok: 0 failure(s)" in r.stdout
    shutil.rmtree(tmp_path, ignore_errors=True)
