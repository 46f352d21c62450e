"""The host side of the C-ABI under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library is rebuilt with the sanitizers on its host code only (device code is compiled as
usual) and linked into a small C driver (tests/host/abi_host_driver.c) that calls every entry point
on the paths that return before any device work: argument and descriptor validation, the Gauss
rule, the workspace query. Any sanitizer report fails the run.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1707_05882_amd", "csrc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.slow
def test_host_abi_under_address_and_undefined_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    base = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    procs = []
    for f in srcs:
        obj = str(tmp_path / (f[:-4] + ".o"))
        procs.append((subprocess.Popen(base + SAN_HOST + ["-c", os.path.join(CSRC, f), "-o", obj],
                                       stdout=subprocess.PIPE, stderr=subprocess.PIPE), obj))
    objs = []
    for p, obj in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-2000:]
        objs.append(obj)
    lib = str(tmp_path / "libvbrdf_san.so")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN_HOST + ["-o", lib] + objs,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "driver")
    r = subprocess.run([clang, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(HERE, "host", "abi_host_driver.c"), lib, "-o", exe,
                        f"-Wl,-rpath,{tmp_path}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
