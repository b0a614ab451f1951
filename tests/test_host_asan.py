"""The library's host code under AddressSanitizer (no GPU).

The library is built a second time with the host part instrumented
(-fsanitize=address on the host compilation only; the device code is the
usual gfx950 build), and a small C program (host_asan_driver.c) calls the
entry points whose argument checks, config validation and workspace sizing
run on the host: valid and invalid 1D, 2D and batch configurations, null
handles and outputs.  Memory errors abort the program; every call must
return the expected status with a message."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers missing")
def test_host_code_is_clean_under_address_sanitizer(tmp_path):
    lib = tmp_path / "libpic_asan.so"
    inc = os.path.join(ROOT, "include")
    build = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
             "-I", inc, os.path.join(ROOT, "paper_1008_1685_amd", "csrc", "pic_lib.hip"), "-o", str(lib)]
    r = subprocess.run(build, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    drv = tmp_path / "host_asan_driver"
    # with its device section compiled in (run with --gpu on a machine with a GPU)
    link = [CLANG, "-Wall", "-Werror", "-DWITH_GPU", "-D__HIP_PLATFORM_AMD__", "-fsanitize=address",
            "-fno-omit-frame-pointer", "-I", inc, "-I", "/opt/rocm/include",
            os.path.join(ROOT, "tests", "host_asan_driver.c"), "-L", str(tmp_path), "-lpic_asan",
            "-L", "/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib",
            "-o", str(drv)]
    r = subprocess.run(link, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    # leak checking is off: the HIP runtime's own start-up allocations are not ours
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = subprocess.run([str(drv)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-3000:])
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "all host checks ran: 0 failed" in r.stdout
