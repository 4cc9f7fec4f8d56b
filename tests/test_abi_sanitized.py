"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer run of the C ABI's argument checks (CPU only).

The library is rebuilt with the host part of every source instrumented (device code as usual), a small
C driver (tests/asan/abi_driver.c) links against it and calls every entry point with arguments the
header says are refused -- NULL plans and pointers, sizes out of range, misaligned buffers, workspaces
too small -- and checks each status; the run fails on any sanitizer report."""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_20870_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

# host-only instrumentation: each sanitizer flag applies to the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.timeout(600)
@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not available")
def test_argument_checks_under_host_sanitizers():
    from paper_2602_20870_amd.build import FLAGS
    work = tempfile.mkdtemp(prefix="fgfrft_asan_")
    try:
        srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))

        def compile_one(src):
            obj = os.path.join(work, os.path.basename(src)[:-4] + ".o")
            flags = [f for f in FLAGS if f != "-O3"] + ["-O1"]
            r = subprocess.run([HIPCC, *flags, *HOST_SAN, "-c", src, "-o", obj], capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
            return obj

        with ThreadPoolExecutor(max_workers=4) as ex:
            objs = list(ex.map(compile_one, srcs))
        lib = os.path.join(work, "libfgfrft_asan.so")
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
        assert "__asan_" in nm and "__ubsan_" in nm          # the host code is instrumented
        drv = os.path.join(work, "abi_driver")
        r = subprocess.run([CLANG, "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-o", drv,
                            os.path.join(ROOT, "tests", "asan", "abi_driver.c"), "-L", work, "-lfgfrft_asan",
                            "-Wl,-rpath," + work], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=120)
        report = r.stdout + r.stderr
        assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
        assert r.returncode == 0 and "all checks passed" in r.stdout, report[-4000:]
    finally:
        shutil.rmtree(work, ignore_errors=True)
