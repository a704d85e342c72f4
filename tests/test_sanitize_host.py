"""AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host
code (FP64 plan generator, C ABI argument checks, host tables), run on the CPU.

Every translation unit is compiled as for the product library, with the
sanitizers on the host side only (``-Xarch_host``; GPU code is built as usual
and never launched), and linked with tests/host_sanitize_driver.cpp, which
calls the host-side entry points and exits non-zero on an unexpected status.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1509_07115_amd", "csrc")


@pytest.mark.slow
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    from paper_1509_07115_amd import build
    try:
        cc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={build.ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([cc, *flags, *san, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj], check=True,
                       stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        return obj

    jobs = max(1, min(len(build.SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(compile_one, build.SOURCES))
    drv = str(tmp_path / "driver.o")
    subprocess.run(["g++", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
                    "-o", drv], check=True)
    exe = str(tmp_path / "driver")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run([cc, f"--offload-arch={build.ARCH}", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", drv, *objs, "-o", exe, "-lpthread", "-L", os.path.join(rocm, "lib"),
                    "-lrocprofiler-sdk-roctx"], check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    env = dict(os.environ)
    # leaks are not checked: the HIP runtime keeps its own allocations when no device is found
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env["HIP_VISIBLE_DEVICES"] = ""   # host paths only, also on a machine with a GPU
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.returncode == 0, r.returncode
    assert "0 failures" in r.stdout
