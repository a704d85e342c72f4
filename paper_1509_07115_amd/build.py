"""Build the HIP library ``libdsbt.so`` in-tree for gfx950.

    python -m paper_1509_07115_amd.build      (or  python paper_1509_07115_amd/build.py)

Every HIP translation unit is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``) and with matrix-core
accumulators kept in VGPRs (``-mllvm -amdgpu-mfma-vgpr-form``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdsbt.so")
SOURCES = ["kernels.hip", "fstage.hip", "mstage_mfma.hip", "mstage_chain.hip", "plan_device.hip", "state.hip",
           "monomial.hip", "angular.hip", "capi.cpp", "autotune.cpp", "angular_capi.cpp", "plan_host.cpp",
           "monomial_host.cpp", "angular_host.cpp"]
ARCH = os.environ.get("DSBT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    # -amdgpu-mfma-vgpr-form: matrix-instruction accumulators in ordinary VGPRs
    # (no v_accvgpr_read per result register)
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form",
             "-I", os.path.join(HERE, "..", "include"), "-Wall", "-Wno-unused-result"]
    tmp = tempfile.mkdtemp(prefix="dsbt_build_")
    try:
        def compile_one(src: str) -> str:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] if src.endswith((".hip", "capi.cpp", "autotune.cpp")) else []
            cmd = [cc, *flags, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            return obj

        # translation units are independent: compile them side by side
        jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            objs = list(pool.map(compile_one, SOURCES))
        out_tmp = LIB + ".tmp"
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", out_tmp, "-lpthread",
               "-L", os.path.join(rocm, "lib"), "-lrocprofiler-sdk-roctx"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
