"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only; the device code is built as usual): a driver program runs cluster
selection on the nocc = 400 lattice and every argument check of the C ABI that
returns before device work, and must finish without a sanitizer report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2106_06149_amd import build as B, synth

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    from concurrent.futures import ThreadPoolExecutor

    def compile_one(src):
        host_code = src in ("osv_api.hip", "devpool.hip")
        obj = str(tmp_path / src.replace(".hip", ".o"))
        cmd = [HIPCC] + B.FLAGS + (SAN if host_code else []) + ["-g", "-c", os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    # the driver is plain host C++ (g++), the link goes through hipcc for the device code
    drv = str(tmp_path / "driver.o")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-I" + os.path.join(B.ROOT, "include"), "-I/opt/rocm/include",
           "-D__HIP_PLATFORM_AMD__", "-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer",
           "-c", os.path.join(HERE, "asan_driver.cpp"), "-o", drv]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_driver")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + SAN[:4] + [drv] + objs + ["-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    cen, _ = synth.workload(4, geometry_only=True)
    cf = tmp_path / "centroids.bin"
    with open(cf, "wb") as fh:
        fh.write(np.int32(cen.shape[0]).tobytes())
        fh.write(np.ascontiguousarray(cen, dtype=np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(cf), "400", "56012", "113438"], capture_output=True, text=True,
                       timeout=600, env=env)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "ok" in r.stdout, out[-4000:]
