"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): every source is compiled with the sanitizers on its host pass
only (device code as usual), linked with tests/sanitize/host_checks.c, and
run; the driver calls the host-only entry points (planners, DG tables,
validation) and any memory or undefined-behaviour error aborts it.  Built
under _build/host_sanitize/, again only when a source changed."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_08684_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_checks.c")
OUT = os.path.join(ROOT, "_build", "host_sanitize")
SOURCES = ["mg_runtime.hip", "mg_kernels.hip", "mg_server.hip", "mg_dg.hip"]

HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _tool(name, fallback):
    return shutil.which(name) or (fallback if os.path.exists(fallback) else None)


def _newer(target, deps):
    return not os.path.exists(target) or any(os.path.getmtime(d) > os.path.getmtime(target) for d in deps)


@pytest.mark.slow
def test_host_code_is_clean_under_address_and_ub_sanitizers():
    hipcc = _tool("hipcc", "/opt/rocm/bin/hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    if not hipcc or not os.path.exists(clang):
        pytest.skip("hipcc / ROCm clang not available")
    os.makedirs(OUT, exist_ok=True)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + \
        [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]

    def compile_one(src):
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        path = os.path.join(CSRC, src)
        if _newer(obj, [path] + headers):
            cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
                   f"-I{INCLUDE}", f"-I{CSRC}", "-c", path, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv_obj = os.path.join(OUT, "host_checks.o")
    if _newer(drv_obj, [DRIVER] + headers):
        r = subprocess.run([clang, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-x", "c",
                            DRIVER, f"-I{INCLUDE}", "-c", "-o", drv_obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    exe = os.path.join(OUT, "host_checks")
    if _newer(exe, objs + [drv_obj]):
        r = subprocess.run([hipcc, "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                            *objs, drv_obj, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host checks passed" in r.stdout
