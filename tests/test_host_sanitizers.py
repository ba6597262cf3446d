"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

The HIP sources are compiled for the host only (no device code), with the sanitizers on the host
pass, and linked with tests/host_sanitize/plan_driver.cpp: every workspace query (dry runs of the solve,
setup, batch, ladder and eigensolver paths), option validation, and the batch planner from four host
threads at once.  Any heap or stack error or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_05897_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2511_05897_amd.build import SOURCES
    # device code compiled as usual (the objects must carry their code objects to link), the
    # sanitizers on the host pass only
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run(["hipcc"] + flags + ["-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, (src, r.stderr[-3000:])
        return obj

    import concurrent.futures
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv_obj = str(tmp_path / "plan_driver.o")
    r = subprocess.run(["hipcc"] + flags[1:] + ["--offload-host-only", "-x", "hip", "-c",
                                                  os.path.join(ROOT, "tests", "host_sanitize",
                                                                          "plan_driver.cpp"), "-o", drv_obj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # link as plain host C++ with the sanitizer runtimes and the HIP runtime library
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cxx = os.path.join(rocm, "lib", "llvm", "bin", "clang++")
    drv = str(tmp_path / "plan_driver")
    r = subprocess.run([cxx, "-fsanitize=address,undefined", drv_obj] + objs +
                       ["-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib"),
                        "-o", drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-5000:])
    assert "plan driver: 0 problems" in r.stdout
