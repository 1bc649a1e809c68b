"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The host C++ sources (argument validation, geometry checks, the Mueller screens with the Eq. 6
regularisation, the anti-aliasing function, the network and GEMM entry points' checks) are built
with g++ -fsanitize=address,undefined; the HIP sources are built as usual (their device code is
not instrumented) and everything is linked with tests/host_sanitize_driver.cpp.  The driver
registers an allocator that always fails, so every creating call does all its host work and stops
at its first device allocation; no GPU is needed.  Any sanitizer report aborts the driver; leak
checking is on.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2206_15117_amd", "csrc")
HOST_SOURCES = ["api.cpp", "mlp_api.cpp", "pswf.cpp", "mueller.cpp"]
HIP_SOURCES = ["kernels_gen.hip", "plan.hip", "grid.hip", "mlp.hip", "clean.hip", "mosaic.hip"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("g++ or the HIP runtime is not installed")
    from concurrent.futures import ThreadPoolExecutor

    from paper_2206_15117_amd import build

    out = tmp_path_factory.mktemp("sanitize")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include")]
    host = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-D__HIP_PLATFORM_AMD__"] + SAN + inc

    def host_obj(src, path):
        obj = str(out / (os.path.basename(src) + ".o"))
        _run(host + ["-c", os.path.join(path, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        hip = [ex.submit(build._compile, s, str(out)) for s in HIP_SOURCES]
        objs = [ex.submit(host_obj, s, CSRC) for s in HOST_SOURCES]
        objs.append(ex.submit(host_obj, "host_sanitize_driver.cpp", HERE))
        objs = [f.result() for f in objs] + [f.result() for f in hip]
    exe = str(out / "host_sanitize_driver")
    _run(["g++"] + SAN + ["-pthread", "-o", exe] + objs +
         ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    return exe


def test_host_code_is_clean_under_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    report = res.stdout + res.stderr
    assert res.returncode == 0, report
    assert "runtime error" not in report and "AddressSanitizer" not in report and "LeakSanitizer" not in report
    assert "0 failures" in res.stdout
    calls = int(res.stdout.split("driver: ")[1].split(" calls")[0])
    assert calls >= 150
