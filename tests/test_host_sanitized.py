"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The join server's admission core (csrc/server_core.h) on a simulated device
  with a virtual clock (tests/host/server_core_test.cpp, g++).
* The library's host sources (engine, cost model, C API, batch, server,
  external join) compiled with the sanitizers on their host side, linked with
  the kernels from the last build, and driven through every host-side entry
  point of hj.h and the argument checks of the device-side ones
  (tests/host/api_host_test.c).
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
CSRC = os.path.join(ROOT, "paper_1307_1955_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1307_1955_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:exitcode=23",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


def test_server_core_virtual_clock(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ is not installed")
    exe = str(tmp_path / "server_core_test")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=undefined", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, os.path.join(HOST, "server_core_test.cpp"), "-o", exe])
    r = _run([exe], env={**os.environ, **SAN_ENV}, timeout=300)
    assert "all checks passed" in r.stdout


HOST_SOURCES = ["engine.cpp", "costmodel.cpp", "hj_api.cpp", "batch.cpp", "server.cpp", "external.cpp"]
KERNEL_OBJECTS = ["scan.o", "shj.o", "phj_partition.o", "phj_join.o", "noalloc.o"]


def test_host_api_sanitized(tmp_path):
    for tool in (HIPCC, CLANG, CLANGXX):
        if not os.path.exists(tool):
            pytest.skip("%s is not installed" % tool)
    kobjs = [os.path.join(BUILD, o) for o in KERNEL_OBJECTS]
    if not all(os.path.exists(o) for o in kobjs):
        pytest.skip("kernel objects not built (run __graft_entry__.build() first)")
    # the sanitizers apply to the host side only (-Xarch_host before each)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    common = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-I", os.path.join(ROOT, "include")]

    def compile_one(src_obj):
        src, obj = src_obj
        _run([HIPCC, *common, *san, "-c", src, "-o", obj])

    jobs = [(os.path.join(CSRC, s), str(tmp_path / (os.path.splitext(s)[0] + ".o"))) for s in HOST_SOURCES]
    jobs.append((os.path.join(HOST, "api_host_devices.cpp"), str(tmp_path / "devices.o")))
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(compile_one, jobs))
    drv = str(tmp_path / "driver.o")
    _run([CLANG, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=undefined", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
          "-c", os.path.join(HOST, "api_host_test.c"), "-o", drv])
    exe = str(tmp_path / "api_host_test")
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv, *[o for _, o in jobs], *kobjs,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lpthread"])
    r = _run([exe], env={**os.environ, **SAN_ENV}, timeout=300)
    assert "all checks passed" in r.stdout
