"""AddressSanitizer and UndefinedBehaviorSanitizer builds, CPU only.

The C oracle is compiled with gcc under both sanitizers (serial and OpenMP)
and driven through every entry point on 4^3 and 5^3 lattices; the library's
host code (every source, the device code compiled as usual but never run) is
compiled with hipcc, the sanitizers applied to the host side only, and driven
through its validation, layout and argument-check paths, none of which reaches
the HIP runtime.  Variants with a planted mistake show that each sanitizer is
live in these builds."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2006_15122_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

GCC_SAN = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-fast-math", "-ffp-contract=off"]
# sanitizers on the host side of each hipcc compile only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=300, **kw)


def _gcc_driver(tmp_path, name, extra):
    exe = str(tmp_path / name)
    r = _run(["gcc", *GCC_SAN, *extra, os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("omp", [False, True], ids=["serial", "openmp"])
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path, omp):
    exe = _gcc_driver(tmp_path, "oracle_san", ["-fopenmp"] if omp else [])
    r = _run([exe])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle driver ok" in r.stdout


@pytest.mark.parametrize("plant, report", [
    (1, "heap-buffer-overflow"),
    (2, "detected memory leaks"),
    (3, "signed integer overflow"),
], ids=["overflow", "leak", "ub"])
def test_oracle_build_reports_a_planted_mistake(tmp_path, plant, report):
    exe = _gcc_driver(tmp_path, f"oracle_plant{plant}", [f"-DPLANT={plant}"])
    r = _run([exe])
    assert r.returncode != 0
    assert report in r.stderr, r.stderr[-4000:]
    if plant == 1:
        # the report names the oracle function that read past the short array
        assert "orc_scalar_kernel" in r.stderr


@pytest.fixture(scope="module")
def host_objects(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    from paper_2006_15122_amd import build_lib

    out = tmp_path_factory.mktemp("host_san")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-Wno-unused-value", *HOST_SAN]

    def compile_one(src):
        obj = str(out / (src + ".o"))
        r = _run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, build_lib.SOURCES))
    return out, objs


def _host_driver(host_objects, plant=0):
    out, objs = host_objects
    drv = str(out / f"host_driver{plant}.o")
    clangxx = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang++")
    clangxx = clangxx if os.path.exists(clangxx) else shutil.which("clang++")
    r = _run([clangxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", f"-DPLANT={plant}", "-I", os.path.join(ROOT, "include"), "-c",
              os.path.join(SAN, "host_driver.cpp"), "-o", drv])
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(out / f"host_san{plant}")
    r = _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN[:4], *objs, drv, "-o", exe, "-lpthread"])
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def test_library_host_code_is_clean_under_asan_and_ubsan(host_objects):
    r = _run([_host_driver(host_objects)])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host driver ok" in r.stdout


def test_library_host_build_reports_a_planted_overflow(host_objects):
    r = _run([_host_driver(host_objects, plant=1)])
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-4000:]
