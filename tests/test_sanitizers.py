"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer: the oracle
run by a C driver over small random inputs, and the C ABI's host-side
argument checks (the library's host code built with the sanitizers; every
call fails its checks before any device work, so no GPU is needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _have_sanitizers():
    return shutil.which("gcc") is not None


@pytest.mark.skipif(not _have_sanitizers(), reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    subprocess.check_call(["gcc"] + SAN + ["-ffp-contract=off", "-fopenmp", "-o", str(exe),
                                           os.path.join(ROOT, "tests", "sanitize_oracle_driver.c"),
                                           os.path.join(ROOT, "oracle", "selscan_oracle.c"), "-lm"])
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "sanitized oracle runs" in r.stdout


HIP_SOURCES = ["ss_walk.hip", "ss_walk_mask.hip", "ss_walk_wide.hip", "ss_walk_batch.hip", "ss_sites.hip",
               "ss_genome.hip", "ss_micro.hip", "ss_capi.hip"]


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_c_abi_host_checks_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The library with its host code instrumented (device code as usual),
    driven through argument checks and workspace sizing only."""
    from concurrent.futures import ThreadPoolExecutor
    hip = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    csrc = os.path.join(ROOT, "paper_1403_6854_amd", "csrc")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]

    def obj(src):
        o = str(tmp_path / (src + ".o"))
        subprocess.check_call([hip, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
                               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                               "-packed-fp32-ops"] + host_san +
                              ["-I", os.path.join(ROOT, "include"), "-I", csrc, "-c",
                               os.path.join(csrc, src), "-o", o],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        return o

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(obj, HIP_SOURCES))
    lib = str(tmp_path / "libselscan_san.so")
    subprocess.check_call([hip, "--offload-arch=gfx950", "-shared", "-fPIC"] + host_san + objs + ["-o", lib],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    clang = "/opt/rocm/llvm/bin/clang"
    drv = str(tmp_path / "capi_san")
    subprocess.check_call([clang, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g",
                           "-O1", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "sanitize_capi_driver.c"), lib,
                           "-Wl,-rpath," + str(tmp_path), "-o", drv])
    r = subprocess.run([drv], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "sanitized host checks passed" in r.stdout
