"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU oracle
and of the library's host code, run on the CPU.

* The oracle (oracle/*.c) with a driver that takes small steps in each of its
  modes (tests/sanitize/oracle_driver.c), built by gcc with
  -fsanitize=address,undefined.
* The library's host translation unit (every entry point's argument checks,
  validation, creation and error reporting) with host-only instrumentation
  (-Xarch_host before each -fsanitize=: the GPU code is built as usual),
  linked with the library's other objects from the last build, and a driver
  that calls every host path that needs no GPU (tests/sanitize/abi_driver.c).

Any out-of-bounds access, use after free, leak or undefined operation on
these paths ends the driver with a sanitizer report and a non-zero status.
"""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
CSRC = os.path.join(ROOT, "paper_1208_2643_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1208_2643_amd", "_build")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r.stdout


@pytest.mark.timeout(300)
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off", "-std=c99",
         os.path.join(ROOT, "oracle", "mpfc_oracle.c"),
         os.path.join(ROOT, "oracle", "mpfc3d_oracle.c"),
         os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    assert "oracle driver ok" in run([exe], env=env)


@pytest.mark.timeout(600)
def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    objs = sorted(glob.glob(os.path.join(BUILD, "launch_*.o")))
    if shutil.which("hipcc") is None or not objs:
        pytest.skip("hipcc or the library's objects (build first) not found")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", *HOST_SAN, "-Xarch_host", "-fno-sanitize-recover=all",
             "-I", os.path.join(ROOT, "include")]
    host = str(tmp_path / "mpfc_san.o")
    drv = str(tmp_path / "abi_driver.o")
    exe = str(tmp_path / "abi_san")
    run(["hipcc", *flags, "-std=c++17", "-c", os.path.join(CSRC, "mpfc.hip"), "-o", host])
    run(["hipcc", "--offload-host-only", *flags, "-x", "c", "-c",
         os.path.join(SAN, "abi_driver.c"), "-o", drv])
    run(["hipcc", "--offload-arch=gfx950", *HOST_SAN, drv, host, *objs, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    assert "abi driver ok" in run([exe], env=env, timeout=120)
