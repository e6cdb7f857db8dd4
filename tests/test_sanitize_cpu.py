"""CPU-only builds under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (oracle/rid_oracle.c) with a driver that runs every function on
  small inputs and its edge cases (k = n = l, k = l = 1, exact rank k, rank
  failure, forced pivots, argument errors, a zero matrix).
* The library's host code (every csrc/*.hip, device code built as usual,
  host code instrumented) with a driver that calls every C entry point with
  a null handle and invalid sizes, pointers and leading dimensions: each must
  return its argument error before touching a device, with no undefined
  arithmetic on the way (sizes near 2^62 included).
No GPU is used: no call reaches the device.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1",
               OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          os.path.join(ROOT, "oracle", "rid_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
          "-o", exe, "-lquadmath", "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "all checks passed" in r.stdout


def test_host_argument_checks_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    from concurrent.futures import ThreadPoolExecutor

    from paper_1205_3830_amd import build as b
    csrc = os.path.join(ROOT, "paper_1205_3830_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", inc,
              "-I", csrc, "-pthread"] + san + ["-c", os.path.join(csrc, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, b.SOURCES))
    drv = str(tmp_path / "abi_driver.o")
    clang = "/opt/rocm/lib/llvm/bin/clang"
    _run([clang, "-g", "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__",
          "-I", "/opt/rocm/include", "-I", inc, "-c", os.path.join(HERE, "abi_driver.c"),
          "-o", drv])
    exe = str(tmp_path / "abi_san")
    _run([HIPCC, "--offload-arch=gfx950", "-g"] + san[:4] + ["-pthread", drv] + objs +
         ["-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=120)
    assert "all checks passed" in r.stdout
