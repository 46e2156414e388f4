"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

- The oracle (oracle/ht_oracle.c), built with gcc and both sanitizers, driven over small, ragged,
  wide-row and sector grids and degenerate hits by tests/sanitize/oracle_driver.c.
- The host side of libht.so: every translation unit is compiled as for the product library, with
  the sanitizers on the host pass only (the device code is unchanged), and linked with
  tests/sanitize/abi_driver.c, which calls the table, tiling, tuning and batch-plan queries and
  every entry point with invalid arguments. None of these calls touches a GPU.

Any sanitizer report aborts the driver (-fno-sanitize-recover=all), and the test fails on a
non-zero exit status.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1507_03074_amd import build as hbuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")

pytestmark = pytest.mark.slow

# sanitizers on the host pass of hipcc only: each -fsanitize flag follows -Xarch_host
HOST_SANITIZE = ["-Xarch_host", "-g",
                 "-Xarch_host", "-fsanitize=address",
                 "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all"]
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\nexit %d\n%s\n%s" % (" ".join(cmd), r.returncode, r.stdout[-4000:],
                                                        r.stderr[-4000:])
    return r


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(SAN, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "ht_oracle.c"), "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "oracle driver: clean" in r.stdout


@pytest.mark.skipif(not os.path.exists(hbuild.hipcc()) and shutil.which("hipcc") is None,
                    reason="needs hipcc")
def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    hipcc = hbuild.hipcc()
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"

    def compile_one(i):
        src, defs = hbuild.UNITS[i]
        obj = str(tmp_path / ("%02d.o" % i))
        _run([hipcc, *hbuild.HIPCC_FLAGS, *HOST_SANITIZE, *defs, "-I", hbuild.INCLUDE, "-I",
              hbuild.CSRC, "-c", os.path.join(hbuild.CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(min(8, len(hbuild.UNITS))) as pool:
        objs = list(pool.map(compile_one, range(len(hbuild.UNITS))))
    drv = str(tmp_path / "abi_driver.o")
    _run([clang, "-x", "c", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", hbuild.INCLUDE, "-c", os.path.join(SAN, "abi_driver.c"), "-o", drv])
    exe = str(tmp_path / "abi_driver")
    _run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-o", exe, drv, *objs])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "abi driver: clean" in r.stdout
