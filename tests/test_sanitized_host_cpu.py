"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The serving pool (fo_pool.cpp) and its fibers (fo_fiber.cpp), built with
  g++ against a recording stand-in for the HIP runtime and the context calls
  (tests/pool_host): results alone and in the mix, budget admission, reuse,
  eviction, teardown with requests running, calls from a foreign thread.  The
  stand-in checks that every stream, device buffer and context is released
  exactly once, on the thread that made it, and never used after release.
* The FP64 oracle (oracle/fo_oracle.c), built with gcc, through every entry
  point on small 2D and 3D meshes (tests/oracle_host).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    return r.returncode, r.stdout + r.stderr


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip("%s not available" % tool)


def test_pool_host_logic_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "pool_host")
    src = os.path.join(ROOT, "tests", "pool_host")
    csrc = os.path.join(ROOT, "paper_2601_05709_amd", "csrc")
    rc, out = _run(["g++", "-std=c++17"] + SAN + ["-I" + src, "-I" + csrc, "-pthread",
                                                  os.path.join(src, "driver.cpp"), os.path.join(src, "stub.cpp"),
                                                  os.path.join(csrc, "fo_pool.cpp"), os.path.join(csrc, "fo_fiber.cpp"),
                                                  "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    print(out)
    assert rc == 0, out
    assert "0 errors, 0 leaks" in out and "0 failed checks" in out


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_host")
    rc, out = _run(["gcc", "-std=c11", "-fopenmp"] + SAN + [os.path.join(ROOT, "tests", "oracle_host", "driver.c"),
                                                           os.path.join(ROOT, "oracle", "fo_oracle.c"), "-lm",
                                                           "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe])
    print(out)
    assert rc == 0, out
    assert "0 failed checks" in out
