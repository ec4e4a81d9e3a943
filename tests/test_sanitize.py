"""Sanitizer builds on the CPU (no device needed).

- The oracle (plain C) built with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer and driven over small random multigraphs
  through every entry point (tests/sanitize/oracle_driver.c).
- The library's host code built with AddressSanitizer and
  UndefinedBehaviorSanitizer (hipcc, host side only; the gfx950 device code
  is built as usual) and driven through every C-ABI path that runs without a
  device: argument checks, error strings, option defaults, and the server's
  creation and destruction when no device is usable
  (tests/sanitize/host_driver.cpp). Leaks reported inside the HIP runtime
  are suppressed; leaks in the library are not.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, "%s\nstdout:\n%s\nstderr:\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-6000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-pthread", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "oracle", "chl_oracle.c"), os.path.join(SAN, "oracle_driver.c"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe, "300"], env=env)
    assert "graphs ok" in r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_host_code_asan_ubsan(tmp_path):
    import importlib
    b = importlib.import_module("paper_1907_00140_amd.build")
    san = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = [f for f in b.FLAGS if f != "-O3"] + ["-O1"]

    def comp(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(["hipcc", "-x", "hip", *flags, *san, "-c", src, "-o", obj])
        return obj

    srcs = [os.path.join(b.CSRC, s) for s in b.SOURCES] + [os.path.join(SAN, "host_driver.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, srcs))
    exe = str(tmp_path / "host_driver")
    _run(["hipcc", "--offload-arch=gfx950", *san, *objs, "-o", exe, "-lpthread"])
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:librocprofiler\n"
                    "leak:libdrm\nleak:libnuma\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", LSAN_OPTIONS="suppressions=%s" % supp,
               UBSAN_OPTIONS="print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = _run([exe], env=env)
    assert "host driver: ok" in r.stdout
