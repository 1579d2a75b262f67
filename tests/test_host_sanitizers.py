"""Host code under AddressSanitizer (with LeakSanitizer) and
UndefinedBehaviorSanitizer, on the CPU:

* the FP64 C oracle (oracle/oracle.c) with tests/sanitize/oracle_driver.c,
  every entry point on small matrices in exactly sized heap buffers (gcc);
* libsvdp's host code (argument checks, workspace carving of every op over
  edge shapes, the schedule tables, status strings) with
  tests/sanitize/lib_driver.cpp: the library sources are compiled with the
  sanitizers on the host side only, the driver reaches no launch, so no GPU
  is needed (hipcc; about a minute).

Both builds go to a temporary directory; a sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
HIPCC = "/opt/rocm/bin/hipcc"
SOURCES = ("api", "kernels", "eigh", "gemm", "prof")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_address_and_undefined_behavior_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
          "-O1", "-std=c99", os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert r.stdout.strip() == "ok"
    assert "Sanitizer" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_library_host_code_under_address_and_undefined_behavior_sanitizers(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    common = ["-fno-omit-frame-pointer", "-g", "-O1", "-std=c++17", "-fPIC",
              "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2609_32505_amd", "csrc")]
    procs, objs = [], []
    for name in SOURCES:
        obj = str(tmp_path / f"{name}.o")
        objs.append(obj)
        cmd = [HIPCC, "--offload-arch=gfx950"] + san + common + [
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-c", os.path.join(ROOT, "paper_2609_32505_amd", "csrc", name + ".hip"), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    for cmd, p in procs:
        out, err = p.communicate(timeout=900)
        assert p.returncode == 0, f"{' '.join(cmd)}\n{err[-3000:]}"
    drv = str(tmp_path / "lib_driver.o")
    _run([HIPCC, "--cuda-host-only"] + san + common +
         ["-c", os.path.join(ROOT, "tests", "sanitize", "lib_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "lib_san")
    _run([HIPCC] + san + [drv] + objs + ["-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert r.stdout.strip().endswith("ok")
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr
