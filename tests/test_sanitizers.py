"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only; GPU code is never
built with a sanitizer):
  * the CPU oracle, every entry point, on a small s/p/d system (gcc);
  * the library's host code (context creation, argument and option validation, the basis
    screening radius, status strings) built with the host half of hipcc under the sanitizers
    and linked with the ordinary kernel objects.  Validation of P (SNK_VALIDATE) needs a
    context, which needs a GPU: it is covered by the GPU tests instead.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2303_14280_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2303_14280_amd", "_build")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=gnu11", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fopenmp", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "snk_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"), timeout=300)
    assert "oracle driver ok" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2303_14280_amd import build as B
    hipcc = B.hipcc()
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang not found")
    kernels = [os.path.join(BUILD, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        B.build()
    # host half only: each -fsanitize flag applies to the host compilation of the sources
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + san
    objs = []
    for src in ("snk_host.cpp", "snk_mlp.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run([hipcc] + flags + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "host_driver.o")
    _run([clang, "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "host_driver.c"), "-o", drv])
    exe = str(tmp_path / "host_driver")
    _run([clang + "++", "-fsanitize=address,undefined", drv] + objs + kernels +
         ["-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "host driver ok" in r.stdout
