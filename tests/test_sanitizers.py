"""AddressSanitizer and UndefinedBehaviorSanitizer builds of host code (CPU).

The C oracle (definition.c, closed_form.c) and the library's host code (the
C-ABI's presets, option and argument checks, workspace sizes, kernel
descriptions) are compiled with -fsanitize=address,undefined and driven by
small C programs (tests/native/*_san_main.c) over valid, degenerate and
invalid inputs.  The library is built as usual with the sanitizers on its
host side only (the drivers take only paths that return before any launch;
GPU code is never built with a sanitizer here).  Any sanitizer report fails
the test.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2507_21686_amd", "csrc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_oracle_under_asan_ubsan():
    tmp = tempfile.mkdtemp(prefix="san_oracle_")
    exe = os.path.join(tmp, "oracle_san")
    srcs = [os.path.join(ROOT, "oracle", "definition.c"), os.path.join(ROOT, "oracle", "closed_form.c"),
            os.path.join(NATIVE, "oracle_san_main.c")]
    r = _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined", "-o", exe] + srcs + ["-lm"])
    assert r.returncode == 0, r.stderr
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_library_host_code_under_asan_ubsan():
    from concurrent.futures import ThreadPoolExecutor
    tmp = tempfile.mkdtemp(prefix="san_capi_")
    names = ("capi", "forward", "adjoint", "adjoint_linear", "operators", "quadrature", "mlp", "serve", "noalloc",
             "refine", "probe")

    def compile_one(name):
        obj = os.path.join(tmp, name + ".o")
        r = _run(["hipcc", "-O3", "-Xarch_host", "-g", "-std=c++17", "--offload-arch=gfx950", "-fno-omit-frame-pointer",
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Wno-unused-command-line-argument", "-c", os.path.join(CSRC, name + ".hip"), "-o", obj])
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, names))
    drv = os.path.join(tmp, "drv.o")
    r = _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-c",
              os.path.join(NATIVE, "capi_san_main.c"), "-o", drv])
    assert r.returncode == 0, r.stderr
    exe = os.path.join(tmp, "capi_san")
    r = _run(["hipcc", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", "-o", exe, drv] + objs)
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    shutil.rmtree(tmp, ignore_errors=True)
