"""Builds the device library ``libsphbi.so`` for gfx950 with hipcc.

The library is built in-tree (next to this file) so that it travels with the
source tree.  Every HIP translation unit is compiled with packed FP32
instructions disabled.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsphbi.so")
SOURCES = ["capi.hip", "forward.hip", "adjoint.hip", "adjoint_linear.hip", "operators.hip", "quadrature.hip", "mlp.hip", "serve.hip", "noalloc.hip", "refine.hip", "probe.hip"]
ARCH = os.environ.get("SPHBI_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd[-3:]) + "\n" + res.stderr[-4000:])
    return res.stderr


def build(verbose: bool = False) -> str:
    """Compile the HIP sources into ``libsphbi.so`` (always recompiles).

    The translation units are compiled to objects in parallel, then linked.
    """
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="sphbi_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in srcs]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            logs = list(ex.map(lambda so: _run(["hipcc"] + FLAGS + ["-c", so[0], "-o", so[1]]), zip(srcs, objs)))
        tmp = LIB + ".tmp"
        logs.append(_run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs))
    if verbose:
        for log in logs:
            if log:
                print(log)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
