"""Builds the gfx950 HIP library (``libmd_gfx950.so``) next to this file.

Every HIP source is compiled with ``-Xclang -target-feature -Xclang -packed-fp32-ops``
(packed FP32 instructions disabled) and linked into one shared library that exports
the C ABI declared in ``include/md.h``.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["md_api.hip", "md_kernels.hip", "md_lj.hip", "md_obs.hip"]
HEADERS = ["md_internal.h"]
LIB = os.path.join(HERE, "libmd_gfx950.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _obj(src: str) -> str:
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def build(force: bool = False, verbose: bool = False) -> str:
    """Compile each source to an object (parallel), then link the shared library."""
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    deps = [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "md.h")]
    dep_time = max(os.path.getmtime(d) for d in deps)
    procs = []
    for src in SOURCES:
        s = os.path.join(CSRC, src)
        o = _obj(src)
        stale = force or not os.path.exists(o) or os.path.getmtime(o) < max(dep_time, os.path.getmtime(s))
        if stale:
            cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", s, "-o", o]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the GPU-only feature flag; that warning is harmless
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr)
        elif verbose and text.strip():
            print(text)
    if failed:
        raise RuntimeError("HIP compilation failed: " + ", ".join(failed))
    objs = [_obj(s) for s in SOURCES]
    if force or procs or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose=True))
