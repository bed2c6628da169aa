"""Build libnurbsdiff.so in-tree with hipcc for gfx950.

Each ``csrc/*.hip`` translation unit (one per degree in u for the uniform
kernels, one per kind and degree class for the persistent kernels, the host
ABI) is compiled in parallel and linked into one shared library.  The
per-request serving binding ``csrc/serve_py.c`` (CPython C API, host code
only) is compiled with the host C compiler into ``_serve_py``.

Packed-FP32 instructions are disabled (``-packed-fp32-ops``): the per-point
arithmetic is plain scalar FP32 FMA.  No fast-math.  The per-point rational
divide multiplies by the hardware reciprocal ``v_rcp_f32`` (1 ulp, far inside
the 1e-5 point tolerance); the divides of the basis recursion and of its knot
derivative take one Newton step on that reciprocal.  Both are written out in
the source.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import sysconfig

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnurbsdiff.so")
OBJ = os.path.join(ROOT, "_build", "obj")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CC = os.environ.get("CC", "gcc")
PYEXT = os.path.join(HERE, "_serve_py" + sysconfig.get_config_var("EXT_SUFFIX"))
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def units():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".hpp", ".inc", ".h", ".c"))] + [os.path.join(ROOT, "include", "nurbsdiff.h")]


def _compile(src, extra, verbose):
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + CFLAGS + list(extra) + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return obj, out


def build(extra=None, out=LIB, verbose=False, jobs=None) -> str:
    """Compile every HIP translation unit and link ``out`` (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    extra = list(extra or [])
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, msg in ex.map(lambda s: _compile(s, extra, verbose), units()):
            objs.append(obj)
            if msg.strip() and verbose:
                print(msg)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    build_pyext(verbose)
    return out


def build_pyext(verbose=False) -> str:
    """Compile the CPython serving binding (host code only)."""
    tmp = PYEXT + ".tmp"
    cmd = [CC, "-O2", "-shared", "-fPIC", "-Wall", "-I", sysconfig.get_paths()["include"], "-o", tmp,
           os.path.join(CSRC, "serve_py.c")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PYEXT)
    return PYEXT


def is_stale() -> bool:
    if not os.path.exists(LIB) or not os.path.exists(PYEXT):
        return True
    t = min(os.path.getmtime(LIB), os.path.getmtime(PYEXT))
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    build(extra=sys.argv[1:], verbose=True)
    print(LIB)
