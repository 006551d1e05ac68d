"""Builds the device library ``libmgx.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmgx.so")
# The diagnostic build: the same sources with per-wave phase timestamps in the step kernels.
LIB_WAVE_TS = os.path.join(PKG, "libmgx_wavets.so")
ARCH = os.environ.get("MGX_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # explicit fused multiply-adds only: identical arithmetic in every kernel variant
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def source_hash(root: str = ROOT) -> str:
    """SHA-256 (first 16 hex digits) over the device library's sources under ``root``: every
    ``*.hip`` and ``*.hpp`` of the package's csrc/ and every ``*.h`` of include/, by relative
    path and content. Compiled into the library and checked when it is loaded."""
    h = hashlib.sha256()
    pkg = os.path.basename(PKG)
    files = sorted(glob.glob(os.path.join(root, pkg, "csrc", "*.hip")) + glob.glob(os.path.join(root, pkg, "csrc", "*.hpp"))
                   + glob.glob(os.path.join(root, "include", "*.h")))
    for f in files:
        h.update(os.path.relpath(f, root).replace(os.sep, "/").encode())
        h.update(b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def build(verbose: bool = False, extra=(), jobs: int = 0, out: str = LIB) -> str:
    """Compile every HIP source into ``out`` (libmgx.so; always recompiles): one object per
    source, compiled in parallel, then linked."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = f".{os.getpid()}"
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(s)[:-4] + tag + ".o") for s in srcs]
    compile_flags = [f for f in FLAGS if f != "-shared"] + [f'-DMGX_BUILD_HASH="{source_hash()}"']
    cmds = [[hipcc, *compile_flags, *extra, "-I", INCLUDE, "-I", CSRC, "-c", s, "-o", o] for s, o in zip(srcs, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        procs = list(ex.map(lambda c: subprocess.run(c), cmds))
    failed = [c[-3] for c, p in zip(cmds, procs) if p.returncode != 0]
    try:
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc -c " + " ".join(failed))
        tmp = out + f".tmp{os.getpid()}"
        subprocess.check_call([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


def build_wave_timestamps(verbose: bool = False) -> str:
    """The diagnostic library libmgx_wavets.so (step kernels record per-wave phase times)."""
    return build(verbose, extra=("-DMGX_WAVE_TIMESTAMPS",), out=LIB_WAVE_TS)


if __name__ == "__main__":
    if sys.argv[1:] == ["--wave-timestamps"]:
        print(build_wave_timestamps(verbose=True))
    else:
        build(verbose=True, extra=sys.argv[1:])
        print(LIB)
