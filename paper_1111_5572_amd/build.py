"""Compile the HIP library (libsnapgpu.so) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("index.hip", "index_gpu.hip", "dups.hip", "align.hip", "server.hip")]
HEADERS = [os.path.join(HERE, "csrc", "snap_internal.h"), os.path.join(ROOT, "include", "snapgpu.h"),
           os.path.join(ROOT, "include", "snapgpu_debug.h")]
LIB = os.path.join(HERE, "libsnapgpu.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed fp32 instructions off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source into libsnapgpu.so (always recompiles unless force=False
    and the library is newer than every source)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(f) for f in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    # one object per source, compiled side by side, then one link
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    with tempfile.TemporaryDirectory(prefix="snapgpu_build_") as tdir:
        objs = [os.path.join(tdir, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [["hipcc", *HIPCC_FLAGS, "-c", "-I", os.path.join(ROOT, "include"), "-o", obj, src]
                for src, obj in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c))
        with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
            for f in [ex.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        link = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *objs]
        if verbose:
            print(" ".join(link))
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
