"""Builds the gfx950 HIP library ``libgsraster.so`` in-tree with hipcc.

    python -m paper_2501_06838_amd.build

Flags: -O3 for gfx950 only; -munsafe-fp-atomics so FP32/FP64 atomic adds on
(coarse-grained) device memory use the hardware instructions; packed FP32
instructions are disabled for every kernel.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgsraster.so")
SOURCES = ["gs_api.hip", "gs_binning.hip", "gs_render.hip", "gs_surrogate.hip", "gs_head.hip",
           "gs_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def command(out=LIB):
    """One hipcc line that compiles and links every source (for reference;
    build() compiles the sources in parallel and links them)."""
    return [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC,
            *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-FP32 feature name: harmless
    noise = "'-packed-fp32-ops' is not a recognized feature"
    text = "\n".join(l for l in res.stdout.splitlines() if noise not in l)
    return res.returncode, text


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel, one hipcc per file) and link
    them into one shared library.  Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    tag = "%d" % os.getpid()
    objs = [os.path.join(CSRC, os.path.splitext(s)[0] + ".%s.o" % tag) for s in SOURCES]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    cmds = [[HIPCC, *compile_flags, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, s),
             "-o", o] for s, o in zip(SOURCES, objs)]
    tmp = LIB + ".tmp" + tag
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            results = list(ex.map(_run, cmds))
        for cmd, (rc, text) in zip(cmds, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if rc != 0:
                raise RuntimeError("hipcc failed:\n" + text)
            if verbose and text.strip():
                print(text)
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        rc, text = _run(link)
        if verbose:
            print(" ".join(link), flush=True)
        if rc != 0:
            raise RuntimeError("hipcc link failed:\n" + text)
        os.replace(tmp, LIB)
    finally:
        for o in objs + [tmp]:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
