"""Build the HIP library libtm.so in-tree for gfx950 with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtm.so")

SOURCES = ["tm_kernels.hip", "tm_runtime.cpp", "tm_server.cpp"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile every source (one hipcc process each, in parallel) and link
    libtm.so; always recompiles."""
    tag = "%d" % os.getpid()
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build_%s_%s.o" % (tag, os.path.splitext(src)[0]))
        cmd = [hipcc()] + _flags() + list(extra_flags or []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    logs = [p.communicate()[0] for p in procs]
    failed = [(src, log) for src, p, log in zip(SOURCES, procs, logs) if p.returncode != 0]
    out_tmp = LIB + ".tmp" + tag
    try:
        if failed:
            raise RuntimeError("hipcc failed:\n" + "\n".join("%s:\n%s" % f for f in failed))
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out_tmp] + objs
        res = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout)
        if verbose:
            for log in logs:
                if log.strip():
                    print(log)
        os.replace(out_tmp, LIB)
    finally:
        for f in objs + [out_tmp]:
            if os.path.exists(f):
                os.remove(f)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
