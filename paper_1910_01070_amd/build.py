"""Build libhr2.so (HIP for gfx950) in-tree.

``python -m paper_1910_01070_amd.build`` compiles the kernels and the host
library with hipcc and links ``paper_1910_01070_amd/libhr2.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libhr2.so")
SOURCES = ["kernels.hip", "api.cpp", "serve.cpp", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-pthread",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    """Compile every source in parallel, then link the shared library."""
    with tempfile.TemporaryDirectory(prefix="hr2build") as tmp:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
        failed = []
        for cmd, p in procs:
            out, _ = p.communicate()
            out = "\n".join(l for l in out.splitlines()
                            if "packed-fp32-ops" not in l and l.strip())
            if p.returncode != 0:
                failed.append((cmd, out))
            elif verbose and out:
                print(out)
        if failed:
            msg = "\n\n".join(" ".join(c) + "\n" + o for c, o in failed)
            raise RuntimeError("hipcc failed:\n" + msg)
        tmp_lib = LIB_PATH + ".tmp"
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread",
                               "-o", tmp_lib, *objs])
        os.replace(tmp_lib, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
