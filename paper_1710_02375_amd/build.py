"""Builds the HIP library libkbc_lbm.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", "kernels.hip"), os.path.join(HERE, "csrc", "engine.hip"),
           os.path.join(HERE, "csrc", "fsi.hip")]
HEADERS = [os.path.join(HERE, "csrc", n) for n in ("lbm_device.hpp", "kbc_node.hpp", "kernels.hpp")]
LIB = os.path.join(HERE, "libkbc_lbm.so")
ARCH = os.environ.get("KBC_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
         # packed FP32 instructions stay disabled on this target
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles every source into libkbc_lbm.so; each source is compiled to
    an object in parallel, then linked.  Returns the library path."""
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        objs.append(obj)
        cmd = ["hipcc"] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
    for cmd, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "not a recognized feature" not in l and l.strip())
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n%s\n%s" % (" ".join(cmd), text))
        if verbose and text:
            print(text)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
