"""Compile the HIP sources of the package into libtdde.so (gfx950) next to this file.

Each source is compiled to an object in parallel, then the objects are linked.
Usage: python -m paper_2512_21697_amd.build    (or call build())
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtdde.so")
# (source, extra flags, object name): the persistent solver is compiled once per variant
SOURCES = [("tdde.hip", [], "tdde"), ("mlp.hip", [], "mlp"), ("split.hip", [], "split")] + [
    ("persistent.hip", [f"-DTDDE_VARIANT={v}"], f"persistent_v{v}") for v in range(4)]
ARCH = os.environ.get("TDDE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="tdde_build_") as tmpd:
        objs, procs = [], []
        for name, extra, oname in SOURCES:
            src = os.path.join(CSRC, name)
            obj = os.path.join(tmpd, oname + ".o")
            cmd = ["hipcc", *FLAGS, *extra, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = False
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                sys.stderr.write(out)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed building libtdde.so")
        tmp = LIB + ".tmp"
        cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libtdde.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
