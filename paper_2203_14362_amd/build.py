"""Compile the HIP sources of the canvas engine into libspade.so (gfx950)."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspade.so")
SOURCES = ["capi.hip", "raster.hip", "probe.hip", "batch.hip", "disk.hip", "layers.hip", "dist.hip", "host.hip", "jobs.hip",
           "buffer.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res.stderr


def build(verbose: bool = False) -> str:
    """Always recompiles (one hipcc per source, in parallel, then one link);
    returns the path of the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tag = "%d" % os.getpid()
    objs = [os.path.join(CSRC, s[:-4] + ".o" + tag) for s in SOURCES]
    cmds = [[hipcc] + HIPCC_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            logs = list(ex.map(_run, cmds))
        tmp = LIB + ".tmp" + tag
        logs.append(_run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs))
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    if verbose:
        print("".join(logs))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
