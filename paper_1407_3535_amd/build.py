"""Compiles libzts.so in-tree with hipcc for gfx950."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libzts.so")
SOURCES = ["zts_kernels.hip", "zts_host.hip", "zts_serve.hip"]
HEADERS = ["zts_device.h", "zts_kernels.h", "zts_shared.h", "zts_runtime.h"]
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-ffp-contract=off",          # every binary64 decision is evaluated exactly as written
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",        # only the ZTS_API entry points are exported
    "-pthread",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def build(force: bool = True, verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(CSRC, h) for h in HEADERS]
                     + [os.path.join(HERE, "..", "include", "zts.h")])
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + srcs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (res.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        sys.stderr.write(errs + "\n")
        raise RuntimeError("hipcc failed (%d)" % res.returncode)
    if verbose and errs.strip():
        sys.stderr.write(errs + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
