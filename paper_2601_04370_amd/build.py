"""Build the HIP library libgwg.so (gfx950) in the package directory.

hipcc compiles the kernels and the host C ABI into one shared library.  The
flags disable packed-FP32 instruction selection and FMA contraction (the
thin-film kernels opt back into contraction locally), and keep
IEEE-conforming division and square root.  The library carries the hash of
the sources it was built from (gwg_source_hash), so a loader can refuse a
library that does not match the sources beside it.
"""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgwg.so")
SOURCES = ["gwg_kernels.hip", "gwg_api.cpp"]
HEADERS = ["gwg_internal.h", "gwg_device.h", "gwg_adjoint.h", "gwg_trace.h", "gwg_launch.h",
           "gwg_fwd_kernel.h", "gwg_bwd_kernel.h", "gwg_memo_kernel.h",
           "gwg_table.h", "gwg_table_kernel.h", "gwg_omega_kernel.h", "gwg_trig_poly.h"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.exists(c) or c == "hipcc"):
            return c
    return "hipcc"


def source_hash() -> str:
    """First 16 hex digits of the SHA-256 over every source file of the
    library (kernels, host code, the C header) and the compile flags, in a
    fixed order."""
    h = hashlib.sha256()
    for path in sources():
        h.update(os.path.relpath(path, ROOT).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = ([hipcc()] + FLAGS + ['-DGWG_SOURCE_HASH="%s"' % source_hash()]
           + ["-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp"] + srcs)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def sources():
    return ([os.path.join(CSRC, s) for s in SOURCES + HEADERS]
            + [os.path.join(ROOT, "include", "gwg.h")])


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
