"""Build the in-tree HIP library paper_1008_1685_amd/libpic.so for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "pic_lib.hip")
OUT = os.path.join(HERE, "libpic.so")
# the STREAM-copy kernel the roofline's measured ceiling comes from
COPY_SRC = os.path.join(HERE, "csrc", "stream_copy.hip")
COPY_OUT = os.path.join(HERE, "libstreamcopy.so")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, out: str = OUT, defines=(), src: str = SRC) -> str:
    """Compile libpic.so; ``defines`` are extra -D options (tuning variants)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, *[f"-D{d}" for d in defines], "-I", os.path.join(ROOT, "include"),
           src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed ({r.returncode})")
    os.replace(tmp, out)
    return out


def build_stream_copy(verbose: bool = False) -> str:
    """Compile libstreamcopy.so (the copy-ceiling measurement)."""
    return build(verbose=verbose, out=COPY_OUT, src=COPY_SRC)


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_stream_copy(verbose=True))
