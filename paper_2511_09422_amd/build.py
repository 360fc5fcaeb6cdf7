"""Build ``liblbfz.so`` in-tree with hipcc for gfx950.

    python -m paper_2511_09422_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/lbfz_api.hip", "csrc/lbfz_2d.hip", "csrc/lbfz_3d.hip", "csrc/lbfz_batch.hip",
           "csrc/lbfz_nn.hip", "csrc/lbfz_copy.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "liblbfz.so")
    tmp = out + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + [os.path.join(HERE, s) for s in SOURCES]
    res = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs:
        print(msgs, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
