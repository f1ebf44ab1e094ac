"""Compile the CPU oracle (test infrastructure) into oracle/libks_oracle.so with gcc.

Plain C11, -O2, no fast-math and no FMA contraction.
"""

from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
CC = os.environ.get("CC", "gcc")


def build() -> Path:
    out = HERE / "libks_oracle.so"
    tmp = HERE / "libks_oracle.so.tmp"
    srcs = sorted(HERE.glob("*.c"))
    cmd = [CC, "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-pthread",
           *map(str, srcs), "-lm", "-o", str(tmp)]
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout)
        raise RuntimeError("oracle build failed: " + " ".join(cmd))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
