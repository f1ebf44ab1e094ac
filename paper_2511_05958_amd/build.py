"""Compile the native libraries in-tree.

* ``paper_2511_05958_amd/libks.so``            HIP kernels + C ABI (gfx950)
* ``paper_2511_05958_amd/synth/libks_synth.so`` seeded input generator (host + gfx950)

Every HIP translation unit is built for gfx950 only, with FMA contraction off
(so that FP64 decisions made from exact integers round identically everywhere)
and with packed-FP32 instruction selection disabled.
"""

from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "--offload-arch=gfx950",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

KS_SOURCES = [
    "csrc/ks_api.hip",
    "csrc/ks_learn.hip",
    "csrc/ks_segment.hip",
    "csrc/ks_probe.hip",
    "csrc/ks_stats.hip",
    "csrc/ks_sweep.hip",
]

TARGETS = {
    "libks": (PKG / "libks.so", [PKG / s for s in KS_SOURCES], [f"-I{ROOT / 'include'}", f"-I{PKG / 'csrc'}"]),
    "synth": (PKG / "synth" / "libks_synth.so", [PKG / "synth" / "synth.hip"], []),
}


def _run(cmd: list[str]) -> None:
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout)
        raise RuntimeError(f"build failed: {' '.join(cmd)}")


def build_hip(name: str) -> Path:
    out, srcs, extra = TARGETS[name]
    tmp = out.with_suffix(".so.tmp")
    _run([HIPCC, *HIP_FLAGS, *extra, *map(str, srcs), "-o", str(tmp)])
    os.replace(tmp, out)
    return out


def build_all() -> list[Path]:
    built = [build_hip("synth")]
    if (PKG / KS_SOURCES[0]).exists():
        built.append(build_hip("libks"))
    return built


if __name__ == "__main__":
    for p in build_all():
        print(p)
