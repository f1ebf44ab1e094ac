"""Compile the native libraries in-tree.

* ``paper_2511_05958_amd/libks.so``            HIP kernels + C ABI (gfx950)
* ``paper_2511_05958_amd/synth/libks_synth.so`` seeded input generator (host + gfx950)

Every HIP translation unit is built for gfx950 only, with FMA contraction off
(so that FP64 decisions made from exact integers round identically everywhere)
and with packed-FP32 instruction selection disabled. libks's sources compile
to objects in parallel (csrc/ks_scan_variants.hip once per scan-kernel
variant, -DKS_SCAN_VARIANT=i) and are then linked into the one library.
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
KS_VARIANT_SOURCE = "csrc/ks_scan_variants.hip"
KS_SCAN_VARIANTS = 6  # ks_host::kNumVariants

TARGETS = {
    "libks": (PKG / "libks.so", [PKG / s for s in KS_SOURCES], [f"-I{ROOT / 'include'}", f"-I{PKG / 'csrc'}"]),
    "synth": (PKG / "synth" / "libks_synth.so", [PKG / "synth" / "synth.hip"], []),
}


def _run(cmd: list[str]) -> None:
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout)
        raise RuntimeError(f"build failed: {' '.join(cmd)}")


def _jobs() -> int:
    try:
        return max(1, min(len(os.sched_getaffinity(0)), int(os.environ.get("MAX_JOBS", "16") or 16)))
    except (AttributeError, ValueError):
        return 4


def _build_libks(out: Path, extra: list[str]) -> None:
    """Objects in parallel, then one link (each object carries its own gfx950 code)."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    cflags = [f for f in HIP_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="ks_build_") as tmpd:
        jobs = []
        for src in KS_SOURCES:
            jobs.append([HIPCC, *cflags, *extra, "-c", str(PKG / src), "-o", str(Path(tmpd) / (Path(src).stem + ".o"))])
        for v in range(KS_SCAN_VARIANTS):
            jobs.append([HIPCC, *cflags, *extra, f"-DKS_SCAN_VARIANT={v}", "-c", str(PKG / KS_VARIANT_SOURCE), "-o",
                         str(Path(tmpd) / f"ks_scan_variant{v}.o")])
        with ThreadPoolExecutor(max_workers=_jobs()) as pool:
            list(pool.map(_run, jobs))
        objs = [j[-1] for j in jobs]
        tmp = out.with_suffix(".so.tmp")
        _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", str(tmp)])
        os.replace(tmp, out)


def build_hip(name: str) -> Path:
    out, srcs, extra = TARGETS[name]
    if name == "libks":
        _build_libks(out, extra)
        return out
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
