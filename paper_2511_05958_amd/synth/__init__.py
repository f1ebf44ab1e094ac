"""Seeded synthetic latency sweeps (input generator; none of the method's arithmetic).

A batch is a packed uint32 buffer of series; series ``t`` is a row-major
``[K][N]`` block at element ``specs[t]['offset']`` (256-byte aligned). The five
workload recipes follow the shapes of the size-benchmark sweeps (rows =
footprints stepped by the fetch granularity, columns = the first N load
latencies of each footprint) with latency levels on the scale of the AMD
load latencies the paper reports (Table 3):

=====  ==========================================================================
recipe  shape and structure
=====  ==========================================================================
1      1 series, K=64, N=256; one change 120 -> 320 cycles at a uniform row
       1..63; lognormal jitter sigma=0.05; no outliers
2      K=256, N=1024; 1-4 plateaus, an ascending subset of {120,300,550,850}
       each x U[0.9,1.1], plateaus >= 8 rows; sigma=0.08; 1% outliers x U[1,5]
3      K=round(logU[32,512]), N=round(logU[64,4096]); 0-4 transitions from
       {120,300,550,850,1300} +-10%, each a 2-row ramp at 1/3 and 2/3 of the
       jump; plateaus >= 4 rows; sigma=0.08; 1% outliers
4      recipe 2 with its own seed (training series)
5      K=1024, N=2048; 1-4 transitions, L0 = 120 x U[0.9,1.1], adjacent ratios
       U[1.05,1.2]; per sample 5% outliers x U[1,5], else 10% Pareto(1, 2.5)
       multipliers, else lognormal sigma=0.08
=====  ==========================================================================
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "libks_synth.so"
SEED_BASE = 2511059580

SERIES_DTYPE = np.dtype(
    [
        ("offset", "<u8"),
        ("K", "<u4"),
        ("N", "<u4"),
        ("sid", "<u4"),
        ("nseg", "<u4"),
        ("nplant", "<u4"),
        ("pad", "<u4"),
        ("seg_start", "<u4", (16,)),
        ("plant", "<u4", (4,)),
        ("seg_level", "<f8", (16,)),
    ],
    align=True,
)
assert SERIES_DTYPE.itemsize == 240

NOISE_DTYPE = np.dtype(
    [("sigma", "<f8"), ("p_out", "<f8"), ("out_lo", "<f8"), ("out_hi", "<f8"),
     ("p_pareto", "<f8"), ("pareto_alpha", "<f8")]
)

DEFAULT_COUNTS = {1: 1, 2: 4096, 3: 16384, 4: 200_000, 5: 8192}

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(str(_LIB_PATH))
        vp = ctypes.c_void_p
        lib.syn_noise_for.argtypes = [ctypes.c_int, vp]
        lib.syn_make_batch.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, vp, vp]
        lib.syn_fill_host.argtypes = [vp, ctypes.c_uint32, vp, ctypes.c_uint32, vp, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_int]
        lib.syn_fill_device.argtypes = [vp, ctypes.c_uint32, vp, ctypes.c_uint32, vp, ctypes.c_uint64,
                                        ctypes.c_uint64, vp]
        lib.syn_philox4x32_10.argtypes = [vp, vp, vp]
        lib.syn_philox4x32_10.restype = None
        lib.syn_math.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.syn_math.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Batch:
    recipe: int
    seed: int
    specs: np.ndarray  # SERIES_DTYPE
    noise: np.ndarray  # NOISE_DTYPE, shape ()
    total_elems: int

    @property
    def num_series(self) -> int:
        return len(self.specs)

    @property
    def sample_bytes(self) -> int:
        """Algorithmic sample bytes: 4 * sum K*N (padding excluded)."""
        return int(4 * np.sum(self.specs["K"].astype(np.uint64) * self.specs["N"].astype(np.uint64)))

    def subset(self, ids) -> "Batch":
        """The given series, repacked from element 0 (same samples, same series ids)."""
        sp = self.specs[np.asarray(ids, dtype=np.int64)].copy()
        off = 0
        for t in range(len(sp)):
            sp[t]["offset"] = off
            off += (int(sp[t]["K"]) * int(sp[t]["N"]) + 63) & ~63
        return Batch(self.recipe, self.seed, sp, self.noise, off)


def seed_for(recipe: int) -> int:
    return (SEED_BASE + recipe) & 0xFFFFFFFF


def make_batch(recipe: int, num_series: int | None = None, seed: int | None = None,
               first_series: int = 0) -> Batch:
    lib = _load()
    if num_series is None:
        num_series = DEFAULT_COUNTS[recipe]
    if seed is None:
        seed = seed_for(recipe)
    specs = np.zeros(num_series, dtype=SERIES_DTYPE)
    noise = np.zeros((), dtype=NOISE_DTYPE)
    total = ctypes.c_uint64(0)
    if lib.syn_noise_for(recipe, noise.ctypes.data) != 0:
        raise ValueError(f"unknown recipe {recipe}")
    if lib.syn_make_batch(recipe, seed, first_series, num_series, _ptr(specs), ctypes.byref(total)) != 0:
        raise ValueError(f"unknown recipe {recipe}")
    return Batch(recipe, seed, specs, noise, int(total.value))


def fill_host(batch: Batch, threads: int | None = None) -> np.ndarray:
    """All samples of the batch as a host uint32 array of length batch.total_elems."""
    lib = _load()
    out = np.zeros(batch.total_elems, dtype=np.uint32)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rc = lib.syn_fill_host(_ptr(batch.specs), batch.num_series, batch.noise.ctypes.data, batch.seed,
                           _ptr(out), 0, out.size, threads)
    if rc != 0:
        raise RuntimeError(f"syn_fill_host failed ({rc})")
    return out


def fill_device(batch: Batch, dst_ptr: int, dst_elems: int, stream: int = 0) -> None:
    """Write the batch's samples into a device buffer (bit-identical to fill_host)."""
    lib = _load()
    rc = lib.syn_fill_device(_ptr(batch.specs), batch.num_series, batch.noise.ctypes.data, batch.seed,
                             ctypes.c_void_p(dst_ptr), 0, dst_elems, ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"syn_fill_device failed ({rc})")


def series_view(samples: np.ndarray, batch: Batch, t: int) -> np.ndarray:
    s = batch.specs[t]
    o, K, N = int(s["offset"]), int(s["K"]), int(s["N"])
    return samples[o:o + K * N].reshape(K, N)


def philox4x32_10(ctr, key) -> tuple[int, int, int, int]:
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib.syn_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return tuple(int(v) for v in o)


def math_fn(which: str, x: float) -> float:
    return _load().syn_math({"exp": 0, "log": 1, "cos2pi": 2}[which], float(x))


def line_experiments(num_exp: int, J: int = 16, A: int = 32, N: int = 256, seed: int = SEED_BASE + 6,
                     stride_step: int = 16) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Cache-line-size experiments (Section "Cache Line Size benchmarks"): for each of
    num_exp caches, J strides stride_step * (j + 1) bytes (stride 0 the pivot, J - 1 the
    MAX) x A array sizes around and above the cache size x N latencies. A stride up to the
    line size L touches every line, so the miss share rises with the array size from 0.3
    to 1; a stride s > L skips lines and reaches L / s of it. Latency = lo + (hi - lo) x
    miss share, hi ~ U[500, 900], lo ~ U[200, 400] cycles, L a power of two drawn from
    the strides below the largest power of two; per sample lognormal jitter sigma 0.05
    and 1% outliers x U[1, 5] (numpy's Generator, seeded).

    Returns (samples uint32 [num_exp * J * A * N], strides uint32 [J], planted L [num_exp])."""
    rng = np.random.default_rng(seed)
    strides = np.array([stride_step * (j + 1) for j in range(J)], np.uint32)
    pow2 = [int(s) for s in strides if (int(s) & (int(s) - 1)) == 0][:-1]
    if not pow2:
        raise ValueError("the strides need two powers of two")
    lines = np.array(pow2, np.uint32)[rng.integers(0, len(pow2), num_exp)]
    hi = rng.uniform(500, 900, num_exp)
    lo = rng.uniform(200, 400, num_exp)
    frac = np.linspace(0.3, 1.0, A)
    share = np.where(strides[None, :, None] <= lines[:, None, None], frac[None, None, :],
                     frac[None, None, :] * (lines[:, None, None] / strides[None, :, None].astype(np.float64)))
    lat = lo[:, None, None] + (hi - lo)[:, None, None] * share          # [E][J][A]
    out = np.empty((num_exp, J, A, N), np.uint32)
    for e in range(num_exp):  # one experiment at a time bounds the temporaries
        x = lat[e][:, :, None] * np.exp(0.05 * rng.standard_normal((J, A, N)))
        o = rng.random((J, A, N)) < 0.01
        x = np.where(o, lat[e][:, :, None] * rng.uniform(1, 5, (J, A, N)), x)
        out[e] = np.clip(np.rint(x), 1, 2**32 - 1).astype(np.uint32)
    return out.reshape(-1), strides, lines
