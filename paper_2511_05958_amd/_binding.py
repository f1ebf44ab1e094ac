"""ctypes binding of libks.so: the C ABI of include/ks.h, same names, marshalling only.

Device buffers are passed as torch CUDA tensors (their data_ptr) or raw
integer addresses; streams as torch.cuda.Stream, a raw hipStream_t address,
or None for torch's current stream. Every step of the computation runs in the
library's HIP kernels; if libks.so is missing, every call raises.
"""

from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "libks.so"

KS_VERSION = 10000
KS_MAX_K = 2048
KS_MAX_N = 1 << 24
KS_CNN_PARAMS = 44993
KS_FEATURE_MAX_N = 1 << 24  # = KS_MAX_N
KS_NOALLOC_MAX_SERIES = 1 << 19
KS_CNN_TRACE_ACTS = 204
KS_CNN_TRACE_GRADS = 193

KS_OK = 0
KS_E_INVALID = -1
KS_E_RANGE = -2
KS_E_STATE = -3
KS_E_HIP = -4
KS_E_MODEL = -5
KS_E_NOMEM = -6

KS_OPT_GRID = 1
KS_OPT_PERSISTENT = 2
KS_OPT_NO_GRAPH = 4

KS_SIGNIFICANT = 1
KS_REFINED = 2
KS_FALLBACK = 4
KS_BAD_SHAPE = 8
KS_OUT_OF_RANGE = 16
KS_SEGMENT_BAD = 0xFFFFFFFF

DESC_DTYPE = np.dtype([("offset", "<u8"), ("K", "<u4"), ("N", "<u4"), ("aux_offset", "<u8")])
RESULT_DTYPE = np.dtype(
    [("cp", "<u4"), ("n", "<u4"), ("m", "<u4"), ("U", "<u4"), ("D", "<f8"), ("lambda", "<f8"),
     ("p", "<f8"), ("flags", "<u4"), ("pad", "<u4")]
)
ROW_STATS_DTYPE = np.dtype([("mean", "<f8"), ("std", "<f8"), ("min", "<u4"), ("p50", "<u4"), ("p95", "<u4"),
                            ("max", "<u4")])
assert DESC_DTYPE.itemsize == 24 and RESULT_DTYPE.itemsize == 48 and ROW_STATS_DTYPE.itemsize == 32

# include/ks_sweep.h
CHECK_DTYPE = np.dtype([("flags", "<u4"), ("disturbed", "<u4"), ("lo", "<i4"), ("hi", "<i4"), ("med_lo", "<u4"),
                        ("med_hi", "<u4"), ("mad_lo", "<u4"), ("mad_hi", "<u4")])
LINE_DTYPE = np.dtype([("line", "<u4"), ("jstar", "<u4"), ("flags", "<u4"), ("pad", "<u4"), ("jump", "<f8")])
assert CHECK_DTYPE.itemsize == 32 and LINE_DTYPE.itemsize == 24
KS_CHECK_EDGE_LOW = 1
KS_CHECK_EDGE_HIGH = 2
KS_CHECK_NO_CHANGE = 4
KS_CHECK_DISTURBED = 8
KS_CHECK_INVALID = 0x80000000
KS_LINE_INCONCLUSIVE = 1
KS_LINE_NO_INCREASE = 2
KS_LINE_NO_MAX_LIKE = 4
KS_LINE_INVALID = 0x80000000


class ks_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("c_alpha", ctypes.c_double), ("max_K", ctypes.c_uint32),
                ("w", ctypes.c_uint32), ("tau", ctypes.c_float), ("opts", ctypes.c_uint32)]


assert ctypes.sizeof(ks_params) == 32


KS_LAUNCH_GRID = 0
KS_LAUNCH_PERSISTENT = 1
KS_LAUNCH_ORDERED = 2


KS_SCAN_VARIANTS = 6


class ks_launch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("chunk_bytes", ctypes.c_uint32), ("graph", ctypes.c_uint32),
                ("variant", ctypes.c_uint32)]


class KsError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ks_status_string(code)} ({code})")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64

_SIGNATURES = {
    "ks_version": ([], ctypes.c_int),
    "ks_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "ks_params_init": ([_vp, ctypes.c_double], ctypes.c_int),
    "ks_ctx_create": ([ctypes.c_int, _vp], ctypes.c_int),
    "ks_ctx_destroy": ([_vp], ctypes.c_int),
    "ks_reserve": ([_vp, _u32, _u64], ctypes.c_int),
    "ks_learn_reserve": ([_vp, _u32, _u32, ctypes.c_int], ctypes.c_int),
    "ks_scan_batch": ([_vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp, _u64, _vp], ctypes.c_int),
    "ks_launch_set": ([_vp, _u32, _u32, _vp], ctypes.c_int),
    "ks_launch_get": ([_vp, _u32, _u32, _vp], ctypes.c_int),
    "ks_autotune": ([_vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "ks_scan_batch_noalloc": ([_vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp, _u64, _vp], ctypes.c_int),
    "ks_model_create": ([_vp, _u64, _vp], ctypes.c_int),
    "ks_model_destroy": ([_vp], ctypes.c_int),
    "ks_model_set_params": ([_vp, _vp], ctypes.c_int),
    "ks_model_get_params": ([_vp, _vp], ctypes.c_int),
    "ks_model_grads": ([_vp, _vp], ctypes.c_int),
    "ks_model_save": ([_vp, ctypes.c_char_p], ctypes.c_int),
    "ks_model_load": ([_vp, ctypes.c_char_p], ctypes.c_int),
    "ks_features": ([_vp, _vp, _u64, _vp, _u32, _u32, _vp, _u64, _vp], ctypes.c_int),
    "ks_cnn_forward": ([_vp, _vp, _vp, _u64, _vp, _u32, _u32, _vp, _u64, _vp], ctypes.c_int),
    "ks_propose": ([_vp, _vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp, _vp, _u64, _vp], ctypes.c_int),
    "ks_refine": ([_vp, _vp, _u32, _u64, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "ks_segment_batch": ([_vp, _vp, _u64, _vp, _u32, _vp, _u32, _u32, _vp, _vp, _vp], ctypes.c_int),
    "ks_probe_read": ([_vp, _u64, _u32, _u32, _vp, _vp], ctypes.c_int),
    "ks_stats_batch": ([_vp, _vp, _u64, _vp, _u32, _u32, _vp, _u64, _vp], ctypes.c_int),
    "ks_check_batch": ([_vp, _vp, _u32, _u32, _vp, _vp, _u64, _u32, _u32, _vp, _vp], ctypes.c_int),
    "ks_align_batch": ([_vp, _vp, _u32, _vp, _vp, _vp, _vp], ctypes.c_int),
    "ks_line_batch": ([_vp, _vp, _u32, _vp, _u64, _u32, _vp, _vp, _vp], ctypes.c_int),
    "ks_train_step": ([_vp, _vp, _vp, _u64, _vp, _vp, _u32, _u32, ctypes.c_float, _vp, _vp], ctypes.c_int),
    "ks_cnn_backward": ([_vp, _vp, _vp, _u64, _vp, _u32, _u32, _vp, _u64, _vp, _vp], ctypes.c_int),
    "ks_cnn_trace": ([_vp, _vp, _vp, _u64, _vp, _u32, _u32, _vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp], ctypes.c_int),
}


def lib():
    """The loaded libks.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is missing: the HIP library must be built (__graft_entry__.build())")
        so = ctypes.CDLL(str(_LIB_PATH))
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(so, name)
            fn.argtypes = args
            fn.restype = res
        _lib = so
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGNATURES)


def _check(code: int, what: str) -> None:
    if code != KS_OK:
        raise KsError(code, what)


def _addr(x, nbytes_min: int | None = None, what: str = "buffer") -> int | None:
    """Device address of a torch tensor / int / None, with a host-side size check."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not x.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if nbytes_min is not None and x.numel() * x.element_size() < nbytes_min:
        raise ValueError(f"{what} holds {x.numel() * x.element_size()} bytes, needs {nbytes_min}")
    return x.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- C ABI


def ks_version() -> int:
    return int(lib().ks_version())


def ks_status_string(code: int) -> str:
    return lib().ks_status_string(code).decode()


def ks_params_init(alpha: float = 0.05) -> ks_params:
    p = ks_params()
    _check(lib().ks_params_init(ctypes.byref(p), alpha), "ks_params_init")
    return p


def ks_ctx_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().ks_ctx_create(device, ctypes.byref(h)), "ks_ctx_create")
    return h


def ks_ctx_destroy(ctx) -> None:
    _check(lib().ks_ctx_destroy(ctx), "ks_ctx_destroy")


def ks_reserve(ctx, max_series: int, max_total_steps: int) -> None:
    _check(lib().ks_reserve(ctx, max_series, max_total_steps), "ks_reserve")


def ks_learn_reserve(ctx, max_series: int, max_K: int = 0, train: bool = False) -> None:
    _check(lib().ks_learn_reserve(ctx, max_series, max_K, 1 if train else 0), "ks_learn_reserve")


def ks_scan_batch(ctx, samples, desc, num_series: int, params: ks_params, out, all_U=None, stream=None,
                  num_samples: int | None = None) -> None:
    """Exact scan of num_series series. samples: uint32 device buffer (int32/uint32 tensor);
    desc: ks_desc[num_series] device buffer; out: ks_result[num_series] device buffer;
    all_U: optional uint32 device buffer for every U_c."""
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    all_U_len = 0 if all_U is None else (all_U.numel() * all_U.element_size() // 4)
    rc = lib().ks_scan_batch(ctx, _addr(samples, 4 * num_samples, "samples"), num_samples,
                             _addr(desc, 24 * num_series, "desc"), num_series, ctypes.byref(params),
                             _addr(out, 48 * num_series, "out"), _addr(all_U, None, "all_U"), all_U_len,
                             _stream(stream))
    _check(rc, "ks_scan_batch")


def ks_scan_batch_noalloc(ctx, samples, desc, num_series: int, params: ks_params, out, all_U=None, stream=None,
                          num_samples: int | None = None) -> None:
    """ks_scan_batch with the ordered plan on the library's fixed device scratch (allocates nothing;
    num_series <= KS_NOALLOC_MAX_SERIES). Calls that overlap in time on one device race."""
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    all_U_len = 0 if all_U is None else (all_U.numel() * all_U.element_size() // 4)
    rc = lib().ks_scan_batch_noalloc(ctx, _addr(samples, 4 * num_samples, "samples"), num_samples,
                                     _addr(desc, 24 * num_series, "desc"), num_series, ctypes.byref(params),
                                     _addr(out, 48 * num_series, "out"), _addr(all_U, None, "all_U"), all_U_len,
                                     _stream(stream))
    _check(rc, "ks_scan_batch_noalloc")


def ks_launch_set(ctx, max_K: int, num_series: int, mode: int = KS_LAUNCH_ORDERED, chunk_bytes: int = 1 << 20,
                  graph: int = 1, variant: int = 0) -> None:
    cfg = ks_launch(mode, chunk_bytes, graph, variant)
    _check(lib().ks_launch_set(ctx, max_K, num_series, ctypes.byref(cfg)), "ks_launch_set")


def ks_launch_get(ctx, max_K: int, num_series: int) -> ks_launch:
    cfg = ks_launch()
    _check(lib().ks_launch_get(ctx, max_K, num_series, ctypes.byref(cfg)), "ks_launch_get")
    return cfg


def ks_autotune(ctx, samples, desc, num_series: int, params: ks_params, out, stream=None,
                num_samples: int | None = None) -> tuple[ks_launch, float]:
    """Time the candidate launch plans on this batch; record and return the fastest (and its ms)."""
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    best = ks_launch()
    ms = ctypes.c_float(0.0)
    rc = lib().ks_autotune(ctx, _addr(samples, 4 * num_samples, "samples"), num_samples,
                           _addr(desc, 24 * num_series, "desc"), num_series, ctypes.byref(params),
                           _addr(out, 48 * num_series, "out"), _stream(stream), ctypes.byref(best),
                           ctypes.byref(ms))
    _check(rc, "ks_autotune")
    return best, float(ms.value)


def _nelem(x, size):
    return 0 if x is None else (x.numel() * x.element_size()) // size


def ks_model_create(ctx, seed: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().ks_model_create(ctx, seed, ctypes.byref(h)), "ks_model_create")
    return h


def ks_model_destroy(model) -> None:
    _check(lib().ks_model_destroy(model), "ks_model_destroy")


def ks_model_set_params(model, params) -> None:
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != KS_CNN_PARAMS:
        raise ValueError(f"expected {KS_CNN_PARAMS} parameters, got {a.size}")
    _check(lib().ks_model_set_params(model, a.ctypes.data), "ks_model_set_params")


def ks_model_get_params(model) -> np.ndarray:
    a = np.zeros(KS_CNN_PARAMS, np.float32)
    _check(lib().ks_model_get_params(model, a.ctypes.data), "ks_model_get_params")
    return a


def ks_model_grads(model) -> np.ndarray:
    a = np.zeros(KS_CNN_PARAMS, np.float32)
    _check(lib().ks_model_grads(model, a.ctypes.data), "ks_model_grads")
    return a


def ks_model_save(model, path) -> None:
    _check(lib().ks_model_save(model, str(path).encode()), "ks_model_save")


def ks_model_load(model, path) -> None:
    _check(lib().ks_model_load(model, str(path).encode()), "ks_model_load")


def ks_features(ctx, samples, desc, num_series: int, max_K: int = 0, features=None, stream=None,
                num_samples: int | None = None) -> None:
    """Feature pass; features (optional): float32 device buffer of 9 floats per row at aux_offset."""
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    rc = lib().ks_features(ctx, _addr(samples, 4 * num_samples, "samples"), num_samples,
                           _addr(desc, 24 * num_series, "desc"), num_series, max_K, _addr(features, None, "features"),
                           _nelem(features, 36), _stream(stream))
    _check(rc, "ks_features")


def ks_cnn_forward(ctx, model, features, desc, num_series: int, max_K: int, logits, stream=None) -> None:
    rc = lib().ks_cnn_forward(ctx, model, _addr(features, None, "features"), _nelem(features, 36),
                              _addr(desc, 24 * num_series, "desc"), num_series, max_K, _addr(logits, None, "logits"),
                              _nelem(logits, 4), _stream(stream))
    _check(rc, "ks_cnn_forward")


def ks_propose(ctx, model, samples, desc, num_series: int, params: ks_params, proposal, confidence, features=None,
               stream=None, num_samples: int | None = None) -> None:
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    rc = lib().ks_propose(ctx, model, _addr(samples, 4 * num_samples, "samples"), num_samples,
                          _addr(desc, 24 * num_series, "desc"), num_series, ctypes.byref(params),
                          _addr(proposal, 4 * num_series, "proposal"), _addr(confidence, 4 * num_series, "confidence"),
                          _addr(features, None, "features"), _nelem(features, 36), _stream(stream))
    _check(rc, "ks_propose")


def ks_refine(ctx, desc, num_series: int, num_samples: int, proposal, confidence, params: ks_params, out,
              stream=None) -> None:
    rc = lib().ks_refine(ctx, _addr(desc, 24 * num_series, "desc"), num_series, num_samples,
                         _addr(proposal, 4 * num_series, "proposal"), _addr(confidence, 4 * num_series, "confidence"),
                         ctypes.byref(params), _addr(out, 48 * num_series, "out"), _stream(stream))
    _check(rc, "ks_refine")


def ks_segment_batch(ctx, samples, desc, num_series: int, params: ks_params, max_levels: int, max_cp: int, cps,
                     counts, stream=None, num_samples: int | None = None) -> None:
    """Every level boundary of each series (binary segmentation). cps: ks_result[num_series * max_cp]
    device buffer; counts: uint32[num_series] device buffer."""
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    rc = lib().ks_segment_batch(ctx, _addr(samples, 4 * num_samples, "samples"), num_samples,
                                _addr(desc, 24 * num_series, "desc"), num_series, ctypes.byref(params), max_levels,
                                max_cp, _addr(cps, 48 * num_series * max_cp, "cps"), _addr(counts, 4 * num_series, "counts"),
                                _stream(stream))
    _check(rc, "ks_segment_batch")


def ks_stats_batch(ctx, samples, desc, num_series: int, max_K: int, out, stream=None,
                   num_samples: int | None = None) -> None:
    """Per-row latency statistics (mean, std, min, p50, p95, max) of every series; out: a device
    buffer of ROW_STATS_DTYPE records, series s at rows aux_offset .. aux_offset + K."""
    if num_samples is None:
        num_samples = samples.numel() * samples.element_size() // 4
    rc = lib().ks_stats_batch(ctx, _addr(samples, 4 * num_samples, "samples"), num_samples,
                              _addr(desc, 24 * num_series, "desc"), num_series, max_K, _addr(out, None, "out"),
                              _nelem(out, 32), _stream(stream))
    _check(rc, "ks_stats_batch")


def ks_check_batch(ctx, desc, num_series: int, max_K: int, results, stats, out, edge: int = 4, k: int = 5,
                   stream=None) -> None:
    """Workflow step 3 on every sweep: outlier check and widening from the detection (ks_result)
    and the per-step statistics (ROW_STATS_DTYPE rows); out: CHECK_DTYPE records (include/ks_sweep.h)."""
    rc = lib().ks_check_batch(ctx, _addr(desc, 24 * num_series, "desc"), num_series, max_K,
                              _addr(results, 48 * num_series, "results"), _addr(stats, None, "stats"),
                              _nelem(stats, 32), edge, k, _addr(out, 32 * num_series, "out"), _stream(stream))
    _check(rc, "ks_check_batch")


def ks_align_batch(measured, total, n: int, segments, aligned, distance, stream=None) -> None:
    """Benchmarked segment sizes aligned to the nearest integer fraction of the reported size
    (uint64 bytes in; uint32 k, float64 aligned size and distance out)."""
    rc = lib().ks_align_batch(_addr(measured, 8 * n, "measured"), _addr(total, 8 * n, "total"), n,
                              _addr(segments, 4 * n, "segments"), _addr(aligned, 8 * n, "aligned"),
                              _addr(distance, 8 * n, "distance"), _stream(stream))
    _check(rc, "ks_align_batch")


def ks_line_batch(ctx, desc, num_exp: int, stats, J: int, strides, out, stream=None) -> None:
    """Cache-line-size scoring of every experiment (K = J A rows of ROW_STATS_DTYPE p50s); out:
    LINE_DTYPE records (include/ks_sweep.h)."""
    rc = lib().ks_line_batch(ctx, _addr(desc, 24 * num_exp, "desc"), num_exp, _addr(stats, None, "stats"),
                             _nelem(stats, 32), J, _addr(strides, 4 * J, "strides"), _addr(out, 24 * num_exp, "out"),
                             _stream(stream))
    _check(rc, "ks_line_batch")


def ks_probe_read(words, grid: int, unroll: int, sink, stream=None) -> None:
    """Read-bandwidth probe over a device buffer (measurement aid, include/ks_probe.h)."""
    n = words.numel() * words.element_size() // 4
    _check(lib().ks_probe_read(_addr(words, 4 * n, "words"), n, grid, unroll, _addr(sink, 4, "sink"), _stream(stream)),
           "ks_probe_read")


def ks_train_step(ctx, model, features, desc, labels, num_series: int, max_K: int, lr: float, loss=None,
                  stream=None) -> None:
    rc = lib().ks_train_step(ctx, model, _addr(features, None, "features"), _nelem(features, 36),
                             _addr(desc, 24 * num_series, "desc"), _addr(labels, 4 * num_series, "labels"), num_series,
                             max_K, lr, _addr(loss, 4, "loss"), _stream(stream))
    _check(rc, "ks_train_step")


def ks_cnn_backward(ctx, model, features, desc, num_series: int, max_K: int, dlogits, grads, stream=None) -> None:
    """Gradient of sum(dlogits * logits) at the model's weights; grads: float32 device buffer of
    KS_CNN_PARAMS values (parameter layout)."""
    rc = lib().ks_cnn_backward(ctx, model, _addr(features, None, "features"), _nelem(features, 36),
                               _addr(desc, 24 * num_series, "desc"), num_series, max_K,
                               _addr(dlogits, None, "dlogits"), _nelem(dlogits, 4),
                               _addr(grads, 4 * KS_CNN_PARAMS, "grads"), _stream(stream))
    _check(rc, "ks_cnn_backward")


def ks_cnn_trace(ctx, model, features, desc, num_series: int, max_K: int, labels=None, dlogits=None, acts=None,
                 grads_in=None, grads=None, stream=None) -> None:
    """Per-layer values of the network: acts (KS_CNN_TRACE_ACTS floats per row), grads_in
    (KS_CNN_TRACE_GRADS floats per row) and the parameter gradient (device float32 buffers)."""
    rows = max(_nelem(acts, 4 * KS_CNN_TRACE_ACTS), _nelem(grads_in, 4 * KS_CNN_TRACE_GRADS))
    if acts is not None and grads_in is not None:
        rows = min(_nelem(acts, 4 * KS_CNN_TRACE_ACTS), _nelem(grads_in, 4 * KS_CNN_TRACE_GRADS))
    rc = lib().ks_cnn_trace(ctx, model, _addr(features, None, "features"), _nelem(features, 36),
                            _addr(desc, 24 * num_series, "desc"), num_series, max_K,
                            _addr(labels, 4 * num_series, "labels"), _addr(dlogits, None, "dlogits"),
                            _nelem(dlogits, 4), _addr(acts, None, "acts"), _addr(grads_in, None, "grads_in"), rows,
                            _addr(grads, 4 * KS_CNN_PARAMS, "grads"), _stream(stream))
    _check(rc, "ks_cnn_trace")


class Model:
    """Owns one ks_model (ks_model_create / ks_model_destroy)."""

    def __init__(self, ctx, seed: int = 0):
        self.handle = ks_model_create(ctx.handle if isinstance(ctx, Context) else ctx, seed)

    def close(self):
        if self.handle is not None:
            ks_model_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- convenience


def make_desc(offsets, Ks, Ns, aux_offsets=None) -> np.ndarray:
    d = np.zeros(len(Ks), DESC_DTYPE)
    d["offset"] = offsets
    d["K"] = Ks
    d["N"] = Ns
    if aux_offsets is None:
        aux = np.zeros(len(Ks), np.uint64)
        if len(Ks):
            aux[1:] = np.cumsum(np.asarray(Ks, np.uint64))[:-1]
        d["aux_offset"] = aux
    else:
        d["aux_offset"] = aux_offsets
    return d


def to_device(a: np.ndarray, device="cuda"):
    """Copy a numpy array's bytes into a device uint8 tensor (uint32 arrays become int32 tensors)."""
    import torch

    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).to(device)
    return torch.from_numpy(a.view(np.uint8).reshape(-1)).to(device)


def empty_results(num_series: int, device="cuda"):
    import torch

    return torch.empty(num_series * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=device)


def results_to_numpy(out) -> np.ndarray:
    return out.cpu().numpy().view(RESULT_DTYPE)


class Context:
    """Owns one ks_ctx (ks_ctx_create / ks_ctx_destroy)."""

    def __init__(self, device: int = 0):
        self.handle = ks_ctx_create(device)

    def close(self):
        if self.handle is not None:
            ks_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
