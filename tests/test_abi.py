"""The C-ABI library on the host: it loads, exports every function include/ks.h declares,
and rejects bad arguments before touching a device (no compute calls, no GPU needed)."""

import ctypes
import re
from pathlib import Path

import pytest

import paper_2511_05958_amd as P

ROOT = Path(__file__).resolve().parent.parent


def declared_functions():
    names = set()
    for h in sorted((ROOT / "include").glob("*.h")):
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(ks_[A-Za-z0-9_]+)\s*\(", text,
                             flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = declared_functions()
    assert "ks_scan_batch" in names and len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps each declared function under the same name
    assert set(names) <= set(P._binding.exported_symbols())
    for n in names:
        assert callable(getattr(P, n)), n


def test_status_and_params_on_host():
    assert P.ks_version() == P.KS_VERSION
    for code in (0, -1, -2, -3, -5, -6, -99):
        assert isinstance(P.ks_status_string(code), str)
    prm = P.ks_params_init(0.05)
    assert abs(prm.c_alpha - 1.8444397270569681) < 1e-15
    assert (prm.max_K, prm.w, prm.opts) == (0, 8, 0) and abs(prm.tau - 0.5) < 1e-7
    with pytest.raises(P.KsError):
        P.ks_params_init(0.0)
    with pytest.raises(P.KsError):
        P.ks_params_init(1.0)


def test_null_arguments_rejected_without_device():
    lib = P.lib()
    prm = P.ks_params_init(0.05)
    assert lib.ks_scan_batch(None, None, 0, None, 0, ctypes.byref(prm), None, None, 0, None) == P.KS_E_INVALID
    assert lib.ks_ctx_destroy(None) == P.KS_E_INVALID
    assert lib.ks_ctx_create(0, None) == P.KS_E_INVALID
    assert lib.ks_reserve(None, 1, 1) == P.KS_E_INVALID
    assert lib.ks_learn_reserve(None, 1, 16, 0) == P.KS_E_INVALID
