"""The C ABI without a GPU: the library loads, exports every declared symbol,
and its host-only calls (defaults, workspace sizing, host validation,
argument checks that fail before any launch) behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2511_06600_amd import _lib, validate_host

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperef.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hef_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_params_default_and_pool_width():
    lib = _lib.load()
    p = _lib.HefParams()
    lib.hef_params_default(C.byref(p))
    assert (p.k, p.b, p.levels, p.orth_passes, p.ckpt_every, p.seed) == (10, 1, 1, 1, 0, 7)
    assert abs(p.percentile - 0.5) < 1e-7 and abs(p.drop_tol - 1e-3) < 1e-9
    assert lib.hef_pool_width(C.byref(p)) == 20
    p.b, p.k = 8, 30
    assert lib.hef_pool_width(C.byref(p)) == 480
    p.flags = _lib.FLAG_STAR_ONLY
    assert lib.hef_pool_width(C.byref(p)) == 240


def _hg(n=100, m=50, nnz=200):
    h = _lib.HefHypergraph()
    h.n, h.m, h.nnz = n, m, nnz
    h.eptr, h.pins, h.w = 0x1000, 0x2000, None   # never dereferenced by sizing
    return h


def test_workspace_size_is_host_only_and_monotone():
    lib = _lib.load()
    p = _lib.HefParams()
    lib.hef_params_default(C.byref(p))
    p.b, p.k = 8, 30
    sizes = []
    for n in (1000, 10_000, 100_000):
        out = C.c_size_t(0)
        st = lib.hef_workspace_size(C.byref(_hg(n, n, 4 * n)), C.byref(p), _lib.OP_RESISTANCE,
                                    C.byref(out))
        assert st == _lib.HEF_OK
        sizes.append(out.value)
    assert sizes[0] < sizes[1] < sizes[2]
    # the pool alone (n x 480 float32) is part of it
    assert sizes[2] > 100_000 * 480 * 4


def test_invalid_parameters_are_rejected_on_the_host():
    lib = _lib.load()
    p = _lib.HefParams()
    lib.hef_params_default(C.byref(p))
    out = C.c_size_t(0)
    p.b = 3
    assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), 0, C.byref(out)) == 6
    p.b, p.k = 16, 20                       # K = 640 > 512
    assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), 0, C.byref(out)) == 6
    p.b, p.k, p.orth_passes = 1, 10, 3
    assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), 0, C.byref(out)) == 1
    assert b"orth_passes" in lib.hef_last_error()
    p.orth_passes = 1
    # the float64 basis: Alg. 1 only, one orthonormalisation pass; basis 3 is unknown
    p.basis = _lib.BASIS_FP64
    assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), _lib.OP_RESISTANCE,
                                  C.byref(out)) == 0
    for op in (_lib.OP_COARSEN, _lib.OP_CLUSTER_LEVEL, _lib.OP_BACKWARD):
        assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), op, C.byref(out)) == 6
        assert b"float64 basis" in lib.hef_last_error()
    p.orth_passes = 2
    assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), _lib.OP_RESISTANCE,
                                  C.byref(out)) == 6
    p.orth_passes, p.basis = 1, 3
    assert lib.hef_workspace_size(C.byref(_hg()), C.byref(p), 0, C.byref(out)) == 1
    p.basis = _lib.BASIS_FP32
    assert lib.hef_workspace_size(None, C.byref(p), 0, C.byref(out)) == 1
    # hef_resistance fails its argument checks before touching the device
    assert lib.hef_resistance(None, C.byref(p), None, None, None, None, None, None, 0, None) == 1
    assert lib.hef_resistance(C.byref(_hg()), C.byref(p), None, None, 0x10, None, None, 0x10, 16,
                              None) == 3


def test_host_validator():
    ok = (5, 2, [0, 3, 5], [0, 2, 4, 1, 3], [1.0, 2.0])
    assert validate_host(*ok) == 0
    assert validate_host(5, 2, [0, 3, 5], [0, 2, 4, 1, 3], None) == 0
    assert validate_host(5, 2, [0, 1, 3], [0, 2, 4], [1.0, 1.0]) == 2        # |e| < 2
    assert validate_host(5, 2, [0, 3, 5], [0, 4, 2, 1, 3], [1.0, 1.0]) == 2  # not increasing
    assert validate_host(5, 2, [0, 3, 5], [0, 2, 2, 1, 3], [1.0, 1.0]) == 2  # duplicate pin
    assert validate_host(5, 2, [0, 3, 5], [0, 2, 5, 1, 3], [1.0, 1.0]) == 2  # out of range
    assert validate_host(5, 2, [0, 3, 5], [0, 2, 4, 1, 3], [1.0, 0.0]) == 2  # w <= 0
    assert validate_host(5, 2, [0, 3, 5], [0, 2, 4, 1, 3], [1.0, np.nan]) == 2
    assert validate_host(5, 2, [1, 3, 5], [0, 2, 4, 1, 3], [1.0, 1.0]) == 2  # eptr[0] != 0


def test_status_strings():
    lib = _lib.load()
    for code in range(7):
        assert lib.hef_status_string(code)
    assert lib.hef_status_string(0) == b"ok"
