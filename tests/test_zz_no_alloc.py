"""hef_resistance_static (no workspace, per-device static scratch) against
hef_resistance on the same inputs: bitwise-identical R, Q_H and pool (both
run the same kernels in the same order), on two calls in a row, the second
with a smaller hypergraph, and a clear error for an input whose scratch
exceeds the static array."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2511_06600_amd as hef
from paper_2511_06600_amd import _lib
from synth import generate
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu


def _both(h, params, with_starts):
    dh = to_device(h)
    xs = xc = None
    if with_starts:
        g = torch.Generator(device="cuda").manual_seed(h.n)
        xs = torch.randn((h.n + h.m, params.b), device="cuda", generator=g)
        xc = torch.randn((h.n, params.b), device="cuda", generator=g)
    R1, q1, c1 = hef.resistance(dh, params, xs, xc, return_pool=True)
    R2, q2, c2 = hef.resistance_static(dh, params, xs, xc, return_pool=True)
    R3, q3, _ = hef.resistance_static(dh, params, xs, xc, return_pool=False)
    torch.cuda.synchronize()
    return (R1, q1, c1), (R2, q2, c2), (R3, q3)


@pytest.mark.parametrize("first,second", [((6000, 6400, 8, 4), (700, 650, 10, 1))])
def test_static_scratch_equals_workspace_path(first, second):
    for i, (n, m, k, b) in enumerate((first, second)):
        h = generate(n, m, 2, 60, 2.5, p_loc=0.7, win=300, weights="lognormal", seed=40 + i)
        params = hef.Params(k=k, b=b)
        need = hef.workspace_bytes(to_device(h), params, _lib.OP_RESISTANCE)
        say(f"case: call {i} n={h.n} m={h.m} nnz={h.nnz} k={k} b={b} workspace={need} bytes")
        assert need <= _lib.STATIC_SCRATCH_BYTES
        ref, got, got_nochi = _both(h, params, with_starts=(i == 0))
        assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
        assert torch.equal(ref[2], got[2])
        assert torch.equal(ref[0], got_nochi[0]) and torch.equal(ref[1], got_nochi[1])
        assert torch.isfinite(got[0]).all() and (got[1] > 0).any()


def test_static_scratch_rejects_large_input():
    h = generate(20000, 21000, 2, 60, 2.5, p_loc=0.7, win=300, seed=44)
    params = hef.Params(k=20, b=4)
    dh = to_device(h)
    need = hef.workspace_bytes(dh, params, _lib.OP_RESISTANCE)
    say(f"case: oversized n={h.n} m={h.m} K={params.K} workspace={need} bytes")
    assert need > _lib.STATIC_SCRATCH_BYTES
    R = torch.full((h.m,), -1.0, device="cuda")
    st = _lib.load().hef_resistance_static(C.byref(dh.c()), C.byref(params.c()), None, None,
                                           R.data_ptr(), None, None,
                                           torch.cuda.current_stream().cuda_stream)
    assert st == 3  # HEF_ERR_WORKSPACE_TOO_SMALL
    assert b"static scratch" in _lib.load().hef_last_error()
    torch.cuda.synchronize()
    assert (R == -1.0).all()  # nothing written
