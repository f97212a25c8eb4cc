"""hef_resistance_static captured into a HIP graph (torch.cuda.graph) and
replayed.  With HEF_FLAG_ASSUME_VALID the call synchronises nothing, its
scratch is the library's static array and its buffers are cleared by fill
kernels, so the graph holds kernel and device-to-device copy nodes only.
Every replay, with eager work of the program and synchronisations between
the replays, must reproduce the eager call bit for bit."""
import pytest
import torch

import paper_2511_06600_amd as hef
from synth import generate
from tests.gpu_common import say, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("basis", ["fp32", "bf16"])
def test_static_entry_replays_in_a_graph(basis):
    h = generate(6000, 6400, 2, 60, 2.5, p_loc=0.7, win=300, weights="lognormal", seed=51)
    params = hef.Params(k=8, b=4, basis=basis, assume_valid=True)
    dh = to_device(h)
    say(f"case: graph capture of hef_resistance_static n={h.n} m={h.m} k=8 b=4 basis={basis}")
    # the eager call (it also looks up the static scratch's device address)
    R0, q0, c0 = hef.resistance_static(dh, params, return_pool=True)
    torch.cuda.synchronize()
    assert torch.isfinite(R0).all() and (q0 > 0).any()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        R1, q1, c1 = hef.resistance_static(dh, params, return_pool=True)
    for rep in range(3):
        # eager work between the replays: clobber the outputs, run other kernels
        R1.fill_(-1.0)
        q1.zero_()
        c1.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"replay {rep}: checked against the eager call (junk {float(junk):.3f})")
        assert torch.equal(R1, R0), f"replay {rep}: R differs"
        assert torch.equal(q1, q0), f"replay {rep}: Q_H differs"
        assert torch.equal(c1, c0), f"replay {rep}: pool differs"
