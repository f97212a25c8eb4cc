"""MI355X-native HyperEF 2.0 hot path: Python binding of libhyperef.so.

Argument marshalling only: every stage runs in the library's HIP kernels;
PyTorch provides device memory (tensors, the workspace) and the stream.
There is no CPU fallback: if the library is missing, importing the
functions below raises.

    hg = DeviceHypergraph.from_arrays(n, m, eptr, pins, w)
    R, qh, chi = resistance(hg, Params(k=30, b=8), return_pool=True)
    cluster, n_clusters, R0, eta = coarsen(hg, Params(k=20, b=4, levels=3))
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import HefError, check, load  # noqa: F401


@dataclass
class Params:
    """Mirror of hef_params (include/hyperef.h)."""
    k: int = 10
    b: int = 1
    levels: int = 1
    percentile: float = 0.5
    local_clustering: bool = True
    basis: str = "fp32"           # "fp32" or "bf16" pool storage ("fp64": debug, resistance only)
    seed: int = 7
    drop_tol: float = 1e-3
    orth_passes: int = 1
    ckpt_every: int = 0           # 0: the adjoint tape keeps every Krylov step
    assume_valid: bool = False
    star_only: bool = False
    clique_only: bool = False
    target_nr: float = 0.0        # node-reduction target of the level loop (0 = off)

    def c(self) -> _lib.HefParams:
        p = _lib.HefParams()
        p.k, p.b, p.levels = self.k, self.b, self.levels
        p.percentile = self.percentile
        p.local_clustering = int(self.local_clustering)
        p.basis = {"fp32": _lib.BASIS_FP32, "bf16": _lib.BASIS_BF16,
                   "fp64": _lib.BASIS_FP64}[self.basis]
        p.seed = self.seed
        p.drop_tol = self.drop_tol
        p.orth_passes = self.orth_passes
        p.ckpt_every = self.ckpt_every
        p.flags = ((_lib.FLAG_ASSUME_VALID if self.assume_valid else 0)
                   | (_lib.FLAG_STAR_ONLY if self.star_only else 0)
                   | (_lib.FLAG_CLIQUE_ONLY if self.clique_only else 0))
        p.target_nr = self.target_nr
        return p

    @property
    def K(self) -> int:
        return load().hef_pool_width(C.byref(self.c()))


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class DeviceHypergraph:
    """A CSR hypergraph resident on the GPU (int32 eptr / pins, float32 w)."""

    def __init__(self, n: int, m: int, eptr: torch.Tensor, pins: torch.Tensor,
                 w: torch.Tensor | None):
        self.n, self.m = int(n), int(m)
        self.eptr, self.pins, self.w = eptr, pins, w
        self.nnz = int(pins.numel())
        self.device = eptr.device

    @classmethod
    def from_arrays(cls, n, m, eptr, pins, w=None, device="cuda") -> "DeviceHypergraph":
        e = torch.as_tensor(np.asarray(eptr, dtype=np.int32), device=device)
        p = torch.as_tensor(np.asarray(pins, dtype=np.int32), device=device)
        ww = None if w is None else torch.as_tensor(np.asarray(w, dtype=np.float32), device=device)
        return cls(n, m, e, p, ww)

    def c(self) -> _lib.HefHypergraph:
        h = _lib.HefHypergraph()
        h.n, h.m, h.nnz = self.n, self.m, self.nnz
        h.eptr, h.pins, h.w = _ptr(self.eptr), _ptr(self.pins), _ptr(self.w)
        return h


def workspace_bytes(hg: DeviceHypergraph, params: Params, op: int) -> int:
    out = C.c_size_t(0)
    check(load().hef_workspace_size(C.byref(hg.c()), C.byref(params.c()), op, C.byref(out)),
          "hef_workspace_size")
    return int(out.value)


def _workspace(hg, params, op):
    nbytes = workspace_bytes(hg, params, op)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=hg.device)


_POOL_DTYPE = {"fp32": torch.float32, "bf16": torch.bfloat16, "fp64": torch.float64}


def resistance(hg: DeviceHypergraph, params: Params, start_star: torch.Tensor | None = None,
               start_clique: torch.Tensor | None = None, return_pool: bool = False):
    """Alg. 1: returns (R [m] float32, qh [K] float64, chi [n, K] or None)."""
    lib = load()
    K = params.K
    R = torch.empty(hg.m, dtype=torch.float32, device=hg.device)
    qh = torch.empty(K, dtype=torch.float64, device=hg.device)
    chi = None
    if return_pool:
        chi = torch.empty((hg.n, K), dtype=_POOL_DTYPE[params.basis], device=hg.device)
    ws = _workspace(hg, params, _lib.OP_RESISTANCE)
    for t, rows in ((start_star, hg.n + hg.m), (start_clique, hg.n)):
        if t is not None:
            assert t.dtype == torch.float32 and t.is_contiguous() and t.shape == (rows, params.b)
    check(lib.hef_resistance(C.byref(hg.c()), C.byref(params.c()), _ptr(start_star),
                             _ptr(start_clique), _ptr(R), _ptr(qh), _ptr(chi), _ptr(ws),
                             ws.numel(), _stream(hg.device)), "hef_resistance")
    return R, qh, chi


def resistance_static(hg: DeviceHypergraph, params: Params,
                      start_star: torch.Tensor | None = None,
                      start_clique: torch.Tensor | None = None, return_pool: bool = False):
    """Alg. 1 through hef_resistance_static (no workspace: the library's
    per-device static scratch); returns what resistance() returns."""
    lib = load()
    K = params.K
    R = torch.empty(hg.m, dtype=torch.float32, device=hg.device)
    qh = torch.empty(K, dtype=torch.float64, device=hg.device)
    chi = None
    if return_pool:
        chi = torch.empty((hg.n, K), dtype=_POOL_DTYPE[params.basis], device=hg.device)
    for t, rows in ((start_star, hg.n + hg.m), (start_clique, hg.n)):
        if t is not None:
            assert t.dtype == torch.float32 and t.is_contiguous() and t.shape == (rows, params.b)
    check(lib.hef_resistance_static(C.byref(hg.c()), C.byref(params.c()), _ptr(start_star),
                                    _ptr(start_clique), _ptr(R), _ptr(qh), _ptr(chi),
                                    _stream(hg.device)), "hef_resistance_static")
    return R, qh, chi


def coarsen(hg: DeviceHypergraph, params: Params):
    """Alg. 2: returns (cluster [n] int32, n_clusters, R0 [m], eta [n_clusters])."""
    lib = load()
    cluster = torch.empty(hg.n, dtype=torch.int32, device=hg.device)
    R0 = torch.empty(hg.m, dtype=torch.float32, device=hg.device)
    eta = torch.empty(max(hg.n, 1), dtype=torch.float32, device=hg.device)
    nc = C.c_int32(0)
    ws = _workspace(hg, params, _lib.OP_COARSEN)
    check(lib.hef_coarsen(C.byref(hg.c()), C.byref(params.c()), _ptr(cluster), C.byref(nc),
                          _ptr(R0), _ptr(eta), _ptr(ws), ws.numel(), _stream(hg.device)),
          "hef_coarsen")
    return cluster, int(nc.value), R0, eta[:int(nc.value)]


def coarsen_levels(hg: DeviceHypergraph, params: Params):
    """Alg. 2 with the per-level record of hef_coarsen_levels: returns
    (cluster, n_clusters, R0, eta, levels), levels a list of dicts with the
    level's sizes n, m, nnz and its R [m], qh [K], rho [K], label [n] and
    eta [n_next] (device tensors)."""
    lib = load()
    cap = params.levels
    K = params.K
    cluster = torch.empty(hg.n, dtype=torch.int32, device=hg.device)
    R0 = torch.empty(hg.m, dtype=torch.float32, device=hg.device)
    eta = torch.empty(max(hg.n, 1), dtype=torch.float32, device=hg.device)
    Rl = torch.empty((cap, max(hg.m, 1)), dtype=torch.float32, device=hg.device)
    ql = torch.empty((cap, max(K, 1)), dtype=torch.float64, device=hg.device)
    rl = torch.empty((cap, max(K, 1)), dtype=torch.float64, device=hg.device)
    ll = torch.empty((cap, max(hg.n, 1)), dtype=torch.int32, device=hg.device)
    el = torch.empty((cap, max(hg.n, 1)), dtype=torch.float32, device=hg.device)
    hn = np.zeros(cap, dtype=np.int32)
    hm = np.zeros(cap, dtype=np.int32)
    hz = np.zeros(cap, dtype=np.int64)
    tr = _lib.HefLevelTrace()
    tr.cap = cap
    tr.n, tr.m, tr.nnz = hn.ctypes.data, hm.ctypes.data, hz.ctypes.data
    tr.R, tr.qh, tr.rho = _ptr(Rl), _ptr(ql), _ptr(rl)
    tr.label, tr.eta = _ptr(ll), _ptr(el)
    nc = C.c_int32(0)
    ws = _workspace(hg, params, _lib.OP_COARSEN)
    check(lib.hef_coarsen_levels(C.byref(hg.c()), C.byref(params.c()), _ptr(cluster),
                                 C.byref(nc), _ptr(R0), _ptr(eta), C.byref(tr), _ptr(ws),
                                 ws.numel(), _stream(hg.device)), "hef_coarsen_levels")
    levels = []
    for lv in range(tr.levels_run):
        n_next = int(hn[lv + 1]) if lv + 1 < tr.levels_run else int(nc.value)
        levels.append(dict(n=int(hn[lv]), m=int(hm[lv]), nnz=int(hz[lv]),
                           R=Rl[lv, :int(hm[lv])], qh=ql[lv, :K], rho=rl[lv, :K],
                           label=ll[lv, :int(hn[lv])], eta=el[lv, :n_next]))
    return cluster, int(nc.value), R0, eta[:int(nc.value)], levels


def rebuild(hg: DeviceHypergraph, label: torch.Tensor, n_clusters: int):
    """Alg. 2's coarse hypergraph of a clustering, as
    (DeviceHypergraph over n_clusters nodes, kept [m'] int32 input ids)."""
    lib = load()
    assert label.dtype == torch.int32 and label.shape == (hg.n,) and label.is_contiguous()
    eptr = torch.empty(hg.m + 1, dtype=torch.int32, device=hg.device)
    pins = torch.empty(max(hg.nnz, 1), dtype=torch.int32, device=hg.device)
    w = torch.empty(max(hg.m, 1), dtype=torch.float32, device=hg.device)
    kept = torch.empty(max(hg.m, 1), dtype=torch.int32, device=hg.device)
    m2 = C.c_int32(0)
    nnz2 = C.c_int64(0)
    ws = _workspace(hg, Params(), _lib.OP_REBUILD)
    check(lib.hef_rebuild(C.byref(hg.c()), _ptr(label), int(n_clusters), _ptr(eptr), _ptr(pins),
                          _ptr(w), _ptr(kept), C.byref(m2), C.byref(nnz2), _ptr(ws), ws.numel(),
                          _stream(hg.device)), "hef_rebuild")
    m2, nnz2 = int(m2.value), int(nnz2.value)
    out = DeviceHypergraph(int(n_clusters), m2, eptr[:m2 + 1], pins[:nnz2], w[:m2])
    return out, kept[:m2]


def rating(hg: DeviceHypergraph, R: torch.Tensor, shift: float = 0.0):
    """Eq. (17) vertex-pair rating: (best [n] int32, rating [n] float64), the
    neighbour of largest sum of w(e) / (R_e - shift) over shared hyperedges."""
    lib = load()
    assert R.dtype == torch.float32 and R.shape == (hg.m,) and R.is_contiguous()
    best = torch.empty(max(hg.n, 1), dtype=torch.int32, device=hg.device)
    val = torch.empty(max(hg.n, 1), dtype=torch.float64, device=hg.device)
    ws = _workspace(hg, Params(), _lib.OP_RATING)
    check(lib.hef_rating(C.byref(hg.c()), _ptr(R), float(shift), _ptr(best), _ptr(val), _ptr(ws),
                         ws.numel(), _stream(hg.device)), "hef_rating")
    return best[:hg.n], val[:hg.n]


def cluster_level(hg: DeviceHypergraph, params: Params, R: torch.Tensor,
                  eta: torch.Tensor | None, chi: torch.Tensor, qh: torch.Tensor):
    """One level of Alg. 2 from given inputs: (cluster [n], n_clusters, eta_out)."""
    lib = load()
    cluster = torch.empty(hg.n, dtype=torch.int32, device=hg.device)
    eta_out = torch.empty(max(hg.n, 1), dtype=torch.float32, device=hg.device)
    nc = C.c_int32(0)
    ws = _workspace(hg, params, _lib.OP_CLUSTER_LEVEL)
    want = torch.bfloat16 if params.basis == "bf16" else torch.float32
    assert chi.dtype == want and chi.shape == (hg.n, params.K) and chi.is_contiguous()
    check(lib.hef_cluster_level(C.byref(hg.c()), C.byref(params.c()), _ptr(R), _ptr(eta),
                                _ptr(chi), _ptr(qh), _ptr(cluster), C.byref(nc), _ptr(eta_out),
                                _ptr(ws), ws.numel(), _stream(hg.device)), "hef_cluster_level")
    return cluster, int(nc.value), eta_out[:int(nc.value)]


def conductance(hg: DeviceHypergraph, label: torch.Tensor, n_clusters: int):
    """Eq. (3) per cluster and Eq. (18): (cut, vol, phi [n_clusters] float64,
    phi_avg float64 scalar tensor) for the partition label [n] int32."""
    lib = load()
    assert label.dtype == torch.int32 and label.shape == (hg.n,) and label.is_contiguous()
    nc = int(n_clusters)
    out = torch.empty(3 * max(nc, 1) + 1, dtype=torch.float64, device=hg.device)
    cut, vol, phi = out[:nc], out[nc:2 * nc], out[2 * nc:3 * nc]
    avg = out[3 * nc:3 * nc + 1]
    ws = _workspace(hg, Params(), _lib.OP_CONDUCTANCE)
    check(lib.hef_conductance(C.byref(hg.c()), _ptr(label), nc, _ptr(cut), _ptr(vol), _ptr(phi),
                              _ptr(avg), _ptr(ws), ws.numel(), _stream(hg.device)),
          "hef_conductance")
    return cut, vol, phi, avg[0]


def resistance_backward(hg: DeviceHypergraph, params: Params, dR: torch.Tensor,
                        start_star: torch.Tensor | None = None,
                        start_clique: torch.Tensor | None = None,
                        tape: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dw for dL/dR = dR (the adjoint of Alg. 1).  With `tape` (the
    workspace returned by resistance_taped for the same hypergraph and
    params) only the reverse sweep runs."""
    lib = load()
    dw = torch.empty(hg.m, dtype=torch.float32, device=hg.device)
    pc = params.c()
    if tape is not None:
        pc.flags |= _lib.FLAG_TAPED
        ws = tape
    else:
        ws = _workspace(hg, params, _lib.OP_BACKWARD)
    check(lib.hef_resistance_backward(C.byref(hg.c()), C.byref(pc), _ptr(start_star),
                                      _ptr(start_clique), _ptr(dR.contiguous()), _ptr(dw),
                                      _ptr(ws), ws.numel(), _stream(hg.device)),
          "hef_resistance_backward")
    return dw


def resistance_taped(hg: DeviceHypergraph, params: Params, start_star: torch.Tensor | None = None,
                     start_clique: torch.Tensor | None = None):
    """The forward of Alg. 1 (FP32 pool) keeping the adjoint's tape: returns
    (R [m] float32, tape workspace for resistance_backward)."""
    lib = load()
    R = torch.empty(hg.m, dtype=torch.float32, device=hg.device)
    ws = _workspace(hg, params, _lib.OP_BACKWARD)
    check(lib.hef_resistance_taped(C.byref(hg.c()), C.byref(params.c()), _ptr(start_star),
                                   _ptr(start_clique), _ptr(R), _ptr(ws), ws.numel(),
                                   _stream(hg.device)), "hef_resistance_taped")
    return R, ws


class HyperEFResistance(torch.autograd.Function):
    """R = HyperEFResistance.apply(w, hg, params[, start_star, start_clique]):
    resistances as a differentiable function of the hyperedge weights.  The
    forward keeps the Krylov tape in its workspace, so the backward runs only
    the reverse sweep."""

    @staticmethod
    def forward(ctx, w, hg, params, start_star=None, start_clique=None):
        h = DeviceHypergraph(hg.n, hg.m, hg.eptr, hg.pins, w.detach().contiguous())
        R, tape = resistance_taped(h, params, start_star, start_clique)
        ctx.h, ctx.params, ctx.tape = h, params, tape
        ctx.starts = (start_star, start_clique)
        return R

    @staticmethod
    def backward(ctx, dR):
        dw = resistance_backward(ctx.h, ctx.params, dR.float(), *ctx.starts, tape=ctx.tape)
        ctx.tape = None
        return dw, None, None, None, None


def debug_apply(hg: DeviceHypergraph, expansion: int, x: torch.Tensor) -> torch.Tensor:
    """y = A x for the normalised star (0) or clique (1) adjacency."""
    lib = load()
    x = x.contiguous()
    y = torch.empty_like(x)
    ws = _workspace(hg, Params(), _lib.OP_APPLY)
    check(lib.hef_debug_apply(C.byref(hg.c()), expansion, x.shape[1], _ptr(x), _ptr(y), _ptr(ws),
                              ws.numel(), _stream(x.device)), "hef_debug_apply")
    return y


def debug_gram(X: torch.Tensor) -> torch.Tensor:
    """X^T X (float64) through the matrix-core Gram kernels."""
    lib = load()
    X = X.contiguous()
    rows, cols = X.shape
    G = torch.empty((cols, cols), dtype=torch.float64, device=X.device)
    nbytes = int(lib.hef_debug_gram_ws(rows, cols))
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=X.device)
    check(lib.hef_debug_gram(_ptr(X), rows, cols, _ptr(G), _ptr(ws), ws.numel(),
                             _stream(X.device)), "hef_debug_gram")
    return G


def start_block(seed: int, level: int, expansion: int, rows: int, b: int,
                device="cuda") -> torch.Tensor:
    """The counter-generator start block on the device."""
    lib = load()
    out = torch.empty((rows, b), dtype=torch.float32, device=device)
    check(lib.hef_start_block(seed, level, expansion, rows, b, _ptr(out), _stream(out.device)),
          "hef_start_block")
    return out


def validate_host(n, m, eptr, pins, w=None) -> int:
    """Host-side structural validation (no GPU needed); returns the status."""
    lib = load()
    e = np.ascontiguousarray(eptr, dtype=np.int32)
    p = np.ascontiguousarray(pins, dtype=np.int32)
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
    return int(lib.hef_validate_host(n, m, e.ctypes.data, p.ctypes.data,
                                     None if ww is None else ww.ctypes.data))


def last_coarsen_levels() -> list:
    """[(n, m, nnz)] of the levels the calling thread's last coarsen estimated."""
    lib = load()
    cap = 64
    n = (C.c_int32 * cap)()
    m = (C.c_int32 * cap)()
    z = (C.c_int64 * cap)()
    k = lib.hef_last_coarsen_levels(C.cast(n, C.c_void_p), C.cast(m, C.c_void_p),
                                    C.cast(z, C.c_void_p), cap)
    return [(n[i], m[i], z[i]) for i in range(min(k, cap))]


def last_coarsen_work() -> list:
    """Per level of the calling thread's last coarsen: the (isolated node,
    candidate cluster) pairs its best-neighbour search screened."""
    lib = load()
    cap = 64
    w = (C.c_int64 * cap)()
    k = lib.hef_last_coarsen_work(C.cast(w, C.c_void_p), cap)
    return [w[i] for i in range(min(k, cap))]


def timing_enable(on: bool = True) -> None:
    """Per-stage HIP-event timing inside the library (profiling aid)."""
    load().hef_timing_enable(1 if on else 0)


def timing_stages(names=None) -> None:
    """Limit the timing events to the named stages (None: the default, every
    stage but the spmm_step span)."""
    lib = load()
    idx = {lib.hef_timing_stage_name(i).decode(): i for i in range(lib.hef_timing_stage_count())}
    if names is None:
        names = [nm for nm in idx if nm != "spmm_step"]
    mask = 0
    for nm in names:
        mask |= 1 << idx[nm]
    lib.hef_timing_stages(mask)


def timing_read(reset: bool = True) -> dict:
    """{stage: (total ms, launches)} of the stages timed since the last reset."""
    lib = load()
    n = lib.hef_timing_stage_count()
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    check(lib.hef_timing_read(C.cast(ms, C.c_void_p), C.cast(cnt, C.c_void_p), n, int(reset)),
          "hef_timing_read")
    return {lib.hef_timing_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}
