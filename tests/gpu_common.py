"""Shared helpers of the GPU tests: seeded inputs on the device and the
parity measures of the resistance estimate."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2511_06600_amd as hef
from synth import start_block


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(h):
    return hef.DeviceHypergraph.from_arrays(h.n, h.m, h.eptr, h.pins, h.w)


def starts(h, b, seed=7, level=0):
    """Start blocks from the shared counter generator (float64 for the oracle,
    float32 device copies of the same values for the library)."""
    Xs = start_block(seed, level, 0, h.n + h.m, b)
    Xc = start_block(seed, level, 1, h.n, b)
    xs = torch.as_tensor(Xs.astype(np.float32), device="cuda")
    xc = torch.as_tensor(Xc.astype(np.float32), device="cuda")
    # the oracle sees exactly the float32 values the library sees
    return Xs.astype(np.float32).astype(np.float64), Xc.astype(np.float32).astype(np.float64), xs, xc


def r_errors(R_gpu: np.ndarray, R_ref: np.ndarray):
    """(norm-relative error, 99.9th percentile and max of the elementwise
    relative error over non-degenerate hyperedges R >= 1e-3 max R)."""
    R_gpu = np.asarray(R_gpu, dtype=np.float64)
    norm = np.linalg.norm(R_gpu - R_ref) / np.linalg.norm(R_ref)
    nz = R_ref >= 1e-3 * R_ref.max()
    rel = np.abs(R_gpu[nz] - R_ref[nz]) / R_ref[nz]
    return float(norm), float(np.quantile(rel, 0.999)), float(rel.max())
