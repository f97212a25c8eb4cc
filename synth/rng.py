"""Counter-based N(0,1) generator for the random Krylov start blocks.

The start vectors x of the Krylov subspaces (Eq. (12): "x is a random vector")
are drawn from this generator.  It is a pure function of
(seed, level, expansion, row, col), so any party that implements the same
published definition gets the same numbers without sharing code:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): ``splitmix64(x) = mix(x + 0x9E3779B97F4A7C15)``
  with ``mix(z) = z3`` where ``z1 = (z ^ z>>30) * 0xBF58476D1CE4E5B9``,
  ``z2 = (z1 ^ z1>>27) * 0x94D049BB133111EB``, ``z3 = z2 ^ z2>>31``, all
  arithmetic modulo 2**64.
* Stream key ``h = splitmix64(splitmix64(seed) + 2*level + expansion)``
  (expansion 0 = star, 1 = clique).
* Element ``i = row*b + col`` of a rows x b block:
  ``a = splitmix64(h + 2i)``, ``c = splitmix64(h + 2i + 1)``,
  ``u1 = ((a >> 11) + 1) * 2**-53`` in (0, 1], ``u2 = (c >> 11) * 2**-53``
  in [0, 1).
* Box-Muller (Box and Muller, 1958): ``z = sqrt(-2 ln u1) * cos(2 pi u2)``,
  evaluated in float64.

The HIP library implements the same definition on the device for calls that
pass no explicit start block.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STAR = 0
CLIQUE = 1


def splitmix64(x):
    """SplitMix64 output for state(s) ``x`` (numpy uint64 array or int)."""
    scalar = np.isscalar(x) or isinstance(x, int)
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return int(z) if scalar else z


def stream_key(seed: int, level: int, expansion: int) -> int:
    base = splitmix64(np.uint64(seed % (1 << 64)))
    return (int(base) + 2 * int(level) + int(expansion)) % (1 << 64)


def std_normal_counter(seed: int, level: int, expansion: int, first: int, count: int) -> np.ndarray:
    """Elements ``first .. first+count-1`` of the flat N(0,1) stream, float64."""
    h = np.uint64(splitmix64(np.uint64(stream_key(seed, level, expansion))))
    i = np.arange(first, first + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        a = splitmix64(h + np.uint64(2) * i)
        c = splitmix64(h + np.uint64(2) * i + np.uint64(1))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (c >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def start_block(seed: int, level: int, expansion: int, rows: int, b: int,
                dtype=np.float64, chunk: int = 1 << 24) -> np.ndarray:
    """A rows x b start block (row-major), element (r, c) = stream[r*b + c]."""
    total = rows * b
    out = np.empty(total, dtype=dtype)
    for lo in range(0, total, chunk):
        hi = min(total, lo + chunk)
        out[lo:hi] = std_normal_counter(seed, level, expansion, lo, hi - lo)
    return out.reshape(rows, b)
