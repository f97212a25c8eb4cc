"""The benchmark's algorithmic counts (the numerators of its rooflines) against
counts written out by enumeration on small shapes, and the figure quoted for
the large2m fused Krylov step; the roofline arithmetic, including a kernel
that was not timed."""
import math

import pytest

import bench


def test_gram_flops_counts_the_tiles_on_and_above_the_diagonal():
    for K in (1, 31, 32, 33, 100, 480, 512):
        T = math.ceil(K / 32)
        tiles = sum(1 for i in range(T) for j in range(T) if j >= i)
        assert bench.gram_flops(7, K) == 2.0 * 7 * 32 * 32 * tiles


def test_apply_flops_counts_the_upper_triangle():
    # column j of R^-1 has j + 1 nonzeros: j + 1 multiply-adds (2 flops
    # each) per row
    for K in (1, 5, 480):
        assert bench.apply_flops(3, K) == 2 * 3 * sum(j + 1 for j in range(K))


def test_lanczos_bytes_block_counts():
    # step j of k reads min(j + 1, 3) blocks of b columns, both expansions
    n, m, b, k = 10, 7, 4, 6
    gram, _ = bench.lanczos_bytes(n, m, b, k)
    rows = (n + m) + n
    assert gram == 4 * b * rows * sum(min(j + 1, 3) for j in range(k + 1))


def test_spmm_step_bytes_at_large2m():
    # the 715 MB per fused Krylov step quoted for level 0 of large2m
    got = bench.spmm_step_bytes(2_000_000, 2_200_000, 7_907_430, 8)
    assert got == pytest.approx(715e6, rel=5e-3)


def test_roofline_entry_rates_and_untimed_kernels():
    e = bench.roofline_entry("hbm", 2e9, 1.0, 4, 8000.0, "GB/s", ["k"])
    assert e["achieved"] == pytest.approx(2000.0) and e["frac"] == pytest.approx(0.25)
    assert e["avg_launch_us"] == pytest.approx(250.0)
    f = bench.roofline_entry("mfma", 3e12, 10.0, 1, 157.3, "TFLOP/s", ["k"])
    assert f["achieved"] == pytest.approx(300.0)
    z = bench.roofline_entry("hbm", 1e9, 0.0, 0, 8000.0, "GB/s", ["k"])
    assert z["achieved"] == 0.0 and z["frac"] == 0.0
