"""Seeded inputs: generator statistics and the start-block counter generator."""
import numpy as np

from synth import generate, make_hypergraph, size_law, splitmix64, start_block
from synth.configs import graph_2uniform


def test_splitmix64_published_sequence():
    # SplitMix64 from state 0 (Steele, Lea, Flood 2014; Vigna's reference
    # splitmix64.c): the first three outputs.
    gamma = 0x9E3779B97F4A7C15
    outs = [splitmix64((i * gamma) % (1 << 64)) for i in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_start_block_is_standard_normal_and_counter_based():
    x = start_block(7, 0, 0, 200_000, 1).ravel()
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1) < 0.01
    # fourth moment of N(0,1) is 3
    assert abs((x ** 4).mean() - 3) < 0.05
    # the block is a window of one flat stream: rows x b reshapes agree
    a = start_block(7, 0, 1, 100, 4).ravel()
    b = start_block(7, 0, 1, 50, 8).ravel()
    assert np.array_equal(a, b)
    # streams for different (level, expansion, seed) differ
    c = start_block(7, 1, 1, 100, 4).ravel()
    d = start_block(8, 0, 1, 100, 4).ravel()
    assert not np.allclose(a, c) and not np.allclose(a, d)


def test_size_law_means():
    s, p = size_law(2, 20, 2.5)
    assert abs((s * p).sum() - 3.50) < 0.01
    s, p = size_law(2, 2000, 2.7828)
    assert abs((s * p).sum() - 3.60) < 0.01


def test_generated_hypergraph_layout():
    h = make_hypergraph("tiny2k")
    assert h.n == 2000 and h.m == 2000
    sz = h.sizes()
    assert sz.min() >= 2 and sz.max() <= 20
    assert abs(sz.mean() - 3.5) < 0.25
    for e in range(h.m):
        mem = h.pins[h.eptr[e]:h.eptr[e + 1]]
        assert (np.diff(mem) > 0).all()
    assert h.pins.min() >= 0 and h.pins.max() < h.n
    assert (h.w == 1).all()


def test_netlist_locality_and_weights():
    h = generate(20000, 21000, 2, 2000, 2.7828, p_loc=0.7, weights="lognormal", seed=3)
    sz = h.sizes()
    assert abs(sz.mean() - 3.6) < 0.15
    # roughly 70% of pins of small nets lie within 500 ids of the net's median pin
    eid = h.edge_ids()
    small = sz[eid] <= 8
    med = np.array([np.median(h.pins[h.eptr[e]:h.eptr[e + 1]]) for e in range(h.m)])
    dist = np.abs(h.pins[small] - med[eid[small]])
    dist = np.minimum(dist, h.n - dist)
    assert (dist < 1000).mean() > 0.6
    lw = np.log(h.w.astype(np.float64))
    assert abs(lw.mean()) < 0.02 and abs(lw.std() - 0.5) < 0.02
    for e in np.nonzero(sz > 100)[0]:
        mem = h.pins[h.eptr[e]:h.eptr[e + 1]]
        assert np.unique(mem).size == mem.size


def test_generator_is_seeded():
    a = generate(5000, 5000, seed=11)
    b = generate(5000, 5000, seed=11)
    assert np.array_equal(a.pins, b.pins) and np.array_equal(a.eptr, b.eptr)


def test_two_uniform_graph():
    g = graph_2uniform(30, 60)
    assert (g.sizes() == 2).all() and g.m == 60
