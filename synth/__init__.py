"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the resistance-estimation method: it only
draws hypergraphs and random start blocks.  Both the CPU oracle and the HIP
path consume what it produces; neither imports the other.
"""
from .rng import splitmix64, start_block, std_normal_counter  # noqa: F401
from .hypergraph import Hypergraph, generate, size_law  # noqa: F401
from .configs import CONFIGS, get_config, make_hypergraph  # noqa: F401
