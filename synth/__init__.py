"""Seeded synthetic inputs shared by the tests, the benchmark and the
oracle checks.  Holds no part of the matching method."""
from .configs import CONFIGS, Pair, PairSpec, make_pair, rest_mesh, tiny_pair  # noqa: F401
from .ilp import generic_ilp  # noqa: F401
