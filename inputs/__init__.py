"""Seeded synthetic inputs for the Sneddon-type workloads.

This module is shared by the oracle, the tests and the benchmark. It holds
no arithmetic of the method itself: it only turns (seed, stream, integer
lattice coordinates) into pseudo-random numbers and states which lattice
points lie on the prescribed crack. Because every value is a pure function
of the node's integer coordinates, two implementations that number their
nodes differently still receive identical inputs.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) applied to a counter built from the seed,
the stream id and the coordinates. Normals use the Box-Muller transform.
"""
from .sneddon import (
    splitmix64,
    uniform01,
    normal,
    crack_mask,
    sneddon_state,
    random_vector,
    bernoulli_mask,
    WorkloadSpec,
    WORKLOADS,
)

__all__ = [
    "splitmix64",
    "uniform01",
    "normal",
    "crack_mask",
    "sneddon_state",
    "random_vector",
    "bernoulli_mask",
    "WorkloadSpec",
    "WORKLOADS",
]
