"""Seeded synthetic inputs for the batched 2x2 SVD and the Kogbetliantz solver.

This module holds none of the SVD method's arithmetic: it only draws numbers.
Both the CPU oracle (through the tests) and the GPU path consume what it
produces.  Everything is deterministic in the seed (numpy PCG64).
"""
from .gen import (  # noqa: F401
    SEED_BASE, KINDS, uniform_real, scaled_law, random_bits, to_trains, kog_matrix,
    kog_problem_set, kog_problem_set_device, round_robin_pairs,
)
