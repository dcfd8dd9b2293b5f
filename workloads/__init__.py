"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This package builds *inputs* only: cloth-like triangle-mesh trajectories that stand in for the
simulator's output, observed point clouds, uniform random words for the sampler, request mixes
for the serving loop. It contains no part of the method's arithmetic (no area weighting, no
inverse-CDF face choice, no barycentric sampling, no nearest-neighbour search, no gradients).
"""
from .gen import (  # noqa: F401
    CONFIGS,
    grid_mesh,
    trajectory,
    observed_cloud,
    sim_uniform_words,
    fd_vertices,
    serving_requests,
    workload,
)
