"""Seeded synthetic inputs for the PPO learning hot path.

This package only draws random numbers and lays them out; it holds none of the
method's arithmetic (no network evaluation, no advantage estimation, no loss).
Both the FP64 oracle and the HIP path consume what it produces, so neither side
can bias the other through its inputs.
"""
from .configs import CONFIGS, NetShape, PPOConfig, get_config
from .rollout import (
    make_rollout,
    make_permutations,
    xavier_theta,
    flat_layout,
)
from .heightfield import HeightField

__all__ = [
    "CONFIGS",
    "NetShape",
    "PPOConfig",
    "get_config",
    "make_rollout",
    "make_permutations",
    "xavier_theta",
    "flat_layout",
    "HeightField",
]
