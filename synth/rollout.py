"""Seeded rollout tensors, initial parameters and epoch permutations.

Everything is drawn from numpy's PCG64 streams spawned from one SeedSequence
per workload, so a workload name plus a seed fixes every array bit for bit.
Layouts are the ones the learner stores (Section 2.2, all data kept on the
device): time-major [T, N, ...] with the environment index contiguous.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .configs import NetShape, PPOConfig
from .heightfield import HeightField, SCAN_X, SCAN_Y

PROPRIO_DIM = 48


def _streams(seed: int, n: int) -> List[np.random.Generator]:
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def flat_layout(net: NetShape) -> List[Tuple[str, Tuple[int, ...], int]]:
    """Parameter order of the flat parameter vector.

    Actor layers W1, b1, ..., W_L, b_L (W row-major [out, in]), the actor's
    log standard deviations [A], then the critic's layers in the same order.
    """
    entries = []
    off = 0
    for prefix, dims in (("actor", net.actor_dims), ("critic", net.critic_dims)):
        for l in range(len(dims) - 1):
            shp = (dims[l + 1], dims[l])
            entries.append((f"{prefix}.W{l + 1}", shp, off))
            off += shp[0] * shp[1]
            entries.append((f"{prefix}.b{l + 1}", (dims[l + 1],), off))
            off += dims[l + 1]
        if prefix == "actor":
            entries.append(("actor.logstd", (net.act_dim,), off))
            off += net.act_dim
    return entries


def param_count(net: NetShape) -> int:
    name, shp, off = flat_layout(net)[-1]
    return off + int(np.prod(shp))


def xavier_theta(net: NetShape, seed: int = 0, logstd: float = 0.0) -> np.ndarray:
    """Flat float32 parameters: Xavier-uniform weights, zero biases.

    W ~ U(-a, a) with a = sqrt(6 / (fan_in + fan_out)); biases 0; log-std set
    to `logstd` (0 means unit exploration noise).
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5EED])))
    theta = np.zeros(param_count(net), dtype=np.float32)
    for name, shp, off in flat_layout(net):
        size = int(np.prod(shp))
        if ".W" in name:
            fan_out, fan_in = shp
            a = np.sqrt(6.0 / (fan_in + fan_out))
            theta[off:off + size] = rng.uniform(-a, a, size=size).astype(np.float32)
        elif name == "actor.logstd":
            theta[off:off + size] = np.float32(logstd)
    return theta


def _observations(cfg: PPOConfig, rng: np.random.Generator, hf, count: int) -> np.ndarray:
    d = cfg.net.obs_dim
    obs = np.empty((count, d), dtype=np.float32)
    if cfg.heightfield:
        assert d == PROPRIO_DIM + SCAN_X * SCAN_Y, d
        obs[:, :PROPRIO_DIM] = rng.standard_normal((count, PROPRIO_DIM), dtype=np.float32)
        obs[:, PROPRIO_DIM:] = hf.scan(rng, count)
    else:
        obs[:] = rng.standard_normal((count, d), dtype=np.float32)
    return obs


def make_rollout(cfg: PPOConfig, seed: int | None = None,
                 with_timeouts: bool = False) -> Dict[str, np.ndarray]:
    """Synthetic rollout storage for one iteration.

    obs [T, N, D] (proprioception ~N(0,1); for rough-terrain shapes the last
    187 columns are height samples from a seeded heightfield), last_obs [N, D]
    (the observation after the final step), rewards [T, N] ~ N(0, 0.1^2),
    dones [T, N] ~ Bernoulli(p) as uint8, and optionally timeouts [T, N]
    (uint8, a subset of dones chosen with probability 1/2).
    """
    seed = cfg.seed if seed is None else seed
    r_obs, r_rew, r_done, r_to, r_last = _streams(seed, 5)
    T, N, D = cfg.n_steps, cfg.n_envs, cfg.net.obs_dim
    hf = HeightField(seed) if cfg.heightfield else None
    obs = _observations(cfg, r_obs, hf, T * N).reshape(T, N, D)
    last_obs = _observations(cfg, r_last, hf, N)
    rewards = (r_rew.standard_normal((T, N)) * cfg.reward_std).astype(np.float32)
    dones = (r_done.random((T, N)) < cfg.done_prob).astype(np.uint8)
    out = dict(obs=obs, last_obs=last_obs, rewards=rewards, dones=dones)
    if with_timeouts:
        out["timeouts"] = (dones.astype(bool) & (r_to.random((T, N)) < 0.5)).astype(np.uint8)
    return out


def make_permutations(batch: int, epochs: int, seed: int = 0) -> np.ndarray:
    """One permutation of [0, B) per epoch, int32 [E, B]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x9E12])))
    return np.stack([rng.permutation(batch).astype(np.int32) for _ in range(epochs)])


def gaussian_like(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2) float32 array (used for teacher-forced test inputs)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x6A55])))
    return (rng.standard_normal(shape) * scale).astype(np.float32)
