"""Workload shapes of the massively parallel PPO set-up.

Batch arithmetic follows the paper's Section 2.2.1 (B = n_robots * n_steps) and
the hyper-parameter table of Appendix A.4 (Table 3): B = 98304 (4096 x 24),
mini-batch 24576, 5 epochs, clip 0.2, entropy coefficient 0.01, gamma 0.99,
lambda 0.95.  Network widths, the activation, the learning rate and the
gradient-norm limit are not given in the paper; the values below are the
workload definitions this project benchmarks.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple


@dataclass(frozen=True)
class NetShape:
    obs_dim: int
    act_dim: int
    hidden: Tuple[int, ...]

    @property
    def actor_dims(self) -> List[int]:
        return [self.obs_dim, *self.hidden, self.act_dim]

    @property
    def critic_dims(self) -> List[int]:
        return [self.obs_dim, *self.hidden, 1]


@dataclass(frozen=True)
class PPOConfig:
    name: str
    n_envs: int
    n_steps: int
    net: NetShape
    epochs: int
    minibatches: int
    gamma: float = 0.99
    lam: float = 0.95
    clip: float = 0.2
    entropy_coef: float = 0.01
    value_coef: float = 1.0
    lr: float = 1e-3
    max_grad_norm: float = 1.0
    reward_std: float = 0.1
    done_prob: float = 1e-3
    heightfield: bool = False
    seed: int = 0

    @property
    def batch(self) -> int:
        return self.n_envs * self.n_steps

    @property
    def minibatch(self) -> int:
        assert self.batch % self.minibatches == 0
        return self.batch // self.minibatches


TINY = PPOConfig(
    name="tiny_64x24_d48_h64x64",
    n_envs=64, n_steps=24, net=NetShape(48, 12, (64, 64)),
    epochs=1, minibatches=1, done_prob=0.02,
)
FLAT = PPOConfig(
    name="flat_4096x24_d48_h512x256x128",
    n_envs=4096, n_steps=24, net=NetShape(48, 12, (512, 256, 128)),
    epochs=5, minibatches=4,
)
ROUGH = PPOConfig(
    name="rough_4096x24_d235_h512x256x128",
    n_envs=4096, n_steps=24, net=NetShape(235, 12, (512, 256, 128)),
    epochs=5, minibatches=4, heightfield=True,
)
LARGE = PPOConfig(
    name="large_16384x24_d235_h1024x512x256",
    n_envs=16384, n_steps=24, net=NetShape(235, 12, (1024, 512, 256)),
    epochs=5, minibatches=8, heightfield=True,
)

# Eight independent sweep-style runs of uneven size, updated together.
SWEEP_ENVS = (512, 1024, 2048, 3072, 4096, 6144, 8192, 8192)
SWEEP_STEPS = (16, 24, 24, 32, 32, 48, 24, 50)


def sweep_runs() -> List[PPOConfig]:
    runs = []
    for r, (n, t) in enumerate(zip(SWEEP_ENVS, SWEEP_STEPS)):
        d = 48 if r % 2 == 0 else 235
        runs.append(PPOConfig(
            name=f"sweep_run{r}_{n}x{t}_d{d}",
            n_envs=n, n_steps=t, net=NetShape(d, 12, (512, 256, 128)),
            epochs=5, minibatches=4, heightfield=(d == 235), seed=r,
        ))
    return runs


# Fig. 4's shapes: at a fixed batch size the number of environments grows from
# 128 to 16384 (T = B / N), next to the 20000 x 50 reference point.  Rough-terrain
# network width; observations are all N(0, 1) here since only timings are taken.
FIG4_BATCHES = (49152, 98304, 196608)
FIG4_ENVS = (128, 256, 512, 1024, 2048, 4096, 8192, 16384)


def fig4_runs() -> List[PPOConfig]:
    runs = []
    for b in FIG4_BATCHES:
        for n in FIG4_ENVS:
            runs.append(PPOConfig(name=f"fig4_b{b}_{n}x{b // n}_d235", n_envs=n, n_steps=b // n,
                                  net=NetShape(235, 12, (512, 256, 128)), epochs=5, minibatches=4))
    runs.append(PPOConfig(name="fig4_20000x50_d235", n_envs=20000, n_steps=50,
                          net=NetShape(235, 12, (512, 256, 128)), epochs=5, minibatches=4))
    return runs


CONFIGS = {c.name: c for c in (TINY, FLAT, ROUGH, LARGE)}
ALIASES = {"tiny": TINY.name, "flat": FLAT.name, "rough": ROUGH.name, "large": LARGE.name}


def get_config(name: str) -> PPOConfig:
    return CONFIGS[ALIASES.get(name, name)]
