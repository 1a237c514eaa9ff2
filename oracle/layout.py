"""Flat parameter layout, as the oracle reads it.

Test infrastructure only (see the package docstring).

The paper fixes no network (Section 2.2 and Appendix A.1 only speak of a
policy and a critic).  This project uses separate actor and critic MLPs with
no shared trunk.  The flat vector holds, in order: actor W1, b1, ..., WL, bL,
the actor's state-independent log standard deviations, then critic W1, b1,
..., WL, bL.  Each W is row-major [out, in].  This is an interface that the
HIP library also implements (independently); tests compare the two.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class NetSpec:
    obs_dim: int
    act_dim: int
    hidden: Tuple[int, ...]

    def dims(self, which: str) -> List[int]:
        out = self.act_dim if which == "actor" else 1
        return [self.obs_dim, *self.hidden, out]


def param_layout(spec: NetSpec) -> Dict[str, Tuple[int, Tuple[int, ...]]]:
    """name -> (offset, shape) for every tensor in the flat vector."""
    table = {}
    pos = 0
    for which in ("actor", "critic"):
        d = spec.dims(which)
        for l in range(1, len(d)):
            table[f"{which}.W{l}"] = (pos, (d[l], d[l - 1]))
            pos += d[l] * d[l - 1]
            table[f"{which}.b{l}"] = (pos, (d[l],))
            pos += d[l]
        if which == "actor":
            table["actor.logstd"] = (pos, (spec.act_dim,))
            pos += spec.act_dim
    table["__total__"] = (pos, ())
    return table


def unpack(theta: np.ndarray, spec: NetSpec):
    """Views of the flat vector as float64 arrays.

    Returns (actor_layers, logstd, critic_layers) where each *_layers is a
    list of (W, b) pairs.
    """
    theta = np.asarray(theta, dtype=np.float64)
    lay = param_layout(spec)
    assert theta.shape == (lay["__total__"][0],), (theta.shape, lay["__total__"])

    def get(name):
        off, shp = lay[name]
        size = int(np.prod(shp))
        return theta[off:off + size].reshape(shp)

    nets = {}
    for which in ("actor", "critic"):
        n_layers = len(spec.dims(which)) - 1
        nets[which] = [(get(f"{which}.W{l}"), get(f"{which}.b{l}")) for l in range(1, n_layers + 1)]
    return nets["actor"], get("actor.logstd"), nets["critic"]
