"""Philox4x32-10 counter-based generator and the Gaussian action noise.

Test infrastructure only (see the package docstring).

The paper does not say how exploration noise is drawn (Section 2.2 only says
the learner is a custom GPU PPO).  This project draws it from Philox4x32-10
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11), written here from that paper's definition:

  * state: four 32-bit counter words c0..c3, two 32-bit key words k0, k1;
  * one round multiplies c0 by 0xD2511F53 and c2 by 0xCD9E8D57 into 64-bit
    products (hi, lo) and forms (hi_b ^ c1 ^ k0, lo_b, hi_a ^ c3 ^ k1, lo_a),
    where a is the c0 product and b the c2 product;
  * the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) modulo
    2^32 between rounds; ten rounds in total.

Uniforms use the top 23 bits plus half a step, u = ((x >> 9) + 1/2) * 2^-23,
which needs 24 significand bits, so it is exact in float32 as well as in
float64, and it is never 0 or 1.  Normals come in pairs from the
Box-Muller transform (Box and Muller, 1958): r = sqrt(-2 ln u_a),
e_a = r cos(2 pi u_b), e_b = r sin(2 pi u_b).

Counter layout for the action noise of env n, action group g (4 dims each),
rollout step t, iteration it:  (n * ceil(A/4) + g, t, it mod 2^32, TAG_ACTION);
key = (seed mod 2^32, seed >> 32).  Dimension j = 4 g + i takes normal i of its
block; draws past A are discarded.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
MUL_A = np.uint64(0xD2511F53)
MUL_B = np.uint64(0xCD9E8D57)
WEYL_0 = np.uint64(0x9E3779B9)
WEYL_1 = np.uint64(0xBB67AE85)
ROUNDS = 10
TAG_ACTION = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds; inputs are integer arrays (or scalars) < 2^32.

    Returns four uint32 arrays broadcast to a common shape.
    """
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for _ in range(ROUNDS):
        prod_a = MUL_A * c0          # < 2^64, exact in uint64
        prod_b = MUL_B * c2
        hi_a, lo_a = prod_a >> np.uint64(32), prod_a & MASK32
        hi_b, lo_b = prod_b >> np.uint64(32), prod_b & MASK32
        c0, c1, c2, c3 = (hi_b ^ c1 ^ k0), lo_b, (hi_a ^ c3 ^ k1), lo_a
        k0 = (k0 + WEYL_0) & MASK32
        k1 = (k1 + WEYL_1) & MASK32
    shape = np.broadcast(c0, c1, c2, c3).shape
    return tuple(np.broadcast_to(v, shape).astype(np.uint32) for v in (c0, c1, c2, c3))


def uniforms(x):
    """Map uint32 draws to (0, 1): ((x >> 9) + 0.5) / 2^23, in float64."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def box_muller(u_a, u_b):
    """Two independent standard normals from two uniforms in (0, 1)."""
    r = np.sqrt(-2.0 * np.log(u_a))
    return r * np.cos(2.0 * np.pi * u_b), r * np.sin(2.0 * np.pi * u_b)


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def action_noise(seed: int, n_envs: int, act_dim: int, t: int, iteration: int,
                 return_raw: bool = False):
    """Standard-normal exploration noise eps[n, j] for one rollout step."""
    groups = (act_dim + 3) // 4
    k0, k1 = seed_key(seed)
    n = np.arange(n_envs, dtype=np.uint64)[:, None]
    g = np.arange(groups, dtype=np.uint64)[None, :]
    ctr0 = n * np.uint64(groups) + g
    x0, x1, x2, x3 = philox4x32_10(ctr0, t, int(iteration) & 0xFFFFFFFF, TAG_ACTION, k0, k1)
    u0, u1, u2, u3 = (uniforms(x) for x in (x0, x1, x2, x3))
    e0, e1 = box_muller(u0, u1)
    e2, e3 = box_muller(u2, u3)
    eps = np.stack([e0, e1, e2, e3], axis=-1).reshape(n_envs, groups * 4)[:, :act_dim]
    if return_raw:
        raw = np.stack([x0, x1, x2, x3], axis=-1).reshape(n_envs, groups * 4)
        return eps, raw
    return eps
