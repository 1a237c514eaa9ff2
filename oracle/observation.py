"""Observation assembly in front of policy inference: the proprioceptive part,
terrain heights sampled around the robot's base, and uniform observation noise.

Test infrastructure only (see the package docstring).

What the paper fixes (Section 3.2, observations; appendix, Table 4, noise
scales): the policy sees proprioceptive measurements followed by terrain
heights sampled on a grid around the base, each the distance between the
terrain surface and the base height; every element gets additive noise drawn
uniformly with a per-component scale.

Readings where the paper is silent (all of them listed with the design notes):
  * the terrain is a height field on a uniform grid (the simulation section
    describes heights on a uniform grid): cell (i, j) holds the height at world
    (i / inv_res, j / inv_res);
  * the scan pattern is a list of body-frame (x, y) offsets, rotated by the
    base heading (yaw only, given as the unit vector (cos, sin)) and translated
    to the base position; a scan point reads the grid cell nearest to it,
    clamped to the grid;
  * the measurement is base_z - h(point), unclipped;
  * noise for column j is scale_j * (2u - 1), uniform on (-scale_j, scale_j),
    with u from Philox4x32-10 at counter (n * ceil(D / 4) + g, t,
    iteration mod 2^32, TAG_OBS_NOISE) for column j = 4 g + i (draw i).

The cell index is a decision that floating point takes, so it is taken in the
device kernel's precision: each of wx = x + (c px - s py) and
wy = y + (s px + c py) is evaluated in float32 with every product and sum
rounded on its own (no fused multiply-add), and the cell is
rint(w * inv_res) in float32 (round half to even), then clamped.  The heights,
the difference and the noise are evaluated in float64.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10, seed_key, uniforms

TAG_OBS_NOISE = 2


def scan_world_points(base: np.ndarray, scan: np.ndarray):
    """World (x, y) of every scan point of every robot, in float32.

    base: [N, 5] (x, y, z, cos(yaw), sin(yaw)); scan: [S, 2] body-frame
    offsets.  Returns wx, wy of shape [N, S].
    """
    f = np.float32
    base = np.asarray(base, dtype=f)
    scan = np.asarray(scan, dtype=f)
    x, y = base[:, 0:1], base[:, 1:2]
    c, s = base[:, 3:4], base[:, 4:5]
    px, py = scan[None, :, 0], scan[None, :, 1]
    # numpy float32 arithmetic rounds each operation on its own
    cx = (c * px).astype(f)
    sy = (s * py).astype(f)
    sx = (s * px).astype(f)
    cy = (c * py).astype(f)
    wx = (x + (cx - sy).astype(f)).astype(f)
    wy = (y + (sx + cy).astype(f)).astype(f)
    return wx, wy


def nearest_cells(wx, wy, inv_res: float, nx: int, ny: int):
    """Index of the grid cell nearest to each world point, clamped to the grid
    (for a rectangular grid the nearest cell of an outside point is the
    clamped one).  The rounding is float32 round-half-to-even."""
    f = np.float32
    r = f(inv_res)
    gi = np.rint((np.asarray(wx, dtype=f) * r).astype(f))
    gj = np.rint((np.asarray(wy, dtype=f) * r).astype(f))
    # fmax/fmin ignore a NaN operand, so a NaN position reads cell 0
    gi = np.fmin(np.fmax(gi, f(0)), f(nx - 1)).astype(np.int64)
    gj = np.fmin(np.fmax(gj, f(0)), f(ny - 1)).astype(np.int64)
    return gi, gj


def height_scan(base: np.ndarray, height: np.ndarray, inv_res: float, scan: np.ndarray) -> np.ndarray:
    """base_z - h(nearest cell of each scan point): [N, S] float64."""
    height = np.asarray(height)
    nx, ny = height.shape
    wx, wy = scan_world_points(base, scan)
    gi, gj = nearest_cells(wx, wy, inv_res, nx, ny)
    z = np.asarray(base, dtype=np.float64)[:, 2:3]
    return z - height.astype(np.float64)[gi, gj]


def obs_noise_unit(seed: int, n_envs: int, dim: int, t: int, iteration: int) -> np.ndarray:
    """2u - 1 for every element of the [N, D] observation, float64 (exact)."""
    groups = (dim + 3) // 4
    k0, k1 = seed_key(seed)
    n = np.arange(n_envs, dtype=np.uint64)[:, None]
    g = np.arange(groups, dtype=np.uint64)[None, :]
    x = philox4x32_10(n * np.uint64(groups) + g, t, int(iteration) & 0xFFFFFFFF, TAG_OBS_NOISE, k0, k1)
    u = np.stack([uniforms(v) for v in x], axis=-1).reshape(n_envs, groups * 4)[:, :dim]
    return 2.0 * u - 1.0


def assemble_obs(proprio: np.ndarray, base: np.ndarray, height, inv_res: float, scan, noise_scale,
                 seed: int, t: int, iteration: int) -> np.ndarray:
    """[N, P + S] float64: proprioception, then the height scan, plus noise.

    height/scan may be None for S = 0; noise_scale None means no noise.
    """
    proprio = np.asarray(proprio, dtype=np.float64)
    N, P = proprio.shape
    parts = [proprio]
    if scan is not None and len(scan) > 0:
        parts.append(height_scan(base, height, inv_res, scan))
    obs = np.concatenate(parts, axis=1)
    if noise_scale is not None:
        scale = np.asarray(noise_scale, dtype=np.float64)
        obs = obs + scale[None, :] * obs_noise_unit(seed, N, obs.shape[1], t, iteration)
    return obs
