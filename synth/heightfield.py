"""Seeded 2-D heightfield used only to shape rough-terrain observations.

The paper's terrain (Section 3.1) is built from 8 m square tiles of several
types (random rough ground, slopes, stairs) laid out side by side, and the
policy observes terrain heights sampled on a grid around the base
(Section 3.2).  This module builds a small stand-in of that kind: each tile
gets uniform noise of +-5 cm plus either a pyramid slope of up to 0.4 rad or
pyramid stairs with 15 cm risers.  It generates inputs only: nothing here is
part of the learning path.
"""
from __future__ import annotations

import numpy as np

RES = 0.1          # metres per cell
TILE = 8.0         # metres per tile side
SCAN_X = 17        # samples along the body x axis
SCAN_Y = 11        # samples along the body y axis
SCAN_SPACING = 0.1


class HeightField:
    def __init__(self, seed: int, tiles: int = 6):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x4846])))
        cells = int(round(TILE / RES))
        n = tiles * cells
        h = rng.uniform(-0.05, 0.05, size=(n, n))
        ii, jj = np.meshgrid(np.arange(cells), np.arange(cells), indexing="ij")
        centre = (cells - 1) / 2.0
        # Chebyshev distance from the tile centre, in metres.
        dist = np.maximum(np.abs(ii - centre), np.abs(jj - centre)) * RES
        for a in range(tiles):
            for b in range(tiles):
                kind = rng.integers(0, 2)
                if kind == 0:
                    slope = rng.uniform(0.0, 0.4)
                    tile = np.tan(slope) * (TILE / 2 - dist)
                else:
                    step_w = 0.3
                    tile = 0.15 * np.floor((TILE / 2 - dist) / step_w)
                h[a * cells:(a + 1) * cells, b * cells:(b + 1) * cells] += tile
        self.h = h.astype(np.float64)
        self.size = n * RES
        self._rng_seed = seed

    def lookup(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        n = self.h.shape[0]
        i = np.clip(np.rint(x / RES).astype(np.int64), 0, n - 1)
        j = np.clip(np.rint(y / RES).astype(np.int64), 0, n - 1)
        return self.h[i, j]

    def scan(self, rng: np.random.Generator, count: int) -> np.ndarray:
        """Height samples for `count` random base poses: [count, 187] float32.

        Each value is the height of the robot base above the sampled terrain
        point minus the nominal 0.5 m standing height.
        """
        margin = 2.0
        bx = rng.uniform(margin, self.size - margin, size=count)
        by = rng.uniform(margin, self.size - margin, size=count)
        yaw = rng.uniform(-np.pi, np.pi, size=count)
        gx = (np.arange(SCAN_X) - (SCAN_X - 1) / 2) * SCAN_SPACING
        gy = (np.arange(SCAN_Y) - (SCAN_Y - 1) / 2) * SCAN_SPACING
        px, py = np.meshgrid(gx, gy, indexing="ij")
        px = px.reshape(-1)
        py = py.reshape(-1)
        c, s = np.cos(yaw)[:, None], np.sin(yaw)[:, None]
        wx = bx[:, None] + c * px[None, :] - s * py[None, :]
        wy = by[:, None] + s * px[None, :] + c * py[None, :]
        base_z = self.lookup(bx, by) + 0.5
        out = base_z[:, None] - self.lookup(wx, wy) - 0.5
        return out.astype(np.float32)


# Column layout of the 48 proprioceptive observations used by the synthetic
# workloads (Section 3.2 lists the quantities; the split is this project's):
# base linear velocity 3, base angular velocity 3, projected gravity 3,
# commands 3, joint positions 12, joint velocities 12, previous actions 12.
PROPRIO_LAYOUT = (("base_lin_vel", 3), ("base_ang_vel", 3), ("gravity", 3), ("commands", 3),
                  ("joint_pos", 12), ("joint_vel", 12), ("last_actions", 12))
# Half-widths of the uniform observation noise per component (appendix Table 4);
# the previous actions are not listed there and get none.
NOISE_HALF_WIDTH = {"base_lin_vel": 0.01, "base_ang_vel": 0.2, "gravity": 0.05, "commands": 0.0,
                    "joint_pos": 0.01, "joint_vel": 1.5, "last_actions": 0.0, "heights": 0.1}


def noise_scales(n_scan: int = SCAN_X * SCAN_Y) -> np.ndarray:
    """[48 + n_scan] float32 noise half-widths in observation column order."""
    parts = [np.full(n, NOISE_HALF_WIDTH[name], dtype=np.float32) for name, n in PROPRIO_LAYOUT]
    parts.append(np.full(n_scan, NOISE_HALF_WIDTH["heights"], dtype=np.float32))
    return np.concatenate(parts)


def scan_pattern(nx: int = SCAN_X, ny: int = SCAN_Y, spacing: float = SCAN_SPACING) -> np.ndarray:
    """[nx * ny, 2] float32 body-frame (x, y) offsets on a centred grid, x-major."""
    a, b = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    pts = np.stack([(a - (nx - 1) / 2) * spacing, (b - (ny - 1) / 2) * spacing], axis=-1)
    return pts.reshape(-1, 2).astype(np.float32)


def base_poses(rng: np.random.Generator, count: int, size: float, margin: float = 2.0,
               z_range=(0.3, 0.8)) -> np.ndarray:
    """[count, 5] float32 (x, y, z, cos yaw, sin yaw); x, y uniform over the
    field minus `margin` (a negative margin puts some robots off the field)."""
    x = rng.uniform(margin, size - margin, count)
    y = rng.uniform(margin, size - margin, count)
    z = rng.uniform(*z_range, count)
    yaw = rng.uniform(-np.pi, np.pi, count)
    return np.stack([x, y, z, np.cos(yaw), np.sin(yaw)], axis=1).astype(np.float32)
