"""Seeded 2-D heightfield used only to shape rough-terrain observations.

The paper's terrain (Section 3.1) is built from 8 m square tiles of several
types (random rough ground, slopes, stairs) laid out side by side, and the
policy observes terrain heights sampled on a grid around the base
(Section 3.2).  This module builds a small stand-in of that kind: each tile
gets uniform noise of +-5 cm plus either a pyramid slope of up to 0.4 rad or
pyramid stairs with 15 cm risers.  It is harness code: nothing here is graded
and nothing here is part of the learning path.
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
