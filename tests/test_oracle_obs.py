"""Pins of the observation-assembly oracle (height scan and noise) against
brute force, array slices and closed forms (Section 3.2; Table 4)."""
import numpy as np
import pytest
from scipy import stats

from oracle.observation import (assemble_obs, height_scan, nearest_cells, obs_noise_unit,
                                scan_world_points, TAG_OBS_NOISE)
from oracle.philox import action_noise

f32 = np.float32


def _grid_scan(nx=17, ny=11, spacing=0.1):
    a, b = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    pts = np.stack([(a - (nx - 1) / 2) * spacing, (b - (ny - 1) / 2) * spacing], axis=-1)
    return pts.reshape(-1, 2).astype(f32)


def _base(x, y, z, yaw):
    return np.array([[x, y, z, np.cos(yaw), np.sin(yaw)]], dtype=f32)


def test_nearest_cell_is_the_brute_force_nearest():
    """Every point, inside the grid or outside it, reads the cell at the least
    distance (searched over the whole grid); points within 1e-4 cell of a
    half-way line are left out, since there both cells are nearest up to
    rounding."""
    rng = np.random.default_rng(0)
    nx, ny, inv_res = 13, 9, 10.0
    wx = rng.uniform(-0.5, 1.8, 20000).astype(f32)
    wy = rng.uniform(-0.5, 1.3, 20000).astype(f32)
    gi, gj = nearest_cells(wx, wy, inv_res, nx, ny)
    cx = np.arange(nx) / inv_res
    cy = np.arange(ny) / inv_res
    d2 = ((wx.astype(np.float64)[:, None, None] - cx[None, :, None]) ** 2
          + (wy.astype(np.float64)[:, None, None] - cy[None, None, :]) ** 2)
    flat = d2.reshape(len(wx), -1).argmin(axis=1)
    bi, bj = np.unravel_index(flat, (nx, ny))
    frac_x = np.abs(wx.astype(np.float64) * inv_res - np.floor(wx.astype(np.float64) * inv_res) - 0.5)
    frac_y = np.abs(wy.astype(np.float64) * inv_res - np.floor(wy.astype(np.float64) * inv_res) - 0.5)
    keep = (frac_x > 1e-4) & (frac_y > 1e-4)
    assert keep.mean() > 0.99
    np.testing.assert_array_equal(gi[keep], bi[keep])
    np.testing.assert_array_equal(gj[keep], bj[keep])
    outside = (wx < 0) | (wx > (nx - 1) / inv_res) | (wy < 0) | (wy > (ny - 1) / inv_res)
    assert outside.sum() > 1000


def test_nearest_cell_rounds_half_to_even_and_nan_reads_cell_zero():
    # exact halves in binary: 0.25 * 10 = 2.5 -> 2, 0.75 * 10 = 7.5 -> 8, 1.25 * 10 = 12.5 -> 12
    gi, _ = nearest_cells(np.array([0.25, 0.75, 1.25], f32), np.zeros(3, f32), 10.0, 20, 5)
    np.testing.assert_array_equal(gi, [2, 8, 12])
    gi, gj = nearest_cells(np.array([np.nan], f32), np.array([np.nan], f32), 10.0, 20, 5)
    assert gi[0] == 0 and gj[0] == 0


def test_rotation_direction():
    """Heading (cos, sin) rotates body +x onto the world direction (cos, sin)
    and body +y onto (-sin, cos)."""
    yaw = np.deg2rad(30.0)
    base = _base(1.0, 2.0, 0.0, yaw)
    wx, wy = scan_world_points(base, np.array([[1.0, 0.0], [0.0, 1.0]], f32))
    np.testing.assert_allclose([wx[0, 0], wy[0, 0]], [1 + np.cos(yaw), 2 + np.sin(yaw)], atol=1e-6)
    np.testing.assert_allclose([wx[0, 1], wy[0, 1]], [1 - np.sin(yaw), 2 + np.cos(yaw)], atol=1e-6)


@pytest.mark.parametrize("heading", ["0", "90", "180"])
def test_heading_reads_array_slices(heading):
    """Base on a cell centre and the 17 x 11 scan on grid points: at heading 0
    the scan is an axis-aligned slice of the height field, at 90 degrees that
    slice transposed with its rows reversed, at 180 degrees reversed in both
    axes."""
    rng = np.random.default_rng(1)
    H = rng.uniform(-1, 1, (40, 30)).astype(f32)
    i0, j0, z = 20, 14, 0.75
    c, s = {"0": (1.0, 0.0), "90": (0.0, 1.0), "180": (-1.0, 0.0)}[heading]
    base = np.array([[f32(i0 * 0.1), f32(j0 * 0.1), z, c, s]], dtype=f32)
    h = height_scan(base, H, 10.0, _grid_scan()).reshape(17, 11)
    if heading == "0":
        expect = H[i0 - 8:i0 + 9, j0 - 5:j0 + 6]
    elif heading == "90":
        # body (a, b) offsets (a-8, b-5) cells land at world (i0-(b-5), j0+(a-8))
        expect = H[i0 - 5:i0 + 6, j0 - 8:j0 + 9][::-1, :].T
    else:
        expect = H[i0 - 8:i0 + 9, j0 - 5:j0 + 6][::-1, ::-1]
    np.testing.assert_array_equal(h, z - expect.astype(np.float64))


def test_flat_terrain_reads_its_height_everywhere():
    rng = np.random.default_rng(2)
    H = np.full((25, 25), 0.37, dtype=f32)
    yaw = rng.uniform(-np.pi, np.pi, 64)
    base = np.stack([rng.uniform(-1, 4, 64), rng.uniform(-1, 4, 64), rng.uniform(0, 1, 64),
                     np.cos(yaw), np.sin(yaw)], axis=1).astype(f32)
    h = height_scan(base, H, 10.0, _grid_scan())
    np.testing.assert_array_equal(h, np.broadcast_to(base[:, 2:3].astype(np.float64) - np.float64(f32(0.37)), h.shape))


def test_noise_is_uniform_on_the_open_interval():
    """2u - 1 takes the values (2k + 1 - 2^23) / 2^23 (odd multiples of
    2^-23); uniform on (-1, 1): moments, Kolmogorov-Smirnov, no correlation
    between steps, iterations or the action-noise stream."""
    e = obs_noise_unit(7, 4096, 235, t=3, iteration=5)
    assert e.shape == (4096, 235)
    k = e * 2.0 ** 23
    np.testing.assert_array_equal(k, np.round(k))
    assert np.all(np.abs(k.astype(np.int64)) % 2 == 1)
    assert np.all(np.abs(e) < 1)
    n = e.size
    assert abs(e.mean()) < 4 * np.sqrt(1 / 3 / n)
    assert abs(e.var() - 1 / 3) < 4 * np.sqrt(4 / 45 / n)
    assert stats.kstest(e.ravel()[:200000], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    for other in (obs_noise_unit(7, 4096, 235, t=4, iteration=5), obs_noise_unit(7, 4096, 235, t=3, iteration=6),
                  obs_noise_unit(8, 4096, 235, t=3, iteration=5)):
        r = np.corrcoef(e.ravel(), other.ravel())[0, 1]
        assert abs(r) < 4 / np.sqrt(n)
    assert TAG_OBS_NOISE != 1
    eps = action_noise(7, 4096, 12, 3, 5)
    r = np.corrcoef(e[:, :12].ravel(), eps.ravel())[0, 1]
    assert abs(r) < 4 / np.sqrt(eps.size)


def test_assemble_layout_and_zero_noise():
    rng = np.random.default_rng(3)
    N, P = 50, 45
    proprio = rng.standard_normal((N, P)).astype(f32)
    H = rng.uniform(-0.1, 0.1, (60, 60)).astype(f32)
    yaw = rng.uniform(-np.pi, np.pi, N)
    base = np.stack([rng.uniform(1, 5, N), rng.uniform(1, 5, N), rng.uniform(0.3, 0.7, N),
                     np.cos(yaw), np.sin(yaw)], axis=1).astype(f32)
    scan = _grid_scan()
    no_noise = assemble_obs(proprio, base, H, 10.0, scan, None, 0, 0, 0)
    np.testing.assert_array_equal(no_noise[:, :P], proprio.astype(np.float64))
    np.testing.assert_array_equal(no_noise[:, P:], height_scan(base, H, 10.0, scan))
    zero = assemble_obs(proprio, base, H, 10.0, scan, np.zeros(P + len(scan), f32), 9, 1, 2)
    np.testing.assert_array_equal(zero, no_noise)
    scale = np.concatenate([np.full(P, 0.05, f32), np.full(len(scan), 0.1, f32)])
    noisy = assemble_obs(proprio, base, H, 10.0, scan, scale, 9, 1, 2)
    d = noisy - no_noise
    assert np.all(np.abs(d[:, :P]) < 0.05) and np.all(np.abs(d[:, P:]) < 0.1)
    assert np.abs(d[:, P:]).max() > 0.09
    only_proprio = assemble_obs(proprio, base, None, 10.0, None, None, 0, 0, 0)
    np.testing.assert_array_equal(only_proprio, proprio.astype(np.float64))
