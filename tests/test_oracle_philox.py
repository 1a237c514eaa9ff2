"""Pins for the oracle's Philox4x32-10 and Gaussian noise (CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

from oracle import philox


ROCRAND_HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    """Philox4x32-10 blocks from rocRAND's implementation (a library routine,
    built for the host from the installed header): an independent reference
    for the oracle's rounds, multipliers, key schedule and word order."""
    if not os.path.exists(ROCRAND_HEADER) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "philox_rocrand_ref.cpp")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src, "-o", exe],
                   check=True, capture_output=True)

    def run(rows):
        text = "".join(" ".join(f"{int(v):x}" for v in r) + "\n" for r in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split()
        return np.array([int(x, 16) for x in out], dtype=np.uint64).reshape(-1, 4)
    return run


def test_matches_rocrand(rocrand_philox):
    """Bit-exact against rocRAND on random counters and keys and on the wrap
    edges: all-zero and all-ones words, counters next to 2^32, keys whose
    Weyl bumps wrap."""
    rng = np.random.default_rng(7)
    rows = [r for r in rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64)]
    m = 0xFFFFFFFF
    rows += [np.array(r, dtype=np.uint64) for r in (
        (0, 0, 0, 0, 0, 0), (m, m, m, m, m, m), (m, 0, m, 0, 0, m), (0, m, 0, m, m, 0),
        (m - 1, 1, 2, 3, 0x9E3779B9, 0xBB67AE85), (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0),
        (1, 0, 0, 0, 0xF0000000, 0xF0000000), (0, 0, 0, 1, 0x61C88647, 0x4498517B))]
    rows = np.stack(rows)
    ref = rocrand_philox(rows)
    got = np.stack(philox.philox4x32_10(rows[:, 0], rows[:, 1], rows[:, 2], rows[:, 3], rows[:, 4], rows[:, 5]),
                   axis=1).astype(np.uint64)
    np.testing.assert_array_equal(got, ref)


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(1)
    c = rng.integers(0, 2**32, size=(4, 50), dtype=np.uint64)
    k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
    vec = philox.philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1])
    for i in range(50):
        sc = philox.philox4x32_10(int(c[0, i]), int(c[1, i]), int(c[2, i]), int(c[3, i]), int(k[0]), int(k[1]))
        assert [int(v[i]) for v in vec] == [int(v) for v in sc]


def test_uniform_map_edges():
    u = philox.uniforms(np.array([0, 511, 512, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] == 2.0 ** -24
    assert u[1] == 2.0 ** -24          # low 9 bits are dropped
    assert u[2] == 1.5 * 2.0 ** -23
    assert u[3] == 1.0 - 2.0 ** -24
    # every value is exactly representable in float32
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_box_muller_polar_identity():
    rng = np.random.default_rng(2)
    ua = rng.uniform(1e-6, 1, 1000)
    ub = rng.uniform(0, 1, 1000)
    ea, eb = philox.box_muller(ua, ub)
    np.testing.assert_allclose(ea ** 2 + eb ** 2, -2.0 * np.log(ua), rtol=1e-12)
    ang = np.mod(np.arctan2(eb, ea), 2 * np.pi)
    np.testing.assert_allclose(ang, 2 * np.pi * ub, atol=1e-9)


def test_uniform_and_normal_statistics():
    n = 1 << 18
    x = philox.philox4x32_10(np.arange(n), 7, 3, 1, 0x1234, 0x5678)
    u = philox.uniforms(np.concatenate(x))
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.002
    eps = philox.action_noise(seed=0, n_envs=20000, act_dim=12, t=3, iteration=5).reshape(-1)
    assert abs(eps.mean()) < 4 / np.sqrt(eps.size)
    assert abs(eps.var() - 1.0) < 0.01
    assert scipy.stats.kstest(eps, "norm").pvalue > 1e-3


def test_action_noise_counter_layout():
    a = philox.action_noise(seed=3, n_envs=8, act_dim=12, t=0, iteration=0)
    b = philox.action_noise(seed=3, n_envs=8, act_dim=12, t=1, iteration=0)
    c = philox.action_noise(seed=3, n_envs=8, act_dim=12, t=0, iteration=1)
    d = philox.action_noise(seed=4, n_envs=8, act_dim=12, t=0, iteration=0)
    assert a.shape == (8, 12)
    for other in (b, c, d):
        assert not np.any(a == other)
    # env n, group g uses counter word 0 = n * 3 + g; check one block directly.
    eps, raw = philox.action_noise(seed=3, n_envs=8, act_dim=12, t=0, iteration=0, return_raw=True)
    x = philox.philox4x32_10(5 * 3 + 2, 0, 0, philox.TAG_ACTION, 3, 0)
    assert [int(v) for v in x] == [int(v) for v in raw[5, 8:12]]
    # A not a multiple of 4: the tail of the last block is discarded.
    e10 = philox.action_noise(seed=3, n_envs=8, act_dim=10, t=0, iteration=0)
    np.testing.assert_array_equal(e10, a[:, :10])
