"""Pins for the oracle's GAE, time-out bootstrap and advantage statistics."""
import json
import os

import numpy as np
import pytest

from oracle import advantage as G
from tests.conftest import GOLDEN


def _random_rollout(T, N, seed, p_done=0.2, timeouts=False):
    rng = np.random.default_rng(seed)
    r = rng.normal(0, 1, (T, N))
    v = rng.normal(0, 1, (T, N))
    d = (rng.random((T, N)) < p_done).astype(np.uint8)
    last = rng.normal(0, 1, N)
    to = (d.astype(bool) & (rng.random((T, N)) < 0.5)).astype(np.uint8) if timeouts else None
    return r, v, d, last, to


def test_hand_worked_example():
    with open(os.path.join(GOLDEN, "gae_hand_t3.json")) as f:
        g = json.load(f)
    adv, ret = G.gae(g["rewards"], g["values"], g["dones"], g["last_values"],
                     g["gamma"], g["lam"], timeouts=g["timeouts"])
    np.testing.assert_allclose(adv, g["advantages"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(ret, g["returns"], rtol=0, atol=1e-12)


def test_lambda_one_is_discounted_return_minus_value():
    T, N, gamma = 9, 5, 0.9
    r, v, d, last, _ = _random_rollout(T, N, 0)
    adv, _ = G.gae(r, v, d, last, gamma, 1.0)
    for n in range(N):
        for t in range(T):
            ret, disc = 0.0, 1.0
            k = t
            while True:
                ret += disc * r[k, n]
                if d[k, n]:
                    break
                disc *= gamma
                k += 1
                if k == T:
                    ret += disc * last[n]
                    break
            assert adv[t, n] == pytest.approx(ret - v[t, n], abs=1e-12)


def test_lambda_zero_is_td_residual():
    T, N, gamma = 7, 6, 0.95
    r, v, d, last, _ = _random_rollout(T, N, 1)
    adv, _ = G.gae(r, v, d, last, gamma, 0.0)
    v_next = np.vstack([v[1:], last[None]])
    delta = r + gamma * (1 - d) * v_next - v
    np.testing.assert_allclose(adv, delta, atol=1e-12)


def test_gamma_zero_and_all_done():
    T, N = 5, 4
    r, v, d, last, to = _random_rollout(T, N, 2, timeouts=True)
    adv, _ = G.gae(r, v, d, last, 0.0, 0.95, timeouts=to)
    np.testing.assert_allclose(adv, r - v, atol=1e-12)
    ones = np.ones((T, N), dtype=np.uint8)
    adv, _ = G.gae(r, v, ones, last, 0.99, 0.95)
    np.testing.assert_allclose(adv, r - v, atol=1e-12)


@pytest.mark.parametrize("with_timeouts", [False, True])
def test_quadratic_brute_force(with_timeouts):
    T, N, gamma, lam = 11, 7, 0.97, 0.9
    r, v, d, last, to = _random_rollout(T, N, 3, timeouts=with_timeouts)
    adv, ret = G.gae(r, v, d, last, gamma, lam, timeouts=to)
    rb = r + (gamma * v * to if to is not None else 0.0)
    v_next = np.vstack([v[1:], last[None]])
    delta = rb + gamma * (1 - d) * v_next - v
    for n in range(N):
        for t in range(T):
            total, weight = 0.0, 1.0
            for l in range(T - t):
                total += weight * delta[t + l, n]
                weight *= gamma * lam * (1 - d[t + l, n])
            assert adv[t, n] == pytest.approx(total, abs=1e-12)
    np.testing.assert_allclose(ret - adv, v, atol=1e-12)


def test_timeout_bootstrap_changes_only_timeout_rewards():
    T, N, gamma, lam = 6, 3, 0.99, 0.95
    r, v, d, last, to = _random_rollout(T, N, 4, p_done=0.5, timeouts=True)
    assert to.sum() > 0
    a1, _ = G.gae(r, v, d, last, gamma, lam, timeouts=to)
    a2, _ = G.gae(r + gamma * v * to, v, d, last, gamma, lam)
    np.testing.assert_allclose(a1, a2, atol=1e-12)


def test_normalisation_moments():
    rng = np.random.default_rng(5)
    a = rng.normal(3.0, 2.0, (24, 64))
    mean, std = G.advantage_stats(a)
    n = a.size
    # unbiased variance from the two-pass definition
    assert std ** 2 == pytest.approx(np.sum((a - a.mean()) ** 2) / (n - 1), rel=1e-12)
    z = G.normalize_advantages(a, mean, std)
    assert abs(z.mean()) < 1e-12
    assert np.std(z, ddof=1) == pytest.approx(std / (std + 1e-8), rel=1e-12)
