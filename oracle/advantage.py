"""Generalized Advantage Estimation with time-out bootstrapping.

Test infrastructure only (see the package docstring).

Section 2.2.1 of the paper uses GAE (Schulman et al., 2016) over short
rollouts of n_steps per robot, with gamma = 0.99 and lambda = 0.95
(Appendix A.4, Table 3).  Section 2.2.2 bootstraps the critic's target on
time-outs: the reward of a transition that ended by time-out is augmented
with the discounted critic prediction.  Reading used here: the stored value
of the current state stands in for the value of the (overwritten) terminal
state, r'_t = r_t + gamma * V_t * timeout_t, and time-outs are also dones.

Recursion over a [T, N] rollout (t-major, env-contiguous), with d_t = 1 when
the episode ended at transition t and V_T = last_values:

  delta_t = r'_t + gamma (1 - d_t) V_{t+1} - V_t
  A_t     = delta_t + gamma lambda (1 - d_t) A_{t+1},   A_T = 0
  R_t     = A_t + V_t            (returns use un-normalised advantages)

Advantages are normalised once per iteration over the whole batch with the
sample mean and the unbiased (ddof = 1) standard deviation:
  A_hat = (A - mean) / (std + 1e-8).
"""
from __future__ import annotations

import numpy as np

ADV_EPS = 1e-8


def gae(rewards, values, dones, last_values, gamma, lam, timeouts=None):
    """Returns (advantages, returns), float64 [T, N]."""
    r = np.asarray(rewards, dtype=np.float64)
    V = np.asarray(values, dtype=np.float64)
    d = np.asarray(dones, dtype=np.float64)
    T, N = r.shape
    if timeouts is not None:
        r = r + gamma * V * np.asarray(timeouts, dtype=np.float64)
    adv = np.zeros((T, N), dtype=np.float64)
    next_value = np.asarray(last_values, dtype=np.float64)
    next_adv = np.zeros(N, dtype=np.float64)
    for t in range(T - 1, -1, -1):
        not_done = 1.0 - d[t]
        delta = r[t] + gamma * not_done * next_value - V[t]
        adv[t] = delta + gamma * lam * not_done * next_adv
        next_value = V[t]
        next_adv = adv[t]
    return adv, adv + V


def advantage_stats(adv):
    """(mean, unbiased std) over every element, float64."""
    a = np.asarray(adv, dtype=np.float64).reshape(-1)
    return float(np.mean(a)), float(np.std(a, ddof=1))


def normalize_advantages(adv, mean, std):
    return (np.asarray(adv, dtype=np.float64) - mean) / (std + ADV_EPS)
