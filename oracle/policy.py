"""Actor-critic forward pass and the diagonal-Gaussian policy.

Test infrastructure only (see the package docstring).

The paper (Section 2.2) runs policy inference for every robot on the GPU and
learns a critic; it names neither the network nor the action distribution.
This oracle evaluates the project's reading of that set-up:

  * each hidden layer: z_l = h_{l-1} W_l^T + b_l, h_l = ELU(z_l) with
    ELU(z) = z for z > 0 and exp(z) - 1 otherwise (alpha = 1);
  * the output layer is linear: actor mean mu in R^A, critic value V in R;
  * the policy is a diagonal Gaussian N(mu, diag(sigma^2)) with a
    state-independent parameter log(sigma) in R^A;
  * log pi(a|s) = sum_j [ -((a_j - mu_j) / sigma_j)^2 / 2 - log sigma_j ]
                  - (A/2) log(2 pi);
  * entropy H = sum_j log sigma_j + (A/2) (1 + log(2 pi)).

Actions are the desired joint positions (Section 3.2); the learner does not
squash or clip them.
"""
from __future__ import annotations

import numpy as np

from .layout import NetSpec, unpack
from .philox import action_noise

LOG_2PI = np.log(2.0 * np.pi)


def elu(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > 0.0, z, np.expm1(np.minimum(z, 0.0)))


def elu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > 0.0, 1.0, np.exp(np.minimum(z, 0.0)))


def mlp_forward(layers, x):
    """Returns (output, zs, hs): pre-activations z_l and inputs h_{l-1}.

    hs[0] is the network input; hs[l] is the input of layer l+1.
    """
    h = np.asarray(x, dtype=np.float64)
    zs, hs = [], [h]
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        if l + 1 < len(layers):
            h = elu(z)
            hs.append(h)
        else:
            h = z
    return h, zs, hs


def gaussian_logp(a, mu, logstd):
    a = np.asarray(a, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    logstd = np.asarray(logstd, dtype=np.float64)
    A = mu.shape[-1]
    zscore = (a - mu) / np.exp(logstd)
    return np.sum(-0.5 * zscore ** 2 - logstd, axis=-1) - 0.5 * A * LOG_2PI


def gaussian_entropy(logstd):
    logstd = np.asarray(logstd, dtype=np.float64)
    A = logstd.shape[-1]
    return np.sum(logstd) + 0.5 * A * (1.0 + LOG_2PI)


def rollout_infer(theta, spec: NetSpec, obs, seed: int, t: int, iteration: int):
    """One policy step for all environments.

    Returns dict(actions [N,A], logp [N], values [N], mu [N,A], eps [N,A]),
    all float64.  The noise eps comes from Philox (see philox.action_noise);
    a = mu + sigma * eps.
    """
    actor, logstd, critic = unpack(theta, spec)
    obs = np.asarray(obs, dtype=np.float64)
    mu, _, _ = mlp_forward(actor, obs)
    v, _, _ = mlp_forward(critic, obs)
    eps = action_noise(seed, obs.shape[0], spec.act_dim, t, iteration)
    actions = mu + np.exp(logstd) * eps
    logp = gaussian_logp(actions, mu, logstd)
    return dict(actions=actions, logp=logp, values=v[:, 0], mu=mu, eps=eps)


def critic_values(theta, spec: NetSpec, obs):
    _, _, critic = unpack(theta, spec)
    v, _, _ = mlp_forward(critic, np.asarray(obs, dtype=np.float64))
    return v[:, 0]
