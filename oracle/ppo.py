"""PPO loss, its analytic gradient, global gradient-norm clipping and Adam.

Test infrastructure only (see the package docstring).

The paper trains with PPO (Schulman et al., 2017) on very large mini-batches
(Section 2.2.1) with clip range 0.2, entropy coefficient 0.01 and 5 epochs
(Appendix A.4, Table 3).  Per mini-batch of M samples with stored actions a,
old log-probabilities lp_old, normalised advantages A_hat and returns R:

  rho_i  = exp(log pi(a_i|s_i) - lp_old_i)
  L_pi   = -(1/M) sum_i min(rho_i A_hat_i, clip(rho_i, 1-eps, 1+eps) A_hat_i)
  L_V    = (1/M) sum_i (R_i - V_i)^2            (value clipping optional)
  H      = entropy of the diagonal Gaussian (state independent)
  L      = L_pi + c_v L_V - c_e H

Analytic gradient (derived from the definitions above):
  dL/dlogp_i = -(1/M) A_hat_i rho_i [active_i], active_i meaning the
      unclipped term attains the min: (A_hat_i >= 0 and rho_i <= 1+eps) or
      (A_hat_i < 0 and rho_i >= 1-eps)   (closed band: ties pass gradient);
  dL/dmu_ij      = dL/dlogp_i (a_ij - mu_ij) / sigma_j^2;
  dL/dlogsigma_j = sum_i dL/dlogp_i ((a_ij - mu_ij)^2 / sigma_j^2 - 1) - c_e;
  dL/dV_i        = (2 c_v / M)(V_i - R_i);
then ordinary back-propagation through each MLP:
  dW_l = dz_l^T h_{l-1},  db_l = sum_rows dz_l,  dh_{l-1} = dz_l W_l,
  dz_{l-1} = dh_{l-1} * ELU'(z_{l-1}).

The gradient is clipped to a global norm (all parameters together):
c = min(1, max_norm / (||g||_2 + 1e-6)), g <- c g.  Adam (Kingma and Ba,
2015, Algorithm 1) with bias correction, beta1 0.9, beta2 0.999, eps 1e-8
outside the square root, no weight decay; the step count runs on across
mini-batches, epochs and iterations.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from .layout import NetSpec, param_layout, unpack  # noqa: F401 (unpack re-exported for tests)
from .policy import elu_grad, gaussian_entropy, gaussian_logp, mlp_forward

CLIP_NORM_EPS = 1e-6


@dataclass
class PPOHyper:
    clip: float = 0.2
    value_coef: float = 1.0
    entropy_coef: float = 0.01
    max_grad_norm: float = 1.0
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    clip_value: bool = False
    # Appendix A.4, Algorithm 1 (0 disables the adaptive rate)
    desired_kl: float = 0.0
    lr_factor: float = 1.5
    lr_min: float = 1e-5
    lr_max: float = 1e-2


def gaussian_kl(mu_old, logstd_old, mu_new, logstd_new):
    """KL(pi_old || pi_new) per sample for diagonal Gaussians:
    sum_j [log(sigma_new/sigma_old) + (sigma_old^2 + (mu_old - mu_new)^2) / (2 sigma_new^2) - 1/2]."""
    mu_old = np.asarray(mu_old, dtype=np.float64)
    mu_new = np.asarray(mu_new, dtype=np.float64)
    ls_old = np.asarray(logstd_old, dtype=np.float64)
    ls_new = np.asarray(logstd_new, dtype=np.float64)
    var_old = np.exp(2.0 * ls_old)
    var_new = np.exp(2.0 * ls_new)
    return np.sum(ls_new - ls_old + (var_old + (mu_old - mu_new) ** 2) / (2.0 * var_new) - 0.5, axis=-1)


def adaptive_lr(lr: float, kl: float, hp: "PPOHyper") -> float:
    """Algorithm 1 of Appendix A.4: divide the rate by the factor when the KL
    exceeds twice the target, multiply it when the KL is below half the
    target, within [lr_min, lr_max]."""
    if kl > 2.0 * hp.desired_kl:
        return max(hp.lr_min, lr / hp.lr_factor)
    if kl < 0.5 * hp.desired_kl:
        return min(hp.lr_max, lr * hp.lr_factor)
    return lr


def _mlp_backward(layers, zs, hs, g_out):
    """Back-propagate dL/d(output) through one MLP; returns [(dW, db)]."""
    grads = [None] * len(layers)
    g_z = g_out
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (g_z.T @ hs[l], g_z.sum(axis=0))
        if l > 0:
            g_h = g_z @ W
            g_z = g_h * elu_grad(zs[l - 1])
    return grads


def ppo_loss_grad(theta, spec: NetSpec, batch: Dict[str, np.ndarray], hp: PPOHyper,
                  want_grad: bool = True, active_override=None, tie_delta: float = 0.0):
    """Loss terms, statistics and the flat gradient for one mini-batch.

    batch: obs [M, D], actions [M, A], logp_old [M], adv [M] (normalised),
    returns [M], and values_old [M] when hp.clip_value is set.

    Clip-edge ties: a sample whose ratio lies within rounding of the clip
    edge that decides its branch may legitimately take either branch in
    another implementation's arithmetic.  With active_override (bool [M],
    the other implementation's branches) and tie_delta (a scalar, or one band
    per sample), samples whose margin is below their band take the
    override's branch; every other sample keeps its own.  The result reports how many samples were adopted that way
    ("ties_adopted") and how many disagree outside the band
    ("disagree_outside", which a checker requires to be zero).
    """
    actor, logstd, critic = unpack(theta, spec)
    obs = np.asarray(batch["obs"], dtype=np.float64)
    a = np.asarray(batch["actions"], dtype=np.float64)
    lp_old = np.asarray(batch["logp_old"], dtype=np.float64)
    adv = np.asarray(batch["adv"], dtype=np.float64)
    ret = np.asarray(batch["returns"], dtype=np.float64)
    M = obs.shape[0]
    eps = hp.clip

    mu, zs_a, hs_a = mlp_forward(actor, obs)
    v_out, zs_c, hs_c = mlp_forward(critic, obs)
    V = v_out[:, 0]
    sigma = np.exp(logstd)

    logp = gaussian_logp(a, mu, logstd)
    ratio = np.exp(logp - lp_old)
    surr_unclipped = ratio * adv
    surr_clipped = np.clip(ratio, 1.0 - eps, 1.0 + eps) * adv
    policy_loss = -np.mean(np.minimum(surr_unclipped, surr_clipped))

    if hp.clip_value:
        v_old = np.asarray(batch["values_old"], dtype=np.float64)
        v_clipped = v_old + np.clip(V - v_old, -eps, eps)
        sq_u = (V - ret) ** 2
        sq_c = (v_clipped - ret) ** 2
        value_loss = np.mean(np.maximum(sq_u, sq_c))
        v_pass = sq_u >= sq_c
    else:
        value_loss = np.mean((ret - V) ** 2)
        v_pass = np.ones(M, dtype=bool)

    entropy = gaussian_entropy(logstd)
    loss = policy_loss + hp.value_coef * value_loss - hp.entropy_coef * entropy

    active = ((adv >= 0.0) & (ratio <= 1.0 + eps)) | ((adv < 0.0) & (ratio >= 1.0 - eps))
    # Distance of each ratio from the clip edge that decides its branch.
    margin = np.where(adv >= 0.0, np.abs(ratio - (1.0 + eps)), np.abs(ratio - (1.0 - eps)))
    ties_adopted = disagree_outside = 0
    if active_override is not None:
        other = np.asarray(active_override, dtype=bool).reshape(M)
        band = margin < tie_delta
        ties_adopted = int(np.sum(band & (other != active)))
        disagree_outside = int(np.sum(~band & (other != active)))
        active = np.where(band, other, active)
    out = dict(
        loss=loss, policy_loss=policy_loss, value_loss=value_loss, entropy=entropy,
        clip_frac=float(np.mean(np.abs(ratio - 1.0) > eps)),
        approx_kl=float(np.mean((ratio - 1.0) - np.log(ratio))),
        ratio=ratio, active=active, margin=margin, mu=mu, values=V, logp=logp,
        ties_adopted=ties_adopted, disagree_outside=disagree_outside,
    )
    if "mu_old" in batch and "logstd_old" in batch:
        out["kl"] = float(np.mean(gaussian_kl(batch["mu_old"], batch["logstd_old"], mu, logstd)))
    if not want_grad:
        return out

    g_logp = -(1.0 / M) * adv * ratio * active
    diff = a - mu
    g_mu = g_logp[:, None] * diff / sigma ** 2
    g_logstd = np.sum(g_logp[:, None] * (diff ** 2 / sigma ** 2 - 1.0), axis=0) - hp.entropy_coef
    g_V = (2.0 * hp.value_coef / M) * (V - ret) * v_pass

    grads_a = _mlp_backward(actor, zs_a, hs_a, g_mu)
    grads_c = _mlp_backward(critic, zs_c, hs_c, g_V[:, None])

    lay = param_layout(spec)
    grad = np.zeros(lay["__total__"][0], dtype=np.float64)

    def put(name, value):
        off, shp = lay[name]
        grad[off:off + int(np.prod(shp))] = np.asarray(value).reshape(-1)

    for which, grads in (("actor", grads_a), ("critic", grads_c)):
        for l, (dW, db) in enumerate(grads, start=1):
            put(f"{which}.W{l}", dW)
            put(f"{which}.b{l}", db)
    put("actor.logstd", g_logstd)
    out["grad"] = grad
    out["g_mu"] = g_mu
    out["g_V"] = g_V
    return out


def clip_coef(grad, max_norm: float):
    """(coefficient, pre-clip global L2 norm)."""
    norm = float(np.sqrt(np.sum(np.asarray(grad, dtype=np.float64) ** 2)))
    return min(1.0, max_norm / (norm + CLIP_NORM_EPS)), norm


def adam_step(theta, m, v, grad, step: int, hp: PPOHyper, lr: Optional[float] = None):
    """One Adam step; `step` counts the steps already taken.  Returns new arrays."""
    lr = hp.lr if lr is None else lr
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    t = step + 1
    m = hp.beta1 * np.asarray(m, dtype=np.float64) + (1.0 - hp.beta1) * g
    v = hp.beta2 * np.asarray(v, dtype=np.float64) + (1.0 - hp.beta2) * g * g
    m_hat = m / (1.0 - hp.beta1 ** t)
    v_hat = v / (1.0 - hp.beta2 ** t)
    theta = theta - lr * m_hat / (np.sqrt(v_hat) + hp.adam_eps)
    return theta, m, v


def minibatch(batch: Dict[str, np.ndarray], idx) -> Dict[str, np.ndarray]:
    """Rows `idx` of every per-sample array; the state-independent old
    log-std (key "logstd_old") is shared by all samples."""
    return {k: (np.asarray(v) if k == "logstd_old" else np.asarray(v)[idx]) for k, v in batch.items()}


def update_epoch(theta, m, v, step: int, spec: NetSpec, batch: Dict[str, np.ndarray],
                 perm, n_minibatches: int, hp: PPOHyper, lr: Optional[float] = None):
    """One epoch: K mini-batch steps of loss/gradient, clip, Adam.

    batch arrays are flattened over the rollout (sample s = t * N + n);
    perm is this epoch's permutation of [0, B).  With hp.desired_kl > 0 and
    the collection-time means and log-std in the batch (mu_old, logstd_old),
    each step first adapts the learning rate from the mini-batch KL at the
    current parameters (Algorithm 1), then takes the Adam step with it.
    Returns (theta, m, v, step, per-step records); each record holds the
    rate it used under "lr".
    """
    B = len(perm)
    assert B % n_minibatches == 0
    M = B // n_minibatches
    lr = hp.lr if lr is None else lr
    records: List[dict] = []
    for k in range(n_minibatches):
        idx = np.asarray(perm[k * M:(k + 1) * M])
        res = ppo_loss_grad(theta, spec, minibatch(batch, idx), hp)
        if hp.desired_kl > 0.0 and "kl" in res:
            lr = adaptive_lr(lr, res["kl"], hp)
        c, norm = clip_coef(res["grad"], hp.max_grad_norm)
        theta, m, v = adam_step(theta, m, v, c * res["grad"], step, hp, lr=lr)
        step += 1
        res["grad_norm"] = norm
        res["clip_coef"] = c
        res["lr"] = lr
        records.append(res)
    return theta, m, v, step, records
