"""Shared inputs for the GPU parity tests: seeded arrays from synth, expected
values from the oracle, device tensors for the HIP path."""
import numpy as np
import pytest
import torch

import synth
from oracle import NetSpec, advantage_stats, gae, normalize_advantages, rollout_infer


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def spec_of(cfg):
    return NetSpec(cfg.net.obs_dim, cfg.net.act_dim, tuple(cfg.net.hidden))


def dev(x, device, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device).contiguous()


def teacher_batch(cfg, theta, B, seed, shift="near", returns="gae"):
    """A batch of B samples whose stored actions / log-probs / values come
    from the oracle policy at `theta`, with controlled log-ratio offsets.

    shift="near": log-ratio offsets U(-0.05, 0.05) (every ratio inside the
    clip band, margin >= 0.14); "mixed": a third of the samples pushed to
    ratios in [1.35, 1.8] or [0.55, 0.74] (outside the band on either side,
    margins >= 0.06 from the clip edges).

    returns="gae": the samples are laid out as a [T, N] rollout with
    rewards ~ N(0, 0.1^2) and dones ~ Bernoulli(1e-3); advantages and
    returns come from the oracle's GAE on the oracle's values (the
    learner's real inputs).  returns="converged": returns = V + N(0, 0.5^2)
    and advantages ~ N(0, 1) (a critic already right on average, which makes
    its true gradient small).
    """
    spec = spec_of(cfg)
    rng = np.random.default_rng(seed)
    if cfg.heightfield:
        obs = synth.make_rollout(cfg, seed=seed)["obs"].reshape(-1, cfg.net.obs_dim)
        reps = -(-B // obs.shape[0])
        obs = np.concatenate([obs] * reps)[:B]
    else:
        obs = synth.rollout.gaussian_like((B, cfg.net.obs_dim), seed=seed)
    ro = rollout_infer(theta, spec, obs, seed=seed, t=0, iteration=0)
    act = ro["actions"].astype(np.float32)
    logp = ro["logp"]
    if shift == "near":
        off = rng.uniform(-0.05, 0.05, B)
    else:
        off = rng.uniform(-0.05, 0.05, B)
        pick = rng.random(B)
        off = np.where(pick < 1 / 6, -rng.uniform(0.3, 0.6, B), off)
        off = np.where((pick >= 1 / 6) & (pick < 1 / 3), rng.uniform(0.3, 0.6, B), off)
    # stored lp_old such that log(rho) = logp - lp_old = off at theta
    lp_old = (logp - off).astype(np.float32)
    values = ro["values"].astype(np.float32)
    if returns == "gae":
        T = 24 if B % 24 == 0 else (8 if B % 8 == 0 else 1)
        N = B // T
        rewards = rng.normal(0, 0.1, (T, N))
        dones = (rng.random((T, N)) < 1e-3).astype(np.uint8)
        last = values.reshape(T, N)[-1] * 0.9 + rng.normal(0, 0.1, N)
        raw, ret = gae(rewards, values.reshape(T, N), dones, last, 0.99, 0.95)
        raw, ret = raw.reshape(B), ret.reshape(B).astype(np.float32)
    else:
        raw = rng.normal(0, 1, B)
        ret = (values + rng.normal(0, 0.5, B)).astype(np.float32)
    m, s = advantage_stats(raw)
    adv = normalize_advantages(raw, m, s).astype(np.float32)
    return dict(obs=obs.astype(np.float32), actions=act, logp=lp_old, adv=adv, returns=ret, values=values)


def oracle_view(batch):
    """Key names of the oracle's batch dictionary."""
    out = dict(obs=batch["obs"], actions=batch["actions"], logp_old=batch["logp"], adv=batch["adv"],
               returns=batch["returns"], values_old=batch["values"])
    for k in ("mu_old", "logstd_old"):
        if k in batch:
            out[k] = batch[k]
    return out


def add_kl_inputs(cfg, theta, batch, seed, shift_scale, logstd_shift=0.03):
    """Collection-time means and log-std for the KL: mu_old = mu(theta) +
    shift_scale[s] * N(0, 1) per sample s (shift_scale is a scalar or a [B]
    array) and logstd_old = logstd + logstd_shift * N(0, 1).  Returns the
    batch with mu_old [B, A] and logstd_old [A] added (float32)."""
    from oracle import mlp_forward, unpack
    spec = spec_of(cfg)
    actor, logstd, _ = unpack(theta, spec)
    mu, _, _ = mlp_forward(actor, batch["obs"].astype(np.float64))
    rng = np.random.default_rng(seed)
    B, A = mu.shape
    scale = np.broadcast_to(np.asarray(shift_scale, dtype=np.float64), (B,))
    out = dict(batch)
    out["mu_old"] = (mu + scale[:, None] * rng.normal(0, 1, (B, A))).astype(np.float32)
    out["logstd_old"] = (np.asarray(logstd, np.float32) + logstd_shift * rng.normal(0, 1, A)).astype(np.float32)
    return out


def bf16_round(x):
    """Round float32 values to the nearest bf16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    return r.view(np.float32).astype(np.float64)


def bf16_split_sum(x):
    """bf16(x) + bf16(x - bf16(x)) for float32 x (the subtraction is exact in
    float32), as float64: the value a weight stored as a bf16 pair carries."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    hi = bf16_round(x32)
    lo = bf16_round((x32.astype(np.float64) - hi).astype(np.float32))
    return hi + lo


def round_hidden_weights(theta, spec):
    """theta with every hidden-layer weight matrix replaced by the value the
    bf16 GEMMs multiply with: bf16(W) for the actor, the bf16 pair
    bf16(W) + bf16(W - bf16(W)) for the critic (biases, output layers and
    log-std stay float32).  A diagnostic: the oracle at these parameters
    separates weight quantisation from everything else."""
    from oracle import param_layout
    lay = param_layout(spec)
    out = np.asarray(theta, dtype=np.float64).copy()
    for which in ("actor", "critic"):
        for l in range(1, len(spec.hidden) + 1):
            off, shp = lay[f"{which}.W{l}"]
            n = int(np.prod(shp))
            w32 = np.asarray(theta[off:off + n], dtype=np.float32)
            out[off:off + n] = bf16_round(w32) if which == "actor" else bf16_split_sum(w32)
    return out
