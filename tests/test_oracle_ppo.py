"""Pins for the oracle's PPO loss, analytic gradient, clipping and Adam."""
import numpy as np
import pytest
import torch

import synth
from oracle import NetSpec, param_layout
from oracle import policy as P
from oracle import ppo as O

TINY = NetSpec(obs_dim=5, act_dim=3, hidden=(4, 3))


def _batch(spec, theta, M, seed, ratio_shift=0.05, adv_sign=None):
    """Batch whose stored log-probs put every ratio near 1 (within +-shift)."""
    rng = np.random.default_rng(seed)
    obs = rng.normal(0, 1, (M, spec.obs_dim))
    actor, logstd, critic = O.unpack(theta, spec)
    mu, _, _ = P.mlp_forward(actor, obs)
    a = mu + np.exp(logstd) * rng.normal(0, 1, mu.shape)
    lp = P.gaussian_logp(a, mu, logstd)
    adv = rng.normal(0, 1, M)
    if adv_sign is not None:
        adv = adv_sign * np.abs(adv)
    return dict(obs=obs, actions=a, logp_old=lp + rng.uniform(-ratio_shift, ratio_shift, M),
                adv=adv, returns=rng.normal(0, 1, M), values_old=rng.normal(0, 1, M))


def _theta(spec, seed):
    n = param_layout(spec)["__total__"][0]
    return np.random.default_rng(seed).normal(0, 0.5, n)


def _loss(theta, spec, batch, hp):
    return O.ppo_loss_grad(theta, spec, batch, hp, want_grad=False)["loss"]


def _fd(theta, spec, batch, hp, coords, h=1e-6):
    g = np.zeros(len(coords))
    for i, c in enumerate(coords):
        tp, tm = theta.copy(), theta.copy()
        tp[c] += h
        tm[c] -= h
        g[i] = (_loss(tp, spec, batch, hp) - _loss(tm, spec, batch, hp)) / (2 * h)
    return g


@pytest.mark.parametrize("clip_value", [False, True])
def test_full_finite_difference_tiny_net(clip_value):
    theta = _theta(TINY, 0)
    batch = _batch(TINY, theta, 9, 1)
    hp = O.PPOHyper(clip_value=clip_value)
    res = O.ppo_loss_grad(theta, TINY, batch, hp)
    assert np.min(res["margin"]) > 100 * 1e-6      # no sample near a clip edge
    fd = _fd(theta, TINY, batch, hp, range(len(theta)))
    np.testing.assert_allclose(res["grad"], fd, rtol=1e-6, atol=1e-9)


def test_finite_difference_with_clipped_samples():
    theta = _theta(TINY, 2)
    batch = _batch(TINY, theta, 12, 6, ratio_shift=0.6)   # many ratios outside the band
    hp = O.PPOHyper()
    res = O.ppo_loss_grad(theta, TINY, batch, hp)
    assert 0 < res["active"].sum() < 12
    assert np.min(res["margin"]) > 1e-4
    fd = _fd(theta, TINY, batch, hp, range(len(theta)))
    np.testing.assert_allclose(res["grad"], fd, rtol=1e-6, atol=1e-9)


@pytest.mark.slow
def test_finite_difference_sampled_at_64x24_shape():
    cfg = synth.get_config("tiny")
    spec = NetSpec(cfg.net.obs_dim, cfg.net.act_dim, tuple(cfg.net.hidden))
    theta = synth.xavier_theta(cfg.net, seed=0).astype(np.float64)
    batch = _batch(spec, theta, cfg.batch, 5)
    hp = O.PPOHyper()
    res = O.ppo_loss_grad(theta, spec, batch, hp)
    assert np.min(res["margin"]) > 100 * 1e-6
    rng = np.random.default_rng(6)
    coords = rng.choice(len(theta), 40, replace=False)
    lay = param_layout(spec)
    coords = np.concatenate([coords, np.arange(lay["actor.logstd"][0], lay["actor.logstd"][0] + 12),
                             [lay["critic.b3"][0]]])
    fd = _fd(theta, spec, batch, hp, coords)
    np.testing.assert_allclose(res["grad"][coords], fd, rtol=1e-6, atol=1e-10)
    # directional derivatives
    for k in range(3):
        u = rng.normal(0, 1, len(theta))
        h = 1e-6
        dd = (_loss(theta + h * u, spec, batch, hp) - _loss(theta - h * u, spec, batch, hp)) / (2 * h)
        assert dd == pytest.approx(res["grad"] @ u, rel=1e-6)


def test_ratio_one_gives_vanilla_policy_gradient():
    theta = _theta(TINY, 7)
    batch = _batch(TINY, theta, 10, 8, ratio_shift=0.0)
    hp = O.PPOHyper(value_coef=0.0, entropy_coef=0.0)
    res = O.ppo_loss_grad(theta, TINY, batch, hp)
    np.testing.assert_allclose(res["ratio"], 1.0, atol=1e-12)
    assert res["policy_loss"] == pytest.approx(-np.mean(batch["adv"]), abs=1e-12)
    M = len(batch["adv"])

    def vanilla(th):
        actor, logstd, _ = O.unpack(th, TINY)
        mu, _, _ = P.mlp_forward(actor, batch["obs"])
        return -np.sum(batch["adv"] * P.gaussian_logp(batch["actions"], mu, logstd)) / M

    h = 1e-6
    for c in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[c] += h
        tm[c] -= h
        assert res["grad"][c] == pytest.approx((vanilla(tp) - vanilla(tm)) / (2 * h), abs=1e-9)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_clip_band(sign):
    theta = _theta(TINY, 9)
    M = 8
    batch = _batch(TINY, theta, M, 10, ratio_shift=0.0, adv_sign=sign)
    hp = O.PPOHyper(value_coef=0.0, entropy_coef=0.0)
    base = O.ppo_loss_grad(theta, TINY, batch, hp)
    eps = hp.clip
    # Active side: ratio = 1 + 2 eps with A > 0, or 1 - 2 eps with A < 0.
    shift = np.log(1 + 2 * eps) if sign > 0 else np.log(1 - 2 * eps)
    active = dict(batch, logp_old=base["logp"] - shift)
    res = O.ppo_loss_grad(theta, TINY, active, hp)
    clipped = (1 + eps) if sign > 0 else (1 - eps)
    assert res["policy_loss"] == pytest.approx(-clipped * np.mean(batch["adv"]), rel=1e-12)
    assert not res["active"].any()
    lay = param_layout(TINY)
    assert np.all(res["grad"][:lay["critic.W1"][0]] == 0.0)
    # Inactive side: ratio = 1 + 2 eps with A < 0: the unclipped term is the min.
    other = dict(batch, adv=-batch["adv"], logp_old=base["logp"] - shift)
    res2 = O.ppo_loss_grad(theta, TINY, other, hp)
    r = 1 + 2 * eps if sign > 0 else 1 - 2 * eps
    assert res2["policy_loss"] == pytest.approx(-r * np.mean(other["adv"]), rel=1e-12)
    assert res2["active"].all()
    np.testing.assert_allclose(res2["ratio"], r, rtol=1e-12)


def test_clip_tie_override():
    """Samples within tie_delta of their clip edge take the override's branch
    (the other implementation's decision), the rest keep their own.  Pinned by
    finite differences: forcing sample i onto the unclipped branch adds
    exactly the gradient of its unclipped surrogate -rho_i A_i / M, evaluated
    here by central differences of a one-sample forward pass."""
    theta = _theta(TINY, 31)
    M = 10
    batch = _batch(TINY, theta, M, 32, ratio_shift=0.0)
    hp = O.PPOHyper(value_coef=0.0, entropy_coef=0.0)
    base = O.ppo_loss_grad(theta, TINY, batch, hp)
    eps = hp.clip
    # samples 0..3 sit just past their deciding clip edge (inside the band,
    # clipped: no gradient), samples 4..9 well inside the band (margin > 0.1)
    edge = np.where(batch["adv"] >= 0, 1.0 + eps, 1.0 - eps)
    want = np.exp(base["logp"] - batch["logp_old"])
    target = want.copy()
    target[:4] = edge[:4] * np.where(batch["adv"][:4] >= 0, 1.0 + 3e-3, 1.0 - 3e-3)
    tb = dict(batch, logp_old=base["logp"] - np.log(target))
    own = O.ppo_loss_grad(theta, TINY, tb, hp)
    assert not own["active"][:4].any() and own["active"][4:].all()
    assert np.all(own["margin"][:4] < 1e-2) and np.all(own["margin"][4:] > 0.1)

    # the other side decided samples 0 and 2 were active, and sample 7 inactive
    other = own["active"].copy()
    other[[0, 2]] = True
    other[7] = False
    res = O.ppo_loss_grad(theta, TINY, tb, hp, active_override=other, tie_delta=2e-2)
    assert res["ties_adopted"] == 2 and res["disagree_outside"] == 1
    assert res["active"][[0, 2]].all() and res["active"][7]

    def unclipped(th, i):
        one = {k: (v[i:i + 1] if k != "logstd_old" else v) for k, v in tb.items()}
        r = O.ppo_loss_grad(th, TINY, one, O.PPOHyper(clip=1e9, value_coef=0.0, entropy_coef=0.0),
                            want_grad=False)
        return r["policy_loss"] / M          # -rho_i A_i / M (one-sample mean)

    h = 1e-6
    expect = own["grad"].copy()
    for c in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[c] += h
        tm[c] -= h
        for i in (0, 2):
            expect[c] += (unclipped(tp, i) - unclipped(tm, i)) / (2 * h)
    np.testing.assert_allclose(res["grad"], expect, rtol=1e-6, atol=1e-9)
    # a zero band adopts nothing
    res0 = O.ppo_loss_grad(theta, TINY, tb, hp, active_override=other, tie_delta=0.0)
    assert res0["ties_adopted"] == 0 and res0["disagree_outside"] == 3
    np.testing.assert_array_equal(res0["grad"], own["grad"])


def test_value_and_entropy_closed_forms():
    theta = _theta(TINY, 11)
    lay = param_layout(TINY)
    off = lay["actor.logstd"][0]
    theta[off:off + 3] = 0.0
    batch = _batch(TINY, theta, 6, 12, ratio_shift=0.0)
    hp = O.PPOHyper()
    res = O.ppo_loss_grad(theta, TINY, batch, hp)
    batch["returns"] = res["values"] - 1.0
    res = O.ppo_loss_grad(theta, TINY, batch, hp)
    assert res["value_loss"] == pytest.approx(1.0, rel=1e-13)
    assert res["entropy"] == pytest.approx(1.5 * (1 + np.log(2 * np.pi)), rel=1e-14)
    assert res["loss"] == pytest.approx(res["policy_loss"] + 1.0 - 0.01 * res["entropy"], rel=1e-13)


def test_clip_coefficient():
    g = np.random.default_rng(13).normal(0, 1, 1000)
    c, norm = O.clip_coef(g, 1.0)
    assert norm == pytest.approx(np.linalg.norm(g), rel=1e-14)
    assert np.linalg.norm(c * g) == pytest.approx(1.0, rel=1e-5)
    c2, _ = O.clip_coef(g * 1e-4, 1.0)
    assert c2 == 1.0


def test_adam_matches_torch_and_first_step():
    rng = np.random.default_rng(14)
    n = 50
    theta0 = rng.normal(0, 1, n)
    hp = O.PPOHyper(lr=1e-3)
    g0 = rng.normal(0, 1, n)
    th1, m1, v1 = O.adam_step(theta0, np.zeros(n), np.zeros(n), g0, 0, hp)
    np.testing.assert_allclose(th1 - theta0, -hp.lr * g0 / (np.abs(g0) + hp.adam_eps), rtol=1e-12)

    p = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=hp.lr, betas=(hp.beta1, hp.beta2), eps=hp.adam_eps)
    th, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
    for s in range(20):
        g = rng.normal(0, 1, n) * (10.0 ** rng.uniform(-4, 1, n))
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        th, m, v = O.adam_step(th, m, v, g, s, hp)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_update_epoch_composes_steps():
    theta = _theta(TINY, 15)
    rng = np.random.default_rng(16)
    B, K = 12, 3
    batch = _batch(TINY, theta, B, 17)
    perm = rng.permutation(B)
    hp = O.PPOHyper()
    n = len(theta)
    th, m, v, step, rec = O.update_epoch(theta, np.zeros(n), np.zeros(n), 4, TINY, batch, perm, K, hp)
    assert step == 7 and len(rec) == K
    th2, m2, v2 = theta, np.zeros(n), np.zeros(n)
    for k in range(K):
        idx = perm[k * 4:(k + 1) * 4]
        r = O.ppo_loss_grad(th2, TINY, O.minibatch(batch, idx), hp)
        c, _ = O.clip_coef(r["grad"], hp.max_grad_norm)
        th2, m2, v2 = O.adam_step(th2, m2, v2, c * r["grad"], 4 + k, hp)
    np.testing.assert_array_equal(th, th2)


def test_gaussian_kl_pins():
    import scipy.integrate
    import scipy.stats
    # one dimension against numeric integration of p log(p / q)
    for mo, so, mn, sn in [(0.0, 1.0, 0.3, 0.8), (1.0, 0.5, -0.2, 1.3), (0.1, 2.0, 0.1, 2.0)]:
        p = scipy.stats.norm(mo, so)
        q = scipy.stats.norm(mn, sn)
        num, _ = scipy.integrate.quad(lambda x: p.pdf(x) * (p.logpdf(x) - q.logpdf(x)), -30, 30, limit=200)
        got = O.gaussian_kl([mo], [np.log(so)], [mn], [np.log(sn)])
        assert got == pytest.approx(num, abs=1e-9)
    rng = np.random.default_rng(20)
    mu = rng.normal(0, 1, (5, 4))
    ls = rng.normal(0, 0.3, 4)
    np.testing.assert_allclose(O.gaussian_kl(mu, ls, mu, ls), 0.0, atol=1e-15)
    # pure mean shift: sum d^2 / (2 sigma^2); pure scale: sum (r^2 - 1)/2 - log r with r = so/sn
    d = rng.normal(0, 1, (5, 4))
    np.testing.assert_allclose(O.gaussian_kl(mu, ls, mu + d, ls), np.sum(d ** 2 / (2 * np.exp(2 * ls)), axis=1),
                               rtol=1e-13)
    r = np.exp(ls - (ls + 0.2))
    np.testing.assert_allclose(O.gaussian_kl(mu, ls, mu, ls + 0.2), np.sum((r ** 2 - 1) / 2 - np.log(r)) * np.ones(5),
                               rtol=1e-12)


def test_adaptive_lr_rule():
    hp = O.PPOHyper(desired_kl=0.01)
    assert O.adaptive_lr(1e-3, 0.021, hp) == pytest.approx(1e-3 / 1.5)
    assert O.adaptive_lr(1e-3, 0.02, hp) == 1e-3          # not above 2 kl*
    assert O.adaptive_lr(1e-3, 0.005, hp) == 1e-3         # not below kl*/2
    assert O.adaptive_lr(1e-3, 0.0049, hp) == pytest.approx(1.5e-3)
    assert O.adaptive_lr(1.2e-5, 1.0, hp) == 1e-5         # lower clamp
    assert O.adaptive_lr(9e-3, 0.0, hp) == 1e-2           # upper clamp


def test_update_epoch_adapts_rate_per_minibatch():
    theta = _theta(TINY, 30)
    B, K = 12, 3
    batch = _batch(TINY, theta, B, 31)
    actor, logstd, _ = O.unpack(theta, TINY)
    mu, _, _ = P.mlp_forward(actor, batch["obs"])
    batch["mu_old"] = mu + 0.05
    batch["logstd_old"] = logstd.copy()
    perm = np.random.default_rng(32).permutation(B)
    hp = O.PPOHyper(desired_kl=0.01, lr=1e-3)
    n = len(theta)
    th, m, v, step, rec = O.update_epoch(theta, np.zeros(n), np.zeros(n), 0, TINY, batch, perm, K, hp)
    lr = hp.lr
    th2, m2, v2 = theta, np.zeros(n), np.zeros(n)
    for k in range(K):
        mb = O.minibatch(batch, perm[k * 4:(k + 1) * 4])
        r = O.ppo_loss_grad(th2, TINY, mb, hp)
        lr = O.adaptive_lr(lr, r["kl"], hp)
        assert rec[k]["lr"] == lr
        c, _ = O.clip_coef(r["grad"], hp.max_grad_norm)
        th2, m2, v2 = O.adam_step(th2, m2, v2, c * r["grad"], k, hp, lr=lr)
    np.testing.assert_array_equal(th, th2)
