"""Pins for the oracle's MLP, Gaussian policy and parameter layout."""
import math

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import layout as L
from oracle import policy as P


def test_param_counts_and_layout_agree_with_input_generator():
    # counts derived by hand from the widths: sum over layers of out*(in+1), plus A log-stds
    expected = {"tiny": 15449, "flat": 380313, "rough": 571801, "large": 1798937}
    for name, count in expected.items():
        cfg = synth.get_config(name)
        spec = L.NetSpec(cfg.net.obs_dim, cfg.net.act_dim, tuple(cfg.net.hidden))
        lay = L.param_layout(spec)
        assert lay["__total__"][0] == count
        for nm, shp, off in synth.flat_layout(cfg.net):
            assert lay[nm] == (off, shp)


def _tiny_net(seed=0, dims=(5, 4, 3, 2)):
    rng = np.random.default_rng(seed)
    return [(rng.normal(0, 1, (dims[i + 1], dims[i])), rng.normal(0, 1, dims[i + 1]))
            for i in range(len(dims) - 1)]


def test_mlp_forward_matches_loops():
    layers = _tiny_net()
    x = np.random.default_rng(1).normal(0, 1, (3, 5))
    out, zs, hs = P.mlp_forward(layers, x)
    for r in range(3):
        h = list(x[r])
        for l, (W, b) in enumerate(layers):
            z = [sum(W[o][i] * h[i] for i in range(len(h))) + b[o] for o in range(len(b))]
            if l + 1 < len(layers):
                h = [zz if zz > 0 else math.exp(zz) - 1.0 for zz in z]
            else:
                h = z
        np.testing.assert_allclose(out[r], h, rtol=1e-13, atol=1e-13)


def test_elu_special_points():
    assert P.elu(0.0) == 0.0
    assert P.elu_grad(0.0) == 1.0           # exp(0) = 1: C1 at the kink
    z = np.linspace(-5, 5, 100)      # excludes the kink at 0
    h = 1e-6
    np.testing.assert_allclose(P.elu_grad(z), (P.elu(z + h) - P.elu(z - h)) / (2 * h), atol=1e-8)
    assert P.elu(-50.0) == pytest.approx(-1.0, abs=1e-15)


def test_logp_matches_scipy_and_closed_forms():
    rng = np.random.default_rng(3)
    A = 12
    mu = rng.normal(0, 1, (10, A))
    logstd = rng.normal(0, 0.3, A)
    a = mu + np.exp(logstd) * rng.normal(0, 1, (10, A))
    ref = scipy.stats.norm.logpdf(a, loc=mu, scale=np.exp(logstd)).sum(axis=1)
    np.testing.assert_allclose(P.gaussian_logp(a, mu, logstd), ref, rtol=1e-13)
    np.testing.assert_allclose(P.gaussian_logp(mu, mu, logstd),
                               -np.sum(logstd) - 0.5 * A * np.log(2 * np.pi), rtol=1e-13)
    ent = scipy.stats.norm(scale=np.exp(logstd)).entropy().sum()
    assert P.gaussian_entropy(logstd) == pytest.approx(ent, rel=1e-13)


def test_entropy_is_negative_expected_logp():
    rng = np.random.default_rng(4)
    A = 4
    logstd = np.array([0.0, -0.5, 0.3, 0.1])
    mu = np.zeros((200000, A))
    a = rng.normal(0, 1, mu.shape) * np.exp(logstd)
    lp = P.gaussian_logp(a, mu, logstd)
    se = lp.std() / np.sqrt(lp.size)
    assert abs(-lp.mean() - P.gaussian_entropy(logstd)) < 5 * se


def test_rollout_infer_consistency():
    cfg = synth.get_config("tiny")
    spec = L.NetSpec(cfg.net.obs_dim, cfg.net.act_dim, tuple(cfg.net.hidden))
    theta = synth.xavier_theta(cfg.net, seed=0, logstd=-0.3)
    obs = synth.rollout.gaussian_like((16, cfg.net.obs_dim), seed=1)
    out = P.rollout_infer(theta, spec, obs, seed=9, t=2, iteration=3)
    logstd = float(np.float32(-0.3))          # the value stored in the float32 vector
    sigma = np.exp(logstd)
    np.testing.assert_allclose(out["actions"], out["mu"] + sigma * out["eps"], rtol=1e-14)
    # log-prob of a = mu + sigma * eps reduces to the standard normal log density of eps
    ref = scipy.stats.norm.logpdf(out["eps"]).sum(axis=1) - cfg.net.act_dim * logstd
    np.testing.assert_allclose(out["logp"], ref, rtol=1e-12)
    np.testing.assert_allclose(out["values"], P.critic_values(theta, spec, obs), rtol=1e-14)
