"""Edge shapes at the limits of the C ABI against the oracle: the longest
horizon, the widest action vector and one not a multiple of four, a single
hidden layer and the most hidden layers, the widest layers, tiny and ragged
batches."""
import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
import synth
from oracle import (NetSpec, PPOHyper, gae, param_layout, ppo_loss_grad, rollout_infer)
from oracle.ppo import minibatch
from tests.gpu_common import dev, oracle_view, require_gpu, teacher_batch
from tests.parity import TOL, assert_close, assert_grad_close

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _cfg(D, A, H):
    return synth.configs.PPOConfig(name=f"edge_d{D}_a{A}_h{'x'.join(map(str, H))}", n_envs=8, n_steps=8,
                                   net=synth.NetShape(D, A, tuple(H)), epochs=1, minibatches=1)


# (obs dim, actions, hidden widths, precision, rows)
SHAPES = [
    (5, 1, (16,), "fp32", 3),                      # smallest net, one action, one hidden layer
    (37, 16, (32, 48, 16, 64), "fp32", 77),        # widest action vector, four hidden layers
    (235, 13, (64, 32), "bf16", 129),              # A not a multiple of 4
    (1000, 12, (2048,), "fp32", 64),               # widest hidden layer, wide input
    (48, 12, (2048, 32), "bf16", 33),
]


@pytest.mark.parametrize("D,A,H,prec,N", SHAPES)
def test_rollout_edges(D, A, H, prec, N):
    d = require_gpu()
    _announce(f"rollout edge D={D} A={A} H={H} {prec} N={N}")
    cfg = _cfg(D, A, H)
    spec = NetSpec(D, A, tuple(H))
    theta = synth.xavier_theta(cfg.net, seed=3, logstd=-0.25)
    obs = synth.rollout.gaussian_like((N, D), seed=5)
    ctx = ppo.Context(D, A, H, prec)
    params = ppo.Params(ctx, theta, device=d)
    out = dict(actions=torch.empty(N, A, device=d), logp=torch.empty(N, device=d),
               values=torch.empty(N, device=d), mu=torch.empty(N, A, device=d))
    ppo.ppo_rollout_infer(ctx, params, dev(obs, d), t=2, seed=99, iteration=4, **out)
    torch.cuda.synchronize()
    ref = rollout_infer(theta, spec, obs, seed=99, t=2, iteration=4)
    tol = TOL[prec]
    assert_close("mu", out["mu"].cpu().numpy(), ref["mu"], tol)
    assert_close("values", out["values"].cpu().numpy(), ref["values"], tol)
    assert_close("logp", out["logp"].cpu().numpy(), ref["logp"], TOL["fp32"])
    eps = (out["actions"] - out["mu"]).cpu().numpy() / np.exp(np.float32(-0.25))
    assert_close("eps", eps, ref["eps"], 1e-5 if prec == "fp32" else 1e-4)


@pytest.mark.parametrize("D,A,H,prec,N", [s for s in SHAPES if s[3] == "fp32"])
def test_loss_grad_edges(D, A, H, prec, N):
    d = require_gpu()
    M = max(N, 2)
    _announce(f"loss_grad edge D={D} A={A} H={H} M={M}")
    cfg = _cfg(D, A, H)
    spec = NetSpec(D, A, tuple(H))
    theta = synth.xavier_theta(cfg.net, seed=4, logstd=-0.2)
    B = 2 * M
    batch = teacher_batch(cfg, theta, B, seed=6, shift="mixed")
    idx = np.random.default_rng(8).permutation(B)[:M].astype(np.int32)
    hp = PPOHyper()
    ref = ppo_loss_grad(theta, spec, minibatch(oracle_view(batch), idx), hp)
    ctx = ppo.Context(D, A, H, prec)
    params = ppo.Params(ctx, theta, device=d)
    tb = {k: dev(v, d) for k, v in batch.items()}
    stats = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    grad = torch.zeros(ctx.param_count, device=d)
    ppo.ppo_loss_grad(ctx, params, tb, dev(idx, d), ppo.UpdateHParams(), stats, grad, ctx.new_workspace(M=M))
    torch.cuda.synchronize()
    assert_grad_close("grad", grad.cpu().numpy(), ref["grad"], TOL[prec], param_layout(spec))


@pytest.mark.parametrize("T,N", [(4096, 3), (4096, 1)])   # 4096 = PPO_MAX_T
def test_gae_longest_horizon(T, N):
    """The longest horizon the ABI takes, with episode ends and time-outs."""
    d = require_gpu()
    _announce(f"gae T={T} N={N}")
    rng = np.random.default_rng(T + N)
    r = rng.normal(0, 0.1, (T, N)).astype(np.float32)
    v = rng.normal(0, 1, (T, N)).astype(np.float32)
    dn = (rng.random((T, N)) < 2e-3).astype(np.uint8)
    to = (dn.astype(bool) & (rng.random((T, N)) < 0.5)).astype(np.uint8)
    last = rng.normal(0, 1, N).astype(np.float32)
    ctx = ppo.Context(8, 2, (16,), "fp32")
    adv, ret = torch.empty(T, N, device=d), torch.empty(T, N, device=d)
    st = torch.empty(2, dtype=torch.float64, device=d)
    ppo.ppo_gae(ctx, dev(r, d), dev(dn, d), dev(v, d), dev(last, d), 0.99, 0.95, adv, ret, st,
                timeouts=dev(to, d), normalize=False)
    torch.cuda.synchronize()
    a_ref, r_ref = gae(r, v, dn, last, 0.99, 0.95, timeouts=to)
    assert_close("adv", adv.cpu().numpy(), a_ref, TOL["fp32"])
    assert_close("returns", ret.cpu().numpy(), r_ref, TOL["fp32"])
