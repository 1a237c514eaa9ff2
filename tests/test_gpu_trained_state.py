"""The gradient of a trained state against the FP64 oracle, with no margin
filtering: the learning iteration of the benchmark workloads (rollout of
4096 environments x 24 steps through the library's own inference, GAE,
then 5 epochs x 4 mini-batches) run for a few iterations on the GPU, after
which one mini-batch's gradient is compared with the oracle's at the same
parameters and inputs.  After several epochs on the same rollout many
ratios sit at the clip edges, so this exercises the clip-edge tie protocol:
the GPU's per-sample ratios are gated against the oracle's, a sample takes
the GPU's branch where the GPU's ratio could lie across the deciding edge
from the oracle's, and every other sample must agree."""
import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
import synth
from oracle import PPOHyper
from oracle.ppo import minibatch
from tests.gpu_common import require_gpu, spec_of
from tests.test_gpu_parity import check_grad_vs_oracle

pytestmark = pytest.mark.gpu


def _train(cfg, prec, iterations, d):
    net = cfg.net
    T, N, D, A = cfg.n_steps, cfg.n_envs, net.obs_dim, net.act_dim
    B, M = cfg.batch, cfg.minibatch
    ctx = ppo.Context(D, A, net.hidden, prec)
    params = ppo.Params(ctx, synth.xavier_theta(net, seed=cfg.seed), lr=cfg.lr, device=d)
    roll = synth.make_rollout(cfg, with_timeouts=True)
    obs = torch.as_tensor(roll["obs"]).to(d)
    last_obs = torch.as_tensor(roll["last_obs"]).to(d)
    rewards = torch.as_tensor(roll["rewards"]).to(d)
    dones = torch.as_tensor(roll["dones"]).to(d)
    timeouts = torch.as_tensor(roll["timeouts"]).to(d)
    actions = torch.empty(T, N, A, device=d)
    logp = torch.empty(T, N, device=d)
    values = torch.empty(T, N, device=d)
    last_v = torch.empty(N, device=d)
    adv = torch.empty(T, N, device=d)
    ret = torch.empty(T, N, device=d)
    st = torch.empty(2, dtype=torch.float64, device=d)
    perms = torch.as_tensor(synth.make_permutations(B, cfg.epochs, seed=cfg.seed)).to(d)
    stats = torch.zeros(cfg.epochs, cfg.minibatches, ppo.PPO_STATS_WIDTH, device=d)
    ws = ctx.new_workspace(N=N, T=T, M=M, device=d)
    hp = ppo.UpdateHParams(clip=cfg.clip, value_coef=cfg.value_coef, entropy_coef=cfg.entropy_coef,
                           max_grad_norm=cfg.max_grad_norm, use_graph=True)
    batch = dict(obs=obs.view(B, D), actions=actions.view(B, A), logp=logp.view(B), adv=adv.view(B),
                 returns=ret.view(B))
    for it in range(iterations):
        for t in range(T):
            ppo.ppo_rollout_infer(ctx, params, obs[t], t, cfg.seed, it, actions=actions[t], logp=logp[t],
                                  values=values[t], ws=ws)
        ppo.ppo_rollout_infer(ctx, params, last_obs, T, cfg.seed, it, values=last_v, ws=ws)
        ppo.ppo_gae(ctx, rewards, dones, values, last_v, cfg.gamma, cfg.lam, adv, ret, st, timeouts=timeouts,
                    normalize=True, ws=ws)
        for e in range(cfg.epochs):
            ppo.ppo_update_epoch(ctx, params, batch, perms[e], cfg.minibatches, hp, stats[e], ws)
    return ctx, params, batch, perms, hp, ws


@pytest.mark.parametrize("name,prec,iterations", [("flat", "bf16", 4), ("rough", "bf16", 3), ("flat", "fp32", 2)])
def test_trained_state_gradient(name, prec, iterations):
    d = require_gpu()
    cfg = synth.get_config(name)
    print(f"[gpu-case] trained state {name} {prec} iterations={iterations}", flush=True)
    ctx, params, batch, perms, hp, ws = _train(cfg, prec, iterations, d)
    M = cfg.minibatch
    idx = perms[0][:M].contiguous()
    grad = torch.zeros(ctx.param_count, device=d)
    stats = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    active = torch.full((M,), 7, dtype=torch.uint8, device=d)
    ratio = torch.full((M,), float("nan"), device=d)
    ppo.ppo_loss_grad(ctx, params, batch, idx, hp, stats, grad, ws, active_out=active, ratio_out=ratio)
    torch.cuda.synchronize()
    theta = params.theta.cpu().numpy().astype(np.float64)
    full = {k: v.cpu().numpy() for k, v in batch.items()}
    mb = minibatch(dict(obs=full["obs"], actions=full["actions"], logp_old=full["logp"], adv=full["adv"],
                        returns=full["returns"]), idx.cpu().numpy())
    hpo = PPOHyper(clip=cfg.clip, value_coef=cfg.value_coef, entropy_coef=cfg.entropy_coef,
                   max_grad_norm=cfg.max_grad_norm, lr=cfg.lr)
    act = active.cpu().numpy()
    assert set(np.unique(act)) <= {0, 1}
    ref = check_grad_vs_oracle(grad.cpu().numpy(), theta, spec_of(cfg), mb, hpo, prec, act.astype(bool),
                               ratio.cpu().numpy())
    # the state really is trained: some samples clipped, some near the edges
    assert ref["clip_frac"] > 0.05
    st = ppo.stats_dict(stats.cpu().numpy())
    assert st["grad_norm"] == pytest.approx(np.linalg.norm(ref["grad"]), rel=2e-2)
