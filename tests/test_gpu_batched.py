"""Uneven concurrent runs updated together (needs an MI355X).

Every run's epoch in ppo_update_batched must equal the same run updated alone
by ppo_update_epoch with the same (128 x 128) tiles, bit for bit, and the
graph-replayed batched epoch must equal its eager launch.  Two network
shapes: hidden (128, 64, 32), which the bf16 fused pass does not cover (step k
of every run together, in grouped layer-by-layer launches), and the sweep
workload's (512, 256, 128), which it does (each run's whole epoch on one of
the side streams; with PPO_BATCHED_GROUPED=1 step k of every run together:
one fused pass per run on the side streams, then the grouped weight-gradient
launch)."""
import os

import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
import synth
from tests.gpu_common import add_kl_inputs, dev, require_gpu, teacher_batch

pytestmark = pytest.mark.gpu

# (n_envs, n_steps, obs_dim): uneven sizes and both observation widths
SHAPES = {
    (128, 64, 32): [(64, 16, 48), (96, 24, 235), (160, 24, 48), (40, 50, 235)],
    (512, 256, 128): [(512, 16, 48), (1024, 24, 235), (768, 24, 48), (400, 50, 235)],
}
K = 4


def _runs(prec, hidden):
    out = []
    for r, (N, T, D) in enumerate(SHAPES[hidden]):
        cfg = synth.configs.PPOConfig(name=f"run{r}", n_envs=N, n_steps=T, net=synth.NetShape(D, 12, hidden),
                                      epochs=1, minibatches=K, seed=r)
        theta = synth.xavier_theta(cfg.net, seed=r, logstd=-0.3)
        batch = teacher_batch(cfg, theta, cfg.batch, seed=10 + r, shift="mixed")
        # collection-time means: KL well above, below and inside the adaptive band per run
        batch = add_kl_inputs(cfg, theta, batch, seed=30 + r, shift_scale=(0.08, 0.004, 0.033, 0.08)[r],
                              logstd_shift=0.01)
        perm = np.random.default_rng(20 + r).permutation(cfg.batch).astype(np.int32)
        out.append((cfg, theta, batch, perm))
    return out


def _state(params):
    return [params.theta.cpu().numpy().copy(), params.adam_m.cpu().numpy().copy(),
            params.adam_v.cpu().numpy().copy(), params.lr.cpu().numpy().copy(), int(params.step[0].item())]


@pytest.fixture
def fixed_tiles(monkeypatch):
    monkeypatch.setenv("PPO_AUTOTUNE", "0")


@pytest.mark.parametrize("prec,desired_kl,hidden,grouped", [
    ("fp32", 0.0, (128, 64, 32), False), ("bf16", 0.0, (128, 64, 32), False), ("bf16", 0.01, (128, 64, 32), False),
    ("bf16", 0.0, (512, 256, 128), False), ("bf16", 0.01, (512, 256, 128), False),
    ("bf16", 0.0, (512, 256, 128), True), ("bf16", 0.01, (512, 256, 128), True)])
def test_batched_equals_solo(prec, desired_kl, hidden, grouped, fixed_tiles, monkeypatch):
    d = require_gpu()
    if grouped:
        monkeypatch.setenv("PPO_BATCHED_GROUPED", "1")
    runs = _runs(prec, hidden)
    print(f"[gpu-case] batched vs solo {prec} desired_kl={desired_kl} hidden={hidden} grouped={grouped} "
          f"runs={SHAPES[hidden]}", flush=True)
    hp = ppo.UpdateHParams(desired_kl=desired_kl)
    ctxs, solo_state, solo_stats = [], [], []
    for cfg, theta, batch, perm in runs:
        ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
        # the sweep shape takes the fused pass in bf16, the small one the grouped GEMMs
        assert (ctx.fused_shape()[0] > 0) == (prec == "bf16" and hidden == (512, 256, 128))
        ctxs.append(ctx)
        params = ppo.Params(ctx, theta, device=d)
        stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
        ws = ctx.new_workspace(M=cfg.minibatch)
        ppo.ppo_update_epoch(ctx, params, {k: dev(v, d) for k, v in batch.items()}, dev(perm, d), K, hp, stats, ws)
        torch.cuda.synchronize()
        solo_state.append(_state(params))
        solo_stats.append(stats.cpu().numpy())

    if desired_kl > 0:
        # run 0 starts far above the band (rate divided), run 1 far below (multiplied)
        assert solo_stats[0][0, 9] == pytest.approx(1e-3 / 1.5, rel=1e-6)
        assert solo_stats[1][0, 9] == pytest.approx(1e-3 * 1.5, rel=1e-6)
    for use_graph in (False, True):
        params, batches, perms, stats, wss = [], [], [], [], []
        for (cfg, theta, batch, perm), ctx in zip(runs, ctxs):
            params.append(ppo.Params(ctx, theta, device=d))
            batches.append({k: dev(v, d) for k, v in batch.items()})
            perms.append(dev(perm, d))
            stats.append(torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d))
            wss.append(ctx.new_workspace(M=cfg.minibatch))
        ppo.ppo_update_batched(ctxs, params, batches, perms, K,
                               ppo.UpdateHParams(use_graph=use_graph, desired_kl=desired_kl), stats, wss)
        torch.cuda.synchronize()
        for r in range(len(runs)):
            got = _state(params[r])
            for a, b in zip(got[:4], solo_state[r][:4]):
                np.testing.assert_array_equal(a, b)
            assert got[4] == solo_state[r][4] == K
            np.testing.assert_array_equal(stats[r].cpu().numpy(), solo_stats[r])


def test_batched_run_against_oracle():
    """One run of the sweep shape (bf16, 235-dim observations) against the
    FP64 oracle: the loss and gradient of its first mini-batch at its initial
    parameters, through the same context and workspace layout the batched
    update uses (per-tensor gate, clip-edge tie protocol)."""
    from oracle import PPOHyper
    from oracle.ppo import minibatch
    from tests.gpu_common import oracle_view, spec_of
    from tests.test_gpu_parity import check_grad_vs_oracle
    d = require_gpu()
    cfg, theta, batch, perm = _runs("bf16", (512, 256, 128))[1]
    print(f"[gpu-case] batched-shape run vs oracle B={cfg.batch} D={cfg.net.obs_dim}", flush=True)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "bf16")
    params = ppo.Params(ctx, theta, device=d)
    M = cfg.minibatch
    idx = perm[:M]
    stats = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    grad = torch.zeros(ctx.param_count, device=d)
    active = torch.zeros(M, dtype=torch.uint8, device=d)
    ratio = torch.zeros(M, device=d)
    ppo.ppo_loss_grad(ctx, params, {k: dev(v, d) for k, v in batch.items()}, dev(idx, d), ppo.UpdateHParams(),
                      stats, grad, ctx.new_workspace(M=M), active_out=active, ratio_out=ratio)
    torch.cuda.synchronize()
    check_grad_vs_oracle(grad.cpu().numpy(), theta, spec_of(cfg), minibatch(oracle_view(batch), idx), PPOHyper(),
                         "bf16", active.cpu().numpy().astype(bool), ratio.cpu().numpy())
