"""HIP path against the FP64 oracle, through the C ABI (needs an MI355X)."""

import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
import synth
from oracle import (PPOHyper, advantage_stats, adam_step, clip_coef, gae, normalize_advantages, param_layout,
                    philox4x32_10, ppo_loss_grad, rollout_infer)
from oracle.ppo import minibatch
from tests.gpu_common import dev, oracle_view, require_gpu, round_hidden_weights, spec_of, teacher_batch
from tests.parity import (TOL, assert_close, assert_grad_close, grad_report, per_tensor_errors, rel_errors,
                          tie_bands)

pytestmark = pytest.mark.gpu


def param_name(spec):
    lay = sorted((off, name) for name, (off, shp) in param_layout(spec).items() if name != "__total__")

    def where(i):
        name = [n for off, n in lay if off <= i][-1]
        return f"({name})"
    return where


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


# ------------------------------------------------------------------ Philox
@pytest.mark.parametrize("seed,c0,c1,c2,c3", [
    (0, 0, 0, 0, 1),
    (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF - 5000, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),   # counter wrap
    (0x123456789ABCDEF0, 77, 23, 4, 1),
])
def test_philox_bit_exact(seed, c0, c1, c2, c3):
    d = require_gpu()
    n = 1 << 20
    _announce(f"philox n={n} seed={seed:#x} c0={c0:#x}")
    out = torch.empty(4 * n, dtype=torch.int32, device=d)
    ppo.ppo_philox_blocks(seed, c0, c1, c2, c3, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(n, 4)
    ctr0 = (np.uint64(c0) + np.arange(n, dtype=np.uint64)) & np.uint64(0xFFFFFFFF)
    ref = np.stack(philox4x32_10(ctr0, c1, c2, c3, seed & 0xFFFFFFFF, seed >> 32), axis=1)
    np.testing.assert_array_equal(got, ref)


# --------------------------------------------------------------------- GAE
GAE_CASES = [
    ("tiny", 0.99, 0.95, True, True),
    ("tiny", 0.99, 1.0, False, False),
    ("tiny", 0.9, 0.0, True, False),
    ("flat", 0.99, 0.95, True, True),
    ("flat", 0.99, 0.95, False, True),
]


@pytest.mark.parametrize("name,gamma,lam,timeouts,normalize", GAE_CASES)
def test_gae(name, gamma, lam, timeouts, normalize):
    d = require_gpu()
    cfg = synth.get_config(name)
    T, N = cfg.n_steps, cfg.n_envs
    _announce(f"gae {name} T={T} N={N} lam={lam} timeouts={timeouts} normalize={normalize}")
    roll = synth.make_rollout(cfg, with_timeouts=True)
    values = synth.rollout.gaussian_like((T, N), seed=11, scale=0.5)
    last = synth.rollout.gaussian_like((N,), seed=12, scale=0.5)
    to = roll["timeouts"] if timeouts else None
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "fp32")
    adv = torch.empty(T, N, device=d)
    ret = torch.empty(T, N, device=d)
    stats = torch.empty(2, dtype=torch.float64, device=d)
    ppo.ppo_gae(ctx, dev(roll["rewards"], d), dev(roll["dones"], d), dev(values, d), dev(last, d), gamma, lam,
                adv, ret, stats, timeouts=dev(to, d) if to is not None else None, normalize=normalize)
    torch.cuda.synchronize()
    a_ref, r_ref = gae(roll["rewards"], values, roll["dones"], last, gamma, lam, timeouts=to)
    mean, std = advantage_stats(a_ref)
    assert_close("returns", ret.cpu().numpy(), r_ref, TOL["fp32"])
    st = stats.cpu().numpy()
    rms = np.sqrt(np.mean(a_ref ** 2))
    assert abs(st[0] - mean) <= TOL["fp32"] * rms
    assert abs(st[1] - std) <= TOL["fp32"] * std
    if normalize:
        assert_close("adv_normalised", adv.cpu().numpy(), normalize_advantages(a_ref, mean, std), TOL["fp32"])
    else:
        assert_close("adv", adv.cpu().numpy(), a_ref, TOL["fp32"])


def test_gae_ragged_small():
    d = require_gpu()
    ctx = ppo.Context(8, 2, (16,), "fp32")
    for T, N in [(1, 2), (3, 1), (5, 65), (64, 130), (100, 3), (384, 130), (1536, 128)]:
        _announce(f"gae ragged T={T} N={N}")
        rng = np.random.default_rng(T * 1000 + N)
        r = rng.normal(0, 1, (T, N)).astype(np.float32)
        v = rng.normal(0, 1, (T, N)).astype(np.float32)
        dn = (rng.random((T, N)) < 0.3).astype(np.uint8)
        to = (dn.astype(bool) & (rng.random((T, N)) < 0.5)).astype(np.uint8)
        last = rng.normal(0, 1, N).astype(np.float32)
        adv = torch.empty(T, N, device=d)
        ret = torch.empty(T, N, device=d)
        st = torch.empty(2, dtype=torch.float64, device=d)
        ppo.ppo_gae(ctx, dev(r, d), dev(dn, d), dev(v, d), dev(last, d), 0.97, 0.9, adv, ret, st,
                    timeouts=dev(to, d), normalize=False)
        torch.cuda.synchronize()
        a_ref, r_ref = gae(r, v, dn, last, 0.97, 0.9, timeouts=to)
        assert_close("adv", adv.cpu().numpy(), a_ref, TOL["fp32"])
        assert_close("returns", ret.cpu().numpy(), r_ref, TOL["fp32"])


# ----------------------------------------------------------- rollout infer
@pytest.mark.parametrize("name,prec,N", [("tiny", "fp32", 64), ("tiny", "bf16", 64), ("flat", "fp32", 4096),
                                         ("flat", "bf16", 4096), ("rough", "bf16", 4096), ("rough", "fp32", 333),
                                         ("large", "bf16", 16384), ("large", "fp32", 1000)])
def test_rollout_infer(name, prec, N):
    d = require_gpu()
    cfg = synth.get_config(name)
    _announce(f"rollout {name} {prec} N={N}")
    spec = spec_of(cfg)
    theta = synth.xavier_theta(cfg.net, seed=0, logstd=-0.4)
    obs = synth.make_rollout(cfg)["obs"][3][:N]
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
    params = ppo.Params(ctx, theta, device=d)
    A = cfg.net.act_dim
    actions = torch.empty(N, A, device=d)
    logp = torch.empty(N, device=d)
    values = torch.empty(N, device=d)
    mu = torch.empty(N, A, device=d)
    ppo.ppo_rollout_infer(ctx, params, dev(obs, d), t=3, seed=42, iteration=7, actions=actions, logp=logp,
                          values=values, mu=mu)
    v_only = torch.empty(N, device=d)
    ppo.ppo_rollout_infer(ctx, params, dev(obs, d), t=3, seed=42, iteration=7, values=v_only)
    torch.cuda.synchronize()
    ref = rollout_infer(theta, spec, obs, seed=42, t=3, iteration=7)
    tol = TOL[prec]
    assert_close("mu", mu.cpu().numpy(), ref["mu"], tol)
    assert_close("values", values.cpu().numpy(), ref["values"], tol)
    assert_close("actions", actions.cpu().numpy(), ref["actions"], tol)
    # log-density of a = mu + sigma eps depends on eps and sigma only
    assert_close("logp", logp.cpu().numpy(), ref["logp"], TOL["fp32"])
    np.testing.assert_array_equal(v_only.cpu().numpy(), values.cpu().numpy())
    # noise recovered from the outputs matches the oracle's Philox/Box-Muller draw
    eps = (actions - mu).cpu().numpy() / np.exp(np.float32(-0.4))
    assert_close("eps", eps, ref["eps"], 1e-5 if prec == "fp32" else 1e-4)


# ------------------------------------------------------ loss and gradient
LOSS_CASES = [("tiny", "fp32", 1536, "near"), ("tiny", "fp32", 1536, "mixed"), ("tiny", "bf16", 1536, "mixed"),
              ("tiny", "fp32", 1000, "mixed"), ("flat", "fp32", 24576, "mixed"), ("flat", "bf16", 24576, "mixed"),
              ("rough", "bf16", 4096, "mixed"), ("rough", "fp32", 2000, "near"),
              ("large", "bf16", 8192, "mixed"),
              # ragged row blocks of the fused bf16 pass (64 rows; 32 for the large widths)
              ("flat", "bf16", 1000, "mixed"), ("rough", "bf16", 777, "near"), ("large", "bf16", 333, "mixed")]


@pytest.mark.parametrize("name,prec,M,shift", LOSS_CASES)
def test_loss_grad(name, prec, M, shift):
    _check_loss_grad(name, prec, M, shift, "gae")


@pytest.mark.parametrize("name,M", [("tiny", 1536), ("flat", 24576)])
def test_loss_grad_bf16_converged_critic(name, M):
    """Returns = V + zero-mean noise: the true critic gradient is small, so a
    systematic shift of V would show in every critic tensor (the critic's
    hidden weights enter its GEMMs as a bf16 pair to keep that shift below
    the tolerance)."""
    _check_loss_grad(name, "bf16", M, "mixed", "converged")


def check_grad_vs_oracle(g, theta, spec, mb, hp, prec, gpu_active=None, gpu_ratio=None):
    """The gradient against the FP64 oracle at theta, per parameter tensor
    (normwise, tol of the precision), and as a whole vector.  With the GPU's
    per-sample ratios and branches (exported by ppo_loss_grad) the ratios are
    gated normwise at the precision's tolerance, each within 5x of it (the
    ratio is an intermediate: with bf16 operands the largest per-sample
    errors over a mini-batch reach several per cent, which a CPU emulation of
    the bf16 rounding points reproduces sample by sample), and a sample takes
    the GPU's branch
    where the GPU's ratio could lie across the deciding clip edge from the
    oracle's (tie_bands); no other sample may disagree.  Elementwise errors
    with the rms floor are printed per tensor; for bf16 the distance to the
    oracle at the effective bf16 weights is printed as a diagnostic.  Returns
    the oracle's result."""
    tol = TOL[prec]
    lay = param_layout(spec)
    band = 0.0
    if gpu_active is not None:
        own = ppo_loss_grad(theta, spec, mb, hp, want_grad=False)
        assert_close("ratio", gpu_ratio, own["ratio"], tol, elementwise=False)
        worst = np.max(np.abs(np.asarray(gpu_ratio, np.float64) / own["ratio"] - 1.0))
        print(f"[parity] ratio: largest per-sample relative error {worst:.2e}")
        assert worst <= 5 * tol, worst
        band = tie_bands(gpu_ratio, own["ratio"])
    ref = ppo_loss_grad(theta, spec, mb, hp, active_override=gpu_active, tie_delta=band)
    if gpu_active is not None:
        print(f"[parity] clip-edge ties adopted from the GPU: {ref['ties_adopted']} "
              f"({int(np.sum(ref['margin'] < band))} samples within their band)")
        assert ref["disagree_outside"] == 0, f"{ref['disagree_outside']} samples decided differently outside the band"
    rep = grad_report(g, ref["grad"], lay)
    print("[parity] per tensor (normwise, elementwise):",
          {k: f"{a:.1e}/{b:.1e}" for k, (a, b) in rep.items()})
    if prec == "bf16":
        ref_q = ppo_loss_grad(round_hidden_weights(theta, spec), spec, mb, hp, active_override=gpu_active,
                              tie_delta=band)
        print("[parity] diagnostic, vs the oracle at the effective bf16 weights:",
              {k: f"{v:.1e}" for k, v in per_tensor_errors(g, ref_q["grad"], lay).items()})
    assert_grad_close(f"grad_{prec}_vs_fp64", g, ref["grad"], tol, lay)
    return ref


def _check_loss_grad(name, prec, M, shift, returns):
    d = require_gpu()
    cfg = synth.get_config(name)
    _announce(f"loss_grad {name} {prec} M={M} {shift} returns={returns}")
    spec = spec_of(cfg)
    theta = synth.xavier_theta(cfg.net, seed=1, logstd=-0.2)
    B = 2 * M
    batch = teacher_batch(cfg, theta, B, seed=5, shift=shift, returns=returns)
    idx = np.random.default_rng(6).permutation(B)[:M].astype(np.int32)
    hp = PPOHyper()
    mb = minibatch(oracle_view(batch), idx)

    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
    params = ppo.Params(ctx, theta, device=d)
    tb = {k: dev(v, d) for k, v in batch.items()}
    stats = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    grad = torch.zeros(ctx.param_count, device=d)
    active = torch.full((M,), 7, dtype=torch.uint8, device=d)
    ratio = torch.full((M,), float("nan"), device=d)
    ws = ctx.new_workspace(M=M)
    ppo.ppo_loss_grad(ctx, params, tb, dev(idx, d), ppo.UpdateHParams(), stats, grad, ws, active_out=active,
                      ratio_out=ratio)
    torch.cuda.synchronize()
    tol = TOL[prec]
    g = grad.cpu().numpy()
    act = active.cpu().numpy()
    assert set(np.unique(act)) <= {0, 1}
    ref = check_grad_vs_oracle(g, theta, spec, mb, hp, prec, act.astype(bool), ratio.cpu().numpy())
    assert np.min(ref["margin"]) > 0.05            # the teacher batch keeps every ratio off the clip edges
    np.testing.assert_array_equal(act.astype(bool), ref["active"])
    st = ppo.stats_dict(stats.cpu().numpy())
    assert st["flags"] == 0.0
    for key in ("policy_loss", "value_loss", "entropy", "loss"):
        assert abs(st[key] - ref[key]) <= tol * (abs(ref[key]) + 0.1), (key, st[key], ref[key])
    assert st["clip_frac"] == pytest.approx(ref["clip_frac"], abs=1e-6)
    assert st["grad_norm"] == pytest.approx(np.linalg.norm(ref["grad"]), rel=tol)
    assert abs(st["approx_kl"] - ref["approx_kl"]) <= max(1e-4, 5 * tol) * (abs(ref["approx_kl"]) + 1e-3)


# ------------------------------------------------------------ update epoch
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_update_epoch_teacher_forced(prec):
    """One mini-batch step (the 64x24 workload: 1 epoch x 1 mini-batch)."""
    d = require_gpu()
    cfg = synth.get_config("tiny")
    _announce(f"update_epoch tiny {prec}")
    spec = spec_of(cfg)
    theta = synth.xavier_theta(cfg.net, seed=0)
    B = cfg.batch
    batch = teacher_batch(cfg, theta, B, seed=9, shift="mixed")
    perm = np.random.default_rng(10).permutation(B).astype(np.int32)
    hp = PPOHyper()
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
    params = ppo.Params(ctx, theta, lr=hp.lr, device=d)
    params.step.fill_(3)
    m0 = synth.rollout.gaussian_like((ctx.param_count,), seed=13, scale=1e-3)
    v0 = np.abs(synth.rollout.gaussian_like((ctx.param_count,), seed=14, scale=1e-5))
    params.adam_m.copy_(dev(m0, d))
    params.adam_v.copy_(dev(v0, d))
    tb = {k: dev(v, d) for k, v in batch.items()}
    stats = torch.zeros(1, ppo.PPO_STATS_WIDTH, device=d)
    ws = ctx.new_workspace(M=B)
    ppo.ppo_update_epoch(ctx, params, tb, dev(perm, d), 1, ppo.UpdateHParams(), stats, ws)
    torch.cuda.synchronize()
    tol = TOL[prec]
    ref = ppo_loss_grad(theta, spec, minibatch(oracle_view(batch), perm), hp)
    g_gpu = params.grad.cpu().numpy().astype(np.float64)
    check_grad_vs_oracle(g_gpu, theta, spec, minibatch(oracle_view(batch), perm), hp, prec)
    # Adam given the device's own gradient (teacher forcing of the optimiser step)
    c, _ = clip_coef(g_gpu, hp.max_grad_norm)
    th_ref, m_ref, v_ref = adam_step(theta, m0, v0, c * g_gpu, 3, hp)
    assert_close("adam_m", params.adam_m.cpu().numpy(), m_ref, TOL["fp32"])
    assert_close("adam_v", params.adam_v.cpu().numpy(), v_ref, TOL["fp32"])
    assert_close("theta", params.theta.cpu().numpy(), th_ref, TOL["fp32"])
    assert int(params.step[0].item()) == 4
    if prec == "bf16":
        sh = params.shadow.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        np.testing.assert_allclose(sh.view(np.float32), params.theta.cpu().numpy(), rtol=2 ** -8)
    st = ppo.stats_dict(stats[0].cpu().numpy())
    assert st["grad_norm"] == pytest.approx(np.linalg.norm(ref["grad"]), rel=tol)


def test_update_epoch_teacher_forced_full_minibatch():
    """The bench's configuration at full size: bf16, the 4096 x 24 network,
    one mini-batch step of 24576 samples through the graph-captured epoch
    (fused pass, weight gradients, reduction, Adam), with the gradient gated
    as for the other bf16 cases and the optimiser state teacher-forced with
    the device's own gradient."""
    d = require_gpu()
    cfg = synth.get_config("flat")
    M = cfg.minibatch
    _announce(f"update_epoch flat bf16 M={M}")
    spec = spec_of(cfg)
    theta = synth.xavier_theta(cfg.net, seed=2, logstd=-0.3)
    batch = teacher_batch(cfg, theta, M, seed=21, shift="mixed")
    perm = np.random.default_rng(22).permutation(M).astype(np.int32)
    hp = PPOHyper()
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "bf16")
    assert ctx.fused_shape()[0] > 0
    params = ppo.Params(ctx, theta, lr=hp.lr, device=d)
    params.step.fill_(7)
    m0 = synth.rollout.gaussian_like((ctx.param_count,), seed=23, scale=1e-3)
    v0 = np.abs(synth.rollout.gaussian_like((ctx.param_count,), seed=24, scale=1e-5))
    params.adam_m.copy_(dev(m0, d))
    params.adam_v.copy_(dev(v0, d))
    tb = {k: dev(v, d) for k, v in batch.items()}
    stats = torch.zeros(1, ppo.PPO_STATS_WIDTH, device=d)
    ws = ctx.new_workspace(M=M)
    ppo.ppo_update_epoch(ctx, params, tb, dev(perm, d), 1, ppo.UpdateHParams(use_graph=True), stats, ws)
    torch.cuda.synchronize()
    mb = minibatch(oracle_view(batch), perm)
    ref = ppo_loss_grad(theta, spec, mb, hp)
    g_gpu = params.grad.cpu().numpy().astype(np.float64)
    check_grad_vs_oracle(g_gpu, theta, spec, mb, hp, "bf16")
    c, _ = clip_coef(g_gpu, hp.max_grad_norm)
    th_ref, m_ref, v_ref = adam_step(theta, m0, v0, c * g_gpu, 7, hp)
    assert_close("adam_m", params.adam_m.cpu().numpy(), m_ref, TOL["fp32"])
    assert_close("adam_v", params.adam_v.cpu().numpy(), v_ref, TOL["fp32"])
    assert_close("theta", params.theta.cpu().numpy(), th_ref, TOL["fp32"])
    assert int(params.step[0].item()) == 8
    st = ppo.stats_dict(stats[0].cpu().numpy())
    assert st["grad_norm"] == pytest.approx(np.linalg.norm(ref["grad"]), rel=TOL["bf16"])
    assert st["policy_loss"] == pytest.approx(ref["policy_loss"], rel=TOL["bf16"], abs=2e-3)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_update_epoch_graph_matches_eager_and_is_deterministic(prec):
    d = require_gpu()
    cfg = synth.get_config("tiny")
    _announce(f"graph vs eager tiny {prec}")
    theta = synth.xavier_theta(cfg.net, seed=2)
    B, K = cfg.batch, 4
    batch = teacher_batch(cfg, theta, B, seed=3, shift="mixed")
    perm = np.random.default_rng(4).permutation(B).astype(np.int32)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
    tb = {k: dev(v, d) for k, v in batch.items()}
    ws = ctx.new_workspace(M=B // K)
    results = []
    for use_graph, reps in ((False, 1), (True, 3)):
        params = ppo.Params(ctx, theta, device=d)
        stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
        for _ in range(reps):
            # replays with host work and synchronisation in between
            ppo.ppo_update_epoch(ctx, params, tb, dev(perm, d), K, ppo.UpdateHParams(use_graph=use_graph),
                                 stats, ws)
            torch.cuda.synchronize()
            results.append((use_graph, params.theta.cpu().numpy().copy(), stats.cpu().numpy().copy()))
    eager_theta, eager_stats = results[0][1], results[0][2]
    # first graph replay starts from the same state as the eager run
    np.testing.assert_array_equal(results[1][1], eager_theta)
    np.testing.assert_array_equal(results[1][2], eager_stats)
    # later replays continue training (step count advanced by K each time)
    assert not np.array_equal(results[2][1], results[1][1])


def test_update_epoch_multi_step_tracks_oracle():
    """Four mini-batch steps in float32, free running (drift reported, loose gate)."""
    d = require_gpu()
    cfg = synth.get_config("tiny")
    spec = spec_of(cfg)
    _announce("update_epoch tiny fp32 K=4 free running")
    theta = synth.xavier_theta(cfg.net, seed=7)
    B, K = cfg.batch, 4
    batch = teacher_batch(cfg, theta, B, seed=8, shift="near")
    perm = np.random.default_rng(9).permutation(B).astype(np.int32)
    hp = PPOHyper()
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "fp32")
    params = ppo.Params(ctx, theta, device=d)
    stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
    ws = ctx.new_workspace(M=B // K)
    ppo.ppo_update_epoch(ctx, params, {k: dev(v, d) for k, v in batch.items()}, dev(perm, d), K,
                         ppo.UpdateHParams(), stats, ws)
    torch.cuda.synchronize()
    from oracle import update_epoch
    n = ctx.param_count
    th, m, v, step, rec = update_epoch(theta, np.zeros(n), np.zeros(n), 0, spec, oracle_view(batch), perm, K, hp)
    st = stats.cpu().numpy()
    for k in range(K):
        assert st[k, 0] == pytest.approx(rec[k]["loss"], rel=1e-4, abs=1e-5)
        assert st[k, 6] == pytest.approx(rec[k]["grad_norm"], rel=1e-4)
    nw, _ = rel_errors(params.theta.cpu().numpy() - theta, th - theta)
    assert nw < 1e-3, nw


@pytest.mark.parametrize("desired_kl", [0.0, 0.01])
def test_profiled_epoch_with_repeats_matches_plain_epoch(desired_kl):
    """The measurement entry point repeats idempotent launches inside its
    event pairs; the epoch's results must equal the plain eager epoch's."""
    d = require_gpu()
    cfg = synth.get_config("tiny")
    _announce(f"profiled epoch reps=3 desired_kl={desired_kl}")
    from tests.gpu_common import add_kl_inputs
    theta = synth.xavier_theta(cfg.net, seed=21)
    B, K = cfg.batch, 4
    batch = add_kl_inputs(cfg, theta, teacher_batch(cfg, theta, B, seed=22, shift="mixed"), seed=23,
                          shift_scale=0.05)
    perm = np.random.default_rng(24).permutation(B).astype(np.int32)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "bf16")
    tb = {k: dev(v, d) for k, v in batch.items()}
    hp = ppo.UpdateHParams(use_graph=False, desired_kl=desired_kl)
    out = []
    for reps in (None, 3):
        params = ppo.Params(ctx, theta, device=d)
        stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
        ws = ctx.new_workspace(M=B // K)
        if reps is None:
            ppo.ppo_update_epoch(ctx, params, tb, dev(perm, d), K, hp, stats, ws)
        else:
            ph = ppo.ppo_update_epoch_profiled(ctx, params, tb, dev(perm, d), K, hp, stats, ws, reps=reps)
            if ctx.fused_shape()[0]:
                assert ph["fused"][1] == K and ph["forward"][1] == 0 and ph["adam"][1] == K
            else:
                assert ph["forward"][1] == K * len(cfg.net.hidden) and ph["adam"][1] == K
        torch.cuda.synchronize()
        out.append((params.theta.cpu().numpy().copy(), params.lr.cpu().numpy().copy(), stats.cpu().numpy().copy()))
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)
