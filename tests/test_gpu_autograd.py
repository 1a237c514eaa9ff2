"""Differentiation through torch.autograd.Function over the hand-written
backward: against the FP64 oracle gradient, against central finite
differences of the library's own loss, and directional derivatives at the
235-dim rough-terrain shape (needs an MI355X)."""
import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
import synth
from oracle import NetSpec, PPOHyper, param_layout, ppo_loss_grad
from oracle.ppo import minibatch
from tests.gpu_common import dev, oracle_view, require_gpu, spec_of, teacher_batch
from tests.parity import TOL, assert_grad_close

pytestmark = pytest.mark.gpu


def _small_setup(seed=0):
    D, A, H = 5, 3, (16, 32)
    spec = NetSpec(D, A, H)
    n = param_layout(spec)["__total__"][0]
    theta = (np.random.default_rng(seed).normal(0, 0.4, n)).astype(np.float32)
    cfg = synth.configs.PPOConfig(name="small", n_envs=8, n_steps=9, net=synth.NetShape(D, A, H), epochs=1,
                                  minibatches=1)
    return spec, theta, cfg


def test_autograd_matches_oracle_gradient():
    d = require_gpu()
    spec, theta, cfg = _small_setup()
    B = 72
    batch = teacher_batch(cfg, theta, B, seed=1, shift="mixed")
    idx = np.random.default_rng(2).permutation(B)[:37].astype(np.int32)
    ctx = ppo.Context(spec.obs_dim, spec.act_dim, spec.hidden, "fp32")
    th = torch.tensor(theta, device=d, requires_grad=True)
    loss = ppo.ppo_loss(ctx, th, {k: dev(v, d) for k, v in batch.items()}, dev(idx, d))
    loss.backward()
    ref = ppo_loss_grad(theta, spec, minibatch(oracle_view(batch), idx), PPOHyper())
    assert float(loss) == pytest.approx(ref["loss"], rel=1e-5, abs=1e-6)
    assert_grad_close("autograd grad", th.grad.cpu().numpy(), ref["grad"], TOL["fp32"], param_layout(spec))
    # chain rule through a downstream scalar
    th2 = torch.tensor(theta, device=d, requires_grad=True)
    (3.0 * ppo.ppo_loss(ctx, th2, {k: dev(v, d) for k, v in batch.items()}, dev(idx, d))).backward()
    np.testing.assert_allclose(th2.grad.cpu().numpy(), 3.0 * th.grad.cpu().numpy(), rtol=1e-6)


def test_autograd_central_differences_float32():
    """Central differences of the library's float32 loss (smoke-level
    tolerance: float32 loss values limit the difference quotient)."""
    d = require_gpu()
    spec, theta, cfg = _small_setup(3)
    B = 72
    batch = teacher_batch(cfg, theta, B, seed=4, shift="near")
    idx = torch.arange(B, dtype=torch.int32, device=d)
    tb = {k: dev(v, d) for k, v in batch.items()}
    ctx = ppo.Context(spec.obs_dim, spec.act_dim, spec.hidden, "fp32")
    ws = ctx.new_workspace(M=B)
    th = torch.tensor(theta, device=d, requires_grad=True)
    ppo.ppo_loss(ctx, th, tb, idx, ws=ws).backward()
    g = th.grad.cpu().numpy().astype(np.float64)
    h = 1e-2
    rng = np.random.default_rng(5)
    coords = rng.choice(theta.size, 60, replace=False)
    fd = []
    for c in coords:
        tp, tm = theta.copy(), theta.copy()
        tp[c] += h
        tm[c] -= h
        lp = float(ppo.ppo_loss(ctx, torch.tensor(tp, device=d), tb, idx, ws=ws))
        lm = float(ppo.ppo_loss(ctx, torch.tensor(tm, device=d), tb, idx, ws=ws))
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    scale = np.sqrt(np.mean(g ** 2))
    assert np.max(np.abs(fd - g[coords])) <= 2e-3 * (np.abs(g[coords]).max() + scale)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_directional_derivatives_rough_shape(prec):
    """Directional derivatives of the FP64 oracle's loss (central differences in
    float64) against <grad, u> of the library's gradient, 235-dim observations."""
    d = require_gpu()
    cfg = synth.get_config("rough")
    spec = spec_of(cfg)
    theta = synth.xavier_theta(cfg.net, seed=6, logstd=-0.3)
    M = 1024
    batch = teacher_batch(cfg, theta, M, seed=7, shift="near")
    idx = np.arange(M, dtype=np.int32)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
    th = torch.tensor(theta, device=d, requires_grad=True)
    ppo.ppo_loss(ctx, th, {k: dev(v, d) for k, v in batch.items()}, dev(idx, d)).backward()
    g = th.grad.cpu().numpy().astype(np.float64)
    ob = minibatch(oracle_view(batch), idx)
    hp = PPOHyper()
    rng = np.random.default_rng(8)
    t64 = theta.astype(np.float64)
    for k in range(8):
        u = rng.normal(0, 1, theta.size)
        u /= np.linalg.norm(u)
        eps = 1e-5
        lp = ppo_loss_grad(t64 + eps * u, spec, ob, hp, want_grad=False)["loss"]
        lm = ppo_loss_grad(t64 - eps * u, spec, ob, hp, want_grad=False)["loss"]
        dd = (lp - lm) / (2 * eps)
        tol = 1e-4 if prec == "fp32" else 3e-2
        assert abs(g @ u - dd) <= tol * (abs(dd) + 0.1 * np.linalg.norm(g)), (k, g @ u, dd)


@pytest.mark.parametrize("prec,name", [("fp32", "tiny"), ("bf16", "flat")])
def test_loss_without_gradient_skips_the_backward(prec, name):
    """Without a gradient wanted (no requires_grad, or under no_grad) the loss
    comes from the loss-only call and equals the loss of the full call; the
    loss-only call leaves the gradient norm at 0 and writes no gradient."""
    d = require_gpu()
    cfg = synth.get_config(name)
    print(f"[gpu-case] loss only {prec} {name}", flush=True)
    theta = synth.xavier_theta(cfg.net, seed=5, logstd=-0.2)
    M = 2048 if name == "flat" else 768
    batch = teacher_batch(cfg, theta, 2 * M, seed=6, shift="mixed")
    idx = dev(np.random.default_rng(7).permutation(2 * M)[:M].astype(np.int32), d)
    tb = {k: dev(v, d) for k, v in batch.items()}
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, prec)
    ws = ctx.new_workspace(M=M)
    th = torch.tensor(theta, device=d, requires_grad=True)
    full = ppo.ppo_loss(ctx, th, tb, idx, ws=ws)
    with torch.no_grad():
        l1 = ppo.ppo_loss(ctx, th, tb, idx, ws=ws)
    l2 = ppo.ppo_loss(ctx, th.detach(), tb, idx, ws=ws)
    assert float(l1) == float(full.detach()) and float(l2) == float(full.detach())
    params = ppo.Params(ctx, theta, device=d)
    st_full = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    st_loss = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    grad = torch.zeros(ctx.param_count, device=d)
    ppo.ppo_loss_grad(ctx, params, tb, idx, ppo.UpdateHParams(), st_full, grad, ws)
    from paper_2109_11978_amd import _abi
    from paper_2109_11978_amd.api import _ptr, _stream, batch_abi
    import ctypes
    b, p, h = batch_abi(tb), params.abi(), ppo.UpdateHParams().abi()
    _abi.check(_abi.load().ppo_loss_grad(ctx.handle, _stream(None), ctypes.byref(p), ctypes.byref(b),
                                         _ptr(idx, torch.int32, "idx"), M, ctypes.byref(h),
                                         _ptr(st_loss, torch.float32, "stats"), None, None, None,
                                         _ptr(ws, torch.uint8, "ws"), ws.numel()))
    torch.cuda.synchronize()
    a, c = st_full.cpu().numpy(), st_loss.cpu().numpy()
    np.testing.assert_array_equal(a[[0, 1, 2, 3, 4, 5, 7]], c[[0, 1, 2, 3, 4, 5, 7]])
    assert a[6] > 0 and c[6] == 0.0
