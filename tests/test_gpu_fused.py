"""The fused per-sample pass of the bf16 update (gather, every hidden layer,
output layers with the PPO loss, input-gradient chain in one launch) on an
MI355X: it must be the path the bf16 step takes for the paper's network
shapes, agree with the layer-by-layer kernels it replaces, and keep the
update deterministic.  Its parity with the FP64 oracle is gated by the loss
and gradient cases of test_gpu_parity (bf16 rows of the flat, rough and large
shapes, including ragged row blocks)."""
import os

import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
import synth
from tests.gpu_common import dev, require_gpu, teacher_batch
from tests.parity import rel_errors

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


class _Fused:
    """Sets PPO_FUSED (and optionally the block shape) for the duration of a
    block; the library reads them at every call."""

    KEYS = ("PPO_FUSED", "PPO_FUSED_ROWS", "PPO_FUSED_THREADS", "PPO_FUSED_PER_CU")

    def __init__(self, on, shape=None):
        self.on = on
        self.shape = shape

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.KEYS}
        os.environ["PPO_FUSED"] = "1" if self.on else "0"
        for k in self.KEYS[1:]:
            os.environ.pop(k, None)
        if self.shape:
            os.environ["PPO_FUSED_ROWS"] = str(self.shape[0])
            os.environ["PPO_FUSED_THREADS"] = str(self.shape[1])
            if len(self.shape) > 2:
                os.environ["PPO_FUSED_PER_CU"] = str(self.shape[2])

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _setup(name, M, seed=1):
    d = require_gpu()
    cfg = synth.get_config(name)
    theta = synth.xavier_theta(cfg.net, seed=seed, logstd=-0.2)
    B = 2 * M
    batch = teacher_batch(cfg, theta, B, seed=seed + 4, shift="mixed")
    idx = np.random.default_rng(seed + 5).permutation(B)[:M].astype(np.int32)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "bf16")
    return d, cfg, theta, batch, idx, ctx


def _loss_grad(ctx, theta, batch, idx, d, fused, hp=None, shape=None):
    params = ppo.Params(ctx, theta, device=d)
    tb = {k: dev(v, d) for k, v in batch.items()}
    stats = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    grad = torch.zeros(ctx.param_count, device=d)
    ws = ctx.new_workspace(M=len(idx))
    with _Fused(fused, shape):
        assert (ctx.fused_shape() == tuple(shape or ctx.fused_shape())[:2]) and (ctx.fused_shape()[0] > 0) == fused
        ppo.ppo_loss_grad(ctx, params, tb, dev(idx, d), hp or ppo.UpdateHParams(), stats, grad, ws)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), stats.cpu().numpy()


# every block shape the library can launch: 64 x 256 three per CU (the first
# layer streamed; for rough's 240-wide inputs with the loss inputs loaded
# after the streamed pair), 64 x 256 and 32 x 256 two per CU and 64 x 512 by
# default, 32 x 512 when asked for
SHAPES = [("flat", 24576, None), ("flat", 1000, (64, 512)), ("rough", 777, None), ("large", 333, None),
          ("flat", 10, (64, 256)), ("large", 31, (32, 512)), ("tiny", 1536, (64, 256)), ("rough", 4096, (64, 512)),
          ("flat", 24576, (64, 256, 2)), ("flat", 1000, (64, 256, 3)), ("flat", 77, (64, 256, 3)),
          ("rough", 24576, (64, 256, 2)), ("rough", 77, (64, 256, 3))]


@pytest.mark.parametrize("name,M,shape", SHAPES)
def test_fused_matches_layered(name, M, shape):
    """Same inputs through both paths: the hidden layers round to bf16 at the
    same points and accumulate in the same k order; the output layers sum in a
    different order, so the two differ by float32 rounding, magnified by the
    bf16 rounding of the gradients downstream of it (a few bf16 ulps)."""
    d, cfg, theta, batch, idx, ctx = _setup(name, M)
    _announce(f"fused vs layered {name} M={M} shape={shape}")
    gf, sf = _loss_grad(ctx, theta, batch, idx, d, True, shape=shape)
    gl, sl = _loss_grad(ctx, theta, batch, idx, d, False)
    nw, ew = rel_errors(gf, gl)
    print(f"grad fused vs layered: normwise {nw:.2e}, worst element {ew:.2e}")
    assert np.all(np.isfinite(gf))
    assert nw < 4e-3, nw
    stf, stl = ppo.stats_dict(sf), ppo.stats_dict(sl)
    for key in ("policy_loss", "value_loss", "entropy", "loss", "approx_kl", "grad_norm"):
        assert abs(stf[key] - stl[key]) <= 2e-3 * (abs(stl[key]) + 1e-3), (key, stf[key], stl[key])
    assert stf["clip_frac"] == stl["clip_frac"]


def test_fused_is_the_bf16_path_and_deterministic():
    d, cfg, theta, batch, idx, ctx = _setup("flat", 4096)
    _announce("fused phase accounting and determinism")
    g1, s1 = _loss_grad(ctx, theta, batch, idx, d, True)
    g2, s2 = _loss_grad(ctx, theta, batch, idx, d, True)
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_array_equal(s1, s2)
    # the profiled epoch names the launches: one fused launch per mini-batch
    params = ppo.Params(ctx, theta, device=d)
    tb = {k: dev(v, d) for k, v in batch.items()}
    perm = dev(np.random.default_rng(3).permutation(len(batch["adv"])).astype(np.int32), d)
    K = 2
    ws = ctx.new_workspace(M=len(batch["adv"]) // K)
    stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
    with _Fused(True):
        ph = ppo.ppo_update_epoch_profiled(ctx, params, tb, perm, K, ppo.UpdateHParams(), stats, ws)
    assert ph["fused"][1] == K
    assert ph["forward"][1] == 0 and ph["head_loss"][1] == 0 and ph["input_grad"][1] == 0
    with _Fused(False):
        ph = ppo.ppo_update_epoch_profiled(ctx, params, tb, perm, K, ppo.UpdateHParams(), stats, ws)
    assert ph["fused"][1] == 0 and ph["forward"][1] == K * len(cfg.net.hidden)


@pytest.mark.parametrize("name,shape", [("flat", None), ("large", None), ("large", (32, 512))])
def test_fused_epoch_graph_matches_eager_and_layered(name, shape):
    """A four-mini-batch epoch: the captured graph replays the eager launches
    bit for bit, and the gradient the fused epoch takes at its last step (at
    parameters three Adam steps in, from weight fragments Adam refreshed in
    place) equals the layer-by-layer gradient at those parameters within the
    single-step tolerance.  The free-running drift between the two paths
    over the epoch is printed, not gated: with mini-batches of 1024 most
    ratios reach a clip edge within a few steps (clip fraction about 0.9), and
    the two paths' float32 summation orders decide some of those ties
    differently, after which their trajectories separate."""
    d = require_gpu()
    cfg = synth.get_config(name)
    _announce(f"fused epoch graph vs eager vs layered {name} shape={shape}")
    theta = synth.xavier_theta(cfg.net, seed=21, logstd=-0.2)
    B = 4096
    batch = teacher_batch(cfg, theta, B, seed=22, shift="mixed")
    perm = np.random.default_rng(23).permutation(B).astype(np.int32)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "bf16")
    K = 4
    M = B // K
    tb = {k: dev(v, d) for k, v in batch.items()}
    ws = ctx.new_workspace(M=M)
    out = {}
    for label, fused, graph in (("eager", True, False), ("graph", True, True), ("layered", False, False)):
        params = ppo.Params(ctx, theta, lr=1e-3, device=d)
        stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
        first = None
        with _Fused(fused, shape if fused else None):
            assert (ctx.fused_shape()[0] > 0) == fused
            for rep in range(2):   # the second graph call replays the captured epoch
                ppo.ppo_update_epoch(ctx, params, tb, dev(perm, d), K, ppo.UpdateHParams(use_graph=graph), stats,
                                     ws)
                if rep == 0:
                    torch.cuda.synchronize()
                    first = (params.theta.cpu().numpy().copy(), params.grad.cpu().numpy().copy(),
                             stats.cpu().numpy().copy())
        torch.cuda.synchronize()
        out[label] = (params.theta.cpu().numpy().copy(), stats.cpu().numpy().copy(), first)
    np.testing.assert_array_equal(out["eager"][0], out["graph"][0])
    np.testing.assert_array_equal(out["eager"][1], out["graph"][1])
    for a, b in zip(out["eager"][2], out["graph"][2]):
        np.testing.assert_array_equal(a, b)
    # parameters after three fused steps (an epoch over the first three
    # mini-batches' rows, in permutation order), then the last mini-batch's
    # gradient by the layer-by-layer path
    params = ppo.Params(ctx, theta, lr=1e-3, device=d)
    stats = torch.zeros(K - 1, ppo.PPO_STATS_WIDTH, device=d)
    head = {k: dev(v[perm[:(K - 1) * M]], d) for k, v in batch.items()}
    with _Fused(True, shape):
        ppo.ppo_update_epoch(ctx, params, head, dev(np.arange((K - 1) * M, dtype=np.int32), d), K - 1,
                             ppo.UpdateHParams(), stats, ws)
    torch.cuda.synchronize()
    g_last_fused = out["eager"][2][1]
    grad = torch.zeros(ctx.param_count, device=d)
    st = torch.zeros(ppo.PPO_STATS_WIDTH, device=d)
    with _Fused(False):
        ppo.ppo_loss_grad(ctx, params, tb, dev(perm[(K - 1) * M:], d), ppo.UpdateHParams(), st, grad, ws)
    torch.cuda.synchronize()
    nw_g, _ = rel_errors(g_last_fused, grad.cpu().numpy())
    nw, _ = rel_errors(out["eager"][2][0] - theta, out["layered"][2][0] - theta)
    nw2, _ = rel_errors(out["eager"][0] - theta, out["layered"][0] - theta)
    print(f"last-step gradient fused vs layered at the same parameters: normwise {nw_g:.2e}; "
          f"free-running parameter drift {nw:.2e} after one epoch, {nw2:.2e} after two")
    assert nw_g < 4e-3, nw_g


@pytest.mark.parametrize("name,N,shape", [("flat", 4096, None), ("rough", 333, (64, 512)), ("large", 31, (32, 512)),
                                          ("flat", 1, None), ("tiny", 64, (64, 256))])
def test_fused_rollout_matches_layered(name, N, shape):
    """Rollout inference through the fused kernel and through the
    layer-by-layer kernels: the Philox draws and the log-densities (functions
    of the draws and log-std only) agree bit for bit; means and values agree
    to float32 rounding of the output layer."""
    d = require_gpu()
    cfg = synth.get_config(name)
    _announce(f"fused rollout vs layered {name} N={N}")
    theta = synth.xavier_theta(cfg.net, seed=3, logstd=-0.4)
    obs = synth.make_rollout(cfg)["obs"][2][:N] if cfg.heightfield else \
        synth.rollout.gaussian_like((N, cfg.net.obs_dim), seed=4)
    ctx = ppo.Context(cfg.net.obs_dim, cfg.net.act_dim, cfg.net.hidden, "bf16")
    params = ppo.Params(ctx, theta, device=d)
    A = cfg.net.act_dim
    res = {}
    for fused in (True, False):
        out = dict(actions=torch.empty(N, A, device=d), logp=torch.empty(N, device=d),
                   values=torch.empty(N, device=d), mu=torch.empty(N, A, device=d))
        v_only = torch.empty(N, device=d)
        a_only = torch.empty(N, A, device=d)
        with _Fused(fused, shape if fused else None):
            assert (ctx.fused_shape()[0] > 0) == fused
            ppo.ppo_rollout_infer(ctx, params, dev(obs, d), t=5, seed=11, iteration=2, **out)
            ppo.ppo_rollout_infer(ctx, params, dev(obs, d), t=5, seed=11, iteration=2, values=v_only)
            ppo.ppo_rollout_infer(ctx, params, dev(obs, d), t=5, seed=11, iteration=2, actions=a_only)
        torch.cuda.synchronize()
        res[fused] = {k: v.cpu().numpy() for k, v in out.items()}
        res[fused]["v_only"] = v_only.cpu().numpy()
        res[fused]["a_only"] = a_only.cpu().numpy()
    f, l = res[True], res[False]
    np.testing.assert_array_equal(f["logp"], l["logp"])
    sigma = np.float32(np.exp(np.float32(-0.4)))
    np.testing.assert_allclose((f["actions"] - f["mu"]) / sigma, (l["actions"] - l["mu"]) / sigma, rtol=0, atol=2e-5)
    for k in ("mu", "values"):
        nw, _ = rel_errors(f[k], l[k])
        assert nw < 1e-5, (k, nw)
    np.testing.assert_array_equal(f["v_only"], f["values"])
    np.testing.assert_array_equal(f["a_only"], f["actions"])


def test_keep_packed_follows_every_weight_change():
    """With PPO_OPT_KEEP_PACKED the rollout reuses the forward weights it
    packed; every path that changes the shadow or reuses the workspace must
    still give what a context that packs on every call gives, bit for bit:
    a repeated call, an update epoch, theta written by torch then repacked,
    a GAE call on the same workspace, and a captured inference graph
    replayed across an update."""
    d = require_gpu()
    _announce("keep-packed rollout")
    cfg = synth.get_config("flat")
    net = cfg.net
    ctx_k = ppo.Context(net.obs_dim, net.act_dim, net.hidden, "bf16")
    ctx_k.keep_packed(True)
    ctx_r = ppo.Context(net.obs_dim, net.act_dim, net.hidden, "bf16")
    params = ppo.Params(ctx_k, synth.xavier_theta(net, seed=5, logstd=-0.3), device=d)
    N, B, K, T = 1000, 4096, 2, 4
    rng = np.random.default_rng(0)
    obs = dev(rng.standard_normal((N, net.obs_dim)).astype(np.float32), d)
    ws = ctx_k.new_workspace(N=N, T=T, M=B // K, device=d)
    ws_r = ctx_r.new_workspace(N=N, device=d)
    A = net.act_dim
    outs = {k: torch.empty(N, A, device=d) for k in ("actions", "mu")}
    outs.update({k: torch.empty(N, device=d) for k in ("logp", "values")})

    def infer(ctx, w):
        ppo.ppo_rollout_infer(ctx, params, obs, 3, 11, 2, ws=w, **outs)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy().copy() for k, v in outs.items()}

    def same_as_reference(tag):
        got = infer(ctx_k, ws)
        ref = infer(ctx_r, ws_r)
        for k in got:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{tag}: {k}")
        return got

    first = same_as_reference("first call")
    again = same_as_reference("cached call")
    np.testing.assert_array_equal(first["mu"], again["mu"])

    batch = dict(obs=dev(rng.standard_normal((B, net.obs_dim)).astype(np.float32), d),
                 actions=dev(rng.standard_normal((B, A)).astype(np.float32), d),
                 logp=dev(rng.normal(-15, 1, B).astype(np.float32), d),
                 adv=dev(rng.standard_normal(B).astype(np.float32), d),
                 returns=dev(rng.standard_normal(B).astype(np.float32), d))
    perm = dev(rng.permutation(B).astype(np.int32), d)
    stats = torch.zeros(K, ppo.PPO_STATS_WIDTH, device=d)
    hp = ppo.UpdateHParams(use_graph=True)
    ppo.ppo_update_epoch(ctx_k, params, batch, perm, K, hp, stats, ws)
    after_update = same_as_reference("after update")
    assert not np.array_equal(after_update["mu"], first["mu"])

    params.theta.mul_(0.9)
    params.pack()
    same_as_reference("after theta written and repacked")

    r = dev(rng.standard_normal((T, N)).astype(np.float32), d)
    v = dev(rng.standard_normal((T, N)).astype(np.float32), d)
    dn = dev((rng.random((T, N)) < 0.1).astype(np.uint8), d)
    last = dev(rng.standard_normal(N).astype(np.float32), d)
    adv, ret = torch.empty(T, N, device=d), torch.empty(T, N, device=d)
    st = torch.empty(2, dtype=torch.float64, device=d)
    ppo.ppo_gae(ctx_k, r, dn, v, last, 0.99, 0.95, adv, ret, st, ws=ws)
    same_as_reference("after GAE on the same workspace")

    # inference captured into a graph packs inside the graph; replays follow updates
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            ppo.ppo_rollout_infer(ctx_k, params, obs, 3, 11, 2, ws=ws, **outs)
    torch.cuda.synchronize()
    for rep in range(2):
        ppo.ppo_update_epoch(ctx_k, params, batch, perm, K, hp, stats, ws)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy().copy() for k, v in outs.items()}
        ref = infer(ctx_r, ws_r)
        for k in got:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"graph replay {rep}: {k}")
        same_as_reference(f"eager after replay {rep}")
