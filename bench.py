#!/usr/bin/env python3
"""Throughput of the PPO learning hot path on one MI355X.

One step = one learning iteration of the massively parallel set-up over a
resident synthetic rollout of 4096 environments x 24 steps (the paper's
Table 3 batch, B = 98304):
  * policy inference + Philox action sampling for each of the 24 steps, and
    the critic on the observation after the last step;
  * GAE with time-out bootstrapping and float64 advantage statistics;
  * the PPO update: 5 epochs x 4 mini-batches of 24576 (forward, loss,
    hand-written backward, float64 global-norm clip, Adam), each epoch
    replayed from a captured HIP graph.
value = B / (time per step), in samples/s, bf16 GEMM operands with float32
accumulation.  The float32 plain path is timed the same way for the speedup.
Also reported: a roofline entry for the dominant kernel (HIP events around
each launch of one eagerly launched epoch), the update's median and IQR over
20 repetitions from the same state, GAE bandwidth on 2^20-environment
rollouts, the copy and bf16-GEMM rates this GPU attains, and the FP64 CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp32]
       python bench.py --config large   (16384 x 24 envs, 235-dim obs, [1024, 512, 256])
       python bench.py --config sweep   (8 uneven runs, batched update vs run after run)
       python bench.py --config fig4    (Fig. 4 shapes: fixed batch, 128 ... 16384 envs)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "PPO update samples/s at 4096 envs x 24 steps, BF16 vs FP32, at stated tol"
HBM_PEAK_GBS = 8000.0
PROFILE_REPS = 10
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="flat")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 plain-path timing")
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the large-GAE bandwidth sweep and the attainable-peak probes")
    ap.add_argument("--quick", action="store_true",
                    help="only the timed steps (for profiler runs): no parts, roofline, fp32 or CPU legs")
    ap.add_argument("--sweep-mode", default="both", choices=["both", "batched", "serial"],
                    help="sweep config: time the batched update, the run-after-run update, or both")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


class Workload:
    """Device-resident rollout storage, parameters and workspaces."""

    def __init__(self, cfg, precision, device):
        import torch
        import paper_2109_11978_amd as ppo
        import synth

        self.cfg = cfg
        net = cfg.net
        self.ctx = ppo.Context(net.obs_dim, net.act_dim, net.hidden, precision)
        T, N, D, A = cfg.n_steps, cfg.n_envs, net.obs_dim, net.act_dim
        B, M = cfg.batch, cfg.minibatch
        roll = synth.make_rollout(cfg, with_timeouts=True)
        self.theta0 = synth.xavier_theta(net, seed=cfg.seed)
        self.params = ppo.Params(self.ctx, self.theta0, lr=cfg.lr, device=device)
        f32 = torch.float32
        self.obs = torch.as_tensor(roll["obs"]).to(device)                  # [T, N, D]
        self.last_obs = torch.as_tensor(roll["last_obs"]).to(device)        # [N, D]
        self.rewards = torch.as_tensor(roll["rewards"]).to(device)
        self.dones = torch.as_tensor(roll["dones"]).to(device)
        self.timeouts = torch.as_tensor(roll["timeouts"]).to(device)
        self.actions = torch.empty(T, N, A, dtype=f32, device=device)
        self.logp = torch.empty(T, N, dtype=f32, device=device)
        self.values = torch.empty(T, N, dtype=f32, device=device)
        self.last_values = torch.empty(N, dtype=f32, device=device)
        self.adv = torch.empty(T, N, dtype=f32, device=device)
        self.returns = torch.empty(T, N, dtype=f32, device=device)
        self.adv_stats = torch.empty(2, dtype=torch.float64, device=device)
        self.perms = torch.as_tensor(synth.make_permutations(B, cfg.epochs, seed=cfg.seed)).to(device)
        self.stats = torch.zeros(cfg.epochs, cfg.minibatches, ppo.PPO_STATS_WIDTH, dtype=f32, device=device)
        self.ws = self.ctx.new_workspace(N=N, T=T, M=M, device=device)
        # one workspace for the whole run, written only through the library
        self.ctx.keep_packed(True)
        self.hp = ppo.UpdateHParams(clip=cfg.clip, value_coef=cfg.value_coef, entropy_coef=cfg.entropy_coef,
                                    max_grad_norm=cfg.max_grad_norm, use_graph=True)
        self.batch = dict(obs=self.obs.view(B, D), actions=self.actions.view(B, A), logp=self.logp.view(B),
                          adv=self.adv.view(B), returns=self.returns.view(B))
        self.iteration = 0
        self.ppo = ppo

    def collect(self):
        ppo, cfg = self.ppo, self.cfg
        for t in range(cfg.n_steps):
            ppo.ppo_rollout_infer(self.ctx, self.params, self.obs[t], t, cfg.seed, self.iteration,
                                  actions=self.actions[t], logp=self.logp[t], values=self.values[t], ws=self.ws)
        ppo.ppo_rollout_infer(self.ctx, self.params, self.last_obs, cfg.n_steps, cfg.seed, self.iteration,
                              values=self.last_values, ws=self.ws)

    def advantages(self):
        self.ppo.ppo_gae(self.ctx, self.rewards, self.dones, self.values, self.last_values, self.cfg.gamma,
                         self.cfg.lam, self.adv, self.returns, self.adv_stats, timeouts=self.timeouts,
                         normalize=True, ws=self.ws)

    def update(self):
        for e in range(self.cfg.epochs):
            self.ppo.ppo_update_epoch(self.ctx, self.params, self.batch, self.perms[e], self.cfg.minibatches,
                                      self.hp, self.stats[e], self.ws)

    def step(self):
        self.collect()
        self.advantages()
        self.update()
        self.iteration += 1


def time_steps(wl, steps, warmup):
    import torch
    for _ in range(warmup):
        wl.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        wl.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_parts(wl, reps=5):
    """Wall time of collection, GAE and update separately (milliseconds)."""
    import torch
    out = {}
    for name, fn in (("rollout_infer", wl.collect), ("gae", wl.advantages), ("update", wl.update)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) / reps * 1e3
    return out


def phase_model(cfg, precision, P):
    """Algorithmic work of one mini-batch step, per phase: useful FLOPs and
    compulsory HBM bytes (every input read once, every output written once,
    at the operand width; split partials and re-reads are not counted)."""
    net, M = cfg.net, cfg.minibatch
    e = 2 if precision == "bf16" else 4
    D, A = net.obs_dim, net.act_dim
    kpad = -(-D // 8) * 8
    H = list(net.hidden)
    L = len(H)
    ins = [D, *H[:-1]]          # useful K of each hidden layer
    ins_pad = [kpad, *H[:-1]]   # stored width of each layer's input
    fwd_f = sum(2 * M * ins[l] * H[l] for l in range(L)) * 2
    fwd_b = (M * kpad * e                                      # gathered input, shared by both nets
             + sum(M * ins_pad[l] * e * 2 for l in range(1, L))  # hidden inputs
             + sum(M * H[l] * e * 2 for l in range(L))           # outputs
             + sum((H[l] * ins_pad[l] * e + H[l] * 4) * 2 for l in range(L)))  # weights, biases
    dx_f = sum(2 * M * H[l] * H[l - 1] for l in range(1, L)) * 2
    dx_b = sum((M * H[l] * e + 2 * M * H[l - 1] * e + H[l] * H[l - 1] * e) * 2 for l in range(1, L))
    dw_f = (sum(2 * M * H[l] * ins[l] for l in range(L)) * 2 + 2 * M * H[-1] * (A + 1))
    dw_b = (M * sum(H) * e * 2 + M * 16 * e * 2                # pre-activation gradients, output-layer gradients
            + M * kpad * e + M * sum(H) * e * 2                 # layer inputs
            + 4 * P)                                            # the gradient
    head_b = M * H[-1] * e * 2 * 2 + M * 16 * e * 2 + M * 4 * (A + 5)
    head_f = M * H[-1] * (A + 1) * 4.0
    # the fused per-sample pass (bf16): the forward, output-layer and
    # input-gradient arithmetic of both networks.  Compulsory bytes: the
    # observation rows, indices and loss inputs it reads and every weight once;
    # the weight-gradient operands it writes (activations, pre-activation and
    # output gradients) are this design's choice, not the method's, and are
    # not counted
    fused_b = (M * D * 4.0 + M * 4.0 + M * 4.0 * (A + 4)
               + sum(H[l] * ins_pad[l] * e + H[l] * 4 for l in range(L)) * 2
               + sum(H[l] * H[l - 1] * e for l in range(1, L)) * 2)
    return {
        "fused": (fwd_f + dx_f + head_f, fused_b),
        "forward": (fwd_f, fwd_b),
        "input_grad": (dx_f, dx_b),
        "weight_grad": (dw_f, dw_b),
        "head_loss": (M * H[-1] * (A + 1) * 4.0, head_b),
        "gather": (0.0, M * D * 4.0 + M * kpad * e + M * 4.0),
        # fused path: one packing launch per epoch, bf16 weights read and written in
        # fragment order (forward, and transposed for the input-gradient chain), per launch
        "pack": (0.0, 2 * 2.0 * (sum(H[l] * ins_pad[l] for l in range(L))
                                 + sum(H[l] * H[l - 1] for l in range(1, L))) * 2),
        "grad_reduce": (0.0, 4.0 * P),
        "adam": (0.0, (30.0 if precision == "bf16" else 28.0) * P),
    }


def code_sha256(path):
    """SHA-256 of a C++/HIP source with its comments and whitespace removed, so
    that recorded counters stay tied to the code rather than to its comments
    (string literals in the kernels hold no comment markers)."""
    import hashlib
    import re
    src = open(path, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return hashlib.sha256("".join(src.split()).encode()).hexdigest()


def recorded_traffic(wl, phase, workload):
    """HBM bytes per launch of the fused, forward or input-gradient phase, from
    the committed rocprofv3 counter summary (per kernel and grid, at the tiles
    this run chose), or None when the summary is missing, lacks one of those
    launches, or was taken on another version of the kernel's code."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"traffic_{workload}.txt")
    if phase not in ("fused", "forward", "input_grad") or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.rsplit(":", 1)
            fields[k.strip()] = v.strip()
    src_name = "k_fused.hip" if phase == "fused" else "k_gemm.hip"
    src = os.path.join(here, "paper_2109_11978_amd", "csrc", src_name)
    sha_key = src_name.replace(".hip", "_code_sha256")
    if fields.get(sha_key) != code_sha256(src):
        return None
    cfg = wl.cfg
    M, H = cfg.minibatch, list(cfg.net.hidden)
    keys = []
    if phase == "fused":
        rows, _ = wl.ctx.fused_shape()
        if rows == 0:
            return None
        keys.append(f"hbm_bytes.fused_update_kernel.{2 * -(-M // rows)}")
    else:
        tiles = wl.ctx.tuning(M, True)
        if phase == "forward":
            sites = [(tiles[f"forward_{l + 1}"], H[l], 0) for l in range(len(H))]
        else:
            sites = [(tiles[f"input_grad_{l + 1}"], H[l - 1], 1) for l in range(len(H) - 1, 0, -1)]
        for tile, cols, epi in sites:
            bm, bn = (int(x) for x in tile.split("x"))
            grid = -(-M // bm) * -(-cols // bn) * 2
            keys.append(f"hbm_bytes.gemm_kernel<bf16,{bm},{bn},0,0,{epi},true>.{grid}")
    vals = [fields.get(k) for k in keys]
    if any(v is None for v in vals):
        return None
    return sum(float(v) for v in vals) / len(vals)


GEMM_PHASES = ("fused", "forward", "input_grad", "weight_grad", "head_loss")


def update_flops(cfg):
    """Useful GEMM FLOPs of one full update (E x B sample passes): the forward
    and the two backward contractions of both networks, output layers
    included; padding (K 48 -> 64, 235 -> 240, head 12 -> 16) and the
    critic's second (residual) weight pass are not counted."""
    net, M = cfg.net, cfg.minibatch
    D, A, H = net.obs_dim, net.act_dim, list(net.hidden)
    ins = [D, *H[:-1]]
    per = 0
    for outs in (A, 1):
        fwd = sum(ins[l] * H[l] for l in range(len(H))) + H[-1] * outs
        dx = sum(H[l] * H[l - 1] for l in range(1, len(H))) + H[-1] * outs
        per += 2 * fwd + 2 * dx + 2 * fwd      # forward, input gradients, weight gradients
    return float(per) * cfg.epochs * cfg.batch


def roofline(wl, precision):
    """Per-phase HIP-event durations of one eager epoch and each phase's
    place under its roof: contractions (the fused pass, the GEMMs, the output
    layers) on the MFMA roof with useful FLOPs, the rest on the HBM roof with
    compulsory bytes; frac = achieved / peak."""
    import torch
    cfg = wl.cfg
    # repeatable launches run PROFILE_REPS times back to back inside their
    # event pair, so the event overhead does not inflate the per-launch time
    prof = wl.ppo.ppo_update_epoch_profiled(wl.ctx, wl.params, wl.batch, wl.perms[0], cfg.minibatches,
                                            wl.hp, wl.stats[0], wl.ws, reps=PROFILE_REPS)
    torch.cuda.synchronize()
    model = phase_model(cfg, precision, wl.ctx.param_count)
    steps = cfg.minibatches
    phases = {}
    per_launch = {}
    for name, (ms, launches) in prof.items():
        if launches == 0:
            continue
        t = ms * 1e-3 / launches
        if name == "gather" and wl.ctx.fused_shape()[0] > 0:
            f, b = model["pack"]          # already per launch
        else:
            f, b = model.get(name, (0.0, 0.0))
            f, b = f * steps / launches, b * steps / launches
        per_launch[name] = (t, f, b)
        if name in GEMM_PHASES and f > 0:
            ach = f / t / 1e12
            phases[name] = {"ms_per_epoch": round(ms, 4), "launches": launches, "us_per_launch": round(t * 1e6, 2),
                            "bound": "mfma", "achieved_tflops": round(ach, 2),
                            "frac": round(ach / MFMA_PEAK_TFLOPS[precision], 4)}
        else:
            ach = b / t / 1e9
            phases[name] = {"ms_per_epoch": round(ms, 4), "launches": launches, "us_per_launch": round(t * 1e6, 2),
                            "bound": "hbm", "achieved_gbs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4)}
    dominant = max(phases, key=lambda k: phases[k]["ms_per_epoch"])
    ph = phases[dominant]
    t, f, b = per_launch[dominant]
    if ph["bound"] == "mfma":
        roof = {"kernel": dominant, "bound": "mfma", "achieved": ph["achieved_tflops"],
                "peak": MFMA_PEAK_TFLOPS[precision], "unit": "TFLOP/s", "frac": ph["frac"]}
    else:
        roof = {"kernel": dominant, "bound": "hbm", "achieved": ph["achieved_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ph["frac"]}
    roof.update({"traffic": recorded_traffic(wl, dominant, cfg.name.split("_")[0]),
                 "algorithmic_flops_per_launch": f, "avg_launch_us": round(t * 1e6, 2)})
    gemm = {k: phases[k].get("achieved_tflops") for k in GEMM_PHASES if k in phases}
    return roof, phases, gemm


def cpu_baseline(wl, precision):
    """The FP64 oracle on the same workload, and the parity of the timed state.

    Sample: one whole learning iteration of the oracle on the rollout the GPU
    holds: the policy step for every one of the 24 rollout steps over all
    4096 environments plus the critic on the observation after the last,
    GAE with time-outs and the advantage statistics, and the full update
    (5 epochs x 4 mini-batches of 24576: loss, gradient, global clip, Adam).
    value = B / that time.

    Parity of the timed state: one mini-batch (the first of epoch 0) through
    ppo_loss_grad at the GPU's current parameters, with its per-sample ratios
    and clip branches, against the oracle at the same parameters and inputs.
    The ratios are compared normwise; a sample takes the GPU's branch where
    the GPU's ratio lies across the deciding clip edge from the oracle's
    (the clip-edge tie protocol); the gradient is compared per parameter
    tensor, normwise (the gate) and elementwise with the rms floor (stated).
    """
    import torch
    import oracle
    from oracle.ppo import minibatch
    cfg = wl.cfg
    net = cfg.net
    spec = oracle.NetSpec(net.obs_dim, net.act_dim, tuple(net.hidden))
    theta = wl.params.theta.cpu().numpy().astype(np.float64)
    obs = wl.obs.cpu().numpy()
    T, N, B, M = cfg.n_steps, cfg.n_envs, cfg.batch, cfg.minibatch
    hp = oracle.PPOHyper(clip=cfg.clip, value_coef=cfg.value_coef, entropy_coef=cfg.entropy_coef,
                         max_grad_norm=cfg.max_grad_norm, lr=cfg.lr)
    P = theta.size
    perms = wl.perms.cpu().numpy()

    t_start = time.perf_counter()
    ro = [oracle.rollout_infer(theta, spec, obs[t], cfg.seed, t, 0) for t in range(T)]
    last = oracle.policy.critic_values(theta, spec, wl.last_obs.cpu().numpy())
    t_inf = time.perf_counter() - t_start
    values = np.stack([r["values"] for r in ro])
    rewards = wl.rewards.cpu().numpy()
    dones = wl.dones.cpu().numpy()
    timeouts = wl.timeouts.cpu().numpy()
    t0 = time.perf_counter()
    adv, ret = oracle.gae(rewards, values, dones, last, cfg.gamma, cfg.lam, timeouts=timeouts)
    mean, std = oracle.advantage_stats(adv)
    adv_n = oracle.normalize_advantages(adv, mean, std)
    t_gae = time.perf_counter() - t0
    full = dict(obs=obs.reshape(B, -1), actions=np.concatenate([r["actions"] for r in ro]),
                logp_old=np.concatenate([r["logp"] for r in ro]), adv=adv_n.reshape(B), returns=ret.reshape(B))
    t0 = time.perf_counter()
    th, m, v, step = theta, np.zeros(P), np.zeros(P), 0
    for e in range(cfg.epochs):
        th, m, v, step, _ = oracle.update_epoch(th, m, v, step, spec, full, perms[e], cfg.minibatches, hp)
    t_upd = time.perf_counter() - t0
    t_iter = time.perf_counter() - t_start

    threads, blas = None, []
    try:
        from threadpoolctl import threadpool_info
        pools = threadpool_info()
        threads = max((i.get("num_threads", 1) for i in pools), default=1)
        blas = [f"{i.get('internal_api')} {i.get('version')} x{i.get('num_threads')}" for i in pools]
    except Exception:
        threads = os.cpu_count()
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass

    # parity of the timed state: the same mini-batch through the HIP path
    dev = wl.params.theta.device
    idx = wl.perms[0][:M].contiguous()
    gstats = torch.zeros(wl.ppo.PPO_STATS_WIDTH, device=dev)
    grad = torch.zeros(P, device=dev)
    active = torch.zeros(M, dtype=torch.uint8, device=dev)
    ratio = torch.zeros(M, device=dev)
    wl.ppo.ppo_loss_grad(wl.ctx, wl.params, wl.batch, idx, wl.hp, gstats, grad, wl.ws, active_out=active,
                         ratio_out=ratio)
    torch.cuda.synchronize()
    gpu_batch = dict(obs=obs.reshape(B, -1), actions=wl.actions.cpu().numpy().reshape(B, -1),
                     logp_old=wl.logp.cpu().numpy().reshape(B), adv=wl.adv.cpu().numpy().reshape(B),
                     returns=wl.returns.cpu().numpy().reshape(B))
    mb = minibatch(gpu_batch, idx.cpu().numpy())
    own = oracle.ppo_loss_grad(theta, spec, mb, hp, want_grad=False)
    rg = ratio.cpu().numpy().astype(np.float64)
    band = np.abs(rg - own["ratio"]) + 1e-7 * np.maximum(1.0, np.abs(own["ratio"]))
    res = oracle.ppo_loss_grad(theta, spec, mb, hp, active_override=active.cpu().numpy().astype(bool),
                               tie_delta=band)
    g = grad.cpu().numpy().astype(np.float64)
    tol = 2e-2 if precision == "bf16" else 1e-5
    normwise, elementwise = {}, {}
    for name, (off, shp) in oracle.param_layout(spec).items():
        if name == "__total__":
            continue
        n = int(np.prod(shp))
        x, r = g[off:off + n], res["grad"][off:off + n]
        normwise[name] = float(np.linalg.norm(x - r) / np.linalg.norm(r))
        rms = float(np.sqrt(np.mean(r * r)))
        elementwise[name] = float(np.max(np.abs(x - r) / (np.abs(r) + rms)))
    ratio_nw = float(np.linalg.norm(rg - own["ratio"]) / np.linalg.norm(own["ratio"]))
    worst = max(normwise, key=normwise.get)
    parity = {"tol": tol, "minibatch": "epoch 0, mini-batch 0, at the parameters after the timed steps",
              "within_tol": bool(max(normwise.values()) <= tol and ratio_nw <= tol and res["disagree_outside"] == 0),
              "gradient_normwise_worst": [worst, round(normwise[worst], 6)],
              "gradient_normwise_total": float(np.linalg.norm(g - res["grad"]) / np.linalg.norm(res["grad"])),
              "gradient_normwise_per_tensor": {k: round(v, 6) for k, v in normwise.items()},
              "gradient_elementwise_rms_floor_per_tensor": {k: round(v, 5) for k, v in elementwise.items()},
              "ratio_normwise": round(ratio_nw, 6),
              "ratio_max_relative": round(float(np.max(np.abs(rg / own["ratio"] - 1.0))), 6),
              "clip_fraction": round(float(res["clip_frac"]), 4),
              "clip_ties_adopted": res["ties_adopted"], "clip_disagreements_outside_band": res["disagree_outside"]}
    base = {"value": round(B / t_iter, 1), "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle, one whole learning iteration: {T} policy steps over {N} envs + the "
                       f"critic on the last observation ({t_inf:.2f} s), GAE over [{T},{N}] ({t_gae:.3f} s), "
                       f"{cfg.epochs} epochs x {cfg.minibatches} mini-batches of {M} ({t_upd:.1f} s); "
                       f"total {t_iter:.1f} s"),
            "update_samples_per_s": round(B / t_upd, 1),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model, "blas": blas}
    return base, parity


def update_distribution(wl, reps=20, warmup=3):
    """Wall time of one full update (HIP events on the launch stream), with the
    parameters and optimiser state restored before every repetition so each
    one sees the same ratios: median and interquartile range in ms."""
    import torch
    p = wl.params
    state = (p.theta, p.adam_m, p.adam_v, p.shadow, p.step, p.lr)
    saved = [t.clone() for t in state]
    times = []
    for r in range(warmup + reps):
        for dst, src in zip(state, saved):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wl.update()
        e1.record()
        e1.synchronize()
        if r >= warmup:
            times.append(e0.elapsed_time(e1))
    for dst, src in zip(state, saved):
        dst.copy_(src)
    p.pack()      # the shadow was written outside the library: refresh it (and the packed copies)
    q25, q50, q75 = np.percentile(times, [25, 50, 75])
    return {"median_ms": round(float(q50), 3), "iqr_ms": round(float(q75 - q25), 3), "reps": reps,
            "samples_per_s_at_median": round(wl.cfg.batch / (q50 * 1e-3), 1)}


def gae_bandwidth(ctx, dev, shapes=((24, 1 << 20), (256, 1 << 20)), reps=5):
    """GAE with time-outs and normalisation on large synthetic rollouts, to show
    how the scan's bandwidth scales once it is no longer cache-resident;
    26 algorithmic bytes per sample."""
    import torch
    import paper_2109_11978_amd as ppo
    out = {}
    for T, N in shapes:
        g = torch.Generator(device=dev)
        g.manual_seed(T)
        r = torch.randn(T, N, device=dev, generator=g) * 0.1
        v = torch.randn(T, N, device=dev, generator=g)
        dn = (torch.rand(T, N, device=dev, generator=g) < 1e-3).to(torch.uint8)
        to = dn & (torch.rand(T, N, device=dev, generator=g) < 0.5).to(torch.uint8)
        last = torch.randn(N, device=dev, generator=g)
        adv, ret = torch.empty_like(r), torch.empty_like(r)
        st = torch.empty(2, dtype=torch.float64, device=dev)
        ws = ctx.new_workspace(N=N, T=T, device=dev)
        run = lambda: ppo.ppo_gae(ctx, r, dn, v, last, 0.99, 0.95, adv, ret, st, timeouts=to,
                                  normalize=True, ws=ws)
        run()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        out[f"T{T}_N{N}"] = {"us": round(t * 1e6, 1), "gbs": round(26 * T * N / t / 1e9, 1)}
        del r, v, dn, to, last, adv, ret, ws
    torch.cuda.empty_cache()
    return out


def obs_assembly_rate(dev, sizes=(4096, 16384, 1 << 20), reps=20):
    """ppo_assemble_obs on the rough-terrain layout (48 proprioceptive columns,
    a 17 x 11 height scan of a 480 x 480 field, Table 4 noise): time per call
    and algorithmic GB/s, 1900 B per robot (proprio 192 B, pose 20 B, 187
    heights 748 B read; 235 floats written)."""
    import torch
    import paper_2109_11978_amd as ppo
    import synth.heightfield as shf
    ctx = ppo.Context(235, 12, (512, 256, 128), "bf16")
    hf = shf.HeightField(seed=0)
    height = torch.as_tensor(hf.h.astype(np.float32)).to(dev)
    scan = torch.as_tensor(shf.scan_pattern()).to(dev)
    noise = torch.as_tensor(shf.noise_scales()).to(dev)
    out = {}
    for N in sizes:
        rng = np.random.default_rng(N)
        proprio = torch.as_tensor(rng.standard_normal((N, 48)).astype(np.float32)).to(dev)
        base = torch.as_tensor(shf.base_poses(rng, N, hf.size)).to(dev)
        obs = torch.empty(N, 235, device=dev)
        run = lambda t: ppo.ppo_assemble_obs(ctx, obs, t, 0, 0, proprio=proprio, base=base, height=height,
                                             scan=scan, noise_scale=noise)
        run(0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for t in range(reps):
            run(t)
        e1.record()
        e1.synchronize()
        t_call = e0.elapsed_time(e1) * 1e-3 / reps
        out[f"N{N}"] = {"us": round(t_call * 1e6, 2), "gbs": round(1900 * N / t_call / 1e9, 1)}
        del proprio, base, obs
    return out


def attainable_peaks(dev):
    """What this GPU reaches on plain library work, next to the published
    peaks: a 1 GiB device-to-device copy (read + write bytes) and a bf16
    8192^3 matrix product through the vendor BLAS."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    a = torch.randn(8192, 8192, device=dev, dtype=torch.bfloat16)
    b = torch.randn(8192, 8192, device=dev, dtype=torch.bfloat16)

    def timed(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    t_copy = timed(lambda: dst.copy_(src), 10)
    t_mm = timed(lambda: torch.mm(a, b), 10)
    del src, dst, a, b
    torch.cuda.empty_cache()
    return {"hbm_copy_gbs": round(2 * n * 4 / t_copy / 1e9, 1), "bf16_gemm_tflops": round(2 * 8192 ** 3 / t_mm / 1e12, 1),
            "published": {"hbm_gbs": HBM_PEAK_GBS, "bf16_tflops": MFMA_PEAK_TFLOPS["bf16"]}}


def fig4_bench(args, dev):
    """Fig. 4's shapes on the rough-terrain network: the parts of one learning
    iteration at fixed batch size as the number of environments grows
    (T = B / N), plus the 20000 x 50 reference point.  The update's time should
    not depend on N at fixed B; collection time falls with T."""
    import torch
    import synth
    rows = []
    total_b, total_t = 0, 0.0
    for cfg in synth.configs.fig4_runs():
        print(f"[fig4] {cfg.name}", file=sys.stderr, flush=True)
        wl = Workload(cfg, "bf16", dev)
        parts = time_parts(wl, reps=2)
        t_iter = sum(parts.values())
        total_b += cfg.batch
        total_t += t_iter * 1e-3
        rows.append({"workload": cfg.name, "n_envs": cfg.n_envs, "n_steps": cfg.n_steps, "batch": cfg.batch,
                     **{f"{k}_ms": round(v, 3) for k, v in parts.items()},
                     "iteration_ms": round(t_iter, 3),
                     "update_samples_per_s": round(cfg.batch / (parts["update"] * 1e-3), 1)})
        del wl
        torch.cuda.empty_cache()
    spread = {}
    for b in synth.configs.FIG4_BATCHES:
        u = [r["update_ms"] for r in rows if r["batch"] == b]
        spread[str(b)] = round(max(u) / min(u), 3)
    out = {"metric": "PPO learning-iteration samples/s over Fig. 4 shapes (fixed batch, growing number of envs)",
           "value": round(total_b / total_t, 1), "unit": "samples/s", "n_gpus": 1, "steps": 2, "warmup": 1,
           "ms_per_step": round(total_t * 1e3 / len(rows), 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "fig4_shapes_d235_h512x256x128", "batches": list(synth.configs.FIG4_BATCHES),
                      "n_envs": list(synth.configs.FIG4_ENVS)},
           "update_time_max_over_min_at_fixed_batch": spread, "rows": rows}
    print(json.dumps(out), flush=True)


def sweep_bench(args, dev):
    """Eight uneven sweep-style runs: per iteration each run collects its own
    rollout (policy steps + GAE); the update is one batched epoch per epoch
    over all runs.  Also times the same updates done run after run."""
    import torch
    import paper_2109_11978_amd as ppo
    import synth
    runs = [Workload(cfg, "bf16", dev) for cfg in synth.configs.sweep_runs()]
    epochs, K = runs[0].cfg.epochs, runs[0].cfg.minibatches
    total_b = sum(w.cfg.batch for w in runs)

    def batched_update():
        for e in range(epochs):
            ppo.ppo_update_batched([w.ctx for w in runs], [w.params for w in runs], [w.batch for w in runs],
                                   [w.perms[e] for w in runs], K, runs[0].hp, [w.stats[e] for w in runs],
                                   [w.ws for w in runs])

    def step():
        for w in runs:
            w.collect()
            w.advantages()
        batched_update()
        for w in runs:
            w.iteration += 1

    if args.sweep_mode == "serial":
        def step():  # noqa: F811 -- the same iteration with run-after-run updates
            for w in runs:
                w.collect()
                w.advantages()
            for w in runs:
                w.update()
                w.iteration += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    s_step = (time.perf_counter() - t0) / args.steps

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t_batched = timed(batched_update) if args.sweep_mode != "serial" else float("nan")
    t_serial = timed(lambda: [w.update() for w in runs]) if args.sweep_mode != "batched" else float("nan")
    t_default = float("nan")
    if args.sweep_mode == "both":
        # the batched update again, from fresh contexts that keep every GEMM site at its
        # default 128 x 128 tile
        tuned = [w.ctx for w in runs]
        os.environ["PPO_AUTOTUNE"] = "0"
        try:
            for w in runs:
                n = w.cfg.net
                w.ctx = ppo.Context(n.obs_dim, n.act_dim, n.hidden, "bf16")
            t_default = timed(batched_update)
        finally:
            del os.environ["PPO_AUTOTUNE"]
            for w, c in zip(runs, tuned):
                w.ctx = c
    rate = lambda t: round(total_b / t, 1) if t == t else None      # None for a leg not timed (NaN)
    ratio = lambda a, b: round(a / b, 3) if a == a and b == b else None
    out = {
        "metric": "PPO update samples/s, 8 uneven sweep runs updated together",
        "value": round(total_b / s_step, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(s_step * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "sweep_8_uneven_runs", "runs": [w.cfg.name for w in runs], "total_batch": total_b},
        "update_samples_per_s_batched": rate(t_batched),
        "update_samples_per_s_run_after_run": rate(t_serial),
        "batched_speedup": ratio(t_serial, t_batched),
        "update_samples_per_s_batched_default_tiles": rate(t_default),
        "autotune_speedup": ratio(t_default, t_batched),
        "sweep_mode": args.sweep_mode,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    import synth
    dev = torch.device("cuda")
    if args.config == "sweep":
        sweep_bench(args, dev)
        return
    if args.config == "fig4":
        fig4_bench(args, dev)
        return
    cfg = synth.get_config(args.config)

    wl = Workload(cfg, "bf16", dev)
    s_step = time_steps(wl, args.steps, args.warmup)
    B = cfg.batch
    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.quick:
        print(json.dumps({"metric": METRIC, "value": round(B / s_step, 1), "unit": "samples/s",
                          "ms_per_step": round(s_step * 1e3, 3), "steps": args.steps, "warmup": args.warmup,
                          "quick": True}), flush=True)
        return
    parts = time_parts(wl)
    upd = update_distribution(wl)
    roof, phases, gemm_tflops = roofline(wl, "bf16")
    out = {
        "metric": METRIC,
        "value": round(B / s_step, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(s_step * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n_envs": cfg.n_envs, "n_steps": cfg.n_steps, "batch": B,
                   "obs_dim": cfg.net.obs_dim, "act_dim": cfg.net.act_dim, "hidden": list(cfg.net.hidden),
                   "epochs": cfg.epochs, "minibatches": cfg.minibatches, "minibatch": cfg.minibatch},
        "update_samples_per_s": round(B / (parts["update"] * 1e-3), 1),
        "update_sample_passes_per_s": round(cfg.epochs * B / (parts["update"] * 1e-3), 1),
        "rollout_env_steps_per_s": round(B / (parts["rollout_infer"] * 1e-3), 1),
        # 26 B per sample: rewards, values, advantages and returns at 4 B, dones and
        # time-outs at 1 B, and the normalisation's second read and write of the advantages
        "gae_gbs": round(26 * B / (parts["gae"] * 1e-3) / 1e9, 1),
        "breakdown_ms": {k: round(v, 3) for k, v in parts.items()},
        "update_ms_median_iqr": upd,
        "roofline": roof,
        # useful GEMM FLOPs of the whole update (forward, input and weight
        # gradients of both networks) over the median update time
        "update_mfma_frac": round(update_flops(cfg) / (upd["median_ms"] * 1e-3) / (MFMA_PEAK_TFLOPS["bf16"] * 1e12), 4),
        "update_useful_tflop": round(update_flops(cfg) / 1e12, 4),
        "phases_bf16": phases,
        "gemm_tflops_bf16": gemm_tflops,
        "autotuned_tiles": {"update": wl.ctx.tuning(cfg.minibatch, True),
                            "rollout": ("fused pass, %d environments x %d threads per workgroup" % wl.ctx.fused_infer_shape()
                                        if wl.ctx.fused_infer_shape()[0] else wl.ctx.tuning(cfg.n_envs, False))},
    }
    if not args.no_fp32:
        wl32 = Workload(cfg, "fp32", dev)
        s32 = time_steps(wl32, args.fp32_steps, 1)
        parts32 = time_parts(wl32, reps=2)
        _, phases32, gemm32 = roofline(wl32, "fp32")
        out["fp32_plain"] = {"value": round(B / s32, 1), "ms_per_step": round(s32 * 1e3, 3),
                             "update_samples_per_s": round(B / (parts32["update"] * 1e-3), 1),
                             "breakdown_ms": {k: round(v, 3) for k, v in parts32.items()},
                             "gemm_tflops_fp32": gemm32}
        out["bf16_speedup_vs_fp32"] = round(s32 / s_step, 2)
        out["bf16_update_speedup_vs_fp32"] = round(parts32["update"] / parts["update"], 2)
        del wl32
    if not args.no_extras:
        out["gae_bandwidth"] = gae_bandwidth(wl.ctx, dev)
        out["obs_assembly"] = obs_assembly_rate(dev)
        out["attainable_peaks"] = attainable_peaks(dev)
    if not args.no_cpu:
        out["cpu_baseline"], out["parity"] = cpu_baseline(wl, "bf16")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
