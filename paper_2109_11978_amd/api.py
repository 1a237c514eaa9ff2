"""Python binding of the C ABI in include/ppo.h.

Argument marshalling only: torch supplies device memory and the current HIP
stream, every computation runs in the HIP library.  The function names match
the C entry points.  There is no fallback path: if the library is missing or
the device is not gfx950 the calls raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import PPO_BF16, PPO_FP32, PPO_STATS_WIDTH, PPOError, check

STATS_FIELDS = ("loss", "policy_loss", "value_loss", "entropy", "clip_frac", "approx_kl", "grad_norm", "flags", "kl",
                "lr")


def _lib():
    return _abi.load()


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, name: str, allow_none: bool = False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclass
class UpdateHParams:
    clip: float = 0.2
    value_coef: float = 1.0
    entropy_coef: float = 0.01
    max_grad_norm: float = 1.0
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    clip_value: bool = False
    use_graph: bool = True
    # KL-adaptive learning rate (Algorithm 1); 0 keeps the rate fixed
    desired_kl: float = 0.0
    lr_factor: float = 1.5
    lr_min: float = 1e-5
    lr_max: float = 1e-2

    def abi(self) -> _abi.HParams:
        return _abi.HParams(self.clip, self.value_coef, self.entropy_coef, self.max_grad_norm, self.beta1,
                            self.beta2, self.adam_eps, int(self.clip_value), int(self.use_graph),
                            self.desired_kl, self.lr_factor, self.lr_min, self.lr_max)


def net_desc(obs_dim: int, act_dim: int, hidden: Sequence[int]) -> _abi.NetDesc:
    h = list(hidden) + [0] * (_abi.PPO_MAX_HIDDEN - len(hidden))
    return _abi.NetDesc(obs_dim, act_dim, len(hidden), (ctypes.c_int32 * _abi.PPO_MAX_HIDDEN)(*h))


def ppo_param_count(obs_dim: int, act_dim: int, hidden: Sequence[int]) -> int:
    n = ctypes.c_int64()
    check(_lib().ppo_param_count(ctypes.byref(net_desc(obs_dim, act_dim, hidden)), ctypes.byref(n)))
    return n.value


def ppo_param_offsets(obs_dim: int, act_dim: int, hidden: Sequence[int]) -> list:
    cap = 4 * (len(hidden) + 1) + 1
    arr = (ctypes.c_int64 * cap)()
    check(_lib().ppo_param_offsets(ctypes.byref(net_desc(obs_dim, act_dim, hidden)), arr, cap))
    return list(arr)


class Context:
    """A network shape and a precision (host-side state of the library)."""

    def __init__(self, obs_dim: int, act_dim: int, hidden: Sequence[int], precision: str = "bf16"):
        if precision not in ("fp32", "bf16"):
            raise ValueError("precision must be 'fp32' or 'bf16'")
        self.obs_dim, self.act_dim, self.hidden = obs_dim, act_dim, tuple(hidden)
        self.precision = precision
        self._desc = net_desc(obs_dim, act_dim, hidden)
        h = ctypes.c_void_p()
        check(_lib().ppo_ctx_create(ctypes.byref(self._desc), PPO_BF16 if precision == "bf16" else PPO_FP32,
                                    ctypes.byref(h)))
        self.handle = h

    def close(self) -> None:
        if self.handle:
            check(_lib().ppo_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return ppo_param_count(self.obs_dim, self.act_dim, self.hidden)

    def param_offsets(self) -> list:
        return ppo_param_offsets(self.obs_dim, self.act_dim, self.hidden)

    def workspace_size(self, N: int = 0, T: int = 0, M: int = 0) -> int:
        n = ctypes.c_size_t()
        check(_lib().ppo_workspace_size(self.handle, N, T, M, ctypes.byref(n)))
        return n.value

    TILE_NAMES = ("128x128", "64x128", "128x64", "64x64")

    def tuning(self, rows: int, update: bool) -> Dict[str, object]:
        """Tile choices the autotuner recorded for `rows` GEMM rows."""
        arr = (ctypes.c_int32 * 18)()
        check(_lib().ppo_ctx_tuning(self.handle, rows, int(update), arr, 18))
        out = {}
        for l in range(len(self.hidden)):
            out[f"forward_{l + 1}"] = self.TILE_NAMES[arr[2 * l]]
        if update:
            for l in range(1, len(self.hidden)):
                out[f"input_grad_{l + 1}"] = self.TILE_NAMES[arr[2 * (4 + l)]]
            out["weight_grad"] = f"{self.TILE_NAMES[arr[16]]} x {arr[17]} half round(s) of splits"
        return out

    def fused_shape(self) -> Tuple[int, int]:
        """(samples, threads) per workgroup of the fused bf16 update pass, or
        (0, 0) when update steps run the layer-by-layer kernels."""
        r, t = ctypes.c_int32(0), ctypes.c_int32(0)
        check(_lib().ppo_fused_shape(self.handle, ctypes.byref(r), ctypes.byref(t)))
        return r.value, t.value

    def fused_infer_shape(self) -> Tuple[int, int]:
        """(environments, threads) per workgroup of bf16 fused inference, or (0, 0)."""
        r, t = ctypes.c_int32(0), ctypes.c_int32(0)
        check(_lib().ppo_fused_infer_shape(self.handle, ctypes.byref(r), ctypes.byref(t)))
        return r.value, t.value

    def keep_packed(self, enable: bool = True) -> None:
        """PPO_OPT_KEEP_PACKED: reuse the forward weights packed into a workspace
        across inference calls.  Only for workspaces kept alive and written by
        this library alone (not the per-call workspaces the binding allocates
        when none is passed)."""
        check(_lib().ppo_ctx_set_option(self.handle, _abi.PPO_OPT_KEEP_PACKED, int(bool(enable))))

    def new_workspace(self, N: int = 0, T: int = 0, M: int = 0, device="cuda") -> torch.Tensor:
        nbytes = self.workspace_size(N, T, M)
        return torch.empty(max(nbytes, 16), dtype=torch.uint8, device=device)


class Params:
    """Device-resident parameters and optimiser state in the flat layout."""

    def __init__(self, ctx: Context, theta0, lr: float = 1e-3, device="cuda", stream=None):
        P = ctx.param_count
        theta0 = torch.as_tensor(np.asarray(theta0, dtype=np.float32)).reshape(-1)
        if theta0.numel() != P:
            raise ValueError(f"theta has {theta0.numel()} entries, the network has {P}")
        self.ctx = ctx
        self.theta = theta0.to(device).contiguous()
        self.grad = torch.zeros(P, dtype=torch.float32, device=device)
        self.adam_m = torch.zeros(P, dtype=torch.float32, device=device)
        self.adam_v = torch.zeros(P, dtype=torch.float32, device=device)
        self.shadow = torch.zeros(P, dtype=torch.int16, device=device)
        self.step = torch.zeros(4, dtype=torch.int32, device=device)
        self.lr = torch.full((4,), lr, dtype=torch.float32, device=device)
        self.pack(stream)

    def pack(self, stream=None) -> None:
        """Refresh the bf16 shadow after theta was written outside the library."""
        ppo_pack_weights(self.ctx, self.theta, self.shadow, stream)

    def abi(self) -> _abi.Params:
        return _abi.Params(_ptr(self.theta, torch.float32, "theta"), _ptr(self.grad, torch.float32, "grad"),
                           _ptr(self.adam_m, torch.float32, "adam_m"), _ptr(self.adam_v, torch.float32, "adam_v"),
                           _ptr(self.shadow, torch.int16, "shadow"), _ptr(self.step, torch.int32, "step"),
                           _ptr(self.lr, torch.float32, "lr"))


def make_batch(obs, actions, logp, adv, returns, values=None, mu_old=None, logstd_old=None) -> _abi.Batch:
    B = obs.shape[0]
    return _abi.Batch(_ptr(obs, torch.float32, "obs"), _ptr(actions, torch.float32, "actions"),
                      _ptr(logp, torch.float32, "logp"), _ptr(adv, torch.float32, "adv"),
                      _ptr(returns, torch.float32, "returns"), _ptr(values, torch.float32, "values", True),
                      _ptr(mu_old, torch.float32, "mu_old", True), _ptr(logstd_old, torch.float32, "logstd_old", True),
                      B)


def batch_abi(batch: Dict[str, torch.Tensor]) -> _abi.Batch:
    """The ABI batch of a dict with keys obs, actions, logp, adv, returns and
    optionally values, mu_old, logstd_old (the caller keeps the tensors alive)."""
    return make_batch(batch["obs"], batch["actions"], batch["logp"], batch["adv"], batch["returns"],
                      batch.get("values"), batch.get("mu_old"), batch.get("logstd_old"))


def ppo_pack_weights(ctx: Context, theta: torch.Tensor, shadow: torch.Tensor, stream=None) -> None:
    check(_lib().ppo_pack_weights(ctx.handle, _stream(stream), _ptr(theta, torch.float32, "theta"),
                                  _ptr(shadow, torch.int16, "shadow")))


def ppo_assemble_obs(ctx: Context, obs: torch.Tensor, t: int, seed: int, iteration: int,
                     proprio: Optional[torch.Tensor] = None, base: Optional[torch.Tensor] = None,
                     height: Optional[torch.Tensor] = None, inv_res: float = 10.0,
                     scan: Optional[torch.Tensor] = None, noise_scale: Optional[torch.Tensor] = None,
                     stream=None) -> None:
    """obs [N, D] <- proprio [N, P], the height scan of `height` [nx, ny] at the
    body-frame points `scan` [S, 2] around each `base` [N, 5] (x, y, z, cos yaw,
    sin yaw), plus uniform noise of half-width noise_scale [D] (None: none)."""
    N, D = obs.shape
    P = 0 if proprio is None else proprio.shape[1]
    if proprio is not None and tuple(proprio.shape) != (N, P):
        raise ValueError(f"proprio must be [{N}, P], got {tuple(proprio.shape)}")
    if noise_scale is not None and tuple(noise_scale.shape) != (D,):
        raise ValueError(f"noise_scale must be [{D}], got {tuple(noise_scale.shape)}")
    terrain = None
    if scan is not None and scan.shape[0] > 0:
        if scan.dim() != 2 or scan.shape[1] != 2:
            raise ValueError(f"scan must be [S, 2], got {tuple(scan.shape)}")
        if base is None or tuple(base.shape) != (N, 5):
            raise ValueError(f"base must be [{N}, 5]")
        if height is None or height.dim() != 2:
            raise ValueError("height must be a 2-D [nx, ny] tensor")
        nx, ny = height.shape
        terrain = _abi.Terrain(_ptr(height, torch.float32, "height"), nx, ny, float(inv_res),
                               _ptr(scan, torch.float32, "scan"), scan.shape[0])
    check(_lib().ppo_assemble_obs(ctx.handle, _stream(stream), _ptr(proprio, torch.float32, "proprio", True), P,
                                  _ptr(base, torch.float32, "base", True),
                                  ctypes.byref(terrain) if terrain is not None else None,
                                  _ptr(noise_scale, torch.float32, "noise_scale", True), N, t, seed, iteration,
                                  _ptr(obs, torch.float32, "obs")))


def ppo_rollout_infer(ctx: Context, params: Params, obs: torch.Tensor, t: int, seed: int, iteration: int,
                      actions=None, logp=None, values=None, mu=None, ws: Optional[torch.Tensor] = None,
                      stream=None) -> None:
    N = obs.shape[0]
    if ws is None:
        ws = ctx.new_workspace(N=N, device=obs.device)
    p = params.abi()
    check(_lib().ppo_rollout_infer(ctx.handle, _stream(stream), ctypes.byref(p), _ptr(obs, torch.float32, "obs"),
                                   N, t, seed, iteration, _ptr(actions, torch.float32, "actions", True),
                                   _ptr(logp, torch.float32, "logp", True),
                                   _ptr(values, torch.float32, "values", True),
                                   _ptr(mu, torch.float32, "mu", True), _ptr(ws, torch.uint8, "ws"), ws.numel()))


def ppo_gae(ctx: Context, rewards, dones, values, last_values, gamma: float, lam: float, adv, returns, adv_stats,
            timeouts=None, normalize: bool = True, ws: Optional[torch.Tensor] = None, stream=None) -> None:
    T, N = rewards.shape
    if ws is None:
        ws = ctx.new_workspace(N=N, T=T, device=rewards.device)
    check(_lib().ppo_gae(ctx.handle, _stream(stream), _ptr(rewards, torch.float32, "rewards"),
                         _ptr(dones, torch.uint8, "dones"), _ptr(timeouts, torch.uint8, "timeouts", True),
                         _ptr(values, torch.float32, "values"), _ptr(last_values, torch.float32, "last_values"),
                         T, N, gamma, lam, _ptr(adv, torch.float32, "adv"), _ptr(returns, torch.float32, "returns"),
                         _ptr(adv_stats, torch.float64, "adv_stats"), int(normalize), _ptr(ws, torch.uint8, "ws"),
                         ws.numel()))


def ppo_gae_noalloc(ctx: Context, rewards, dones, values, last_values, gamma: float, lam: float, adv, returns,
                    adv_stats, timeouts=None, normalize: bool = True, stream=None) -> None:
    """ppo_gae without a workspace: the library's fixed per-device scratch
    holds the statistics partials (N <= PPO_GAE_NOALLOC_MAX_N)."""
    T, N = rewards.shape
    check(_lib().ppo_gae_noalloc(ctx.handle, _stream(stream), _ptr(rewards, torch.float32, "rewards"),
                                 _ptr(dones, torch.uint8, "dones"), _ptr(timeouts, torch.uint8, "timeouts", True),
                                 _ptr(values, torch.float32, "values"),
                                 _ptr(last_values, torch.float32, "last_values"), T, N, gamma, lam,
                                 _ptr(adv, torch.float32, "adv"), _ptr(returns, torch.float32, "returns"),
                                 _ptr(adv_stats, torch.float64, "adv_stats"), int(normalize)))


def ppo_update_epoch(ctx: Context, params: Params, batch: Dict[str, torch.Tensor], perm: torch.Tensor,
                     n_minibatches: int, hp: UpdateHParams, stats: torch.Tensor, ws: torch.Tensor,
                     stream=None) -> None:
    b = batch_abi(batch)
    p = params.abi()
    h = hp.abi()
    check(_lib().ppo_update_epoch(ctx.handle, _stream(stream), ctypes.byref(p), ctypes.byref(b),
                                  _ptr(perm, torch.int32, "perm"), n_minibatches, ctypes.byref(h),
                                  _ptr(stats, torch.float32, "stats"), _ptr(ws, torch.uint8, "ws"), ws.numel()))


def ppo_update_batched(ctxs: Sequence[Context], params: Sequence[Params], batches: Sequence[Dict[str, torch.Tensor]],
                       perms: Sequence[torch.Tensor], n_minibatches: int, hp: UpdateHParams,
                       stats: Sequence[torch.Tensor], ws: Sequence[torch.Tensor], stream=None) -> None:
    """One epoch of R independent runs through shared grouped launches."""
    R = len(ctxs)
    c_ctx = (ctypes.c_void_p * R)(*[c.handle.value for c in ctxs])
    c_par = (_abi.Params * R)(*[p.abi() for p in params])
    c_bat = (_abi.Batch * R)(*[batch_abi(b) for b in batches])
    c_perm = (ctypes.c_void_p * R)(*[_ptr(p, torch.int32, "perm") for p in perms])
    c_stats = (ctypes.c_void_p * R)(*[_ptr(s, torch.float32, "stats") for s in stats])
    c_ws = (ctypes.c_void_p * R)(*[_ptr(w, torch.uint8, "ws") for w in ws])
    c_wsb = (ctypes.c_size_t * R)(*[w.numel() for w in ws])
    h = hp.abi()
    check(_lib().ppo_update_batched(c_ctx, R, _stream(stream), c_par, c_bat, c_perm, n_minibatches,
                                    ctypes.byref(h), c_stats, c_ws, c_wsb))


def ppo_loss_grad(ctx: Context, params: Params, batch: Dict[str, torch.Tensor], idx: torch.Tensor,
                  hp: UpdateHParams, stats: torch.Tensor, grad_out: torch.Tensor, ws: torch.Tensor,
                  stream=None, active_out: Optional[torch.Tensor] = None,
                  ratio_out: Optional[torch.Tensor] = None) -> None:
    """active_out (uint8 [M]) and ratio_out (float32 [M]), both optional,
    receive each row's surrogate branch and probability ratio."""
    b = batch_abi(batch)
    p = params.abi()
    h = hp.abi()
    for name, t in (("active_out", active_out), ("ratio_out", ratio_out)):
        if t is not None and t.numel() != idx.numel():
            raise ValueError(f"{name} needs one entry per mini-batch row")
    check(_lib().ppo_loss_grad(ctx.handle, _stream(stream), ctypes.byref(p), ctypes.byref(b),
                               _ptr(idx, torch.int32, "idx"), idx.numel(), ctypes.byref(h),
                               _ptr(stats, torch.float32, "stats"), _ptr(grad_out, torch.float32, "grad_out"),
                               _ptr(active_out, torch.uint8, "active_out", True),
                               _ptr(ratio_out, torch.float32, "ratio_out", True), _ptr(ws, torch.uint8, "ws"),
                               ws.numel()))


def ppo_update_epoch_profiled(ctx: Context, params: Params, batch: Dict[str, torch.Tensor], perm: torch.Tensor,
                              n_minibatches: int, hp: UpdateHParams, stats: torch.Tensor, ws: torch.Tensor,
                              stream=None, reps: int = 1) -> Dict[str, tuple]:
    """Eager epoch with HIP events around each launch (repeatable launches
    enqueued `reps` times inside their events); returns {phase: (ms, launches)}."""
    b = batch_abi(batch)
    p = params.abi()
    h = hp.abi()
    n = len(_abi.PHASES)
    ms = (ctypes.c_float * n)()
    cnt = (ctypes.c_int32 * n)()
    check(_lib().ppo_update_epoch_profiled(ctx.handle, _stream(stream), ctypes.byref(p), ctypes.byref(b),
                                           _ptr(perm, torch.int32, "perm"), n_minibatches, ctypes.byref(h),
                                           _ptr(stats, torch.float32, "stats"), _ptr(ws, torch.uint8, "ws"),
                                           ws.numel(), reps, ms, cnt))
    return {name: (ms[i], cnt[i]) for i, name in enumerate(_abi.PHASES)}


def ppo_gemm_check(precision: str, a_mode: int, b_mode: int, epilogue: int, M: int, N: int, K: int,
                   A: torch.Tensor, lda: int, B: torch.Tensor, ldb: int, C: torch.Tensor, ldc: int,
                   bias=None, H=None, ldh: int = 0, rowsum=None, splits: int = 1, tile: int = 0,
                   stream=None) -> None:
    """One launch of the library GEMM (verification entry point)."""
    et = torch.int16 if precision == "bf16" else torch.float32
    ct = torch.float32 if epilogue == 2 else et
    check(_lib().ppo_gemm_check(_stream(stream), PPO_BF16 if precision == "bf16" else PPO_FP32, a_mode, b_mode,
                                epilogue, M, N, K, _ptr(A, et, "A"), lda, _ptr(B, et, "B"), ldb, _ptr(C, ct, "C"),
                                ldc, _ptr(bias, torch.float32, "bias", True), _ptr(H, et, "H", True), ldh,
                                _ptr(rowsum, torch.float32, "rowsum", True), splits, tile))


def ppo_philox_blocks(seed: int, c0: int, c1: int, c2: int, c3: int, out: torch.Tensor, stream=None) -> None:
    n = out.numel() // 4
    check(_lib().ppo_philox_blocks(_stream(stream), seed, c0, c1, c2, c3, n, _ptr(out, torch.int32, "out")))


def stats_dict(row) -> Dict[str, float]:
    row = [float(x) for x in row]
    return dict(zip(STATS_FIELDS, row))
