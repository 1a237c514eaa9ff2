"""MI355X (gfx950) learning hot path of massively parallel PPO.

Hand-written HIP kernels behind the C ABI of include/ppo.h; this package is
the thin Python binding over it (torch provides device memory and streams).
"""
from ._abi import (PPO_BF16, PPO_E_HIP, PPO_E_INVAL, PPO_E_NOMEM, PPO_E_SHAPE, PPO_E_UNSUPPORTED, PPO_FP32,
                   PPO_OK, PPO_STATS_WIDTH, PPOError, LIB_PATH, load)
from .api import (Context, Params, UpdateHParams, make_batch, ppo_assemble_obs, ppo_gae, ppo_gae_noalloc, ppo_loss_grad, ppo_pack_weights,
                  ppo_param_count, ppo_param_offsets, ppo_philox_blocks, ppo_rollout_infer, ppo_update_epoch,
                  ppo_update_epoch_profiled, ppo_update_batched, ppo_gemm_check, stats_dict, STATS_FIELDS)
from .autograd import PPOLoss, ppo_loss

__all__ = [
    "PPO_BF16", "PPO_FP32", "PPO_OK", "PPO_E_INVAL", "PPO_E_SHAPE", "PPO_E_UNSUPPORTED", "PPO_E_HIP",
    "PPO_E_NOMEM", "PPO_STATS_WIDTH", "PPOError", "LIB_PATH", "load",
    "Context", "Params", "UpdateHParams", "make_batch", "ppo_assemble_obs", "ppo_gae", "ppo_gae_noalloc", "ppo_loss_grad", "ppo_pack_weights",
    "ppo_param_count", "ppo_param_offsets", "ppo_philox_blocks", "ppo_rollout_infer", "ppo_update_epoch",
    "ppo_update_epoch_profiled", "ppo_update_batched", "ppo_gemm_check",
    "stats_dict", "STATS_FIELDS", "PPOLoss", "ppo_loss",
]
