"""ctypes declarations mirroring include/ppo.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libppo_mi355x.so")

PPO_OK = 0
PPO_E_INVAL = -1
PPO_E_SHAPE = -2
PPO_E_UNSUPPORTED = -3
PPO_E_HIP = -4
PPO_E_NOMEM = -5
PPO_FP32 = 0
PPO_BF16 = 1
PPO_MAX_HIDDEN = 4
PPO_STATS_WIDTH = 10
PPO_OPT_KEEP_PACKED = 1
PPO_GAE_NOALLOC_MAX_N = 1 << 21
PHASES = ("gather", "forward", "head_loss", "input_grad", "weight_grad", "grad_reduce", "adam", "fused")

ERROR_NAMES = {
    PPO_E_INVAL: "PPO_E_INVAL", PPO_E_SHAPE: "PPO_E_SHAPE", PPO_E_UNSUPPORTED: "PPO_E_UNSUPPORTED",
    PPO_E_HIP: "PPO_E_HIP", PPO_E_NOMEM: "PPO_E_NOMEM",
}


class NetDesc(ctypes.Structure):
    _fields_ = [("obs_dim", c_int32), ("act_dim", c_int32), ("n_hidden", c_int32),
                ("hidden", c_int32 * PPO_MAX_HIDDEN)]


class Params(ctypes.Structure):
    _fields_ = [("theta", c_void_p), ("grad", c_void_p), ("adam_m", c_void_p), ("adam_v", c_void_p),
                ("shadow", c_void_p), ("step", c_void_p), ("lr", c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("obs", c_void_p), ("actions", c_void_p), ("logp", c_void_p), ("adv", c_void_p),
                ("returns", c_void_p), ("values", c_void_p), ("mu_old", c_void_p), ("logstd_old", c_void_p),
                ("B", c_int32)]


class HParams(ctypes.Structure):
    _fields_ = [("clip", c_float), ("value_coef", c_float), ("entropy_coef", c_float),
                ("max_grad_norm", c_float), ("beta1", c_float), ("beta2", c_float), ("adam_eps", c_float),
                ("clip_value", c_int32), ("use_graph", c_int32), ("desired_kl", c_float), ("lr_factor", c_float),
                ("lr_min", c_float), ("lr_max", c_float)]


class Terrain(ctypes.Structure):
    _fields_ = [("height", c_void_p), ("nx", c_int32), ("ny", c_int32), ("inv_res", c_float),
                ("scan", c_void_p), ("n_scan", c_int32)]


EXPORTS = {
    "ppo_last_error": (c_char_p, []),
    "ppo_ctx_create": (c_int32, [POINTER(NetDesc), c_int32, POINTER(c_void_p)]),
    "ppo_ctx_destroy": (c_int32, [c_void_p]),
    "ppo_ctx_set_option": (c_int32, [c_void_p, c_int32, c_int32]),
    "ppo_param_count": (c_int32, [POINTER(NetDesc), POINTER(c_int64)]),
    "ppo_param_offsets": (c_int32, [POINTER(NetDesc), POINTER(c_int64), c_int32]),
    "ppo_workspace_size": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "ppo_pack_weights": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ppo_rollout_infer": (c_int32, [c_void_p, c_void_p, POINTER(Params), c_void_p, c_int32, c_int32, c_uint64,
                                    c_uint32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    "ppo_gae": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                          c_float, c_float, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_size_t]),
    "ppo_gae_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                  c_int32, c_float, c_float, c_void_p, c_void_p, c_void_p, c_int32]),
    "ppo_update_epoch": (c_int32, [c_void_p, c_void_p, POINTER(Params), POINTER(Batch), c_void_p, c_int32,
                                   POINTER(HParams), c_void_p, c_void_p, c_size_t]),
    "ppo_loss_grad": (c_int32, [c_void_p, c_void_p, POINTER(Params), POINTER(Batch), c_void_p, c_int32,
                                POINTER(HParams), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    "ppo_update_epoch_profiled": (c_int32, [c_void_p, c_void_p, POINTER(Params), POINTER(Batch), c_void_p, c_int32,
                                            POINTER(HParams), c_void_p, c_void_p, c_size_t, c_int32,
                                            POINTER(c_float), POINTER(c_int32)]),
    "ppo_gemm_check": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32,
                                 c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                                 c_int32, c_void_p, c_int32, c_int32]),
    "ppo_update_batched": (c_int32, [POINTER(c_void_p), c_int32, c_void_p, POINTER(Params), POINTER(Batch),
                                     POINTER(c_void_p), c_int32, POINTER(HParams), POINTER(c_void_p),
                                     POINTER(c_void_p), POINTER(c_size_t)]),
    "ppo_ctx_tuning": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int32), c_int32]),
    "ppo_fused_shape": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "ppo_fused_infer_shape": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "ppo_assemble_obs": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, POINTER(Terrain), c_void_p,
                                   c_int32, c_int32, c_uint64, c_uint32, c_void_p]),
    "ppo_philox_blocks": (c_int32, [c_void_p, c_uint64, c_uint32, c_uint32, c_uint32, c_uint32, c_int64,
                                    c_void_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Loads the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2109_11978_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PPOError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


def check(code: int) -> None:
    if code != PPO_OK:
        msg = load().ppo_last_error()
        raise PPOError(code, msg.decode() if msg else "")
