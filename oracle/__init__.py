"""FP64 CPU oracle for the PPO learning hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written from the paper (Rudin et al., "Learning to Walk in Minutes
Using Massively Parallel Deep Reinforcement Learning", CoRL 2021) and the
textbook definitions it builds on (PPO, GAE, Adam, Philox).  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  The product path (the HIP library and its Python binding) never imports,
links or executes anything here, and this package imports nothing from the
product path.

Every function evaluates in float64 on float32-valued inputs upcast to
float64, step by step in the order of the definitions it cites, with no
blocking, fusion or reordering beyond what a library matmul does.

Parity status per function (what pins it; see tests/test_oracle_*.py):
  philox4x32_10     rocRAND's Philox4x32-10 (a library routine, built for the host)
                    bit for bit on 2000 random blocks and the wrap edges; statistics
  uniforms/normals  closed form of the 24-bit uniform map; moment tests
  mlp_forward       pure-Python loop brute force on a tiny net
  gaussian_logp     scipy.stats.norm.logpdf sum; entropy vs Monte Carlo
  gae               lambda=1 / lambda=0 / gamma=0 closed forms, O(T^2) brute
                    force, hand-worked T=3 example (tests/golden/)
  ppo_loss_grad     central finite differences (full on a tiny net, sampled
                    coordinates and directions at the 64x24 workload);
                    vanilla policy-gradient special case at ratio 1; zero
                    policy gradient on the active clip side
  clip_coef         numpy.linalg.norm; post-clip norm equals the limit
  adam_step         torch.optim.Adam in float64 on CPU; first-step closed form
  gaussian_kl       numeric integration of the 1-D KL (scipy.integrate.quad);
                    zero for equal distributions; pure mean shift and pure
                    scale closed forms
  adaptive_lr       the thresholds and clamps of Algorithm 1, case by case
  update_epoch      composition of the above (no independent pin beyond its
                    parts: parity unpinned as a whole against the paper, which
                    prints no intermediate values)
  assemble_obs      nearest cell against a brute-force search over the whole
                    grid; heading 0, 90 and 180 degrees against plain array
                    slices; flat terrain; noise bounds, moments and
                    independence of the streams
"""
from .philox import philox4x32_10, uniforms, box_muller, action_noise
from .layout import NetSpec, param_layout, unpack
from .policy import elu, elu_grad, mlp_forward, gaussian_logp, gaussian_entropy, rollout_infer
from .advantage import gae, advantage_stats, normalize_advantages
from .observation import assemble_obs, height_scan, scan_world_points, nearest_cells, obs_noise_unit
from .ppo import (
    PPOHyper,
    ppo_loss_grad,
    clip_coef,
    adam_step,
    update_epoch,
    gaussian_kl,
    adaptive_lr,
)

__all__ = [
    "philox4x32_10", "uniforms", "box_muller", "action_noise",
    "NetSpec", "param_layout", "unpack",
    "elu", "elu_grad", "mlp_forward", "gaussian_logp", "gaussian_entropy", "rollout_infer",
    "gae", "advantage_stats", "normalize_advantages",
    "assemble_obs", "height_scan", "scan_world_points", "nearest_cells", "obs_noise_unit",
    "PPOHyper", "ppo_loss_grad", "clip_coef", "adam_step", "update_epoch", "gaussian_kl", "adaptive_lr",
]
