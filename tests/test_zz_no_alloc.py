"""The allocation-free GAE entry point against ppo_gae, through the C ABI:
bit-identical advantages, returns and statistics on two calls in a row, the
second with a smaller rollout (the library's fixed scratch then holds the
first call's partials past the second call's blocks)."""
import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
from tests.gpu_common import dev, require_gpu

pytestmark = pytest.mark.gpu


def _rollout(T, N, seed):
    rng = np.random.default_rng(seed)
    r = rng.normal(0, 0.1, (T, N)).astype(np.float32)
    v = rng.normal(0, 1, (T, N)).astype(np.float32)
    dn = (rng.random((T, N)) < 0.01).astype(np.uint8)
    to = (dn.astype(bool) & (rng.random((T, N)) < 0.5)).astype(np.uint8)
    last = rng.normal(0, 1, N).astype(np.float32)
    return r, dn, to, v, last


@pytest.mark.parametrize("normalize", [True, False])
def test_gae_noalloc_matches_workspace_entry_point(normalize):
    d = require_gpu()
    ctx = ppo.Context(48, 12, (64, 64), "fp32")
    # second call smaller in both T and N; the last shape has a ragged block
    for T, N in ((24, 40000), (7, 1000), (3, 257)):
        print(f"[gpu-case] gae_noalloc T={T} N={N} normalize={normalize}", flush=True)
        r, dn, to, v, last = [dev(x, d) for x in _rollout(T, N, seed=T * 7919 + N)]
        out = []
        for fn in ("ws", "noalloc"):
            adv = torch.full((T, N), float("nan"), device=d)
            ret = torch.full((T, N), float("nan"), device=d)
            st = torch.full((2,), float("nan"), dtype=torch.float64, device=d)
            if fn == "ws":
                ppo.ppo_gae(ctx, r, dn, v, last, 0.99, 0.95, adv, ret, st, timeouts=to, normalize=normalize)
            else:
                ppo.ppo_gae_noalloc(ctx, r, dn, v, last, 0.99, 0.95, adv, ret, st, timeouts=to,
                                    normalize=normalize)
            torch.cuda.synchronize()
            out.append((adv.cpu().numpy(), ret.cpu().numpy(), st.cpu().numpy()))
        for a, b in zip(out[0], out[1]):
            assert np.all(np.isfinite(b))
            np.testing.assert_array_equal(a, b)


def test_gae_noalloc_rejects_past_its_scratch():
    d = require_gpu()
    ctx = ppo.Context(48, 12, (64, 64), "fp32")
    N = ppo._abi.PPO_GAE_NOALLOC_MAX_N + 1
    x = torch.zeros(1, N, device=d)
    u = torch.zeros(1, N, dtype=torch.uint8, device=d)
    st = torch.zeros(2, dtype=torch.float64, device=d)
    with pytest.raises(ppo.PPOError):
        ppo.ppo_gae_noalloc(ctx, x, u, x, x[0], 0.99, 0.95, x, x, st)
