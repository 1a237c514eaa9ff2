"""C-ABI checks that need no GPU: the library loads, exports everything the
header declares, agrees with the oracle on the parameter layout, and rejects
misuse with the documented codes before enqueuing anything."""
import ctypes
import os
import re

import pytest

import paper_2109_11978_amd as ppo
from paper_2109_11978_amd import _abi
from paper_2109_11978_amd.api import net_desc
from oracle import NetSpec, param_layout
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ppo.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="library not built")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ppo_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    lib = ppo.load()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_abi.EXPORTS)


@pytest.mark.parametrize("shape", [(48, 12, (64, 64)), (48, 12, (512, 256, 128)), (235, 12, (512, 256, 128)),
                                   (235, 12, (1024, 512, 256)), (7, 3, (16,)), (5, 16, (32, 48, 16, 64))])
def test_layout_matches_oracle(shape):
    D, A, H = shape
    spec = NetSpec(D, A, H)
    lay = param_layout(spec)
    assert ppo.ppo_param_count(D, A, H) == lay["__total__"][0]
    offs = ppo.ppo_param_offsets(D, A, H)
    names = [f"actor.{k}{l}" for l in range(1, len(H) + 2) for k in ("W", "b")] + ["actor.logstd"] + \
            [f"critic.{k}{l}" for l in range(1, len(H) + 2) for k in ("W", "b")]
    assert offs == [lay[n][0] for n in names]


def _code(fn, *args):
    return fn(*args)


def test_context_validation():
    lib = ppo.load()
    h = ctypes.c_void_p()
    for bad in [(0, 12, (64,)), (48, 0, (64,)), (48, 17, (64,)), (48, 12, (60,)), (48, 12, (4096,)),
                (48, 12, (64, 64, 64, 64, 64)[:4] + ())]:
        D, A, H = bad
        if len(H) <= 4 and all(x % 16 == 0 and 16 <= x <= 2048 for x in H) and 1 <= D and 1 <= A <= 16:
            continue
        rc = lib.ppo_ctx_create(ctypes.byref(net_desc(D, A, H)), 0, ctypes.byref(h))
        assert rc == ppo.PPO_E_SHAPE, bad
    rc = lib.ppo_ctx_create(ctypes.byref(net_desc(48, 12, (64,))), 7, ctypes.byref(h))
    assert rc == ppo.PPO_E_INVAL
    assert b"precision" in lib.ppo_last_error()


def test_workspace_size_grows():
    ctx = ppo.Context(48, 12, (512, 256, 128), "bf16")
    a = ctx.workspace_size(N=4096, T=24, M=24576)
    b = ctx.workspace_size(N=4096, T=24, M=49152)
    assert 0 < a < b
    f = ppo.Context(48, 12, (512, 256, 128), "fp32").workspace_size(N=4096, T=24, M=24576)
    assert f > a


FAKE = 0x10000  # aligned, never dereferenced: validation fails before any enqueue


def _params(lib_ctx_bf16=True):
    return _abi.Params(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE)


def _batch(B, obs=FAKE):
    return _abi.Batch(obs, FAKE, FAKE, FAKE, FAKE, None, None, None, B)


def test_misuse_codes():
    lib = ppo.load()
    ctx = ppo.Context(48, 12, (64, 64), "bf16")
    p = _params()
    hp = ppo.UpdateHParams().abi()
    ws = ctx.workspace_size(N=64, T=24, M=1536)
    stats = FAKE
    # N = 0
    assert lib.ppo_rollout_infer(ctx.handle, None, ctypes.byref(p), FAKE, 0, 0, 0, 0, FAKE, FAKE, FAKE, None,
                                 FAKE, ws) == ppo.PPO_E_SHAPE
    # misaligned obs
    assert lib.ppo_rollout_infer(ctx.handle, None, ctypes.byref(p), FAKE + 4, 64, 0, 0, 0, FAKE, FAKE, FAKE,
                                 None, FAKE, ws) == ppo.PPO_E_INVAL
    # value-only mode without values
    assert lib.ppo_rollout_infer(ctx.handle, None, ctypes.byref(p), FAKE, 64, 0, 0, 0, None, None, None, None,
                                 FAKE, ws) == ppo.PPO_E_INVAL
    # B % K != 0
    b = _batch(1536)
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 5, ctypes.byref(hp),
                                stats, FAKE, ws) == ppo.PPO_E_SHAPE
    assert b"divisible" in lib.ppo_last_error()
    # perm NULL
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), None, 1, ctypes.byref(hp),
                                stats, FAKE, ws) == ppo.PPO_E_SHAPE
    # misaligned obs in the batch
    b2 = _batch(1536, obs=FAKE + 8)
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b2), FAKE, 1, ctypes.byref(hp),
                                stats, FAKE, ws) == ppo.PPO_E_INVAL
    # workspace too small
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 1, ctypes.byref(hp),
                                stats, FAKE, 1024) == ppo.PPO_E_NOMEM
    # bad hyper-parameters
    bad = ppo.UpdateHParams(clip=0.0).abi()
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 1, ctypes.byref(bad),
                                stats, FAKE, ws) == ppo.PPO_E_INVAL
    # value clipping without stored values
    vc = ppo.UpdateHParams(clip_value=True).abi()
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 1, ctypes.byref(vc),
                                stats, FAKE, ws) == ppo.PPO_E_INVAL
    # GAE: T out of range, T*N < 2, gamma out of range
    assert lib.ppo_gae(ctx.handle, None, FAKE, FAKE, None, FAKE, FAKE, 0, 64, 0.99, 0.95, FAKE, FAKE, FAKE, 1,
                       FAKE, ws) == ppo.PPO_E_SHAPE
    assert lib.ppo_gae(ctx.handle, None, FAKE, FAKE, None, FAKE, FAKE, 1, 1, 0.99, 0.95, FAKE, FAKE, FAKE, 1,
                       FAKE, ws) == ppo.PPO_E_SHAPE
    assert lib.ppo_gae(ctx.handle, None, FAKE, FAKE, None, FAKE, FAKE, 24, 64, 1.5, 0.95, FAKE, FAKE, FAKE, 1,
                       FAKE, ws) == ppo.PPO_E_INVAL
    # allocation-free GAE: the same checks, and N past its fixed scratch
    assert lib.ppo_gae_noalloc(ctx.handle, None, FAKE, FAKE, None, FAKE, FAKE, 0, 64, 0.99, 0.95, FAKE, FAKE,
                               FAKE, 1) == ppo.PPO_E_SHAPE
    assert lib.ppo_gae_noalloc(ctx.handle, None, FAKE, FAKE, None, FAKE, FAKE, 24, 64, 0.99, 1.5, FAKE, FAKE,
                               FAKE, 1) == ppo.PPO_E_INVAL
    assert lib.ppo_gae_noalloc(ctx.handle, None, FAKE + 4, FAKE, None, FAKE, FAKE, 24, 64, 0.99, 0.95, FAKE,
                               FAKE, FAKE, 1) == ppo.PPO_E_INVAL
    assert lib.ppo_gae_noalloc(ctx.handle, None, FAKE, FAKE, None, FAKE, FAKE, 1, _abi.PPO_GAE_NOALLOC_MAX_N + 1,
                               0.99, 0.95, FAKE, FAKE, FAKE, 1) == ppo.PPO_E_SHAPE
    assert b"PPO_GAE_NOALLOC_MAX_N" in lib.ppo_last_error()
    # loss_grad: M larger than B
    assert lib.ppo_loss_grad(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 2000, ctypes.byref(hp),
                             FAKE, FAKE, None, None, FAKE, ws) == ppo.PPO_E_SHAPE
    # loss_grad: misaligned gradient output
    assert lib.ppo_loss_grad(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 100, ctypes.byref(hp),
                             FAKE, FAKE + 4, None, None, FAKE, ws) == ppo.PPO_E_INVAL
    assert lib.ppo_loss_grad(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 100, ctypes.byref(hp),
                             FAKE, FAKE, FAKE + 1, FAKE + 2, FAKE, ws) == ppo.PPO_E_INVAL
    assert b"ratio_out" in lib.ppo_last_error()
    # philox count
    assert lib.ppo_philox_blocks(None, 0, 0, 0, 0, 0, 0, FAKE) == ppo.PPO_E_SHAPE
    # null context
    assert lib.ppo_ctx_destroy(None) == ppo.PPO_E_INVAL


def test_batched_rejects_mismatched_runs():
    a = ppo.Context(48, 12, (64, 32), "bf16")
    b = ppo.Context(48, 12, (64,), "bf16")
    import ctypes
    from paper_2109_11978_amd import _abi
    lib = ppo.load()
    ctxs = (ctypes.c_void_p * 2)(a.handle.value, b.handle.value)
    pars = (_abi.Params * 2)()
    bats = (_abi.Batch * 2)()
    arr = (ctypes.c_void_p * 2)(0x10000, 0x10000)
    wsb = (ctypes.c_size_t * 2)(1 << 30, 1 << 30)
    h = ppo.UpdateHParams().abi()
    for i in range(2):
        pars[i] = _abi.Params(0x10000, 0x10000, 0x10000, 0x10000, 0x10000, 0x10000, 0x10000)
        bats[i] = _abi.Batch(0x10000, 0x10000, 0x10000, 0x10000, 0x10000, None, None, None, 64)
    rc = lib.ppo_update_batched(ctxs, 2, None, pars, bats, arr, 4, ctypes.byref(h), arr, arr, wsb)
    assert rc == ppo.PPO_E_SHAPE
    assert b"hidden layers" in lib.ppo_last_error()


def test_adaptive_rate_validation():
    lib = ppo.load()
    ctx = ppo.Context(48, 12, (64, 64), "bf16")
    p = _params()
    ws = ctx.workspace_size(N=64, T=24, M=1536)
    b = _batch(1536)
    # desired_kl > 0 needs the collection-time means
    h = ppo.UpdateHParams(desired_kl=0.01).abi()
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b), FAKE, 1, ctypes.byref(h),
                                FAKE, FAKE, ws) == ppo.PPO_E_INVAL
    assert b"mu_old" in lib.ppo_last_error()
    # mu_old without logstd_old
    b2 = _abi.Batch(FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, None, 1536)
    assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b2), FAKE, 1, ctypes.byref(h),
                                FAKE, FAKE, ws) == ppo.PPO_E_INVAL
    # bad rule parameters
    b3 = _abi.Batch(FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, 1536)
    for bad in (ppo.UpdateHParams(desired_kl=-1.0), ppo.UpdateHParams(desired_kl=0.01, lr_factor=0.5),
                ppo.UpdateHParams(desired_kl=0.01, lr_min=0.0), ppo.UpdateHParams(desired_kl=0.01, lr_max=1e-6),
                ppo.UpdateHParams(desired_kl=float("nan"))):
        hb = bad.abi()
        assert lib.ppo_update_epoch(ctx.handle, None, ctypes.byref(p), ctypes.byref(b3), FAKE, 1, ctypes.byref(hb),
                                    FAKE, FAKE, ws) == ppo.PPO_E_INVAL, bad


@pytest.mark.parametrize("shape,prec,env,expect", [
    ((48, 12, (512, 256, 128)), "bf16", {}, (64, 256)),
    ((235, 12, (512, 256, 128)), "bf16", {}, (64, 256)),
    # a 1024-wide layer needs eight feature blocks per wave over four waves,
    # which takes a workgroup's whole register file: 8 waves alone on a CU
    ((235, 12, (1024, 512, 256)), "bf16", {}, (64, 512)),
    ((235, 12, (1024, 512, 256)), "bf16", {"PPO_FUSED_ROWS": "32", "PPO_FUSED_THREADS": "512"}, (32, 512)),
    ((48, 12, (512, 256, 128)), "bf16", {"PPO_FUSED_ROWS": "64"}, (64, 256)),
    ((48, 12, (512, 256, 128)), "bf16", {"PPO_FUSED_ROWS": "32"}, (32, 256)),
    ((48, 12, (512, 256, 128)), "bf16", {"PPO_FUSED_ROWS": "64", "PPO_FUSED_THREADS": "512"}, (64, 512)),
    ((235, 12, (1024, 512, 256)), "bf16", {"PPO_FUSED_ROWS": "64"}, (64, 512)),
    ((235, 12, (1024, 512, 256)), "bf16", {"PPO_FUSED_THREADS": "256"}, (0, 0)),
    ((48, 12, (512, 256, 128)), "bf16", {"PPO_FUSED": "0"}, (0, 0)),
    ((48, 12, (512, 256, 128)), "fp32", {}, (0, 0)),
    ((48, 12, (64, 64)), "bf16", {}, (64, 256)),        # two feature blocks: two waves each over 64 rows
    ((48, 12, (64, 64)), "bf16", {"PPO_FUSED_ROWS": "64", "PPO_FUSED_THREADS": "256"}, (64, 256)),
    ((48, 12, (32, 32)), "bf16", {}, (0, 0)),           # one feature block for four waves
    # three workgroups per CU stream the first layer in 128-feature chunks
    ((48, 12, (512, 256, 128)), "bf16", {"PPO_FUSED_PER_CU": "3"}, (64, 256)),
    ((48, 12, (512, 256, 128)), "bf16", {"PPO_FUSED_PER_CU": "2"}, (64, 256)),
    ((235, 12, (512, 256, 128)), "bf16", {"PPO_FUSED_PER_CU": "3"}, (64, 256)),  # loss inputs deferred to the head
    ((48, 12, (64, 64)), "bf16", {"PPO_FUSED_PER_CU": "3"}, (0, 0)),           # first layer narrower than a chunk
    ((40, 12, (512, 256, 128)), "bf16", {}, (0, 0)),    # input width not a multiple of 16
    ((48, 12, (384, 256, 128)), "bf16", {}, (0, 0)),    # 12 feature blocks over 4 waves: 3 per wave
])
def test_fused_shape_selection(monkeypatch, shape, prec, env, expect):
    """Which bf16 update steps take the fused per-sample pass, and its block
    shape (host-side rule; no GPU needed)."""
    for k in ("PPO_FUSED", "PPO_FUSED_ROWS", "PPO_FUSED_THREADS", "PPO_FUSED_PER_CU"):
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    D, A, H = shape
    ctx = ppo.Context(D, A, H, prec)
    assert ctx.fused_shape() == expect


def test_assemble_obs_validation():
    """Observation assembly rejects bad shapes and pointers before any device work."""
    lib = ppo.load()
    ctx = ppo.Context(235, 12, (64, 64), "bf16")
    terr = _abi.Terrain(FAKE, 480, 480, 10.0, FAKE, 187)
    call = lambda **kw: lib.ppo_assemble_obs(
        ctx.handle, None, kw.get("proprio", FAKE), kw.get("P", 48), kw.get("base", FAKE),
        ctypes.byref(kw.get("terrain", terr)) if kw.get("terrain", terr) is not None else None,
        kw.get("noise", None), kw.get("N", 4096), kw.get("t", 0), 0, 0, kw.get("obs", FAKE))
    assert call(P=47) == ppo.PPO_E_SHAPE                 # 47 + 187 != 235
    assert b"obs_dim" in lib.ppo_last_error()
    assert call(terrain=None) == ppo.PPO_E_SHAPE         # 48 + 0 != 235
    assert call(N=0) == ppo.PPO_E_SHAPE
    assert call(N=1 << 30) == ppo.PPO_E_SHAPE            # N * ceil(D/4) >= 2^31
    assert call(N=(1 << 24) + 1) == ppo.PPO_E_SHAPE
    assert call(t=-1) == ppo.PPO_E_SHAPE
    assert call(obs=None) == ppo.PPO_E_INVAL
    assert call(obs=FAKE + 4) == ppo.PPO_E_INVAL
    assert call(base=None) == ppo.PPO_E_INVAL
    assert call(proprio=None) == ppo.PPO_E_INVAL
    assert call(noise=FAKE + 8) == ppo.PPO_E_INVAL
    for bad in (_abi.Terrain(FAKE, 0, 480, 10.0, FAKE, 187), _abi.Terrain(FAKE, 480, (1 << 24) + 1, 10.0, FAKE, 187)):
        assert call(terrain=bad) == ppo.PPO_E_SHAPE
    for inv_res in (0.0, -10.0, float("inf"), float("nan")):
        assert call(terrain=_abi.Terrain(FAKE, 480, 480, inv_res, FAKE, 187)) == ppo.PPO_E_INVAL
    assert call(terrain=_abi.Terrain(None, 480, 480, 10.0, FAKE, 187)) == ppo.PPO_E_INVAL
    assert call(terrain=_abi.Terrain(FAKE, 480, 480, 10.0, None, 187)) == ppo.PPO_E_INVAL


def test_ctx_set_option_validation():
    lib = ppo.load()
    ctx = ppo.Context(48, 12, (64, 64), "bf16")
    assert lib.ppo_ctx_set_option(None, _abi.PPO_OPT_KEEP_PACKED, 1) == ppo.PPO_E_INVAL
    assert lib.ppo_ctx_set_option(ctx.handle, 99, 1) == ppo.PPO_E_INVAL
    assert lib.ppo_ctx_set_option(ctx.handle, _abi.PPO_OPT_KEEP_PACKED, 2) == ppo.PPO_E_INVAL
    assert lib.ppo_ctx_set_option(ctx.handle, _abi.PPO_OPT_KEEP_PACKED, 1) == ppo.PPO_OK
    assert lib.ppo_ctx_set_option(ctx.handle, _abi.PPO_OPT_KEEP_PACKED, 0) == ppo.PPO_OK


def test_fused_infer_shape_selection(monkeypatch):
    """bf16 inference prefers 32 rows x 256 threads (two workgroups per CU)
    where that block fits; shapes forced through the environment apply to
    both inference and the update."""
    for k in ("PPO_FUSED", "PPO_FUSED_ROWS", "PPO_FUSED_THREADS", "PPO_FUSED_PER_CU"):
        monkeypatch.delenv(k, raising=False)
    flat = ppo.Context(48, 12, (512, 256, 128), "bf16")
    assert flat.fused_infer_shape() == (32, 256)
    assert flat.fused_shape() == (64, 256)
    for H in ((1024, 512, 256), (64, 64)):
        assert ppo.Context(235, 12, H, "bf16").fused_infer_shape() == (0, 0)
    assert ppo.Context(48, 12, (512, 256, 128), "fp32").fused_infer_shape() == (0, 0)
    monkeypatch.setenv("PPO_FUSED_ROWS", "64")
    monkeypatch.setenv("PPO_FUSED_THREADS", "512")
    assert flat.fused_infer_shape() == (64, 512)
    monkeypatch.setenv("PPO_FUSED", "0")
    assert flat.fused_infer_shape() == (0, 0)
