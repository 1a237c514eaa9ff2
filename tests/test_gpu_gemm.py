"""The library's GEMM kernel on its own, every operand mode and epilogue,
against float64 NumPy products of the exact same (already rounded) operands.

bf16 operands are exact in float32, so the only differences are float32
accumulation order and the final rounding of the output; ragged M/N/K,
unaligned leading dimensions and split sums over K are covered."""
import numpy as np
import pytest
import torch

import paper_2109_11978_amd as ppo
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu


def to_bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def from_bf16_bits(b):
    return (b.astype(np.uint32) << 16).view(np.float32)


def operand(shape, prec, rng, scale=1.0):
    x = (rng.standard_normal(shape) * scale).astype(np.float32)
    if prec == "bf16":
        bits = to_bf16_bits(x)
        return from_bf16_bits(bits).astype(np.float64), torch.as_tensor(bits.view(np.int16)).cuda()
    return x.astype(np.float64), torch.as_tensor(x).cuda()


def output_values(t, prec):
    a = t.cpu().numpy()
    return from_bf16_bits(a.view(np.uint16)).astype(np.float64) if prec == "bf16" else a.astype(np.float64)


def acc_tol(K):
    """float32 accumulation of K exact products: a few ulps of the partial
    sums, which grow like sqrt(K) times a term (relative to the rms output)."""
    return 8 * 2.0 ** -24 * np.sqrt(K)


def check(got, ref, prec, what, K):
    rms = np.sqrt(np.mean(ref ** 2)) + 1e-30
    # one rounding of the output to the operand type plus float32 accumulation
    tol = (2.0 ** -8 if prec == "bf16" else 0.0) * np.abs(ref) + acc_tol(K) * rms
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} wrong; first at {np.argwhere(bad)[0]}: "
                           f"got {got[bad][0]}, expected {ref[bad][0]}")


FWD = [(1, 16, 8), (100, 64, 48), (333, 200, 235), (4103, 512, 48), (257, 128, 512), (64, 48, 7),
       (129, 80, 192), (77, 144, 320)]   # 3 and 5 bf16 k-slabs: odd tails of the two-slab pipeline


TILES = [0, 1, 2, 3]   # 128x128, 64x128, 128x64, 64x64


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("M,N,K", FWD)
def test_forward_bias_elu(prec, M, N, K, tile):
    require_gpu()
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    lda = -(-K // 8) * 8          # padded rows like the gathered observations
    a, ta = operand((M, lda), prec, rng)
    a[:, K:] = 0.0
    ta = ta.view(M, lda)
    b, tb = operand((N, K), prec, rng, scale=1 / np.sqrt(K))   # ldb = K (unaligned when K % 8 != 0)
    bias = rng.standard_normal(N).astype(np.float32)
    C = torch.zeros(M, N, dtype=tb.dtype, device="cuda")
    ppo.ppo_gemm_check(prec, 0, 0, 0, M, N, K, ta, lda, tb, K, C, N, bias=torch.as_tensor(bias).cuda(), tile=tile)
    torch.cuda.synchronize()
    z = a[:, :K] @ b.T + bias
    ref = np.where(z > 0, z, np.expm1(np.minimum(z, 0)))
    check(output_values(C, prec), ref, prec, "forward", K)


DX = [(1, 16, 16), (300, 48, 64), (1536, 64, 64), (4100, 256, 128), (777, 512, 256), (200, 64, 192)]


@pytest.mark.parametrize("b_mode", [0, 1])
@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("M,N,K", DX)
def test_input_grad_delu(prec, M, N, K, tile, b_mode):
    """b_mode 1: W [out=K, in=N] read transposed; b_mode 0: the staged W^T [N, K]."""
    require_gpu()
    rng = np.random.default_rng(M + 11 * N + K)
    a, ta = operand((M, K), prec, rng)
    w, tw = operand((K, N), prec, rng, scale=1 / np.sqrt(K))   # W[out=K][in=N]: B stored transposed
    z = rng.standard_normal((M, N)).astype(np.float32)
    hval = np.where(z > 0, z, np.expm1(np.minimum(z, 0))).astype(np.float32)
    if prec == "bf16":
        hb = to_bf16_bits(hval)
        hv = from_bf16_bits(hb).astype(np.float64)
        th = torch.as_tensor(hb.view(np.int16)).cuda()
    else:
        hv = hval.astype(np.float64)
        th = torch.as_tensor(hval).cuda()
    C = torch.zeros(M, N, dtype=ta.dtype, device="cuda")
    if b_mode == 1:
        ppo.ppo_gemm_check(prec, 0, 1, 1, M, N, K, ta, K, tw, N, C, N, H=th, ldh=N, tile=tile)
    else:
        twt = tw.t().contiguous()   # [N, K]
        ppo.ppo_gemm_check(prec, 0, 0, 1, M, N, K, ta, K, twt, K, C, N, H=th, ldh=N, tile=tile)
    torch.cuda.synchronize()
    ref = (a @ w) * np.where(hv > 0, 1.0, hv + 1.0)
    check(output_values(C, prec), ref, prec, "input_grad", K)


DW = [(12, 64, 1536, 12, 16), (1, 64, 1536, 12, 16), (64, 48, 1536, 12, 64), (512, 48, 24576, 16, 512),
      (256, 512, 24576, 16, 256), (128, 256, 1000, 5, 128), (12, 128, 24576, 16, 16), (1, 128, 24576, 16, 16),
      (64, 235, 700, 3, 64)]


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("M,N,K,splits,lda", DW)
def test_weight_grad_partials(prec, M, N, K, splits, lda, tile):
    require_gpu()
    rng = np.random.default_rng(M + 13 * N + K + splits)
    a_store, ta = operand((K, lda), prec, rng)     # dz stored [samples][lda], first M columns used
    ldb = -(-N // 8) * 8
    b_store, tb = operand((K, ldb), prec, rng)
    bk = 64 if prec == "bf16" else 32
    kps = -(-(-(-K // splits)) // bk) * bk
    used = -(-K // kps)
    C = torch.full((used, M, N), float("nan"), dtype=torch.float32, device="cuda")
    rs = torch.full((used, M), float("nan"), dtype=torch.float32, device="cuda")
    ppo.ppo_gemm_check(prec, 1, 1, 2, M, N, K, ta, lda, tb, ldb, C, N, rowsum=rs, splits=splits, tile=tile)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    rows = rs.cpu().numpy().astype(np.float64)
    A = a_store[:, :M]
    Bm = b_store[:, :N]
    for s in range(used):
        k0, k1 = s * kps, min(K, (s + 1) * kps)
        ref = A[k0:k1].T @ Bm[k0:k1]
        rms = np.sqrt(np.mean(ref ** 2))
        assert np.max(np.abs(got[s] - ref)) <= acc_tol(k1 - k0) * rms + 1e-30, f"split {s}"
        rref = A[k0:k1].sum(axis=0)
        assert np.max(np.abs(rows[s] - rref)) <= 1e-5 * (np.sqrt(np.mean(rref ** 2)) + 1.0), f"rowsum {s}"
    total = got.sum(axis=0)
    ref = A.T @ Bm
    assert np.linalg.norm(total - ref) <= 1e-6 * np.linalg.norm(ref) * np.sqrt(used)
