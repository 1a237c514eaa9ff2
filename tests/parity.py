"""Tolerance rule for float outputs of the HIP path against the FP64 oracle.

Per output tensor x with oracle value r and tolerance tol (1e-5 for the
float32 path, 2e-2 for bf16 GEMM operands):
  normwise     ||x - r||_2 / ||r||_2 <= tol
  elementwise  |x - r| <= tol * (|r| + rms(r))
The rms floor keeps entries near zero (cancelling sums, noise near 0) from
failing on a meaningless relative error.

Outputs that are sums over the mini-batch (the parameter gradient) are gated
normwise per parameter tensor (every W, b and the log-std vector) instead of
elementwise: single entries can be the small difference of large partial
sums (the log-std gradient minus the entropy coefficient, for one), where
float32 accumulation alone leaves 1e-5 of the partial sums but more than
1e-5 of the entry.  With bf16 operands, rounding the hidden weights shifts
every sample's outputs in a correlated way, so such sums also carry a
systematic error that grows with the batch; kernel bugs are caught apart
from that by the GEMM tests on exactly representable operands.
"""
import numpy as np

TOL = {"fp32": 1e-5, "bf16": 2e-2}


def rel_errors(x, ref):
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    r = np.asarray(ref, dtype=np.float64).reshape(-1)
    rms = np.sqrt(np.mean(r * r)) if r.size else 0.0
    norm = np.linalg.norm(r)
    normwise = np.linalg.norm(x - r) / norm if norm > 0 else np.linalg.norm(x - r)
    elem = np.max(np.abs(x - r) / (np.abs(r) + rms + 1e-300)) if r.size else 0.0
    return normwise, elem


def worst_element(x, ref):
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    r = np.asarray(ref, dtype=np.float64).reshape(-1)
    rms = np.sqrt(np.mean(r * r))
    i = int(np.argmax(np.abs(x - r) / (np.abs(r) + rms + 1e-300)))
    return i, x[i], r[i], rms


def assert_close(name, x, ref, tol, where=None, elementwise=True):
    """`where(i)` may name flat index i (e.g. the parameter tensor it belongs to)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert x.shape == ref.shape, (name, x.shape, ref.shape)
    assert np.all(np.isfinite(x)), f"{name}: non-finite output"
    nw, el = rel_errors(x, ref)
    if not (nw <= tol and (el <= tol or not elementwise)):
        i, xi, ri, rms = worst_element(x, ref)
        loc = where(i) if where else ""
        raise AssertionError(f"{name}: normwise {nw:.3e}, elementwise {el:.3e} > tol {tol:.1e}; worst at "
                             f"{i} {loc}: got {xi:.9g}, expected {ri:.9g}, rms {rms:.3g}")
    print(f"[parity] {name}: normwise {nw:.2e} elementwise {el:.2e} (tol {tol:.0e})")
    return nw, el


def per_tensor_errors(x, ref, layout):
    """{tensor name: normwise error} for a flat parameter-shaped vector."""
    out = {}
    for name, (off, shp) in layout.items():
        if name == "__total__":
            continue
        n = int(np.prod(shp))
        out[name] = rel_errors(x[off:off + n], ref[off:off + n])[0]
    return out


def assert_grad_close(name, x, ref, tol, layout):
    """Normwise per parameter tensor and over the whole vector."""
    per = per_tensor_errors(np.asarray(x, np.float64), np.asarray(ref, np.float64), layout)
    nw, el = rel_errors(x, ref)
    print(f"[parity] {name}: normwise {nw:.2e} (elementwise {el:.2e}); per tensor "
          + ", ".join(f"{k} {v:.1e}" for k, v in per.items()))
    bad = {k: v for k, v in per.items() if not v <= tol}
    assert nw <= tol and not bad, f"{name}: normwise {nw:.3e}, tensors over {tol:.0e}: {bad}"
    return per


def tie_bands(gpu_ratio, ref_ratio):
    """Per-sample clip-edge bands for the oracle's tie protocol: a sample may
    take the GPU's branch when the GPU's ratio (itself gated against the
    oracle's) could lie on the other side of the deciding edge, i.e. when the
    oracle's margin is below the distance between the two ratios, plus the
    float32 rounding of the edge 1 +- clip on the GPU (a few 1e-8)."""
    g = np.asarray(gpu_ratio, np.float64)
    r = np.asarray(ref_ratio, np.float64)
    return np.abs(g - r) + 1e-7 * np.maximum(1.0, np.abs(r))


def grad_report(x, ref, layout):
    """{tensor: (normwise, elementwise with the rms floor)} of a gradient."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    out = {}
    for name, (off, shp) in layout.items():
        if name == "__total__":
            continue
        n = int(np.prod(shp))
        out[name] = rel_errors(x[off:off + n], ref[off:off + n])
    return out
