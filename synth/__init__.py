"""Seeded synthetic inputs for the quaternion T-product.

This module only draws random numbers and lays them out.  It holds none of
the T-product arithmetic, so both the FP64 oracle (through the tests) and the
GPU path consume the very same tensors without sharing any computation.

Storage convention (shared by every consumer): a quaternion tensor X of size
rows x cols x p is a float array of shape (4, p, rows, cols).  Plane c holds
the c-th real component of X = a + b i + c j + d k, i.e. (a, b, c, d).  In the
Cayley-Dickson form X = X1 + X2 j (Section 2.2) this is
X1 = a + b i and X2 = c + d i, so the planes are (Re X1, Im X1, Re X2, Im X2).
Face k (0-based) is X[:, k].

Draws use numpy's PCG64 bit generator; a tensor is drawn as one float64 array
of shape (4, p, rows, cols) in C order, then cast by the caller if needed.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "quat_tensor",
    "face_scales",
    "config_inputs",
    "batch_problem_sizes",
    "batch_problem_inputs",
    "CONFIGS",
    "BATCH_P_CHOICES",
]

# The five workloads the method is exercised on.  Seeds follow
# 1000 * config + tensor index (A = 0, B = 1, target C = 2); the second draw of
# the precision workload uses 3010/3011.
CONFIGS = {
    1: dict(name="c1_8x8x8_p8", m=8, n=8, s=8, p=8, dist="normal"),
    2: dict(name="c2_256x256x256_p64", m=256, n=256, s=256, p=64, dist="uniform"),
    3: dict(name="c3_1024x1024x1024_p32", m=1024, n=1024, s=1024, p=32, dist="normal"),
    5: dict(name="c5_512x64x512_p100", m=512, n=64, s=512, p=100, dist="normal"),
}

BATCH_P_CHOICES = (8, 12, 16, 30, 32, 45, 64)


def quat_tensor(rows: int, cols: int, p: int, seed: int, dist: str = "normal") -> np.ndarray:
    """Random quaternion tensor, shape (4, p, rows, cols), float64.

    dist = "normal": every real component i.i.d. N(0, 1).
    dist = "uniform": every real component i.i.d. U[0, 1) (colour-video-like
    non-negative pixel values; the zero frequency then dominates).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (4, p, rows, cols)
    if dist == "normal":
        return rng.standard_normal(shape)
    if dist == "uniform":
        return rng.random(shape)
    raise ValueError(f"unknown distribution {dist!r}")


def face_scales(p: int) -> np.ndarray:
    """Deterministic per-face scale grid 10**(-3 + 6 k / (p - 1)), k = 0..p-1.

    Spans 1e-3 .. 1e3 with both end points hit (p = 1 gives [1e-3]).
    """
    if p == 1:
        return np.array([1e-3])
    k = np.arange(p, dtype=np.float64)
    return 10.0 ** (-3.0 + 6.0 * k / (p - 1))


def config_inputs(cfg: int, draw: int = 1, scale: float | None = None):
    """Inputs (A, B) -- and for workload 5 also the target T -- as float64.

    cfg   : 1, 2, 3 or 5 (workload 4 is a batch, see batch_problem_*).
    draw  : 1 = plain draw; 2 = (workload 3 only) the same distribution with
            every face k of A and of B multiplied by face_scales(p)[k].
    scale : optional integer divisor to shrink m, n, s (keeps p) for quick
            test runs of the same distribution.
    """
    c = CONFIGS[cfg]
    m, n, s, p = c["m"], c["n"], c["s"], c["p"]
    if scale:
        m, n, s = max(1, m // scale), max(1, n // scale), max(1, s // scale)
    if draw == 1:
        sa, sb = 1000 * cfg, 1000 * cfg + 1
    elif draw == 2:
        if cfg != 3:
            raise ValueError("the scaled second draw exists for workload 3 only")
        sa, sb = 1000 * cfg + 10, 1000 * cfg + 11
    else:
        raise ValueError("draw must be 1 or 2")
    A = quat_tensor(m, n, p, sa, c["dist"])
    B = quat_tensor(n, s, p, sb, c["dist"])
    if draw == 2:
        w = face_scales(p)[None, :, None, None]
        A = A * w
        B = B * w
    if cfg == 5:
        T = quat_tensor(m, s, p, 1000 * cfg + 2, c["dist"])
        return A, B, T
    return A, B


def batch_problem_sizes(count: int = 512, seed: int = 4000, lo: int = 16, hi: int = 256,
                        p_choices=BATCH_P_CHOICES):
    """Sizes of the ragged batch: m, n, s ~ U{lo..hi}, p ~ U(p_choices).

    Returns an int array of shape (count, 4) with columns (m, n, s, p).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mns = rng.integers(lo, hi + 1, size=(count, 3))
    ps = rng.choice(np.asarray(p_choices, dtype=np.int64), size=count)
    return np.concatenate([mns, ps[:, None]], axis=1).astype(np.int64)


def batch_problem_inputs(i: int, m: int, n: int, s: int, p: int, base_seed: int = 4_100_000):
    """Inputs (A, B) of problem i of the batch, N(0, 1) components, float64."""
    rng = np.random.Generator(np.random.PCG64(base_seed + i))
    A = rng.standard_normal((4, p, m, n))
    B = rng.standard_normal((4, p, n, s))
    return A, B
