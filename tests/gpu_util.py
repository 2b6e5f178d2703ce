"""Shared helpers of the GPU tests: device transfer and error measures."""
import numpy as np
import torch

import oracle


def device():
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no ROCm GPU visible")
    return torch.device("cuda:0")


def to_dev(x: np.ndarray, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device(), dtype)


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().double().cpu().numpy()


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    return oracle.rel_frob(got, ref)


def sample_indices(p, rows, cols, count, seed, per_face=False):
    """Random output positions (k, i, j); per_face=True draws count per face."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if per_face:
        k = np.repeat(np.arange(p), count)
        n = p * count
    else:
        k = rng.integers(0, p, count)
        n = count
    i = rng.integers(0, rows, n)
    j = rng.integers(0, cols, n)
    return k, i, j


def sampled_rel_err(C_got: np.ndarray, A: np.ndarray, B: np.ndarray, k, i, j) -> float:
    """Relative Frobenius error over sampled entries, oracle entries computed
    one by one from the definition."""
    ref = oracle.tprod_entries(A, B, k, i, j)
    got = C_got[:, k, i, j]
    return float(np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
