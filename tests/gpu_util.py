"""Helpers for GPU parity tests: move element-major numpy limbs to and from
limb-planar device tensors (marshalling only)."""
import sys

import numpy as np

import moma_inputs as mi


def to_dev(x):
    import torch
    return torch.from_numpy(mi.to_planar(x).view(np.int32)).to("cuda:0")


def from_dev(t):
    return mi.from_planar(t.cpu().numpy().view(np.uint32))


def say(*a):
    """Name the case before a GPU step, flushed, so a failure can be attributed."""
    print(*a, flush=True)
    sys.stdout.flush()


def sample_indices(n, k, seed):
    rng = np.random.default_rng(seed)
    head = np.arange(min(n, 64))
    tail = np.arange(max(0, n - 64), n)
    mid = rng.integers(0, n, size=k) if n else np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate([head, tail, mid]).astype(np.int64))
