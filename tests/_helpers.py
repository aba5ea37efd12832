"""Shared helpers of the GPU parity tests (the oracle side and the GPU side each build their own operator)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_freq_relerr(A, B):
    """max over frequencies and columns of ||A[j,c] - B[j,c]|| / ||B[j,c]||."""
    d = np.linalg.norm(A - B, axis=-1)
    n = np.linalg.norm(B, axis=-1)
    return float((d / np.maximum(n, 1e-300)).max())


def mode_alignment(X, Y):
    """min over (j, i) of |<x, y>| / (|x| |y|): 1 when the modes agree up to a phase factor."""
    num = np.abs(np.sum(np.conj(X) * Y, axis=-1))
    den = np.linalg.norm(X, axis=-1) * np.linalg.norm(Y, axis=-1)
    return float((num / den).min())


def gpu_tensor(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
