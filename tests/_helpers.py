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


def mode_errors(X, Y, gains, gap=1e-6):
    """Per-mode error of modes X against reference modes Y, both (k, N) for one frequency, with the reference
    gains (k,) sorted descending.  A mode is unique up to a phase factor, so a simple mode's error is
    min over phi of ||x e^{i phi} - y|| / ||y|| (both normalised).  Modes whose gains lie within a relative gap
    `gap` of each other span a subspace but are not unique one by one; each mode of such a cluster gets the
    distance between the cluster's orthogonal projectors (2-norm), which is the sine of the largest principal
    angle.  Returns an array (k,)."""
    X = np.asarray(X, complex)
    Y = np.asarray(Y, complex)
    k = X.shape[0]
    Xn = X / np.linalg.norm(X, axis=1, keepdims=True)
    Yn = Y / np.linalg.norm(Y, axis=1, keepdims=True)
    out = np.zeros(k)
    i = 0
    while i < k:
        j = i + 1
        while j < k and (gains[j - 1] - gains[j]) < gap * gains[j - 1]:
            j += 1
        if j == i + 1:
            c = np.vdot(Xn[i], Yn[i])
            ph = c / abs(c) if abs(c) > 0 else 1.0
            out[i] = np.linalg.norm(Xn[i] * ph - Yn[i])
        else:
            Qx = np.linalg.qr(X[i:j].T)[0]
            Qy = np.linalg.qr(Y[i:j].T)[0]
            resid = Qy - Qx @ (Qx.conj().T @ Qy)  # the part of the reference subspace outside span X
            out[i:j] = float(np.linalg.norm(resid, 2))
        i = j
    return out
