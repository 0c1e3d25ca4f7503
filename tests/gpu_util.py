"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel2(a, b):
    """||a - b||_2 / ||b||_2: the measure of the reduced-precision error bounds."""
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel(a, b):
    """The FP64 parity measure (results within 1e-12): the larger of
    ||a - b||_2 / ||b||_2 and max|a - b| / max|b|, so that a wrong value at a
    few entries (a corner or boundary DoF) is not diluted by the rest of a
    long vector."""
    a, b = np.asarray(a), np.asarray(b)
    mb = np.abs(b).max() if b.size else 0.0
    mi = (np.abs(a - b).max() if b.size else 0.0) / (mb if mb > 0 else 1.0)
    return max(rel2(a, b), mi)


def announce(*what):
    print("[gpu case]", *what, flush=True)
    sys.stdout.flush()
