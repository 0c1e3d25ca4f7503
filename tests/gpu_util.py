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


def rel(a, b):
    """||a - b||_2 / ||b||_2 (the parity measure: FP64 results within 1e-12)."""
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def announce(*what):
    print("[gpu case]", *what, flush=True)
    sys.stdout.flush()
