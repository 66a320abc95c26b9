"""Helpers for the GPU parity tests: host <-> column-major device tensors."""
import numpy as np
import torch


def dev_colmajor(A, dtype=torch.float64, ld=None):
    """Copy a 2-D numpy array to a column-major device tensor (n x m)."""
    A = np.asarray(A)
    n, m = A.shape
    ld = n if ld is None else ld
    base = torch.zeros((max(m, 1), max(ld, 1)), dtype=dtype, device="cuda")
    if n > 0 and m > 0:
        base[:m, :n] = torch.from_numpy(np.ascontiguousarray(A.T)).to(device="cuda", dtype=dtype)
    return base[:m, :n].t()


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()
