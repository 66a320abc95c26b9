"""POD(S, eps) by a thin SVD of the snapshot matrix (Def. 2.1, Def. 2.5).

The POD modes and singular values of a snapshot multiset are the left singular
vectors and singular values of the snapshot map e_m -> s_m (Def. 2.1), i.e. of
the matrix whose columns are the snapshots.  This oracle takes them from
LAPACK's divide-and-conquer SVD and never forms the Gram matrix, whose
condition number is the square of the snapshot map's (Rem. 2.3).

Truncation (Def. 2.5, with Thm. 2.4): N is the smallest N' in {0..|S|} with
sum_{n > N'} sigma_n^2 <= eps^2 (inclusive bound).  For eps = 0 no SVD is done
and the input is returned with all singular values set to 1.
"""
from __future__ import annotations

import numpy as np


def tail_sums(sigma) -> np.ndarray:
    """tail[N'] = sum_{n > N'} sigma_n^2 for N' = 0..len(sigma), in float64,
    accumulated from the smallest term upwards."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    t = np.zeros(len(s2) + 1)
    acc = 0.0
    for i in range(len(s2) - 1, -1, -1):
        acc += s2[i]
        t[i] = acc
    return t


def truncation_rank(sigma, eps) -> int:
    """Def. 2.5: smallest N' with sum_{n>N'} sigma_n^2 <= eps^2."""
    t = tail_sums(sigma)
    e2 = float(eps) ** 2
    for N in range(len(t)):
        if t[N] <= e2:
            return N
    return len(t) - 1  # unreachable: t[-1] == 0


def pod(S, eps):
    """Return ``(sigma, U)``: the first N singular values (descending) and the
    corresponding modes (columns of U).  ``eps == 0`` is the pass-through
    POD(S, 0) = {(1, s)}."""
    S = np.asarray(S, dtype=np.float64)
    n, m = S.shape
    if eps == 0.0:
        return np.ones(m), S.copy()
    if m == 0:
        return np.zeros(0), np.zeros((n, 0))
    U, s, _ = np.linalg.svd(S, full_matrices=False)
    N = truncation_rank(s, eps)
    return s[:N].copy(), U[:, :N].copy()


def pod_full(S):
    """All singular values and left singular vectors (thin SVD)."""
    S = np.asarray(S, dtype=np.float64)
    if S.shape[1] == 0:
        return np.zeros(0), np.zeros((S.shape[0], 0))
    U, s, _ = np.linalg.svd(S, full_matrices=False)
    return s, U


def pod_rank(S, eps) -> int:
    """|POD(S, eps)| without returning the modes."""
    S = np.asarray(S, dtype=np.float64)
    if eps == 0.0:
        return S.shape[1]
    if S.shape[1] == 0:
        return 0
    s = np.linalg.svd(S, compute_uv=False)
    return truncation_rank(s, eps)
