"""Accuracy metrics and the paper's inequalities, all in float64.

* projection error sum_s ||s - P s||^2 with P the orthogonal projection onto a
  span (the left side of Thm. 2.4 / Thm. 3.3).  It is always evaluated from
  the residual ``R = S - Q (Q^T S)``, re-projected once, never as
  ``||S||^2 - ||Q^T S||^2``, which cancels catastrophically.
* subspace error ``e_sub(r) = ||(I - U_r U_r^T) Q_r||_2`` between the leading
  r reference modes and an orthonormal basis of the leading r test modes.
* checks of Thm. 3.3 (error bound), Thm. 3.4 (mode bound) and Thm. 3.5
  (global mean error, global and local mode bounds).
"""
from __future__ import annotations

import math

import numpy as np

from . import hapod as _hapod
from . import pod as _pod
from . import tree as _tree

U64 = 2.0 ** -53


def orthonormality_error(U) -> float:
    U = np.asarray(U, dtype=np.float64)
    if U.shape[1] == 0:
        return 0.0
    return float(np.max(np.abs(U.T @ U - np.eye(U.shape[1]))))


def orth_basis(U) -> np.ndarray:
    """Orthonormal basis of span(U) by Householder QR (LAPACK geqrf)."""
    U = np.asarray(U, dtype=np.float64)
    if U.shape[1] == 0:
        return U.copy()
    Q, _ = np.linalg.qr(U, mode="reduced")
    return Q


def residual(S, U) -> np.ndarray:
    """S - P_span(U) S, projected twice."""
    S = np.asarray(S, dtype=np.float64)
    Q = orth_basis(U)
    if Q.shape[1] == 0:
        return S.copy()
    R = S - Q @ (Q.T @ S)
    R -= Q @ (Q.T @ R)
    return R


def projection_error(S, U) -> float:
    """sum_{s in S} ||s - P_span(U) s||^2."""
    R = residual(S, U)
    return float(np.sum(R * R))


def mean_projection_error(S, U) -> float:
    S = np.asarray(S)
    return projection_error(S, U) / max(S.shape[1], 1)


def subspace_error(U_ref, U_test, r) -> float:
    """||(I - U_ref,r U_ref,r^T) Q_test,r||_2 (sine of the largest principal
    angle between the two r-dimensional spans).  ``U_ref`` must have
    orthonormal columns."""
    if r == 0:
        return 0.0
    Ur = np.asarray(U_ref, dtype=np.float64)[:, :r]
    Q = orth_basis(np.asarray(U_test, dtype=np.float64)[:, :r])
    R = Q - Ur @ (Ur.T @ Q)
    R -= Ur @ (Ur.T @ R)
    return float(np.linalg.norm(R, 2))


def sigma_rel_error(sig_ref, sig_test, r) -> float:
    if r == 0:
        return 0.0
    a = np.asarray(sig_ref, dtype=np.float64)[:r]
    b = np.asarray(sig_test, dtype=np.float64)[:r]
    return float(np.max(np.abs(a - b) / a))


def resolved_rank(sig_ref, n_test, unit_roundoff, tau) -> int:
    """#{k <= min(N_ref, N_test) : sigma_k^2 >= (10 u / tau) sigma_1^2}: the
    leading modes a Gram matrix in the given precision can resolve to a
    subspace error of about tau."""
    s = np.asarray(sig_ref, dtype=np.float64)
    lim = min(len(s), int(n_test))
    if lim == 0:
        return 0
    thr = (10.0 * unit_roundoff / tau) * s[0] ** 2
    return int(np.sum(s[:lim] ** 2 >= thr))


def rounding_slack(S) -> float:
    """Absolute slack for evaluating projection errors of S in float64."""
    S = np.asarray(S, dtype=np.float64)
    if S.size == 0:
        return 0.0
    col = np.sqrt(np.sum(S * S, axis=0))
    return float(S.shape[1] * (64.0 * S.shape[0] * U64 * col.max()) ** 2)


def check_node_bounds(parent, leaf_data, eps, results):
    """Thm. 3.3 and Thm. 3.4 at every node.  Returns a list of dicts."""
    out = []
    for a in range(len(parent)):
        St = _hapod.subtree_snapshots(parent, a, leaf_data)
        sig, U = results[a]
        below = _tree.nodes_below(parent, a)
        rhs = sum(eps[g] ** 2 for g in below)
        lhs = projection_error(St, U)
        slack = rounding_slack(St)
        n_pod = _pod.pod_rank(St, eps[a])
        out.append(dict(node=a, err=lhs, bound=rhs, err_ok=lhs <= rhs * (1 + 1e-9) + slack,
                        modes=len(sig), pod_modes=n_pod, modes_ok=len(sig) <= n_pod))
    return out


def check_global_bounds(parent, leaf_cols, leaf_data, eps_star, omega, results):
    """Thm. 3.5: mean error <= eps*^2, |HAPOD| <= |MPOD(S, omega eps*)| and the
    local mode bound at every non-root node."""
    root = _tree.validate(parent)
    lev = _tree.levels(parent)
    LT = lev[root]
    S = _hapod.subtree_snapshots(parent, root, leaf_data)
    m = S.shape[1]
    sig, U = results[root]
    mean_err = projection_error(S, U) / m
    slack = rounding_slack(S) / m
    n_mpod = _pod.pod_rank(S, math.sqrt(m) * omega * eps_star)
    local = []
    if LT > 1:
        delta = (LT - 1) ** -0.5 * math.sqrt(1 - omega ** 2) * eps_star
        for a in range(len(parent)):
            if a == root:
                continue
            St = _hapod.subtree_snapshots(parent, a, leaf_data)
            bound = _pod.pod_rank(St, math.sqrt(St.shape[1]) * delta)
            local.append(dict(node=a, modes=len(results[a][0]), bound=bound,
                              ok=len(results[a][0]) <= bound))
    return dict(mean_err=mean_err, mean_ok=mean_err <= eps_star ** 2 * (1 + 1e-9) + slack,
                modes=len(sig), mpod_modes=n_mpod, modes_ok=len(sig) <= n_mpod,
                local=local)
