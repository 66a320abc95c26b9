"""Low-rank factorisation of the accumulated snapshot map (Rem. 3.8).

Test infrastructure: only the tests, the bench's CPU baseline and the smoke
check use this module; the GPU library shares no code with it.

The literal HAPOD recursion (Def. 3.2) keeping, at every node, the right
singular vectors of its snapshot map as Lambda_alpha (Def. 3.9): the first
N_alpha right singular vectors for eps(alpha) > 0, the identity for
eps(alpha) = 0.  The accumulated map of right vectors is
Lambda~_alpha = Lambda_alpha at a leaf and
Lambda~_alpha = diag(Lambda~_beta over the children) Lambda_alpha above, the
children's blocks in the order their modes enter S_alpha (ascending node id,
as in hapod.node_input).  With W the matrix of Lambda~_rho,
S~ ~ U diag(sigma) W^T, W^T W = I (Lem. 3.10), and the squared Frobenius
error is at most the sum of eps(gamma)^2 over all nodes (eq. of Rem. 3.8).
"""
from __future__ import annotations

import numpy as np

from . import hapod as _hapod
from . import pod as _pod
from . import tree as _tree


def hapod_factor(parent, leaf_data, eps):
    """Return ``{node: (sigma, U, W, rows)}``.  ``W`` is |S~_alpha| x N_alpha;
    ``rows[i] = (leaf, j)``: row i of W belongs to column j of leaf_data[leaf]
    (the enumeration of S~_alpha that matches Lambda~_alpha)."""
    _tree.validate(parent)
    ch = _tree.children(parent)
    res = {}
    plain = {}
    for a in _tree.postorder(parent):
        S_a = _hapod.node_input(parent, plain, a, leaf_data)
        m = S_a.shape[1]
        if eps[a] == 0.0:
            sigma, U = np.ones(m), S_a.copy()
            Lam = np.eye(m)
        elif m == 0:
            sigma, U, Lam = np.zeros(0), np.zeros((S_a.shape[0], 0)), np.zeros((0, 0))
        else:
            Uf, s, Vt = np.linalg.svd(S_a, full_matrices=False)
            N = _pod.truncation_rank(s, eps[a])
            sigma, U, Lam = s[:N].copy(), Uf[:, :N].copy(), Vt[:N].T.copy()
        plain[a] = (sigma, U)
        if not ch[a]:
            W = Lam
            rows = [(a, j) for j in range(m)]
        else:
            blocks, rows, c0 = [], [], 0
            for b in ch[a]:
                Wb, rb = res[b][2], res[b][3]
                Nb = Wb.shape[1]
                blocks.append(Wb @ Lam[c0:c0 + Nb, :])
                rows.extend(rb)
                c0 += Nb
            W = np.vstack(blocks) if blocks else np.zeros((0, Lam.shape[1]))
        res[a] = (sigma, U, W, rows)
    return res


def ordered_snapshots(leaf_data, rows):
    """The accumulated snapshot matrix in the enumeration ``rows``."""
    return np.stack([np.asarray(leaf_data[l], dtype=np.float64)[:, j] for l, j in rows], axis=1)


def rows_in_leaf_order(W, rows):
    """W with its rows sorted by (leaf, column)."""
    order = sorted(range(len(rows)), key=lambda i: rows[i])
    return W[order]
