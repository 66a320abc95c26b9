"""The literal node-by-node HAPOD recursion (Def. 3.2).

HAPOD(alpha) = POD(S_alpha, eps(alpha)) where S_alpha is the snapshot set of
a leaf, or, at an inner node, the union over the children beta of the scaled
modes sigma_n * phi_n of HAPOD(beta).  Nodes are visited children first.

Column order of S_alpha (the paper treats it as a multiset, so any order is
admissible): children in ascending node id, each child's modes in descending
singular value.
"""
from __future__ import annotations

import numpy as np

from . import pod as _pod
from . import tree as _tree


def node_input(parent, results, alpha, leaf_data):
    """S_alpha as an n x m float64 matrix."""
    ch = _tree.children(parent)
    if not ch[alpha]:
        return np.asarray(leaf_data[alpha], dtype=np.float64)
    blocks = []
    for b in ch[alpha]:
        sig, U = results[b]
        blocks.append(U * sig[None, :])
    return np.hstack(blocks)


def hapod(parent, leaf_data, eps):
    """Run the recursion; returns ``{node: (sigma, U)}`` for every node.

    ``leaf_data[leaf]`` is the n x m_leaf matrix D^{-1}(leaf); ``eps[node]``
    the local tolerance.
    """
    _tree.validate(parent)
    results = {}
    for a in _tree.postorder(parent):
        S_a = node_input(parent, results, a, leaf_data)
        results[a] = _pod.pod(S_a, eps[a])
    return results


def subtree_snapshots(parent, alpha, leaf_data):
    """S~_alpha: all original snapshots below alpha, leaves in ascending id."""
    below = _tree.nodes_below(parent, alpha)
    ch = _tree.children(parent)
    return np.hstack([np.asarray(leaf_data[g], dtype=np.float64)
                      for g in below if not ch[g]])
