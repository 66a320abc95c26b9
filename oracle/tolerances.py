"""Local HAPOD tolerances (Thm. 3.5 and the incremental case of Sec. 3.2).

For a target l2-mean error eps* and a trade-off parameter 0 <= omega <= 1:

* root:      eps(rho)   = sqrt(|S|) * omega * eps*
* otherwise: eps(alpha) = sqrt(|S~_alpha|) * (L_T - 1)^(-1/2)
                          * sqrt(1 - omega^2) * eps*

where |S~_alpha| counts the original snapshots below alpha and L_T is the
depth (level of the root).  Nodes listed in ``zero_nodes`` get eps = 0, the
usual choice for the data nodes beta_l of an incremental (chain) tree, whose
POD is then the pass-through POD(S, 0).
"""
from __future__ import annotations

import math

from . import tree as _tree


def hapod_tolerances(parent, leaf_cols, eps_star, omega, zero_nodes=()):
    if eps_star < 0 or not (0.0 <= omega <= 1.0):
        raise ValueError("need eps_star >= 0 and 0 <= omega <= 1")
    root = _tree.validate(parent)
    lev = _tree.levels(parent)
    acc = _tree.acc_counts(parent, leaf_cols)
    LT = lev[root]
    total = acc[root]
    eps = [0.0] * len(parent)
    for a in range(len(parent)):
        if a == root:
            eps[a] = math.sqrt(total) * omega * eps_star
        else:
            # LT >= 2 whenever a non-root node exists
            eps[a] = (math.sqrt(acc[a]) / math.sqrt(LT - 1)
                      * math.sqrt(1.0 - omega * omega) * eps_star)
    for z in zero_nodes:
        eps[z] = 0.0
    return eps
