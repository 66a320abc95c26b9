"""Rooted trees as parent arrays (Def. 3.1).

A tree over nodes ``0..N-1`` is given by ``parent[i]`` (the unique node whose
children include ``i``) with ``parent[root] = -1``.  A parent array already
satisfies the "at most one parent" condition of Def. 3.1; the connectivity
condition (every non-root node reaches the root) is checked by walking up.
"""
from __future__ import annotations


class TreeError(ValueError):
    pass


def validate(parent) -> int:
    """Check Def. 3.1 for a parent array; return the root id."""
    n = len(parent)
    if n == 0:
        raise TreeError("empty tree")
    roots = [i for i, p in enumerate(parent) if p == -1]
    if len(roots) != 1:
        raise TreeError(f"expected exactly one root, found {len(roots)}")
    for i, p in enumerate(parent):
        if p != -1 and not (0 <= p < n):
            raise TreeError(f"parent[{i}] = {p} out of range")
        if p == i:
            raise TreeError(f"node {i} is its own parent")
    root = roots[0]
    # connectivity: each walk upwards must reach the root within n steps
    for i in range(n):
        j, steps = i, 0
        while j != root:
            j = parent[j]
            steps += 1
            if steps > n:
                raise TreeError(f"node {i} is on a cycle / not connected to the root")
    return root


def children(parent):
    """Children lists in ascending node id (the set C(alpha) of Def. 3.1)."""
    ch = [[] for _ in parent]
    for i, p in enumerate(parent):
        if p != -1:
            ch[p].append(i)
    return ch


def leaves(parent):
    """Leaf set: nodes with no children."""
    ch = children(parent)
    return [i for i in range(len(parent)) if not ch[i]]


def nodes_below(parent, alpha):
    """N_T(alpha) = {alpha} union the nodes below each child (recursive)."""
    ch = children(parent)
    out, stack = [], [alpha]
    while stack:
        a = stack.pop()
        out.append(a)
        stack.extend(ch[a])
    return sorted(out)


def levels(parent):
    """Level map L(alpha) = max({L(beta) : beta child} u {0}) + 1.

    Leaves have level 1 and the depth of the tree is the root's level.
    """
    validate(parent)
    ch = children(parent)
    lev = [0] * len(parent)
    # children before parents, iteratively (chains can be deep)
    for a in postorder(parent):
        lev[a] = max([lev[b] for b in ch[a]] + [0]) + 1
    return lev


def postorder(parent):
    """Nodes in an order where every child precedes its parent."""
    root = validate(parent)
    ch = children(parent)
    out, stack = [], [(root, False)]
    while stack:
        a, done = stack.pop()
        if done:
            out.append(a)
        else:
            stack.append((a, True))
            for b in reversed(ch[a]):
                stack.append((b, False))
    return out


def acc_counts(parent, leaf_cols):
    """|S~_alpha|: number of original snapshots assigned to leaves below alpha.

    ``leaf_cols[i]`` is |D^{-1}(i)| for leaves and ignored for inner nodes.
    """
    ch = children(parent)
    cnt = [0] * len(parent)
    for a in postorder(parent):
        cnt[a] = int(leaf_cols[a]) if not ch[a] else sum(cnt[b] for b in ch[a])
    return cnt
