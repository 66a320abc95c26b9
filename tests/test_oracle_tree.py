"""Pins of the oracle's tree handling (Def. 3.1) and tolerances (Thm. 3.5)."""
import math

import pytest

import synth
from oracle import tolerances, tree


# ---- Def. 3.1 validation ------------------------------------------------------
@pytest.mark.parametrize("parent", [
    [],                 # empty
    [1, 0],             # no root (cycle)
    [-1, -1],           # two roots
    [3, -1, 1, 0],      # 0->3->0 cycle, disconnected from root 1
    [5, -1],            # out of range
    [0, -1],            # self parent
])
def test_invalid_trees_rejected(parent):
    with pytest.raises(tree.TreeError):
        tree.validate(parent)


# ---- levels, by inspection of the paper's two special trees ------------------
def test_levels_star():
    parent = synth.star_tree(4)
    assert tree.levels(parent) == [1, 1, 1, 1, 2]
    assert tree.leaves(parent) == [0, 1, 2, 3]


def test_levels_chain_matches_incremental_figure():
    # alpha_1..alpha_3 = 0,1,2 ; beta_1, beta_2 = 3, 4 ; root alpha_3
    parent, chunk = synth.chain_tree(3)
    assert parent == [1, 2, -1, 1, 2]
    assert tree.levels(parent) == [1, 2, 3, 1, 1]
    assert chunk == {0: 0, 3: 1, 4: 2}


def test_levels_irregular():
    #        6
    #      /   \
    #     4     5
    #    / \    |
    #   0   1   2      3 -> 6 directly
    parent = [4, 4, 5, 6, 6, 6, -1]
    assert tree.levels(parent) == [1, 1, 1, 1, 2, 2, 3]
    assert tree.nodes_below(parent, 4) == [0, 1, 4]
    assert tree.nodes_below(parent, 6) == list(range(7))


def test_balanced_tree_shape():
    parent = synth.balanced_tree(1024, 3)
    lev = tree.levels(parent)
    assert lev.count(1) == 1024 and lev.count(2) == 32 and lev.count(3) == 1


def test_acc_counts_brute_force():
    parent = [4, 4, 5, 6, 6, 6, -1]
    cols = [3, 5, 7, 11, 0, 0, 0]
    acc = tree.acc_counts(parent, cols)
    leaves = set(tree.leaves(parent))
    for a in range(len(parent)):
        brute = sum(cols[g] for g in tree.nodes_below(parent, a) if g in leaves)
        assert acc[a] == brute


# ---- Thm. 3.5 tolerances: the level-sum argument of its proof ------------------
def _level_sum_check(parent, cols, eps_star, omega):
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    root = tree.validate(parent)
    total = tree.acc_counts(parent, cols)[root]
    lev = tree.levels(parent)
    LT = lev[root]
    # the root takes omega^2 of the budget ...
    assert eps[root] ** 2 == pytest.approx(total * omega ** 2 * eps_star ** 2, rel=1e-14)
    # ... each non-root level at most 1/(LT-1) of the rest, because the
    # subtrees of one level are disjoint
    for l in range(1, LT):
        s = sum(eps[a] ** 2 for a in range(len(parent)) if lev[a] == l)
        assert s <= total * (1 - omega ** 2) * eps_star ** 2 / (LT - 1) * (1 + 1e-12)
    assert sum(e * e for e in eps) <= total * eps_star ** 2 * (1 + 1e-12)


def test_tolerances_level_sums():
    _level_sum_check(synth.star_tree(4), [64] * 4 + [0], 1e-6, 0.75)
    _level_sum_check([4, 4, 5, 6, 6, 6, -1], [3, 5, 7, 11, 0, 0, 0], 0.1, 0.5)
    p, chunk = synth.chain_tree(6)
    _level_sum_check(p, [10] * len(p), 1e-3, 0.9)
    _level_sum_check(synth.balanced_tree(27, 4), [4] * 40, 2e-2, 0.3)


def test_star_leaves_use_the_whole_non_root_budget():
    # in a star every leaf is at level 1 and they partition S: equality
    eps = tolerances.hapod_tolerances(synth.star_tree(4), [64] * 4 + [0], 1e-6, 0.75)
    assert sum(e * e for e in eps[:4]) == pytest.approx(256 * (1 - 0.75 ** 2) * 1e-12, rel=1e-13)


def test_tolerances_weight_by_subtree_snapshots_not_inputs():
    # level-2 node 4 has 8 original snapshots below it; its input column count
    # is data dependent and must not enter
    parent = [4, 4, 5, 6, 6, 6, -1]
    cols = [3, 5, 7, 11, 0, 0, 0]
    eps = tolerances.hapod_tolerances(parent, cols, 1.0, 0.0)
    assert eps[4] ** 2 == pytest.approx(8 / 2.0, rel=1e-14)      # LT - 1 = 2
    assert eps[3] ** 2 == pytest.approx(11 / 2.0, rel=1e-14)


def test_zero_nodes_and_extremes():
    p, chunk = synth.chain_tree(4)
    betas = [b for b in chunk if b != 0]
    eps = tolerances.hapod_tolerances(p, [8] * len(p), 1e-2, 0.75, zero_nodes=betas)
    assert all(eps[b] == 0.0 for b in betas)
    eps0 = tolerances.hapod_tolerances(p, [8] * len(p), 1e-2, 0.0)
    root = tree.validate(p)
    assert eps0[root] == 0.0                                   # omega = 0
    eps1 = tolerances.hapod_tolerances(p, [8] * len(p), 1e-2, 1.0)
    assert all(eps1[a] == 0.0 for a in range(len(p)) if a != root)
    with pytest.raises(ValueError):
        tolerances.hapod_tolerances(p, [8] * len(p), -1.0, 0.5)
    with pytest.raises(ValueError):
        tolerances.hapod_tolerances(p, [8] * len(p), 1.0, 1.5)


def test_valid_deep_parent_chain():
    assert tree.validate([2, 0, -1, 1]) == 2     # 3 -> 1 -> 0 -> 2


def test_single_node_tree():
    eps = tolerances.hapod_tolerances([-1], [9], 0.5, 0.75)
    assert eps == [pytest.approx(3 * 0.75 * 0.5)]
    assert math.isfinite(eps[0])
