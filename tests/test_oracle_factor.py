"""Pins of the oracle's factorisation of the snapshot map (Rem. 3.8, Lem. 3.10).

The accumulated right vectors are orthonormal, reproduce the snapshots when
nothing is truncated, satisfy the Frobenius bound of Rem. 3.8 on several tree
shapes, and reduce to the truncated SVD at a single node.
"""
import numpy as np
import pytest

import synth
from oracle import factor, hapod, pod, tolerances, tree


def low_rank_data(n, m, r, seed, decay=0.7):
    rng = np.random.default_rng(seed)
    A = np.linalg.qr(rng.standard_normal((n, r)))[0]
    return A @ np.diag(decay ** np.arange(r)) @ rng.standard_normal((r, m))


def split(S, cols):
    out, c0 = [], 0
    for c in cols:
        out.append(S[:, c0:c0 + c])
        c0 += c
    return out


def shaped(shape, S, per):
    m = S.shape[1]
    k = m // per
    if shape == "star":
        parent = synth.star_tree(k)
        data = dict(enumerate(split(S, [per] * k)))
        zero = ()
    elif shape == "chain":
        parent, chunk = synth.chain_tree(k)
        blocks = split(S, [per] * k)
        data = {leaf: blocks[c] for leaf, c in chunk.items()}
        zero = tuple(b for b in chunk if b != 0)
    else:
        parent = synth.balanced_tree(k, 3)
        data = dict(enumerate(split(S, [per] * k)))
        zero = ()
    return parent, data, zero


def test_single_node_is_truncated_svd():
    S = low_rank_data(50, 18, 14, 1) + 1e-3 * np.random.default_rng(2).standard_normal((50, 18))
    eps = 0.05
    res = factor.hapod_factor([-1], {0: S}, [eps])
    sig, U, W, rows = res[0]
    assert rows == [(0, j) for j in range(18)]
    # U diag(sigma) W^T is the rank-N truncated SVD: U U^T S
    np.testing.assert_allclose(U @ np.diag(sig) @ W.T, U @ (U.T @ S), atol=1e-12)
    s_ref, _ = pod.pod(S, eps)
    np.testing.assert_allclose(sig, s_ref, rtol=1e-12)


@pytest.mark.parametrize("shape", ["star", "chain", "balanced"])
def test_lossless_tree_reproduces_snapshots(shape):
    S = np.random.default_rng(7).standard_normal((60, 24))
    parent, data, zero = shaped(shape, S, 4)
    eps = [0.0 if a in zero else 1e-300 for a in range(len(parent))]
    res = factor.hapod_factor(parent, data, eps)
    root = tree.validate(parent)
    sig, U, W, rows = res[root]
    St = factor.ordered_snapshots(data, rows)
    np.testing.assert_allclose(U @ np.diag(sig) @ W.T, St, atol=1e-10 * np.abs(S).max())
    np.testing.assert_allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-12)
    assert sorted(rows) == [(l, j) for l in sorted(data) for j in range(data[l].shape[1])]


@pytest.mark.parametrize("shape", ["star", "chain", "balanced"])
def test_frobenius_bound_of_remark_3_8(shape):
    S = low_rank_data(80, 48, 20, 3, decay=0.6) + 1e-4 * np.random.default_rng(4).standard_normal((80, 48))
    parent, data, zero = shaped(shape, S, 6)
    cols = [data[a].shape[1] if a in data else 0 for a in range(len(parent))]
    eps = tolerances.hapod_tolerances(parent, cols, 2e-3, 0.7, zero_nodes=zero)
    res = factor.hapod_factor(parent, data, eps)
    root = tree.validate(parent)
    sig, U, W, rows = res[root]
    St = factor.ordered_snapshots(data, rows)
    err2 = np.linalg.norm(St - U @ np.diag(sig) @ W.T) ** 2
    bound = sum(e * e for e in eps)
    assert err2 <= bound * (1 + 1e-10)
    # truncation really happened, so the bound is not trivially met
    assert len(sig) < St.shape[1]
    assert err2 > 0.0
    # Lem. 3.10: the accumulated right vectors are orthonormal
    np.testing.assert_allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-11)
    # the left factor is the plain recursion's
    plain = hapod.hapod(parent, data, eps)
    np.testing.assert_array_equal(plain[root][0], sig)


def test_rows_in_leaf_order_sorts_by_leaf_then_column():
    W = np.arange(8.0).reshape(4, 2)
    rows = [(3, 0), (1, 1), (1, 0), (3, 1)]
    out = factor.rows_in_leaf_order(W, rows)
    np.testing.assert_array_equal(out, W[[2, 1, 0, 3]])
