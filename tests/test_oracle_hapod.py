"""Pins of the oracle's HAPOD recursion (Def. 3.2) and of the paper's bounds.

Special cases that reduce to a plain POD, exact low-rank data, equivariance,
and the inequalities of Thm. 3.3, 3.4 and 3.5 on several tree shapes.
"""
import math

import numpy as np
import pytest

import synth
from oracle import coeff, hapod, metrics, pod, tolerances, tree


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


def test_single_node_equals_pod():
    S = low_rank_data(60, 20, 15, 1) + 1e-3 * np.random.default_rng(2).standard_normal((60, 20))
    res = hapod.hapod([-1], {0: S}, [0.05])
    s, U = pod.pod(S, 0.05)
    np.testing.assert_array_equal(res[0][0], s)
    np.testing.assert_array_equal(res[0][1], U)


def test_passthrough_leaves_give_pod_of_all():
    # eps(leaves) = 0: the root input is the snapshot matrix itself
    S = low_rank_data(50, 24, 12, 3) + 1e-4 * np.random.default_rng(4).standard_normal((50, 24))
    parent = synth.star_tree(3)
    blocks = split(S, [8, 8, 8])
    res = hapod.hapod(parent, dict(enumerate(blocks)), [0.0, 0.0, 0.0, 0.02])
    s, U = pod.pod(S, 0.02)
    np.testing.assert_allclose(res[3][0], s, rtol=1e-12)
    assert metrics.subspace_error(U, res[3][1], len(s)) < 1e-10


@pytest.mark.parametrize("shape", ["star", "chain", "balanced"])
def test_exact_low_rank_span_recovered(shape):
    r = 6
    S = low_rank_data(40, 48, r, 5)
    if shape == "star":
        parent = synth.star_tree(4)
        data = dict(enumerate(split(S, [12] * 4)))
    elif shape == "chain":
        parent, chunk = synth.chain_tree(4)
        blocks = split(S, [12] * 4)
        data = {leaf: blocks[c] for leaf, c in chunk.items()}
    else:
        parent = synth.balanced_tree(8, 3)
        data = dict(enumerate(split(S, [6] * 8)))
    eps = [1e-9] * len(parent)
    res = hapod.hapod(parent, data, eps)
    root = tree.validate(parent)
    s, U = res[root]
    s_ref, U_ref = pod.pod(S, 1e-9)
    assert len(s) == r == len(s_ref)
    np.testing.assert_allclose(s, s_ref, rtol=1e-9)
    assert metrics.subspace_error(U_ref, U, r) < 1e-9


def test_sigma_invariant_under_column_order():
    S = low_rank_data(30, 16, 10, 8) + 1e-3 * np.random.default_rng(9).standard_normal((30, 16))
    parent = synth.star_tree(2)
    eps = [0.01, 0.01, 0.02]
    a = hapod.hapod(parent, {0: S[:, :8], 1: S[:, 8:]}, eps)
    perm = np.random.default_rng(1).permutation(8)
    b = hapod.hapod(parent, {0: S[:, 8:][:, perm], 1: S[:, :8]}, eps)
    np.testing.assert_allclose(a[2][0], b[2][0], rtol=1e-10)


def _workloads():
    rng = np.random.default_rng(21)
    n = 70
    S = (np.linalg.qr(rng.standard_normal((n, n)))[0][:, :60]
         @ np.diag(np.exp(-np.arange(60) / 6.0)) @ rng.standard_normal((60, 64)))
    star = (synth.star_tree(4), dict(enumerate(split(S, [16] * 4))), [16] * 4 + [0], ())
    p, chunk = synth.chain_tree(4)
    blocks = split(S, [16] * 4)
    chain = (p, {leaf: blocks[c] for leaf, c in chunk.items()},
             [16 if i in chunk else 0 for i in range(len(p))],
             tuple(b for b in chunk if b != 0))
    pb = synth.balanced_tree(8, 3)
    bal = (pb, dict(enumerate(split(S, [8] * 8))), [8] * 8 + [0] * (len(pb) - 8), ())
    return [star, chain, bal]


@pytest.mark.parametrize("omega", [0.0, 0.5, 0.75, 0.95, 1.0])
@pytest.mark.parametrize("eps_star", [1e-3, 1e-2, 1e-1])
@pytest.mark.parametrize("which", [0, 1, 2])
def test_theorems_3_3_3_4_3_5(which, eps_star, omega):
    parent, data, cols, zero = _workloads()[which]
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega, zero_nodes=zero)
    res = hapod.hapod(parent, data, eps)
    for rec in metrics.check_node_bounds(parent, data, eps, res):
        assert rec["err_ok"], rec            # Thm. 3.3
        assert rec["modes_ok"], rec          # Thm. 3.4
    g = metrics.check_global_bounds(parent, cols, data, eps_star, omega, res)
    assert g["mean_ok"], g                   # Thm. 3.5, mean error
    if omega > 0:
        assert g["modes_ok"], g              # Thm. 3.5, mode count vs MPOD
    for rec in g["local"]:
        if eps[rec["node"]] > 0:
            assert rec["ok"], rec            # Thm. 3.5, local mode bound


def test_coefficient_space_equals_explicit():
    n, m, K, tau = 300, 48, 40, 6.0
    C = synth.sinusoid_coeffs(m, K, seed=5)
    S = synth.sinusoid(n, m, K, tau, 0.0, seed=5)
    B = coeff.coefficient_matrix(C, n, tau)
    parent = synth.star_tree(3)
    cols = [16] * 3 + [0]
    eps = tolerances.hapod_tolerances(parent, cols, 1e-4, 0.75)
    ex = hapod.hapod(parent, dict(enumerate(split(S, [16] * 3))), eps)
    co = coeff.hapod_coeff(parent, dict(enumerate(split(B, [16] * 3))), eps)
    s_ex, U_ex = ex[3]
    s_co, U_co = co[3]
    assert len(s_ex) == len(s_co)
    np.testing.assert_allclose(s_ex, s_co, rtol=1e-9)
    rows = np.arange(n)
    U_lift = coeff.sine_basis_rows(rows, n, K) @ U_co
    r = int(np.sum(s_ex > 1e-6 * s_ex[0]))
    assert metrics.subspace_error(U_ex, U_lift, r) < 1e-8


def test_sine_basis_is_orthonormal():
    n, K = 257, 60
    Phi = coeff.sine_basis_rows(np.arange(n), n, K)
    assert metrics.orthonormality_error(Phi) < 1e-13
    # and it reproduces the generator: S = Phi B exactly (noise free)
    C = synth.sinusoid_coeffs(5, K, seed=1)
    S = synth.sinusoid(n, 5, K, 7.0, 0.0, seed=1)
    np.testing.assert_allclose(Phi @ coeff.coefficient_matrix(C, n, 7.0), S, atol=1e-12)
