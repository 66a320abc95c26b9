"""Pins of the oracle's POD(S, eps) (Def. 2.1, Def. 2.5, Thm. 2.4).

None of these re-evaluate the oracle's own formula: they compare it with
closed forms (prescribed singular values and exactly orthonormal sine bases),
exact dyadic arithmetic, a different LAPACK routine (symmetric eigensolver),
and brute-force optimality on tiny inputs.
"""
import math

import numpy as np
import pytest

from oracle import metrics, pod


def dst_basis(n, r):
    """Exactly orthonormal columns: sqrt(2/(n+1)) sin(i k pi/(n+1))."""
    i = np.arange(1, n + 1)[:, None]
    k = np.arange(1, r + 1)[None, :]
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * i * k / (n + 1))


def signed_perm(n, seed):
    rng = np.random.default_rng(seed)
    P = np.eye(n)[rng.permutation(n)]
    return P * rng.choice([-1.0, 1.0], size=n)[None, :]


# ---- truncation rule, exact dyadic arithmetic -------------------------------
@pytest.mark.parametrize("eps,expect", [
    (0.5, 2),        # tail after 2 = 0.25 = eps^2 exactly: inclusive bound keeps 2
    (0.4999, 3),     # just below the tie: one more mode
    (1.5, 1),        # tail after 1 = 1.25 <= 2.25, tail after 0 = 5.25 > 2.25
    (3.0, 0),        # everything fits: N = 0
    (1e-300, 3),     # all nonzero values kept
])
def test_truncation_rank_dyadic(eps, expect):
    sigma = np.array([2.0, 1.0, 0.5])  # squares 4, 1, 0.25 are exact
    assert pod.truncation_rank(sigma, eps) == expect


def test_truncation_zero_singular_values_dropped():
    sigma = np.array([4.0, 1.0, 0.0, 0.0])
    assert pod.truncation_rank(sigma, 1e-300) == 2
    assert list(pod.tail_sums(sigma)) == [17.0, 1.0, 0.0, 0.0, 0.0]


# ---- pass-through ------------------------------------------------------------
def test_eps_zero_is_passthrough():
    S = np.arange(12.0).reshape(4, 3)
    sig, U = pod.pod(S, 0.0)
    assert np.array_equal(sig, np.ones(3))
    assert np.array_equal(U, S)


def test_empty_input():
    sig, U = pod.pod(np.zeros((5, 0)), 0.3)
    assert sig.shape == (0,) and U.shape == (5, 0)


# ---- closed form: prescribed singular values on orthonormal sine bases -------
@pytest.mark.parametrize("n,m", [(64, 12), (200, 40), (30, 30)])
def test_pod_matches_prescribed_svd(n, m):
    r = min(n, m)
    sigma = 3.0 * 0.5 ** np.arange(r)            # well separated
    Q1 = dst_basis(n, r)
    Q2 = dst_basis(m, m)[:, :r]
    S = Q1 @ np.diag(sigma) @ Q2.T
    # eps between tail(5) and tail(4): closed form N = 5
    t4 = np.sum(sigma[4:] ** 2)
    t5 = np.sum(sigma[5:] ** 2)
    eps = math.sqrt(0.5 * (t4 + t5))
    s, U = pod.pod(S, eps)
    assert len(s) == 5
    np.testing.assert_allclose(s, sigma[:5], rtol=1e-13)
    assert metrics.subspace_error(Q1, U, 5) < 1e-12
    assert metrics.orthonormality_error(U) < 1e-13


def test_pod_signed_permutation_exact_values():
    # S = P1 diag(sigma) P2^T with signed permutations: every singular value is
    # a dyadic number, modes are +-unit vectors.
    sigma = np.array([8.0, 4.0, 2.0, 1.0, 0.5])
    P1 = signed_perm(9, 1)[:, :5]
    P2 = signed_perm(5, 2)
    S = P1 @ np.diag(sigma) @ P2.T
    s, U = pod.pod(S, 1.2)       # eps^2 = 1.44: tail(3) = 1.25 fits, tail(2) = 5.25 does not
    assert len(s) == 3
    np.testing.assert_allclose(s, sigma[:3], rtol=1e-15)
    assert metrics.subspace_error(P1, U, 3) < 1e-15


# ---- Thm. 2.4 and an independent LAPACK routine --------------------------------
def test_singular_values_match_symmetric_eigensolver():
    rng = np.random.default_rng(7)
    S = rng.standard_normal((50, 8)) @ np.diag(2.0 ** -np.arange(8))
    s, _ = pod.pod_full(S)
    lam = np.linalg.eigvalsh(S.T @ S)[::-1]
    np.testing.assert_allclose(s ** 2, lam, rtol=1e-10)


def test_seym_error_identity_and_brute_force_optimality():
    rng = np.random.default_rng(3)
    S = rng.standard_normal((6, 5)) @ np.diag([3.0, 2.0, 1.0, 0.3, 0.1])
    s_all, U_all = pod.pod_full(S)
    for N in range(0, 6):
        err = metrics.projection_error(S, U_all[:, :N])
        np.testing.assert_allclose(err, np.sum(s_all[N:] ** 2), rtol=1e-10, atol=1e-14)
        # no random N-dimensional subspace does better (Thm. 2.4, min over X)
        for _ in range(200):
            X = rng.standard_normal((6, N))
            assert metrics.projection_error(S, X) >= err * (1 - 1e-12) - 1e-14


def test_truncated_pod_meets_eps():
    rng = np.random.default_rng(11)
    S = rng.standard_normal((80, 30)) @ np.diag(np.exp(-np.arange(30) / 3.0))
    for eps in [1e-3, 1e-2, 0.1, 1.0]:
        s, U = pod.pod(S, eps)
        err = metrics.projection_error(S, U)
        assert err <= eps ** 2 * (1 + 1e-10)
        if len(s) > 0:      # minimality: one mode fewer violates the bound
            assert metrics.projection_error(S, U[:, :-1]) > eps ** 2
