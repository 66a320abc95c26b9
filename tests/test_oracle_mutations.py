"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, through monkeypatch)
and checks that at least one pin test from ``test_oracle_*`` then fails.
"""
import numpy as np
import pytest

from oracle import hapod, pod, tolerances, tree
import test_oracle_hapod as th
import test_oracle_pod as tp
import test_oracle_tree as tt


def _strict_rank(sigma, eps):
    t = pod.tail_sums(sigma)
    for N in range(len(t)):
        if t[N] < float(eps) ** 2:          # '<' instead of '<='
            return N
    return len(t) - 1


def _off_by_one_tail(sigma):
    t = np.zeros(len(sigma) + 1)
    s2 = np.asarray(sigma, float) ** 2
    for i in range(len(s2)):
        t[i] = s2[i + 1:].sum() if i + 1 < len(s2) else 0.0   # drops sigma_{N'+1}
    return t


def _unscaled_input(parent, results, alpha, leaf_data):
    ch = tree.children(parent)
    if not ch[alpha]:
        return np.asarray(leaf_data[alpha], float)
    return np.hstack([results[b][1] for b in ch[alpha]])      # U instead of U Sigma


def _right_vectors_pod(S, eps):
    # SVD of the transposed snapshot matrix: returns right singular vectors
    S = np.asarray(S, float)
    if eps == 0.0:
        return np.ones(S.shape[1]), S.copy()
    U, s, Vt = np.linalg.svd(S.T, full_matrices=False)
    N = pod.truncation_rank(s, eps)
    return s[:N], U[:, :N]


def _no_depth_factor(parent, leaf_cols, eps_star, omega, zero_nodes=()):
    root = tree.validate(parent)
    acc = tree.acc_counts(parent, leaf_cols)
    eps = [np.sqrt(acc[a]) * (omega if a == root else np.sqrt(1 - omega ** 2)) * eps_star
           for a in range(len(parent))]
    for z in zero_nodes:
        eps[z] = 0.0
    return eps


def _fails(fn, *args):
    try:
        fn(*args)
    except Exception:       # a failed assertion or a shape error both count
        return True
    return False


def test_strict_inequality_is_caught(monkeypatch):
    monkeypatch.setattr(pod, "truncation_rank", _strict_rank)
    assert _fails(tp.test_truncation_rank_dyadic, 0.5, 2)


def test_off_by_one_tail_is_caught(monkeypatch):
    monkeypatch.setattr(pod, "tail_sums", _off_by_one_tail)
    assert _fails(tp.test_truncation_rank_dyadic, 1.5, 1) or \
        _fails(tp.test_truncation_zero_singular_values_dropped)


def test_missing_sigma_scaling_is_caught(monkeypatch):
    monkeypatch.setattr(hapod, "node_input", _unscaled_input)
    assert _fails(th.test_exact_low_rank_span_recovered, "star")


def test_transposed_operand_is_caught(monkeypatch):
    monkeypatch.setattr(pod, "pod", _right_vectors_pod)
    assert _fails(tp.test_pod_matches_prescribed_svd, 64, 12)


def test_missing_depth_factor_is_caught(monkeypatch):
    monkeypatch.setattr(tolerances, "hapod_tolerances", _no_depth_factor)
    assert _fails(tt.test_tolerances_level_sums)
