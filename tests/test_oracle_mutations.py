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


# ---- metrics: planted mistakes caught by test_oracle_metrics --------------------
import test_oracle_metrics as tm  # noqa: E402
from oracle import metrics  # noqa: E402


def _wrong_slice_subspace_error(U_ref, U_test, r):
    if r == 0:
        return 0.0
    Ur = np.asarray(U_ref, float)[:, 1:r + 1]                # off by one column
    Q = metrics.orth_basis(np.asarray(U_test, float)[:, :r])
    R = Q - Ur @ (Ur.T @ Q)
    return float(np.linalg.norm(R, 2))


def _cos_form_subspace_error(U_ref, U_test, r):
    # sqrt(1 - sigma_min(U^T Q)^2): the form with a sqrt(u) floor
    if r == 0:
        return 0.0
    Ur = np.asarray(U_ref, float)[:, :r]
    Q = metrics.orth_basis(np.asarray(U_test, float)[:, :r])
    c = np.linalg.svd(Ur.T @ Q, compute_uv=False).min()
    return float(np.sqrt(max(0.0, 1.0 - c * c)))


def _self_residual(S, U):
    S = np.asarray(S, float)
    Q = metrics.orth_basis(S)                                 # projects on span(S): cancels to 0
    return S - Q @ (Q.T @ S)


def _sigma_not_squared(sig_ref, n_test, unit_roundoff, tau):
    s = np.asarray(sig_ref, float)
    lim = min(len(s), int(n_test))
    if lim == 0:
        return 0
    thr = (10.0 * unit_roundoff / tau) * s[0] ** 2
    return int(np.sum(s[:lim] >= thr))                        # sigma in place of sigma^2


def _node_bounds_always_ok(parent, leaf_data, eps, results):
    out = metrics._orig_check_node_bounds(parent, leaf_data, eps, results)
    for c in out:
        c["err_ok"] = True
    return out


def _global_mean_always_ok(parent, leaf_cols, leaf_data, eps_star, omega, results):
    g = metrics._orig_check_global_bounds(parent, leaf_cols, leaf_data, eps_star, omega, results)
    g["mean_ok"] = True
    return g


def test_wrong_reference_slice_is_caught(monkeypatch):
    monkeypatch.setattr(metrics, "subspace_error", _wrong_slice_subspace_error)
    assert _fails(tm.test_subspace_error_prescribed_angle, 0.1)


def test_cosine_form_floor_is_caught(monkeypatch):
    monkeypatch.setattr(metrics, "subspace_error", _cos_form_subspace_error)
    assert _fails(tm.test_subspace_error_prescribed_angle, 1e-13)


def test_cancelling_residual_is_caught(monkeypatch):
    monkeypatch.setattr(metrics, "residual", _self_residual)
    assert _fails(tm.test_projection_error_known_residual)


def test_sigma_for_sigma_squared_is_caught(monkeypatch):
    monkeypatch.setattr(metrics, "resolved_rank", _sigma_not_squared)
    assert _fails(tm.test_resolved_rank_dyadic_closed_form)


def test_error_check_always_true_is_caught(monkeypatch):
    monkeypatch.setattr(metrics, "_orig_check_node_bounds", metrics.check_node_bounds, raising=False)
    monkeypatch.setattr(metrics, "check_node_bounds", _node_bounds_always_ok)
    assert _fails(tm.test_node_bounds_reject_one_mode_too_few)


def test_mean_check_always_true_is_caught(monkeypatch):
    monkeypatch.setattr(metrics, "_orig_check_global_bounds", metrics.check_global_bounds, raising=False)
    monkeypatch.setattr(metrics, "check_global_bounds", _global_mean_always_ok)
    assert _fails(tm.test_global_bound_rejects_tolerances_without_depth_factor)
