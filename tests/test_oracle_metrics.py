"""Pins of the oracle's accuracy metrics and theorem checks.

Every expected value here is non-zero and fixed by the mathematics, not by
re-evaluating the metric's own formula:

* ``subspace_error``: two spans with one prescribed principal angle theta
  have ||(I - U U^T) Q||_2 = sin(theta) (the largest principal angle's sine),
  including angles far below sqrt(u), where the cos-based form has a floor.
* ``resolved_rank``: a dyadic spectrum sigma_k = 2^-k with a threshold that is
  an exact power of two has a closed-form count.
* ``projection_error``: a residual that is known exactly (unit vectors).
* ``check_node_bounds`` / ``check_global_bounds`` (Thm. 3.3, 3.4, 3.5): they
  accept the oracle's own HAPOD and reject a result with one mode too few
  (error above the bound), one mode too many (above the mode bound), and a
  HAPOD run with tolerances that lack the depth factor (L_T - 1)^(-1/2) of
  Thm. 3.5 on a deep tree.
"""
import math

import numpy as np
import pytest

import synth
from oracle import hapod, metrics, pod, tolerances, tree


def unit(n, i):
    e = np.zeros(n)
    e[i] = 1.0
    return e


# ---- subspace error: prescribed principal angles ------------------------------
@pytest.mark.parametrize("theta", [0.7, 0.1, 1e-3, 1e-9, 1e-13, math.pi / 2])
def test_subspace_error_prescribed_angle(theta):
    n = 6
    U_ref = np.column_stack([unit(n, 0), unit(n, 1), unit(n, 4)])
    tilted = math.cos(theta) * unit(n, 1) + math.sin(theta) * unit(n, 2)
    # the test modes are neither normalised nor orthogonal: only their span counts
    U_test = np.column_stack([2.0 * unit(n, 0), 3.0 * tilted + 0.5 * unit(n, 0), unit(n, 5)])
    got = metrics.subspace_error(U_ref, U_test, 2)
    assert abs(got - math.sin(theta)) <= 4e-16 + 1e-12 * math.sin(theta)
    # r = 1 compares span{e1} with span{e1}: no angle
    assert metrics.subspace_error(U_ref, U_test, 1) <= 1e-16
    # r = 3 adds e5 against e6: a right angle
    assert abs(metrics.subspace_error(U_ref, U_test, 3) - 1.0) <= 1e-15


def test_subspace_error_two_angles_takes_the_largest():
    n = 8
    a, b = 0.3, 0.05
    U_ref = np.column_stack([unit(n, 0), unit(n, 1)])
    U_test = np.column_stack([math.cos(a) * unit(n, 0) + math.sin(a) * unit(n, 2),
                              math.cos(b) * unit(n, 1) + math.sin(b) * unit(n, 3)])
    assert abs(metrics.subspace_error(U_ref, U_test, 2) - math.sin(a)) <= 1e-15


# ---- resolved rank: dyadic spectrum --------------------------------------------
def test_resolved_rank_dyadic_closed_form():
    u = 2.0 ** -53
    sig = 2.0 ** -np.arange(30.0)            # sigma_k^2 = 4^-k, exact
    # threshold (10 u / tau) sigma_1^2 = 2^-20: sigma_k^2 >= 2^-20 <=> k <= 10
    tau = 10.0 * u * 2.0 ** 20
    assert metrics.resolved_rank(sig, 30, u, tau) == 11
    # the count is capped by the test's rank
    assert metrics.resolved_rank(sig, 7, u, tau) == 7
    # sigma scaled by 3: the threshold is relative to sigma_1^2
    assert metrics.resolved_rank(3.0 * sig, 30, u, tau) == 11
    # the boundary is inclusive: 2^-20 itself counts
    assert metrics.resolved_rank(sig[:11], 30, u, tau) == 11
    assert metrics.resolved_rank(np.zeros(0), 5, u, tau) == 0


# ---- projection error: exactly known residuals -----------------------------------
def test_projection_error_known_residual():
    n = 5
    S = np.column_stack([3.0 * unit(n, 0) + 4.0 * unit(n, 1), 2.0 * unit(n, 2), unit(n, 0)])
    U = unit(n, 0)[:, None]
    # residuals: 4 e2 (16), 2 e3 (4), 0
    assert metrics.projection_error(S, U) == 20.0
    assert metrics.mean_projection_error(S, U) == 20.0 / 3
    assert metrics.projection_error(S, np.zeros((n, 0))) == 9 + 16 + 4 + 1


# ---- Thm. 3.3 / 3.4 per node, Thm. 3.5 globally -----------------------------------
def graded(n, m, seed, rate=0.35):
    """Columns with a smoothly decaying spectrum, so that a minimal truncation
    ends close to its tolerance."""
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.standard_normal((n, m)))[0]
    return Q @ np.diag(np.exp(-rate * np.arange(m))) @ rng.standard_normal((m, m))


def star_case():
    parent = synth.star_tree(3)
    cols = [10, 10, 10, 0]
    S = graded(40, 30, 1)
    data = {i: S[:, 10 * i:10 * (i + 1)] for i in range(3)}
    return parent, cols, data, 1e-1, 0.6


def test_node_bounds_accept_the_oracle():
    parent, cols, data, eps_star, omega = star_case()
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    res = hapod.hapod(parent, data, eps)
    checks = metrics.check_node_bounds(parent, data, eps, res)
    assert all(c["err_ok"] and c["modes_ok"] for c in checks)
    # the leaves truncate: their errors are non-zero and within the bound
    assert all(0.0 < checks[i]["err"] <= checks[i]["bound"] for i in range(3))


def test_node_bounds_reject_one_mode_too_few():
    parent, cols, data, eps_star, omega = star_case()
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    res = hapod.hapod(parent, data, eps)
    sig, U = res[1]
    assert len(sig) > 0
    bad = dict(res)
    bad[1] = (sig[:-1], U[:, :-1])            # the minimal rank minus one (Def. 2.5)
    checks = metrics.check_node_bounds(parent, data, eps, bad)
    assert not checks[1]["err_ok"]
    assert checks[0]["err_ok"] and checks[2]["err_ok"]


def test_node_bounds_reject_one_mode_too_many():
    parent, cols, data, eps_star, omega = star_case()
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    res = hapod.hapod(parent, data, eps)
    s_all, U_all = pod.pod_full(data[2])
    N = len(res[2][0])
    assert N < 10
    bad = dict(res)
    bad[2] = (s_all[:N + 1], U_all[:, :N + 1])
    checks = metrics.check_node_bounds(parent, data, eps, bad)
    assert checks[2]["err_ok"] and not checks[2]["modes_ok"]


def test_global_bounds_accept_the_oracle_and_reject_mistakes():
    parent, cols, data, eps_star, omega = star_case()
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    res = hapod.hapod(parent, data, eps)
    g = metrics.check_global_bounds(parent, cols, data, eps_star, omega, res)
    assert g["mean_ok"] and g["modes_ok"] and all(x["ok"] for x in g["local"])
    assert 0.0 < g["mean_err"] <= eps_star ** 2
    root = 3
    sig, U = res[root]
    # root modes cut until the mean error exceeds eps*^2
    bad = dict(res)
    k = len(sig)
    while k > 0 and metrics.mean_projection_error(np.hstack([data[i] for i in range(3)]), U[:, :k]) <= eps_star ** 2:
        k -= 1
    bad[root] = (sig[:k], U[:, :k])
    assert not metrics.check_global_bounds(parent, cols, data, eps_star, omega, bad)["mean_ok"]
    # more root modes than |MPOD(S, omega eps*)|
    S = np.hstack([data[i] for i in range(3)])
    s_all, U_all = pod.pod_full(S)
    over = dict(res)
    over[root] = (s_all[:g["mpod_modes"] + 1], U_all[:, :g["mpod_modes"] + 1])
    assert not metrics.check_global_bounds(parent, cols, data, eps_star, omega, over)["modes_ok"]
    # a leaf with more modes than its local bound allows
    s1, U1 = pod.pod_full(data[1])
    loc = dict(res)
    b1 = [x for x in g["local"] if x["node"] == 1][0]["bound"]
    assert b1 < 10
    loc[1] = (s1[:b1 + 1], U1[:, :b1 + 1])
    assert not [x for x in metrics.check_global_bounds(parent, cols, data, eps_star, omega, loc)["local"]
                if x["node"] == 1][0]["ok"]


def test_global_bound_rejects_tolerances_without_depth_factor():
    """A deep chain truncated with sqrt(|S~|) sqrt(1 - omega^2) eps* at every
    node (no (L_T - 1)^(-1/2)) accumulates about L_T - 1 local budgets and
    breaks the mean-error bound of Thm. 3.5; with the factor it holds."""
    chunks, per = 8, 6
    S = graded(60, chunks * per, 5, rate=0.12)
    parent, chunk = synth.chain_tree(chunks)
    data = {leaf: S[:, per * c:per * (c + 1)] for leaf, c in chunk.items()}
    cols = [per if a in chunk else 0 for a in range(len(parent))]
    zero = tuple(b for b in chunk if b != 0)
    eps_star, omega = 2e-2, 0.5
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega, zero_nodes=zero)
    res = hapod.hapod(parent, data, eps)
    assert metrics.check_global_bounds(parent, cols, data, eps_star, omega, res)["mean_ok"]
    root = tree.validate(parent)
    acc = tree.acc_counts(parent, cols)
    loose = [0.0 if a in zero else
             math.sqrt(acc[a]) * (omega if a == root else math.sqrt(1 - omega ** 2)) * eps_star
             for a in range(len(parent))]
    res_loose = hapod.hapod(parent, data, loose)
    g = metrics.check_global_bounds(parent, cols, data, eps_star, omega, res_loose)
    assert not g["mean_ok"], g["mean_err"] / eps_star ** 2
