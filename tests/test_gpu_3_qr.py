"""GPU parity of the QR-based local POD (hapod_node_pod_qr) against the SVD
oracle (Def. 2.5 by LAPACK's SVD of S itself).

The method of snapshots resolves singular values only to about
sqrt(u) sigma_1 (its Gram matrix squares the condition number, Rem. 2.3);
the QR route keeps them to about u sigma_1.  Checked here on graded,
rank-deficient and noisy low-rank inputs with prescribed singular values:
equal ranks, |sigma_k - sigma_k(oracle)| <= 1e-13 sigma_1, each mode within
the perturbation bound c u sigma_1 / gap_k of the oracle's, orthonormal
modes; and the Gram route's error on the same inputs shown to be orders of
magnitude larger.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from gpu_util import dev_colmajor, host  # noqa: E402
from oracle import metrics, pod  # noqa: E402

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_05210_amd as m
    return m


def prescribed(n, sig, seed, noise=0.0):
    """S = Q_1 diag(sig) Q_2^T with Haar-like orthonormal factors."""
    rng = np.random.default_rng(seed)
    m = len(sig)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((m, m)))
    S = (Q1 * sig) @ Q2.T
    if noise:
        S = S + noise * rng.standard_normal((n, m))
    return S


def check_against_oracle(S, s_qr, U_qr, eps, tag):
    s_ref, U_ref = pod.pod(S, eps)
    s_all = np.linalg.svd(S, compute_uv=False)
    assert len(s_qr) == len(s_ref), (tag, len(s_qr), len(s_ref))
    s1 = s_all[0]
    err = np.max(np.abs(s_qr - s_ref)) if len(s_ref) else 0.0
    assert err <= 1e-13 * s1, (tag, err / s1)
    assert metrics.orthonormality_error(U_qr) <= 1e-13
    # mode k against the oracle's: sin(angle) <= c u sigma_1 / gap_k (Wedin),
    # gap_k the distance of sigma_k to every other singular value of S
    N = len(s_ref)
    for k in range(N):
        others = np.delete(s_all, k)
        gap = np.min(np.abs(others - s_all[k])) if len(others) else s1
        # sine of the angle as the norm of the rejection (1 - cos^2 would
        # lose half the digits)
        c = float(U_qr[:, k] @ U_ref[:, k])
        sin_k = float(np.linalg.norm(U_qr[:, k] - c * U_ref[:, k]))
        bound = 200.0 * math.sqrt(S.shape[1]) * U64 * s1 / gap
        assert sin_k <= max(bound, 1e-12), (tag, k, sin_k, bound)
    return err / s1


@pytest.mark.parametrize("m", [60, 200])
def test_graded_spectrum_to_1e14(hp, m):
    """sigma_k = 10^(-14 k / (m - 1)): condition 1e14, far beyond what a
    Gram matrix holds in FP64."""
    n = 4096
    sig = 10.0 ** (-14.0 * np.arange(m) / (m - 1))
    S = prescribed(n, sig, seed=m)
    eps = math.sqrt(np.sum(sig[sig < 1e-11] ** 2)) * 1.0001
    print(f"graded m={m}", flush=True)
    s_qr, U_qr, info = hp.hapod_node_pod_qr(dev_colmajor(S), eps)
    rel = check_against_oracle(S, s_qr, host(U_qr), eps, "graded")
    s_g, _ = hp.hapod_node_pod("fp64", dev_colmajor(S), eps)
    r = min(len(s_g), len(s_qr))
    gram_err = np.max(np.abs(s_g[:r] - s_qr[:r])) / sig[0]
    print(f"  rank {len(s_qr)}, passes {info['passes']}, sweeps {info['sweeps']}, "
          f"QR sigma err {rel:.1e}, Gram route {gram_err:.1e} (rank {len(s_g)})")
    assert info["passes"] >= 3
    assert gram_err > 1e3 * max(rel, 1e-16)


@pytest.mark.parametrize("m,rank", [(64, 30), (200, 90)])
def test_rank_deficient(hp, m, rank):
    """Exactly rank-deficient S: the shifted passes lift the null directions
    until Q is orthonormal; the rank and the kept sigma are the oracle's."""
    n = 3000
    sig = np.r_[10.0 ** (-6.0 * np.arange(rank) / (rank - 1)), np.zeros(m - rank)]
    S = prescribed(n, sig, seed=rank)
    eps = 1e-9
    print(f"rank-deficient m={m} rank={rank}", flush=True)
    s_qr, U_qr, info = hp.hapod_node_pod_qr(dev_colmajor(S), eps)
    rel = check_against_oracle(S, s_qr, host(U_qr), eps, "rankdef")
    print(f"  rank {len(s_qr)}, passes {info['passes']}, sweeps {info['sweeps']}, sigma err {rel:.1e}")
    assert len(s_qr) == rank


def test_noisy_low_rank_scaled_modes(hp):
    """Low rank plus 1e-10 noise; scaled modes sigma_k phi_k (Def. 3.2)."""
    n, m = 5000, 96
    sig = np.r_[10.0 ** (-4.0 * np.arange(40) / 39), np.zeros(m - 40)]
    S = prescribed(n, sig, seed=5, noise=1e-10)
    eps = 1e-6  # above the noise's ~6e-8 tail, below the smallest signal sigma (1e-4)
    s_qr, W, info = hp.hapod_node_pod_qr(dev_colmajor(S), eps, scaled=True)
    W = host(W)
    U = W / s_qr
    check_against_oracle(S, s_qr, U, eps, "noisy")
    np.testing.assert_allclose(np.linalg.norm(W, axis=0), s_qr, rtol=1e-13)


def test_agrees_with_method_of_snapshots_when_well_conditioned(hp):
    """On a sinusoid snapshot set whose kept spectrum lies well above
    sqrt(u) sigma_1 both routes give the same POD."""
    n, m = 4096, 128
    S = synth.sinusoid(n, m, 40, 6.0, 0.0, seed=3)
    eps = 1e-4 * np.linalg.norm(S)
    s_qr, U_qr, _ = hp.hapod_node_pod_qr(dev_colmajor(S), eps)
    s_g, U_g = hp.hapod_node_pod("fp64", dev_colmajor(S), eps)
    assert len(s_qr) == len(s_g)
    np.testing.assert_allclose(s_qr, s_g, rtol=1e-10, atol=1e-12 * s_qr[0])
    r = metrics.resolved_rank(s_qr, len(s_qr), U64, 1e-8)
    assert metrics.subspace_error(host(U_qr), host(U_g), r) <= 1e-8
    check_against_oracle(S, s_qr, host(U_qr), eps, "sinusoid")


@pytest.mark.parametrize("n,m", [(50, 1), (300, 7), (1000, 129), (2048, 512), (160, 150)])
def test_shapes(hp, n, m):
    """One column, odd widths (the padding index of the round-robin Jacobi
    order), the first width past the LDS-resident Jacobi, the largest width,
    and a nearly square S."""
    rng = np.random.default_rng(n + m)
    S = rng.standard_normal((n, m)) * (0.5 ** np.arange(m) if m > 1 else 1.0) ** 0.05
    eps = 1e-6 * np.linalg.norm(S)
    print(f"shape n={n} m={m}", flush=True)
    s_qr, U_qr, info = hp.hapod_node_pod_qr(dev_colmajor(S), eps)
    check_against_oracle(S, s_qr, host(U_qr), eps, f"shape {n}x{m}")
    print(f"  rank {len(s_qr)}, passes {info['passes']}, sweeps {info['sweeps']}")


def test_zero_tiny_and_duplicate_columns(hp):
    """An exactly zero column, a column whose Gram diagonal underflows, a
    column 1e-98 of its neighbours and an exact duplicate: the first pass
    works on the equilibrated Gram, zero columns factor as unit columns
    (singular value 0); the result is the oracle's."""
    rng = np.random.default_rng(0)
    n, m = 1500, 40
    S = rng.standard_normal((n, m)) * (0.7 ** np.arange(m))
    S[:, 5] = 0.0
    S[:, 9] *= 1e-98
    S[:, 17] *= 1e-170
    S[:, 20] = S[:, 3]
    eps = 1e-12 * np.linalg.norm(S)
    s_qr, U_qr, info = hp.hapod_node_pod_qr(dev_colmajor(S), eps)
    print(f"  zero/tiny/duplicate: rank {len(s_qr)}, passes {info['passes']}, sweeps {info['sweeps']}")
    check_against_oracle(S, s_qr, host(U_qr), eps, "zero/tiny")


def test_passthrough_and_limits(hp):
    S = np.random.default_rng(0).standard_normal((40, 6))
    s, U, info = hp.hapod_node_pod_qr(dev_colmajor(S), 0.0)
    np.testing.assert_array_equal(s, np.ones(6))
    np.testing.assert_array_equal(host(U), S)
    s, U, info = hp.hapod_node_pod_qr(dev_colmajor(np.zeros((40, 0))), 1e-3)
    assert len(s) == 0
    with pytest.raises(hp.HapodError):
        hp.hapod_node_pod_qr(dev_colmajor(np.zeros((600, 513))), 1e-3)
    with pytest.raises(hp.HapodError):  # no orthonormal Q with more columns than rows
        hp.hapod_node_pod_qr(dev_colmajor(np.ones((5, 6))), 1e-3)
    with pytest.raises(hp.HapodError):
        bad = S.copy()
        bad[3, 2] = np.nan
        hp.hapod_node_pod_qr(dev_colmajor(bad), 1e-3)


# ------------------------------------------------------------ tree level ----
def _tree_run(hp, parent, data, n, eps_star, omega, zero=(), **kw):
    from oracle import tolerances
    leaf_cols = [data[i].shape[1] if i in data else 0 for i in range(len(parent))]
    ov = None
    if zero:
        ov = [-1.0] * len(parent)
        for z in zero:
            ov[z] = 0.0
    plan = hp.Plan(parent, leaf_cols, n, eps_star, omega, prec="fp64", eps_override=ov, **kw)
    plan.run({k: dev_colmajor(v) for k, v in data.items()})
    sig, U = plan.modes()
    eps = tolerances.hapod_tolerances(parent, leaf_cols, eps_star, omega, zero_nodes=zero)
    return plan, sig, host(U), eps


def _split(S, cols):
    out, c0 = [], 0
    for c in cols:
        out.append(S[:, c0:c0 + c])
        c0 += c
    return out


@pytest.mark.parametrize("shape", ["balanced", "star", "chain"])
def test_tree_qr_route_matches_oracle_below_the_gram_floor(hp, shape):
    """A graded spectrum down to 1e-13 and eps* = 1e-9: every node's
    truncation falls where the method of snapshots cannot resolve.  With
    qr_pod every node's rank is the oracle's (literal Def. 3.2 recursion with
    LAPACK SVDs), the root's sigma agree to 64 L_T sqrt(m) u sigma_1, and the mean
    squared projection error meets Thm. 3.5's eps*^2."""
    from oracle import hapod, tree
    n = 3000
    if shape == "balanced":
        leaves, per = 27, 12
        parent = synth.balanced_tree(leaves, 4)
        cols, zero = [per] * leaves, ()
    elif shape == "star":
        leaves, per = 4, 64
        parent = synth.star_tree(leaves)
        cols, zero = [per] * leaves, ()
    else:
        leaves, per = 6, 40
        parent, chunk = synth.chain_tree(leaves)
        cols, zero = [per] * leaves, tuple(b for b in chunk if b != 0)
    m = sum(cols)
    sig = 10.0 ** (-13.0 * np.arange(m) / (m - 1))
    S = prescribed(n, sig, seed=m + len(parent))
    blocks = _split(S, cols)
    if shape == "chain":
        data = {leaf: blocks[c] for leaf, c in chunk.items()}
    else:
        data = dict(enumerate(blocks))
    eps_star, omega = 1e-9, 0.75
    print(f"tree qr {shape}", flush=True)
    plan, s_gpu, U, eps = _tree_run(hp, parent, data, n, eps_star, omega, zero=zero, qr_pod=True)
    data64 = {k: np.asarray(v) for k, v in data.items()}
    ref = hapod.hapod(parent, data64, eps)
    root = tree.validate(parent)
    ranks = plan.ranks()
    want = [len(ref[a][0]) for a in range(len(parent))]
    assert list(ranks) == want
    s_ref = ref[root][0]
    # each level's SVD of R (one-sided Jacobi, backward stable) and its
    # products move sigma by about sqrt(m) u sigma_1 times a small constant
    # (64 here), and the levels' errors add up
    lev = tree.levels(parent)
    m_max = max(int(plan.node_stats()["m_in"][a]) for a in range(len(parent)))
    bound = 64.0 * lev[root] * math.sqrt(m_max) * U64 * s_ref[0]
    assert np.max(np.abs(s_gpu - s_ref)) <= bound, (np.max(np.abs(s_gpu - s_ref)) / s_ref[0], bound / s_ref[0])
    assert metrics.orthonormality_error(U) <= 1e-13
    S_all = np.hstack([data64[k] for k in sorted(data64)])
    err_qr = metrics.mean_projection_error(S_all, U)
    plan_g, s_g, U_g, _ = _tree_run(hp, parent, data, n, eps_star, omega, zero=zero)
    err_g = metrics.mean_projection_error(S_all, U_g)
    print(f"  root rank {len(s_gpu)} (Gram route {len(s_g)}), mean error / eps*^2: QR {err_qr / eps_star**2:.3f}, "
          f"Gram {err_g / eps_star**2:.3f}, ranks off in the Gram route: "
          f"{sum(int(a != b) for a, b in zip(plan_g.ranks(), want))}")
    assert err_qr <= eps_star ** 2


def test_tree_qr_route_wide_root_takes_the_gram_route(hp):
    """Leaves of 128 columns take the QR route; the 640-column root is
    beyond it and takes the method of snapshots; the leaves' ranks are the
    oracle's and the root's modes span the oracle's leading ones."""
    from oracle import hapod, tree
    n, leaves, per = 2048, 5, 128
    S = synth.sinusoid(n, leaves * per, 400, 40.0, 1e-10, seed=4)
    parent = synth.star_tree(leaves)
    data = dict(enumerate(_split(S, [per] * leaves)))
    plan, s_gpu, U, eps = _tree_run(hp, parent, data, n, 1e-7, 0.75, qr_pod=True)
    ref = hapod.hapod(parent, data, eps)
    ranks = plan.ranks()
    assert list(ranks[:leaves]) == [len(ref[a][0]) for a in range(leaves)]
    assert plan.node_stats()["m_in"][leaves] > 512
    root = tree.validate(parent)
    r = metrics.resolved_rank(ref[root][0], len(s_gpu), U64, 1e-6)
    assert metrics.subspace_error(ref[root][1], U, r) <= 1e-6


def test_tree_qr_route_plan_rules(hp):
    for kw in ({"prec": "fp32"}, {"prec": "bf16x3"}, {"prec": "fp64", "right_vectors": True}):
        with pytest.raises(hp.HapodError):
            hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5, qr_pod=True, **kw)


def test_tree_qr_route_uneven_leaf_heights(hp):
    """Leaves of different heights (implicit zero rows below each) under a
    3-level tree, every node on the QR route: the gathered inputs read only
    the rows each column holds, inner nodes hold the most of their
    children's, and the root's modes are zero-filled below its own height.
    Every node's rank is the oracle's (zero-padded leaves), the root's sigma
    within 1e-12 sigma_1, and the modes orthonormal."""
    from oracle import hapod, tolerances, tree
    n = 6000
    specs = synth.uneven_leaf_specs(16, seed=5, rows_range=(700, 4000), cols_range=(8, 40))
    parent = synth.balanced_tree(16, 3)
    cols = [sp["cols"] for sp in specs] + [0] * (len(parent) - 16)
    rows = [sp["rows"] for sp in specs] + [0] * (len(parent) - 16)
    data = {i: synth.uneven_leaf(sp, n) for i, sp in enumerate(specs)}
    eps_star, omega = 1e-6, 0.75
    plan = hp.Plan(parent, cols, n, eps_star, omega, prec="fp64", leaf_rows=rows, qr_pod=True)
    plan.run({i: dev_colmajor(d) for i, d in data.items()})
    sig, U = plan.modes()
    U = host(U)
    full = {i: np.vstack([d, np.zeros((n - d.shape[0], d.shape[1]))]) for i, d in data.items()}
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    ref = hapod.hapod(parent, full, eps)
    root = tree.validate(parent)
    assert plan.node_stats()["m_in"].max() <= 512  # every node within the QR route
    assert list(plan.ranks()) == [len(ref[a][0]) for a in range(len(parent))]
    s_ref = ref[root][0]
    assert np.max(np.abs(sig - s_ref)) <= 1e-12 * s_ref[0]
    assert metrics.orthonormality_error(U) <= 1e-13
    assert np.all(U[max(rows):] == 0.0)
