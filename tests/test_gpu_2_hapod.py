"""GPU HAPOD runs (Def. 3.2 with the Thm. 3.5 tolerances) against the oracle.

Comparison contract for results whose tail lies below what a Gram matrix can
resolve: subspace error of the leading r_res modes, where r_res counts the
oracle's modes with sigma_k^2 >= (10 u_p / tau) sigma_1^2 (u_p the unit
roundoff of the Gram's precision; tau = 1e-6 for FP64, 1e-4 for the FP32 and
split-BF16 forms), singular-value error on the same modes, and the paper's
bounds where the precision can certify them.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from gpu_util import dev_colmajor, host  # noqa: E402
from oracle import hapod, metrics, pod, tolerances, tree  # noqa: E402


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_05210_amd as m
    return m


ELEM = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.float32}


UP = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -24}
TAU = {"fp64": 1e-6, "fp32": 1e-4, "bf16x3": 1e-4}


def sigma_within_bound(s_ref, s_gpu, r, u_p, n, eps, root):
    """|sigma_k - sigma_ref,k| for k < r within
      2 sqrt(sum_{gamma != root} eps(gamma)^2)   (both results are singular
          values of approximations of the snapshot map within that Frobenius
          distance, Thm. 3.3, so by Weyl each is that close to the exact ones)
    + 4 sqrt(n) u_p sigma_1^2 / sigma_k          (a Gram perturbation of
          ~sqrt(n) u_p lambda_1 moves sigma_k by that much)."""
    a = np.asarray(s_ref[:r])
    b = np.asarray(s_gpu[:r])
    delta = math.sqrt(sum(e * e for i, e in enumerate(eps) if i != root))
    tol = 2.0 * delta + 4.0 * math.sqrt(n) * u_p * a[0] ** 2 / a
    bad = np.nonzero(np.abs(a - b) > tol)[0]
    if len(bad):
        print("sigma outside bound at", bad[:8], (np.abs(a - b) / tol)[bad[:8]])
    return len(bad) == 0


def split_cols(S, cols):
    out, c0 = [], 0
    for c in cols:
        out.append(S[:, c0:c0 + c])
        c0 += c
    return out


def run_both(hp, parent, leaf_data, n, eps_star, omega, prec, zero=(), reorth=True, **kw):
    leaf_cols = [leaf_data[i].shape[1] if i in leaf_data else 0 for i in range(len(parent))]
    ov = None
    if zero:
        ov = [-1.0] * len(parent)
        for z in zero:
            ov[z] = 0.0
    plan = hp.Plan(parent, leaf_cols, n, eps_star, omega, prec=prec, reorth=reorth, eps_override=ov, **kw)
    dev = {k: dev_colmajor(v, ELEM[prec]) for k, v in leaf_data.items()}
    plan.run(dev)
    sig, U = plan.modes()
    eps = tolerances.hapod_tolerances(parent, leaf_cols, eps_star, omega, zero_nodes=zero)
    data64 = {k: (v.astype(np.float32).astype(np.float64) if prec != "fp64" else v) for k, v in leaf_data.items()}
    ref = hapod.hapod(parent, data64, eps)
    return plan, sig, host(U), ref, eps, leaf_cols, data64


@pytest.mark.parametrize("prec,autotune", [("fp64", False), ("fp32", False), ("bf16x3", False),
                                           ("fp64", True), ("fp32", True)])
def test_star_4096x256(hp, prec, autotune):
    """The 4096 x 256 star workload: 4 leaves x 64 sinusoid snapshots (also
    with the Gram tiles chosen by timing)."""
    print(f"star4096x256 {prec} autotune {autotune}", flush=True)
    w = synth.WORKLOADS["star4096x256"]
    S = synth.sinusoid(w.n, w.num_snapshots, w.K, w.tau, w.noise_std, w.seed)
    parent = synth.star_tree(4)
    data = dict(enumerate(split_cols(S, w.leaf_cols)))
    plan, sig, U, ref, eps, cols, data64 = run_both(hp, parent, data, w.n, w.eps_star, w.omega, prec,
                                                     autotune=autotune)
    root = 4
    s_ref, U_ref = ref[root]
    ranks = plan.ranks()
    if prec == "fp64":
        assert list(ranks[:4]) == [len(ref[i][0]) for i in range(4)]
        # The root's truncation falls below the FP64 Gram's rounding floor
        # (its last modes have sigma^2 near u lambda_1): the rank may differ
        # from the oracle's only where the oracle's own tail at the GPU's rank
        # lies within the m u lambda_1 that the computed tail sums are known to.
        No, Ng = len(s_ref), int(ranks[root])
        if No != Ng:
            s_full = pod.pod_full(hapod.node_input(parent, ref, root, data64))[0]
            tail = pod.tail_sums(s_full)
            band = len(s_full) * UP["fp64"] * s_full[0] ** 2
            gap = abs(tail[min(Ng, len(s_full))] - eps[root] ** 2)
            print(f"  root rank {Ng} (oracle {No}), |tail - eps^2| = {gap:.3e}, m u lambda_1 = {band:.3e}")
            assert gap <= band, (Ng, No, gap, band)
    r = metrics.resolved_rank(s_ref, len(sig), UP[prec], TAU[prec])
    assert r >= (100 if prec == "fp64" else 20)
    e_sub = metrics.subspace_error(U_ref, U, r)
    s_err = metrics.sigma_rel_error(s_ref, sig, r)
    print(f"  rank {len(sig)} (oracle {len(s_ref)}), r_res {r}, e_sub {e_sub:.2e}, sigma err {s_err:.2e}")
    assert e_sub <= TAU[prec]
    assert sigma_within_bound(s_ref, sig, r, UP[prec] if prec == "fp64" else 3 * 2.0 ** -17, w.n, eps, root)
    assert metrics.orthonormality_error(U) <= (1e-12 if prec == "fp64" else 1e-5)
    if prec == "fp64":
        # FP64 keeps the modes down to its rounding floor: the mean-error bound of
        # Thm. 3.5 holds at this tolerance
        S64 = np.hstack([data64[i] for i in range(4)])
        assert metrics.mean_projection_error(S64, U) <= w.eps_star ** 2


def test_chain_bumps_fp64(hp):
    """Incremental HAPOD (chain tree, eps(beta) = 0) on Gaussian bumps."""
    n, chunks, cols = 2048, 8, 32
    S = synth.bumps(n, chunks * cols, seed=4)
    parent, chunk = synth.chain_tree(chunks)
    blocks = split_cols(S, [cols] * chunks)
    data = {leaf: blocks[c] for leaf, c in chunk.items()}
    zero = tuple(b for b in chunk if b != 0)
    eps_star = 1e-3 * math.sqrt(np.mean(np.sum(S * S, axis=0)))
    plan, sig, U, ref, eps, leaf_cols, data64 = run_both(hp, parent, data, n, eps_star, 0.75, "fp64", zero=zero)
    root = tree.validate(parent)
    s_ref, U_ref = ref[root]
    r = metrics.resolved_rank(s_ref, len(sig), UP["fp64"], 1e-6)
    assert metrics.subspace_error(U_ref, U, r) <= 1e-6
    assert sigma_within_bound(s_ref, sig, r, UP["fp64"], n, eps, root)
    np.testing.assert_array_equal(plan.ranks()[list(zero)], [cols] * len(zero))
    # Thm. 3.5: l2-mean projection error of all snapshots
    assert metrics.mean_projection_error(S, U) <= eps_star ** 2


def test_chain_block_structured_gram(hp):
    """Chain of 128-column chunks with the block-structured Gram (FP64): the
    raw chunk goes first, the previous node's scaled modes fill the next
    tile, whose Gram block is set to diag(sigma^2) instead of computed.  Same
    oracle bounds as the literal Gram, and the same ranks."""
    from oracle import metrics
    n, chunks, cols = 4096, 6, 128
    S = synth.bumps(n, chunks * cols, seed=11)
    parent, chunk = synth.chain_tree(chunks)
    blocks = split_cols(S, [cols] * chunks)
    data = {leaf: blocks[c] for leaf, c in chunk.items()}
    zero = tuple(b for b in chunk if b != 0)
    eps_star = 1e-3 * math.sqrt(np.mean(np.sum(S * S, axis=0)))
    plan, sig, U, ref, eps, leaf_cols, data64 = run_both(hp, parent, data, n, eps_star, 0.75, "fp64", zero=zero,
                                                         block_gram=True)
    plan0, sig0, U0, *_ = run_both(hp, parent, data, n, eps_star, 0.75, "fp64", zero=zero)
    root = tree.validate(parent)
    s_ref, U_ref = ref[root]
    r = metrics.resolved_rank(s_ref, len(sig), UP["fp64"], TAU["fp64"])
    assert metrics.subspace_error(U_ref, U, r) <= TAU["fp64"]
    assert list(plan.ranks()) == list(plan0.ranks())
    assert metrics.subspace_error(U0, U, r) <= TAU["fp64"]
    assert sigma_within_bound(s_ref, sig, r, UP["fp64"], n, eps, root)
    assert metrics.mean_projection_error(S, U) <= eps_star ** 2


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_block_structured_gram_needs_fp64(hp, prec):
    with pytest.raises(hp.HapodError):
        hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5, prec=prec, block_gram=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_balanced_three_levels(hp, prec):
    n = 3000
    leaves, per = 27, 12
    S = synth.sinusoid(n, leaves * per, 60, 8.0, 1e-10, seed=9)
    parent = synth.balanced_tree(leaves, 4)
    data = dict(enumerate(split_cols(S, [per] * leaves)))
    plan, sig, U, ref, eps, cols, data64 = run_both(hp, parent, data, n, 1e-4, 0.5, prec)
    root = tree.validate(parent)
    s_ref, U_ref = ref[root]
    r = metrics.resolved_rank(s_ref, len(sig), UP[prec], TAU[prec])
    assert metrics.subspace_error(U_ref, U, r) <= TAU[prec]
    if prec == "fp64":
        # A rank may differ from the oracle's only where the decision is below
        # what an FP64 Gram resolves: each of a node's m computed eigenvalues
        # carries an absolute error of about u lambda_1 (backward error of the
        # eigensolver on a Gram formed in FP64), so its tail sums are known to
        # m u lambda_1, and the oracle's tail at the GPU's rank must lie that
        # close to eps^2.
        ranks = plan.ranks()
        for a in range(len(parent)):
            No, Ng = len(ref[a][0]), int(ranks[a])
            if No == Ng:
                continue
            s_full = pod.pod_full(hapod.node_input(parent, ref, a, data64))[0]
            tail = pod.tail_sums(s_full)
            m_a = len(s_full)
            band = m_a * UP["fp64"] * s_full[0] ** 2
            gap = abs(tail[min(Ng, m_a)] - eps[a] ** 2)
            print(f"  node {a}: rank {Ng} (oracle {No}), |tail - eps^2| = {gap:.3e}, m u lambda_1 = {band:.3e}")
            assert gap <= band, (a, Ng, No, gap, band)


@pytest.mark.parametrize("L", [5, 6])
def test_full_rank_leaves(hp, L):
    """Leaves whose POD keeps every snapshot (rank m: their scaled modes are
    S V for a square orthogonal V): the root's rank and sigma as the literal
    HAPOD's, modes within the Gram route's accuracy, and the same with the
    right vectors kept.  A rank-20 signal plus noise 1e-2 (full-rank leaves);
    omega = 0.999 leaves the leaves too little of the budget to drop a noise
    mode, while the root drops all of them: 240 inputs (every eigenpair from
    the Householder reduction) and 288 (Lanczos, which leaves part of the
    271 noise eigenvalues near 0.1 out: their energy, trace minus the
    returned eigenvalues, counts as discarded, so the rank is still 17)."""
    from oracle import hapod as ohapod
    n, c = 1024, 48
    rng = np.random.default_rng(12)
    sg = 10.0 * np.exp(-np.arange(20) / 4.0)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, 20)))
    Q2, _ = np.linalg.qr(rng.standard_normal((L * c, 20)))
    S = (Q1 * sg) @ Q2.T * math.sqrt(L * c) + 1e-2 * rng.standard_normal((n, L * c))
    data = {i: S[:, i * c:(i + 1) * c] for i in range(L)}
    parent = synth.star_tree(L)
    cols = [c] * L + [0]
    eps_star, omega = 0.4, 0.999
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    ref = ohapod.hapod(parent, data, eps)
    assert all(len(ref[i][0]) == c for i in range(L))  # every leaf keeps all its columns
    prec = "fp64"
    dev = {i: dev_colmajor(v) for i, v in data.items()}
    plan = hp.Plan(parent, cols, n, eps_star, omega, prec=prec)
    plan.run(dev)
    sig, U = plan.modes()
    ranks = plan.ranks()
    assert list(ranks[:L]) == [c] * L
    s_ref, U_ref = ref[L]
    with_v = hp.Plan(parent, cols, n, eps_star, omega, prec=prec, right_vectors=True)
    with_v.run(dev)
    sig2, U2 = with_v.modes()
    print(f"  full-rank leaves {prec}: root rank {len(sig)} (oracle {len(s_ref)}, with right vectors {len(sig2)})")
    assert len(sig) == len(s_ref)
    np.testing.assert_allclose(sig, s_ref, rtol=1e-10)
    r = metrics.resolved_rank(s_ref, len(sig), UP[prec], TAU[prec])
    assert metrics.subspace_error(U_ref, host(U), r) <= TAU[prec]
    assert len(sig2) == len(sig)
    np.testing.assert_allclose(sig2, sig, rtol=1e-12)
    assert metrics.subspace_error(host(U2), host(U), len(sig)) <= 1e-10
    # the leaves' own columns handed to the root (same span and Gram
    # spectrum as S V), read from the row-block layout
    blocks = {i: hp.to_blocks(v) for i, v in dev.items()}
    passed = hp.Plan(parent, cols, n, eps_star, omega, prec=prec, leaf_layout="blocks", leaf_passthrough=True)
    passed.run(blocks)
    sig3, U3 = passed.modes()
    assert [passed.route(i) for i in range(L)] == ["full_leaf"] * L
    assert list(passed.ranks()[:L]) == [c] * L
    assert len(sig3) == len(sig)
    np.testing.assert_allclose(sig3, s_ref, rtol=1e-10)
    np.testing.assert_allclose(sig3, sig, rtol=1e-11)
    assert metrics.subspace_error(host(U3), host(U), len(sig)) <= 1e-10


def test_leaf_blocks_layout_and_passthrough_mixed(hp):
    """Leaves in the row-block layout (n = 1000: a partial last block) give
    the column-major run's result; with leaf_passthrough the full-rank leaves
    hand their columns up while a leaf of rank 5 takes its lift, and the
    root keeps the same rank and sigma."""
    n, c, L = 1000, 40, 4
    rng = np.random.default_rng(7)
    data = {i: rng.standard_normal((n, c)) for i in range(L)}
    data[2] = rng.standard_normal((n, 5)) @ rng.standard_normal((5, c))  # rank 5
    parent = synth.star_tree(L)
    cols = [c] * L + [0]
    eps_star, omega = 1e-6, 0.7
    dev = {i: dev_colmajor(v) for i, v in data.items()}
    ref = hp.Plan(parent, cols, n, eps_star, omega, prec="fp64")
    ref.run(dev)
    sig, U = ref.modes()
    blocks = {i: hp.to_blocks(v) for i, v in dev.items()}
    B = blocks[1].cpu().numpy()
    np.testing.assert_array_equal(B[7, 3, 99], data[1][7 * 128 + 99, 3])   # element (r, j) at [r // 128, j, r % 128]
    assert B.shape == (8, c, 128) and not B[7, :, n - 7 * 128:].any()       # rows past n zero
    for passthrough in (False, True):
        plan = hp.Plan(parent, cols, n, eps_star, omega, prec="fp64", leaf_layout="blocks",
                       leaf_passthrough=passthrough)
        plan.run(blocks)
        sig2, U2 = plan.modes()
        routes = [plan.route(i) for i in range(L)]
        print(f"  blocks layout, passthrough {passthrough}: leaf ranks {list(plan.ranks()[:L])}, routes {routes}, "
              f"root rank {len(sig2)} (column-major {len(sig)})")
        assert list(plan.ranks()[:L]) == list(ref.ranks()[:L])
        assert routes == (["full_leaf", "full_leaf", "snapshots", "full_leaf"] if passthrough else ["snapshots"] * L)
        assert len(sig2) == len(sig)
        np.testing.assert_allclose(sig2, sig, rtol=1e-11)
        assert metrics.subspace_error(host(U2), host(U), len(sig)) <= 1e-10


def test_single_node_tree_equals_node_pod(hp):
    S = synth.sinusoid(500, 40, 30, 5.0, 0.0, seed=2)
    plan = hp.Plan([-1], [40], 500, 1e-3, 0.9, prec="fp64")
    plan.run({0: dev_colmajor(S)})
    sig, U = plan.modes()
    eps = math.sqrt(40) * 0.9 * 1e-3
    s2, U2 = hp.hapod_node_pod("fp64", dev_colmajor(S), eps)
    np.testing.assert_array_equal(sig, s2)
    np.testing.assert_array_equal(host(U), host(U2))


def test_omega_zero_root_passthrough(hp):
    S = synth.sinusoid(300, 24, 20, 5.0, 0.0, seed=1)
    parent = synth.star_tree(2)
    data = {0: S[:, :12], 1: S[:, 12:]}
    plan = hp.Plan(parent, [12, 12, 0], 300, 1e-2, 0.0, prec="fp64")
    plan.run({k: dev_colmajor(v) for k, v in data.items()})
    sig, U = plan.modes()
    eps = tolerances.hapod_tolerances(parent, [12, 12, 0], 1e-2, 0.0)
    ref = hapod.hapod(parent, data, eps)
    np.testing.assert_array_equal(sig, np.ones(len(ref[2][0])))
    W = np.hstack([ref[b][1] * ref[b][0] for b in (0, 1)])
    r = metrics.resolved_rank(ref[0][0], 12, 2.0 ** -53, 1e-6)
    assert metrics.subspace_error(metrics.orth_basis(W), host(U), min(r, host(U).shape[1])) < 1e-6


def test_rerun_is_bitwise_identical(hp):
    w = synth.WORKLOADS["star4096x256"]
    S = synth.sinusoid(w.n, 256, w.K, w.tau, w.noise_std, 0)
    data = {i: dev_colmajor(S[:, 64 * i:64 * (i + 1)]) for i in range(4)}
    plan = hp.Plan(synth.star_tree(4), [64] * 4 + [0], w.n, w.eps_star, w.omega, prec="fp64")
    plan.run(data)
    s1, U1 = plan.modes()
    plan.run(data)
    s2, U2 = plan.modes()
    np.testing.assert_array_equal(s1, s2)
    assert torch.equal(U1, U2)


def test_error_paths_leave_plan_usable(hp):
    S = synth.sinusoid(200, 20, 10, 4.0, 0.0, seed=3)
    data = {0: dev_colmajor(S[:, :10]), 1: dev_colmajor(S[:, 10:])}
    plan = hp.Plan(synth.star_tree(2), [10, 10, 0], 200, 1e-3, 0.5)
    with pytest.raises(hp.HapodError) as e:
        plan.run(lambda leaf: (_ for _ in ()).throw(KeyError(leaf)))
    assert e.value.status == 7
    bad = S[:, :10].copy()
    bad[5, 3] = np.inf
    with pytest.raises(hp.HapodError) as e:
        plan.run({0: dev_colmajor(bad), 1: data[1]})
    assert e.value.status == 5
    plan.run(data)
    assert len(plan.modes()[0]) > 0
    # a cap below the leaf level's own scratch fails at plan time; one above
    # it but below what the run needs (the leaves' modes alone take 2 x 200 x
    # rank doubles) fails in the run, and the plan stays usable
    with pytest.raises(hp.HapodError) as e:
        hp.Plan(synth.star_tree(2), [10, 10, 0], 200, 1e-3, 0.5, mem_cap_bytes=4096)
    assert e.value.status == 3
    capped = hp.Plan(synth.star_tree(2), [10, 10, 0], 200, 1e-3, 0.5, mem_cap_bytes=6000)
    with pytest.raises(hp.HapodError) as e:
        capped.run(data)
    assert e.value.status == 3
    plan.run(data)
    assert len(plan.modes()[0]) > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_star_wide_root_coefficient_oracle(hp, prec):
    """Sinusoid star whose root (16 x 64 = 1024 inputs) takes the Lanczos
    eigensolver; checked against the exact coefficient-space HAPOD."""
    from oracle import coeff
    n, leaves, per, K, tau = 16384, 16, 64, 400, 20.0
    C = synth.sinusoid_coeffs(leaves * per, K, seed=7)
    S = synth.sinusoid(n, leaves * per, K, tau, 0.0, seed=7)
    parent = synth.star_tree(leaves)
    cols = [per] * leaves + [0]
    eps_star, omega = 1e-5, 0.75
    plan = hp.Plan(parent, cols, n, eps_star, omega, prec=prec)
    plan.run({i: dev_colmajor(S[:, i * per:(i + 1) * per], ELEM[prec]) for i in range(leaves)})
    sig, U = plan.modes()
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    B = coeff.coefficient_matrix(C, n, tau)
    ref = coeff.hapod_coeff(parent, dict(enumerate(split_cols(B, cols[:leaves]))), eps)
    s_ref, UB = ref[leaves]
    r = metrics.resolved_rank(s_ref, len(sig), UP[prec], TAU[prec])
    U_ref = coeff.sine_basis_rows(np.arange(n), n, K) @ UB
    e_sub = metrics.subspace_error(U_ref, host(U), r)
    print(f"  wide root {prec}: rank {len(sig)} (oracle {len(s_ref)}), r_res {r}, e_sub {e_sub:.2e}")
    assert r >= (150 if prec == "fp64" else 40)
    assert e_sub <= TAU[prec]


@pytest.mark.parametrize("prec,wave", [("fp64", 0), ("fp64", 5), ("fp32", 7), ("bf16x3", 0)])
def test_uneven_leaves_balanced_tree(hp, prec, wave):
    """Leaves of different heights (implicit zero rows) and widths, mixed
    families, under a 3-level balanced tree; optional launch waves."""
    n = 6000
    specs = synth.uneven_leaf_specs(16, seed=3, rows_range=(700, n), cols_range=(8, 40))
    parent = synth.balanced_tree(16, 3)
    cols = [sp["cols"] for sp in specs] + [0] * (len(parent) - 16)
    rows = [sp["rows"] for sp in specs] + [0] * (len(parent) - 16)
    data = {i: synth.uneven_leaf(sp, n) for i, sp in enumerate(specs)}
    if prec != "fp64":
        data = {i: d.astype(np.float32).astype(np.float64) for i, d in data.items()}
    eps_star, omega = 1e-3, 0.75
    plan = hp.Plan(parent, cols, n, eps_star, omega, prec=prec, leaf_rows=rows, leaf_wave=wave)
    calls = []

    def provider(leaf):
        calls.append(leaf)
        return dev_colmajor(data[leaf], ELEM[prec])
    plan.run(provider)
    assert sorted(calls) == list(range(16))
    sig, U = plan.modes()
    full = {i: np.vstack([d, np.zeros((n - d.shape[0], d.shape[1]))]) for i, d in data.items()}
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    ref = hapod.hapod(parent, full, eps)
    root = tree.validate(parent)
    s_ref, U_ref = ref[root]
    r = metrics.resolved_rank(s_ref, len(sig), UP[prec], TAU[prec])
    e_sub = metrics.subspace_error(U_ref, host(U), r)
    print(f"  uneven {prec} wave {wave}: rank {len(sig)} (oracle {len(s_ref)}), r_res {r}, e_sub {e_sub:.2e}")
    assert r >= 10 and e_sub <= TAU[prec]
    if prec == "fp64":
        S = np.hstack([full[i] for i in range(16)])
        assert metrics.mean_projection_error(S, host(U)) <= eps_star ** 2


def test_chain_streamed_through_one_buffer(hp):
    """Incremental HAPOD whose provider copies each chunk into the same device
    buffer: leaves are fetched just before the group that reads them."""
    n, chunks, per = 4096, 12, 24
    S = synth.bumps(n, chunks * per, seed=8)
    parent, chunk = synth.chain_tree(chunks)
    zero = [b for b in chunk if b != 0]
    cols = [per if i in chunk else 0 for i in range(len(parent))]
    ov = [-1.0] * len(parent)
    for z in zero:
        ov[z] = 0.0
    eps_star = 1e-3 * math.sqrt(np.mean(np.sum(S * S, axis=0)))
    plan = hp.Plan(parent, cols, n, eps_star, 0.75, prec="fp64", eps_override=ov, mem_cap_bytes=256 << 20)
    buf = dev_colmajor(np.zeros((n, per)))
    order = []

    def provider(leaf):
        c = chunk[leaf]
        order.append(c)
        buf.copy_(dev_colmajor(S[:, c * per:(c + 1) * per]))
        return buf
    plan.run(provider)
    assert order == list(range(chunks))          # one chunk per level, in order
    sig, U = plan.modes()
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, 0.75, zero_nodes=zero)
    blocks = {leaf: S[:, c * per:(c + 1) * per] for leaf, c in chunk.items()}
    ref = hapod.hapod(parent, blocks, eps)
    root = tree.validate(parent)
    s_ref, U_ref = ref[root]
    r = metrics.resolved_rank(s_ref, len(sig), UP["fp64"], 1e-6)
    assert metrics.subspace_error(U_ref, host(U), r) <= 1e-6
    assert metrics.mean_projection_error(S, host(U)) <= eps_star ** 2


def test_release_call_waits_for_forwarded_leaf_data(hp):
    """The provider's release call (leaf = -1) may only come once no leaf
    handed over is read again.  Leaves 0 and 1 have eps = 0 and sit under a
    pass-through node (eps = 0), so their data is read by the root's group,
    two groups after leaves 2 and 3.  The provider overwrites every buffer it
    handed out with NaN when told to release: a read after that would turn
    into a NaN Gram diagonal (E_NUMERIC) or wrong modes."""
    n, per = 2048, 20
    parent = [4, 4, 5, 5, 6, 6, -1]
    S = synth.sinusoid(n, 4 * per, 60, 6.0, 1e-10, seed=21)
    data = {i: np.ascontiguousarray(S[:, i * per:(i + 1) * per]) for i in range(4)}
    cols = [per] * 4 + [0, 0, 0]
    eps = tolerances.hapod_tolerances(parent, cols, 1e-4, 0.75)
    ov = [-1.0] * 7
    for z in (0, 1, 4):
        ov[z] = 0.0
        eps[z] = 0.0
    plan = hp.Plan(parent, cols, n, 1e-4, 0.75, prec="fp64", eps_override=ov)
    handed, events = [], []

    class Provider:
        def __call__(self, leaf):
            t = dev_colmajor(data[leaf])
            handed.append(t)
            events.append(leaf)
            return t

        def release(self):
            events.append(-1)
            for t in handed:
                t.fill_(float("nan"))
            handed.clear()

    plan.run(Provider(), hold=False)
    # leaves 2, 3 (level 1) and their release; 0, 1 fetched by the
    # pass-through node's group and released only after the root's group
    assert events == [2, 3, -1, 0, 1, -1]
    ref = hapod.hapod(parent, data, eps)
    s_ref, U_ref = ref[6]
    sig, U = plan.modes()
    r = metrics.resolved_rank(s_ref, len(sig), UP["fp64"], 1e-6)
    assert metrics.subspace_error(U_ref, host(U), r) <= 1e-6


def test_split_twins_in_groups_match_single_arena(hp, monkeypatch):
    """Split-BF16 nodes of 256 or more columns read a pre-split twin of their
    input; when the twins of a level do not fit the arena together they are
    made and consumed group by group.  The result is bitwise the same."""
    n, per = 4096, 300
    S = synth.sinusoid(n, 3 * per, 120, 12.0, 1e-10, seed=33).astype(np.float32)
    leaves = {i: dev_colmajor(np.ascontiguousarray(S[:, i * per:(i + 1) * per]), torch.float32)
              for i in range(3)}
    parent = synth.star_tree(3)
    cols = [per] * 3 + [0]

    def run():
        plan = hp.Plan(parent, cols, n, 1e-3, 0.75, prec="bf16x3")
        plan.run(leaves)
        sig, U = plan.modes()
        return sig, host(U), plan.ranks()

    s1, U1, r1 = run()
    twin = n * per * 4
    monkeypatch.setenv("HAPOD_TWIN_BUDGET", str(twin + twin // 2))   # one twin per group
    s2, U2, r2 = run()
    assert list(r1) == list(r2)
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(U1, U2)
    # no room for any twin: the leaves split in registers, into the same
    # hi/lo pairs and the same product order
    monkeypatch.setenv("HAPOD_TWIN_BUDGET", "1")
    s3, U3, r3 = run()
    assert list(r1) == list(r3)
    np.testing.assert_array_equal(s1, s3)
    np.testing.assert_array_equal(U1, U3)


def _right_vector_case(name):
    if name == "star":
        n = 2048
        S = synth.sinusoid(n, 256, 90, 6.0, 1e-9, seed=21)
        parent = synth.star_tree(5)
        data = dict(enumerate(split_cols(S, [64] * 4)))
        data[4] = np.zeros((n, 16))  # a leaf of rank 0: its rows of W are zero
        return parent, data, n, 1e-4, 0.5, (), {}
    if name in ("chain", "chain_block"):
        n, chunks, cols = 2048, 5, 48
        S = synth.bumps(n, chunks * cols, seed=5)
        parent, chunk = synth.chain_tree(chunks)
        blocks = split_cols(S, [cols] * chunks)
        data = {leaf: blocks[c] for leaf, c in chunk.items()}
        zero = tuple(b for b in chunk if b != 0)
        eps_star = 1e-3 * math.sqrt(np.mean(np.sum(S * S, axis=0)))
        return parent, data, n, eps_star, 0.75, zero, {"block_gram": name == "chain_block"}
    n, leaves, per = 1500, 27, 12
    S = synth.sinusoid(n, leaves * per, 60, 8.0, 1e-10, seed=9)
    parent = synth.balanced_tree(leaves, 4)
    return parent, dict(enumerate(split_cols(S, [per] * leaves))), n, 1e-4, 0.5, (), {}


@pytest.mark.parametrize("name", ["star", "chain", "chain_block", "balanced"])
def test_right_singular_vectors(hp, name):
    """Rem. 3.8 / Def. 3.9: W composed on the device from the nodes' kept
    eigenvectors.  Pinned three ways: W^T W = I (Lem. 3.10); U diag(sigma) =
    S~ W, which the method of snapshots makes hold to rounding at every node
    and hence for the composition; the squared Frobenius error of
    U diag(sigma) W^T at most the sum of eps(gamma)^2.  Against the oracle's
    factorisation: the span of the resolved columns of W."""
    from oracle import factor
    print(f"right vectors {name}", flush=True)
    parent, data, n, eps_star, omega, zero, kw = _right_vector_case(name)
    plan, sig, U, ref, eps, leaf_cols, data64 = run_both(hp, parent, data, n, eps_star, omega, "fp64", zero=zero,
                                                         reorth=False, right_vectors=True, **kw)
    W = host(plan.right_vectors())
    S = np.hstack([data64[k] for k in sorted(data)])
    N = len(sig)
    assert W.shape == (S.shape[1], N)
    assert metrics.orthonormality_error(W) <= 1e-10
    norm_s = np.linalg.norm(S)
    assert np.linalg.norm(U * sig - S @ W) <= 1e-10 * norm_s
    err2 = np.linalg.norm(S - (U * sig) @ W.T) ** 2
    assert err2 <= sum(e * e for e in eps) * (1 + 1e-6) + metrics.rounding_slack(S)
    if name == "star":
        np.testing.assert_array_equal(W[256:], 0.0)
    root = tree.validate(parent)
    fac = factor.hapod_factor(parent, data64, eps)
    W_ref = factor.rows_in_leaf_order(fac[root][2], fac[root][3])
    assert W_ref.shape[1] == len(ref[root][0])
    r = metrics.resolved_rank(ref[root][0], N, UP["fp64"], TAU["fp64"])
    assert r >= 10
    assert metrics.subspace_error(W_ref, W, r) <= TAU["fp64"]
    print(f"  N {N} (oracle {W_ref.shape[1]}), r {r}, err^2/bound {err2 / sum(e * e for e in eps):.3f}")


def test_right_vectors_need_the_option(hp):
    S = synth.sinusoid(256, 16, 10, 5.0, 0.0, seed=3)
    plan = hp.Plan(synth.star_tree(2), [8, 8, 0], 256, 1e-3, 0.5, prec="fp64")
    with pytest.raises(hp.HapodError):
        plan.right_vectors()  # no run yet
    plan.run({0: dev_colmajor(S[:, :8]), 1: dev_colmajor(S[:, 8:])})
    with pytest.raises(hp.HapodError):
        plan.right_vectors()  # plan made without right_vectors


def test_autotune_cache_file(hp, tmp_path):
    """With autotune and a cache file the tuned tile of each node class is
    written back after the run (compute mode, width class, height class,
    tile per line) and a plan made later reads it without error; a corrupt
    line is ignored."""
    n, L, c = 3000, 3, 40
    S = synth.sinusoid(n, L * c, 60, 8.0, 0.0, seed=9)
    data = dict(enumerate(split_cols(S, [c] * L)))
    path = tmp_path / "tiles.txt"
    path.write_text("not a line\n")
    plan = hp.Plan(synth.star_tree(L), [c] * L + [0], n, 1e-6, 0.75, prec="fp32", autotune=True,
                   autotune_cache=str(path))
    plan.run({k: dev_colmajor(v, torch.float32) for k, v in data.items()})
    lines = [ln.split() for ln in path.read_text().splitlines() if ln.strip()]
    assert lines and all(len(ln) == 4 for ln in lines)
    # the leaves' class: FP32 compute, width 48 (40 rounded up to 16), height 2^12
    assert any(ln[0] == "1" and ln[1] == "48" and ln[2] == "12" and ln[3] in ("16", "32", "64", "128")
               for ln in lines), lines
    hp.Plan(synth.star_tree(L), [c] * L + [0], n, 1e-6, 0.75, prec="fp32", autotune=True, autotune_cache=str(path))


def test_device_driven_rank_growth_reruns_the_batch(hp):
    """Leaves of 65..256 columns take the device-driven batch: outputs sized
    before the ranks are known, for the ranks of the plan's previous run.  A
    second run whose ranks grow past them (rank-10 data, then rank-60 data)
    must redo the batch with the ranks read back first; its modes equal,
    bitwise, those of a fresh plan run once on the second data set (sized
    for m), and stay within the oracle's bounds."""
    n, L, c = 3000, 2, 100
    lo = synth.sinusoid(n, L * c, 10, 1e9, 0.0, seed=21)     # 10 equal-weight modes
    hi = synth.sinusoid(n, L * c, 60, 1e9, 0.0, seed=22)     # 60
    eps = 1e-8 * np.linalg.norm(hi)
    plan = hp.Plan(synth.star_tree(L), [c] * L + [0], n, eps, 0.75)
    data_lo = {k: dev_colmajor(v) for k, v in enumerate(split_cols(lo, [c] * L))}
    data_hi = {k: dev_colmajor(v) for k, v in enumerate(split_cols(hi, [c] * L))}
    plan.run(data_lo)
    s_lo, _ = plan.modes()
    assert len(s_lo) == 10
    assert plan.batch_stats() == {"device": 2, "host": 0, "reruns": 0}
    plan.run(data_hi)
    s1, U1 = plan.modes()
    # leaves (10 -> 60) and root (10 -> 60) both outgrow their outputs
    assert plan.batch_stats() == {"device": 0, "host": 0, "reruns": 2}
    fresh = hp.Plan(synth.star_tree(L), [c] * L + [0], n, eps, 0.75)
    fresh.run(data_hi)
    s2, U2 = fresh.modes()
    assert fresh.batch_stats() == {"device": 2, "host": 0, "reruns": 0}
    assert len(s1) == len(s2) == 60
    np.testing.assert_array_equal(s1, s2)
    assert torch.equal(U1, U2)
    s_ref, U_ref = pod.pod(hi, eps)
    np.testing.assert_allclose(s1, s_ref[:60], rtol=1e-10)
    assert metrics.subspace_error(U_ref, host(U1), 60) < 1e-8


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_graph_levels_replays_match_eager_runs(hp, prec):
    """graph_levels: every device-driven batch (leaves of 100 columns, root of
    4 x their rank) is captured as a hipGraph and launched as one.  Run 1
    captures (outputs sized for m), run 2 captures again (outputs now sized
    for the ranks of run 1), later runs replay.  Between the runs, eager work
    on the same stream (another plan, torch arithmetic) and synchronisations;
    every run's modes equal, bitwise, those of a plan without graphs."""
    n, L, c = 5000, 4, 100
    S = synth.sinusoid(n, L * c, 40, 8.0, 1e-9, seed=31)
    dt = torch.float64 if prec == "fp64" else torch.float32
    data = {k: dev_colmajor(v, dt) for k, v in enumerate(split_cols(S, [c] * L))}
    eps = 1e-6 * np.linalg.norm(S)
    eager = hp.Plan(synth.star_tree(L), [c] * L + [0], n, eps, 0.75, prec=prec)
    eager.run(data)
    s0, U0 = eager.modes()
    assert eager.batch_stats()["device"] == 2
    gp = hp.Plan(synth.star_tree(L), [c] * L + [0], n, eps, 0.75, prec=prec, graph_levels=True)
    seen = []
    for r in range(5):
        gp.run(data)
        st = gp.graph_stats()
        seen.append((st["captures"], st["replays"]))
        s, U = gp.modes()
        np.testing.assert_array_equal(s, s0)
        assert torch.equal(U, U0), f"run {r}"
        # eager work between the replays
        eager.run(data)
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        assert float((x * x).sum()) > 0.0
        torch.cuda.synchronize()
    assert seen[0] == (2, 0) and seen[1] == (2, 0), seen
    assert all(sr == (0, 2) for sr in seen[2:]), seen
    assert gp.graph_stats()["ms"] > 0.0
