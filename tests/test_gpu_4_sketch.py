"""GPU parity of the sketched local POD (randomized range finder with the
residual counted as discarded energy) against the SVD oracle.

A wide node's Gram matrix knows sigma_k^2 only to about u sigma_1^2
(Rem. 2.3), so the method of snapshots cannot place a truncation whose tail
lies below that.  The sketched route forms every quantity from S and Q
themselves; checked here: the oracle's rank (Def. 2.5 on LAPACK's singular
values of S), sigma_k within 1e-13 sigma_1, each mode within a Wedin-type
perturbation bound of the oracle's, orthonormal modes, the certified
projection error ||S - U U^T S||_F^2 <= eps^2 (the property Thm. 3.3 - 3.5
use), and at tree level the literal HAPOD's root rank and Thm. 3.5's mean
error where the Gram route over-keeps.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from gpu_util import dev_colmajor, host  # noqa: E402
from oracle import hapod, metrics, pod, tolerances  # noqa: E402

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_05210_amd as m
    return m


def wide_lowrank(n, m, sig, seed, noise=0.0):
    """S = Q_1 diag(sig) Q_2^T (n x m, rank len(sig)) plus optional noise."""
    rng = np.random.default_rng(seed)
    r = len(sig)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, r)))
    Q2, _ = np.linalg.qr(rng.standard_normal((m, r)))
    S = (Q1 * sig) @ Q2.T
    if noise:
        S = S + noise * rng.standard_normal((n, m))
    return S


def check_node(S, s_g, U_g, eps, info, tag, rank_slack=0):
    """Rank, singular values, modes and the certified error of one node."""
    s_all, U_all = pod.pod_full(S)
    N_ref = pod.truncation_rank(s_all, eps)
    N = len(s_g)
    s1 = s_all[0]
    print(f"  {tag}: rank {N} (oracle {N_ref}), residual {info['residual']:.3e}, eps^2 {eps * eps:.3e}, "
          f"passes {info['passes_y']}/{info['passes_b']}, sweeps {info['sweeps']}")
    # the residual r is part of the discarded energy: the rank is the
    # oracle's unless r moves the tail across eps^2
    assert N_ref <= N <= N_ref + rank_slack, (tag, N, N_ref)
    k = min(N, N_ref)
    # sigma_k(B) <= sigma_k(S) <= sigma_k(B) + ||(I - Q Q^T) S||_2 (B = Q^T S:
    # interlacing, then Weyl), and ||(I - Q Q^T) S||_2 <= sqrt(r): the sketch's
    # singular values are those of S to within sqrt(r) plus rounding
    miss = math.sqrt(max(info["residual"], 0.0))
    err = np.max(np.abs(s_g[:k] - s_all[:k])) if k else 0.0
    assert err <= 1e-13 * s1 + miss, (tag, err / s1, miss / s1)
    assert metrics.orthonormality_error(U_g) <= 1e-12, tag
    # mode j against the oracle's: sin(angle) <= (c u sigma_1 + sqrt(r)) / gap_j
    # (Wedin), gap_j the distance of sigma_j to every other singular value of S
    for j in range(k):
        gap = np.min(np.abs(np.delete(s_all, j) - s_all[j]))
        c = abs(float(U_all[:, j] @ U_g[:, j]))
        sin = math.sqrt(max(0.0, 1.0 - c * c)) if c < 1 else 0.0
        bound = (200.0 * math.sqrt(S.shape[1]) * U64 * s1 + 2.0 * miss) / max(gap, 1e-300)
        assert sin <= max(bound, 1e-7), (tag, j, sin, bound)
    # certified: the projection error of the kept modes is at most eps^2
    pe = metrics.projection_error(S, U_g)
    assert pe <= eps * eps * (1 + 1e-6) + metrics.rounding_slack(S), (tag, pe, eps * eps)


@pytest.mark.parametrize("kind", ["sparse_sign", "gaussian"])
@pytest.mark.parametrize("n,m,r,ell", [(3000, 1200, 300, 384), (3001, 1000, 200, 256), (2048, 4096, 100, 128)])
def test_sketch_node_graded(hp, n, m, r, ell, kind):
    """Exact rank r < ell, singular values graded 10^(-k/20): the truncation
    sits at sigma ~ 1e-10 sigma_1, far below the Gram floor.  Both test
    matrices hold the whole range (r < ell), so neither falls back."""
    print(f"sketch node n={n} m={m} r={r} ell={ell} {kind}", flush=True)
    sig = 10.0 ** (-np.arange(r) / 20.0)
    S = wide_lowrank(n, m, sig, seed=n + m)
    # eps^2 between the tails at k = 2r/3 and k + 1 (sigma_k = 1e-10 for r = 300)
    t = pod.tail_sums(sig)
    k = (2 * r) // 3
    eps = math.sqrt(0.5 * (t[k] + t[k + 1]))
    Sd = dev_colmajor(S)
    s_g, U_g, info = hp.hapod_node_pod_sketch(Sd, eps, ell, seed=7, kind=kind)
    torch.cuda.synchronize()
    assert info["kind"] == kind
    check_node(S, s_g, host(U_g), eps, info, f"graded {n}x{m} {kind}")
    # the method of snapshots on the same node: its tail sums near eps^2 are
    # rounding noise of the Gram (~ m u sigma_1^2 >> eps^2)
    s_m, _ = hp.hapod_node_pod("fp64", Sd, eps)
    print(f"  method of snapshots: rank {len(s_m)} (oracle {pod.truncation_rank(pod.pod_full(S)[0], eps)})")


def test_sketch_node_noisy_scaled_and_rerun(hp):
    """Noisy low-rank data (the residual is the noise energy and enters the
    truncation), scaled modes, zero columns, bitwise-identical rerun."""
    n, m, r = 2500, 900, 150
    sig = 1e3 * np.exp(-np.arange(r) / 8.0)
    S = wide_lowrank(n, m, sig, seed=11, noise=1e-9)
    clean = wide_lowrank(n, m, sig, seed=11)
    for z in (5, 700):
        S[:, z] = 0.0
        clean[:, z] = 0.0
    noise_energy = float(np.sum((S - clean) ** 2))
    # eps^2 = 10x the noise energy, below sigma_150^2 = 1e6 e^-37.25 = 6.6e-11:
    # every signal mode is kept and the noise alone is discarded
    eps = math.sqrt(10.0 * noise_energy)
    Sd = dev_colmajor(S)
    s1, W1, i1 = hp.hapod_node_pod_sketch(Sd, eps, 256, seed=3, scaled=True, kind="gaussian")
    s2, W2, i2 = hp.hapod_node_pod_sketch(Sd, eps, 256, seed=3, scaled=True, kind="gaussian")
    torch.cuda.synchronize()
    assert np.array_equal(s1, s2) and torch.equal(W1, W2) and i1["residual"] == i2["residual"]
    # the sparse sign map: certified the same way, its sums in a fixed order
    # (bitwise-identical rerun)
    s3, W3, i3 = hp.hapod_node_pod_sketch(Sd, eps, 256, seed=3, scaled=True)
    s4, W4, i4 = hp.hapod_node_pod_sketch(Sd, eps, 256, seed=3, scaled=True)
    torch.cuda.synchronize()
    assert i3["kind"] == "sparse_sign" and i3["residual"] <= eps * eps
    assert np.array_equal(s3, s4) and torch.equal(W3, W4) and i3["residual"] == i4["residual"]
    check_node(S, s3, host(W3) / s3[None, :], eps, i3, "noisy scaled, sparse sign", rank_slack=1)
    W = host(W1)
    U = W / s1[None, :]
    assert i1["residual"] <= eps * eps
    # the residual of a 256-column sketch of rank-150 data is about the noise
    # energy: the noise outside the sketch's span plus the signal its slightly
    # tilted span misses, within (1 + k / (p - 1)) = 2.4 of the noise energy in
    # expectation for k = 150 signal modes and p = 106 spare columns (Halko,
    # Martinsson & Tropp, Thm. 10.5)
    assert 0.3 * noise_energy <= i1["residual"] <= 5.0 * noise_energy, (i1["residual"], noise_energy)
    check_node(S, s1, U, eps, i1, "noisy scaled", rank_slack=1)
    # scaled modes are sigma_k u_k
    assert np.allclose(np.linalg.norm(W, axis=0), s1, rtol=1e-12)
    # unscaled modes: the error of the kept modes is computed from the modes
    # themselves (rank chosen with eps^2 / 64 left for the residual); with
    # eps^2 = 1.05 r that reserve is too small (the noise directions B holds
    # carry about 0.1 r), so r of the whole basis is taken and the rank set
    # anew -- both certified against the projection error.  With only
    # 0.05 r of the budget left for B's tail, the tight case keeps most of
    # the noise directions the sketch holds (the rank exceeds the oracle's
    # where r moves the tail across eps^2)
    for e2, tag, slack in ((eps * eps, "noisy unscaled", 1), (1.05 * i1["residual"], "noisy unscaled, tight budget", 256)):
        s5, U5, i5 = hp.hapod_node_pod_sketch(Sd, math.sqrt(e2), 256, seed=3, scaled=False, kind="gaussian")
        assert abs(i5["residual"] - i1["residual"]) <= 1e-6 * e2, (tag, i5["residual"], i1["residual"])
        check_node(S, s5, host(U5), math.sqrt(e2), i5, tag, rank_slack=slack)


@pytest.mark.parametrize("kind", ["sparse_sign", "gaussian"])
def test_sketch_node_rank_beyond_sketch_fails(hp, kind):
    """A rank the sketch cannot hold: HAPOD_E_UNSUPPORTED, residual reported
    (the sparse sign map first falls back to the Gaussian, which fails too)."""
    n, m, r = 1500, 800, 400
    sig = np.exp(-np.arange(r) / 100.0)
    S = wide_lowrank(n, m, sig, seed=5)
    eps = math.sqrt(pod.tail_sums(sig)[350])
    with pytest.raises(hp.HapodError) as ei:
        hp.hapod_node_pod_sketch(dev_colmajor(S), eps, 128, kind=kind)
    assert ei.value.status == 8
    assert "residual" in hp.hapod_last_error()
    # the abandoned attempts' buffers went back: a node that fits runs next
    sig2 = 10.0 ** (-np.arange(100) / 20.0)
    S2 = wide_lowrank(1024, 600, sig2, seed=6)
    eps2 = math.sqrt(pod.tail_sums(sig2)[60])
    s_g, U_g, info = hp.hapod_node_pod_sketch(dev_colmajor(S2), eps2, 128, kind=kind)
    torch.cuda.synchronize()
    check_node(S2, s_g, host(U_g), eps2, info, f"after a failure, {kind}")


def test_sketch_node_argument_errors(hp):
    S = dev_colmajor(np.ones((300, 200)))
    for ell in (100, 640, 256):  # not a tile multiple / too wide / above m
        with pytest.raises(hp.HapodError) as ei:
            hp.hapod_node_pod_sketch(S, 1.0, ell)
        assert ei.value.status == 8
    with pytest.raises(hp.HapodError) as ei:
        hp.hapod_node_pod_sketch(S, 0.0, 128)
    assert ei.value.status == 1


def sinus_star(n, leaves, cols, K, tau, noise, seed):
    S = synth.sinusoid(n, leaves * cols, K, tau, noise, seed)
    return S, {i: S[:, i * cols:(i + 1) * cols] for i in range(leaves)}


def test_tree_sketch_root_meets_the_bound(hp):
    """16 leaves x 64 sinusoid snapshots at n = 4096 (K = 200, decay e^-k/10,
    noise 1e-10), eps* = 1e-6, omega = 0.75: the 1024-input root takes the
    sketched route.  Its rank is the literal HAPOD's, its singular values
    agree to 1e-12 sigma_1, the mean error meets Thm. 3.5, while the Gram
    route's root decision lies below its floor."""
    print("tree sketch root 4096 x 1024", flush=True)
    n, L, c = 4096, 16, 64
    S, data = sinus_star(n, L, c, 200, 10.0, 1e-10, seed=21)
    parent = synth.star_tree(L)
    cols = [c] * L + [0]
    eps_star, omega = 1e-6, 0.75
    eps = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    ref = hapod.hapod(parent, data, eps)
    s_ref, U_ref = ref[L]
    dev = {i: dev_colmajor(v) for i, v in data.items()}
    out = {}
    blocks = {i: hp.to_blocks(v) for i, v in dev.items()}
    for name, kw in (("sketch", dict(sketch_cols=256)), ("gram", {}),
                     ("passed", dict(sketch_cols=256, leaf_layout="blocks", leaf_passthrough=True))):
        plan = hp.Plan(parent, cols, n, eps_star, omega, prec="fp64", **kw)
        plan.run(blocks if name == "passed" else dev)
        sig, U = plan.modes()
        out[name] = (sig, host(U), plan.ranks(), plan.sketch_stats(), [plan.route(i) for i in range(L)])
        del plan
    # full-rank leaves handing their own columns (row-block layout) to the
    # sketched root: the same rank, sigma to the residual's level
    sig_p, U_p, ranks_p, st_p, routes_p = out["passed"]
    print(f"  leaf passthrough: routes {set(routes_p)}, root rank {len(sig_p)} (sketch {len(out['sketch'][0])}), "
          f"residual {st_p['residual']:.3e}")
    assert all(r == ("full_leaf" if ranks_p[i] == c else "snapshots") for i, r in enumerate(routes_p))
    assert "full_leaf" in routes_p
    assert len(sig_p) == len(out["sketch"][0])
    assert np.max(np.abs(sig_p - out["sketch"][0])) <= 1e-12 * sig_p[0] + math.sqrt(st_p["residual"])
    assert metrics.mean_projection_error(S, U_p) <= eps_star ** 2
    sig, U, ranks, st, _ = out["sketch"]
    assert st is not None and st["ell"] == 256
    assert st["kind"] == "sparse_sign"  # K = 200 sinusoid modes fit the 256 columns
    assert list(ranks[:L]) == [len(ref[i][0]) for i in range(L)]
    # the root's own input is the literal HAPOD's up to the leaves' rounding;
    # its rank within the one the residual can add
    root_in = hapod.node_input(parent, ref, L, data)
    s_in = pod.pod_full(root_in)[0]
    t_in = pod.tail_sums(s_in)
    print(f"  sketch: root rank {len(sig)} (oracle {len(s_ref)}), residual {st['residual']:.3e}, "
          f"eps^2 {eps[L] ** 2:.3e}; gram route rank {len(out['gram'][0])}")
    # t_S(N) <= r + t_B(N) <= eps^2: the rank is at least the oracle's, and
    # exceeds it only where the residual r moves the tail across eps^2
    assert t_in[len(sig)] <= eps[L] ** 2 * (1 + 1e-9)
    assert len(s_ref) <= len(sig) <= len(s_ref) + 1
    k = min(len(sig), len(s_ref))
    assert np.max(np.abs(sig[:k] - s_ref[:k])) <= 1e-12 * s_ref[0] + math.sqrt(st["residual"])
    # leading subspaces: e_sub(r) <= 2 (||(I - Q Q^T) S||_2 + rounding) /
    # (sigma_r - sigma_{r+1}) (Wedin).  The sketch misses of S mostly the part
    # of the noise outside its span, so ||(I - Q Q^T) S||_2 is about the
    # noise's spectral norm (bounded by std (sqrt(n) + sqrt(m) + 6)); the last
    # kept modes, 1e-6 apart, are defined to that level only
    from oracle import coeff
    e_noise = coeff.weyl_noise_bound(n, L * c, 1e-10)
    for r in sorted({len(s_ref) // 4, len(s_ref) // 2, (3 * len(s_ref)) // 4, len(s_ref)}):
        gap = s_in[r - 1] - s_in[r]
        es = metrics.subspace_error(U_ref, U, r)
        bound = 2.0 * (e_noise + 1e-12 * s_in[0]) / gap
        print(f"  e_sub({r}) = {es:.2e}, bound {bound:.2e}")
        assert es <= bound, (r, es, bound)
    # the Gram contract's resolved rank (sigma_k^2 >= 10 u / tau sigma_1^2) to tau = 1e-6
    r_res = metrics.resolved_rank(s_ref, len(sig), U64, 1e-6)
    assert metrics.subspace_error(U_ref, U, r_res) <= 1e-6
    mean_err = metrics.mean_projection_error(S, U)
    print(f"  mean error {mean_err:.3e} (eps*^2 {eps_star ** 2:.1e}); gram route "
          f"{metrics.mean_projection_error(S, out['gram'][1]):.3e}")
    assert mean_err <= eps_star ** 2
    assert metrics.orthonormality_error(U) <= 1e-12


def test_tree_sketch_inner_nodes_and_uneven_rows(hp):
    """A three-level tree (36 leaves of 64 sinusoid snapshots, K = 50, arity
    6) whose inner nodes (scaled modes, about 300 inputs each) and root take
    the sketched route, leaves of uneven declared height (1200 .. 3000 rows;
    the snapshots themselves live on the first 1200 rows, so every node's
    data stays in one 50-dimensional space while the kernels see columns of
    different row counts): every sketched node's residual within its eps^2,
    the root's rank the literal HAPOD's, the mean error within Thm. 3.5."""
    print("tree sketch inner nodes", flush=True)
    n, L, c, h0 = 3000, 36, 64, 1200
    parent = synth.balanced_tree(L, 3)
    rng = np.random.default_rng(4)
    heights = [int(h) for h in rng.integers(h0, n + 1, size=L)]
    data = {}
    for i in range(L):
        S = np.zeros((n, c))
        S[:h0] = synth.sinusoid(h0, c, 50, 8.0, 1e-11, seed=100 + i)
        data[i] = S
    cols = [c] * L + [0] * (len(parent) - L)
    rows = heights + [0] * (len(parent) - L)
    eps_star, omega = 1e-7, 0.5
    plan = hp.Plan(parent, cols, n, eps_star, omega, prec="fp64", sketch_cols=128, leaf_rows=rows)
    dev = {i: dev_colmajor(v[:heights[i]]) for i, v in data.items()}
    plan.run(dev)
    sig, U = plan.modes()
    U = host(U)
    eps, lev, acc = plan.query()
    took = [a for a in range(len(parent)) if plan.sketch_stats(a) is not None]
    assert len(took) == len(parent) - L, took  # every inner node and the root
    for a in took:
        assert plan.sketch_stats(a)["residual"] <= eps[a] ** 2
    ref = hapod.hapod(parent, data, list(eps))
    root = len(parent) - 1
    S_all = np.hstack([data[i] for i in range(L)])
    mean_err = metrics.mean_projection_error(S_all, U)
    print(f"  sketched nodes {took}, root rank {len(sig)} (oracle {len(ref[root][0])}), "
          f"mean error {mean_err:.3e} (eps*^2 {eps_star ** 2:.1e})")
    assert abs(len(sig) - len(ref[root][0])) <= 1
    assert mean_err <= eps_star ** 2
    assert np.all(U[max(heights):] == 0.0)


def test_sketch_option_rules(hp):
    parent = synth.star_tree(2)
    for kw in (dict(prec="fp32", sketch_cols=256), dict(sketch_cols=100), dict(sketch_cols=1024),
               dict(sketch_cols=256, right_vectors=True)):
        with pytest.raises(hp.HapodError) as ei:
            hp.Plan(parent, [64, 64, 0], 1000, 1e-3, 0.5, **kw)
        assert ei.value.status == 1


def test_plan_routes_workspace_and_node_pod(hp):
    """The route each node took, the pool's peak against the worst-case
    estimate, and hapod_plan_node_pod reproducing a node of the run: a leaf
    (method of snapshots) and the root (sketched) on the same inputs the run
    gave them; an omega = 0 root reports the pass-through route."""
    n, L, c = 4096, 16, 64
    S, data = sinus_star(n, L, c, 200, 10.0, 1e-10, seed=21)
    parent = synth.star_tree(L)
    cols = [c] * L + [0]
    plan = hp.Plan(parent, cols, n, 1e-6, 0.75, prec="fp64", sketch_cols=256)
    dev = {i: dev_colmajor(v) for i, v in data.items()}
    plan.run(dev)
    assert plan.route(-1) == "sketch" and plan.route(0) == "snapshots"
    worst, peak = plan.workspace()
    assert 0 < peak <= worst, (peak, worst)
    ranks = plan.ranks()
    sig_root, U = plan.modes()
    # a leaf through the plan's node POD: its rank and singular values
    s0, W0 = plan.node_pod(0, dev[0])
    s0_run, _ = plan.modes(0, with_U=False)
    assert len(s0) == ranks[0]
    assert np.max(np.abs(s0 - s0_run)) <= 1e-12 * s0_run[0]
    # the root's POD on the leaves' scaled modes (each leaf lossless here, so
    # the node POD of every leaf gives the run's root input up to rounding)
    ins = [plan.node_pod(i, dev[i])[1] for i in range(L)]
    root_in = torch.cat(ins, dim=1).contiguous().t().contiguous().t()
    sr, Ur = plan.node_pod(-1, root_in)
    assert abs(len(sr) - len(sig_root)) <= 1
    k = min(len(sr), len(sig_root))
    st = plan.sketch_stats(-1)
    assert np.max(np.abs(sr[:k] - sig_root[:k])) <= 1e-12 * sig_root[0] + math.sqrt(st["residual"])
    # omega = 0: the root passes its inputs through
    p0 = hp.Plan(parent, cols, n, 1e-6, 0.0, prec="fp64")
    p0.run(dev)
    assert p0.route(-1) == "passthrough" and p0.route(3) == "snapshots"


def test_subtrees_as_streams_equal_the_unsharded_run(hp):
    """The sharding the design describes (each GPU a subtree, one transfer per
    cross-GPU edge), rehearsed on one GPU: the 16 leaves of a star split into
    two groups, each group's leaf PODs issued on a stream of its own through
    hapod_plan_node_pod (what a shard would run), the root's POD on the
    gathered scaled modes afterwards.  Ranks equal the unsharded run's at
    every node, the root's singular values and modes agree to rounding."""
    n, L, c = 4096, 16, 64
    S, data = sinus_star(n, L, c, 200, 10.0, 1e-10, seed=33)
    parent = synth.star_tree(L)
    cols = [c] * L + [0]
    plan = hp.Plan(parent, cols, n, 1e-6, 0.75, prec="fp64", sketch_cols=256)
    dev = {i: dev_colmajor(v) for i, v in data.items()}
    plan.run(dev)
    ranks = plan.ranks()
    sig_run, U_run = plan.modes()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = {}
    for shard, st in enumerate(streams):
        with torch.cuda.stream(st):
            for i in range(shard * L // 2, (shard + 1) * L // 2):
                s_i, W_i = plan.node_pod(i, dev[i])
                outs[i] = (s_i, W_i)
    for st in streams:
        st.synchronize()
    for i in range(L):
        assert len(outs[i][0]) == ranks[i]
    root_in = torch.cat([outs[i][1] for i in range(L)], dim=1).contiguous().t().contiguous().t()
    s_root, U_root = plan.node_pod(-1, root_in)
    assert len(s_root) == len(sig_run)
    st_run = plan.sketch_stats(-1)
    assert np.max(np.abs(s_root - sig_run)) <= 1e-12 * sig_run[0] + math.sqrt(st_run["residual"])
    # modes: the leading subspace with a clear gap agrees to rounding
    r = metrics.resolved_rank(sig_run, len(sig_run), U64, 1e-6)
    assert metrics.subspace_error(host(U_run), host(U_root), r) <= 1e-6
