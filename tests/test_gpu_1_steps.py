"""GPU parity of every method-of-snapshots step, through the C ABI.

Gram (Rem. 2.3): bitwise on integer data, rounding-bounded on random data.
Eigensolve: eigenvalues/residual/orthonormality against LAPACK within
c m u ||G||.  Truncation (Def. 2.5): exact ranks.  Lift and
re-orthonormalisation: against NumPy.  Node POD: against the SVD oracle.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import dev_colmajor, host  # noqa: E402


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_05210_amd as m
    return m


U64 = 2.0 ** -53
U32 = 2.0 ** -24
ELEM = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.float32}

GRAM_SHAPES = [(1, 1), (7, 3), (100, 17), (4096, 64), (5000, 130), (3000, 256), (2049, 300), (64, 129), (1000, 600),
               (300, 520)]


# ---------------------------------------------------------------- Gram ------
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n,m", GRAM_SHAPES)
def test_gram_integer_bitwise(hp, prec, n, m):
    print(f"gram int {prec} n={n} m={m}", flush=True)
    rng = np.random.default_rng(n * 1000 + m)
    A = rng.integers(-32, 33, size=(n, m)).astype(np.int64)
    exact = (A.T @ A).astype(np.float64)          # |entries| < 2^24: exact in all forms
    G = hp.hapod_gram(prec, dev_colmajor(A, ELEM[prec]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(G), exact)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gram_padded_leading_dimension(hp, prec):
    rng = np.random.default_rng(5)
    A = rng.integers(-16, 17, size=(333, 70)).astype(np.float64)
    G = hp.hapod_gram(prec, dev_colmajor(A, ELEM[prec], ld=337))   # odd ld: unaligned columns
    np.testing.assert_array_equal(host(G), A.T @ A)


@pytest.mark.parametrize("prec,u,c", [("fp64", U64, 4.0), ("fp32", U32, 4.0), ("bf16x3", 2.0 ** -17, 4.0)])
@pytest.mark.parametrize("n,m", [(4096, 64), (20000, 200), (777, 131)])
def test_gram_random_within_rounding(hp, prec, u, c, n, m):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((n, m)) * np.exp(-np.arange(m) / 20.0)
    if prec != "fp64":
        A = A.astype(np.float32).astype(np.float64)
    G = host(hp.hapod_gram(prec, dev_colmajor(A, ELEM[prec])))
    ref = A.T @ A
    nrm = np.sqrt(np.diag(ref))
    bound = c * n * u * np.outer(nrm, nrm) if prec == "fp64" else c * math.sqrt(n) * u * np.outer(nrm, nrm) * 8
    assert np.all(np.abs(G - ref) <= bound + 1e-300)
    np.testing.assert_array_equal(G, G.T)


def test_gram_empty_rows(hp):
    A = np.zeros((0, 5))
    G = hp.hapod_gram("fp64", dev_colmajor(A))
    np.testing.assert_array_equal(host(G), np.zeros((5, 5)))


# ---------------------------------------------------------------- eigh ------
def prescribed(m, lam, seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((m, m)))
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("m", [1, 2, 3, 16, 63, 64, 127, 128, 129, 200, 255, 256])
def test_eigh_against_lapack(hp, m):
    print(f"eigh m={m}", flush=True)
    lam = 4.0 * 0.8 ** np.arange(m)
    G0 = prescribed(m, lam, m)
    G0 = 0.5 * (G0 + G0.T)
    lam_g, V, sweeps = hp.hapod_eigh(dev_colmajor(G0))
    lam_g, V = host(lam_g), host(V)
    ref = np.linalg.eigvalsh(G0)[::-1]
    nrm = np.abs(ref).max()
    tol = 50 * max(m, 1) * U64 * nrm
    assert np.all(np.diff(lam_g) <= 0)
    np.testing.assert_allclose(lam_g, ref, atol=tol, rtol=0)
    assert np.abs(G0 @ V - V * lam_g).max() <= tol
    assert np.abs(V.T @ V - np.eye(m)).max() <= 50 * max(m, 1) * U64
    # sign convention: largest |entry| of every column positive
    idx = np.argmax(np.abs(V), axis=0)
    assert np.all(V[idx, np.arange(m)] > 0)
    assert sweeps <= 60


def test_eigh_repeated_and_negative_eigenvalues(hp):
    m = 40
    lam = np.array([3.0] * 5 + [1.0] * 10 + [0.0] * 5 + list(-1e-3 * np.arange(1, 21)))
    G0 = prescribed(m, lam, 3)
    G0 = 0.5 * (G0 + G0.T)
    lam_g, V, _ = hp.hapod_eigh(dev_colmajor(G0))
    lam_g, V = host(lam_g), host(V)
    np.testing.assert_allclose(lam_g, np.sort(lam)[::-1], atol=1e-13)
    assert np.abs(G0 @ V - V * lam_g).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(m)).max() < 1e-13


def test_eigh_diagonal_is_exact(hp):
    d = np.array([0.5, 4.0, 2.0, 4.0, 1.0])
    lam_g, V, sweeps = hp.hapod_eigh(dev_colmajor(np.diag(d)))
    np.testing.assert_array_equal(host(lam_g), [4.0, 4.0, 2.0, 1.0, 0.5])
    # ties keep index order: columns e_1, e_3
    P = host(V)
    np.testing.assert_array_equal(P[:, 0], np.eye(5)[1])
    np.testing.assert_array_equal(P[:, 1], np.eye(5)[3])
    assert sweeps == 1


# ------------------------------------------------------------ truncation ----
@pytest.mark.parametrize("eps,expect", [(0.5, 2), (0.4999, 3), (1.5, 1), (3.0, 0), (1e-300, 3)])
def test_truncate_dyadic(hp, eps, expect):
    from oracle import pod
    lam = torch.tensor([4.0, 1.0, 0.25], dtype=torch.float64, device="cuda")
    N, info = hp.hapod_truncate(lam, eps)
    assert N == expect == pod.truncation_rank(np.array([2.0, 1.0, 0.5]), eps)


def test_truncate_clamps_negative_values(hp):
    lam = torch.tensor([9.0, 4.0, 1.0, 1e-3, -1e-3, -2.0], dtype=torch.float64, device="cuda")
    N, info = hp.hapod_truncate(lam, math.sqrt(1.0015))
    assert N == 2            # tail(2) = 1 + 1e-3 <= 1.0015 < tail(1); negatives count 0
    assert info[3] == 2 and info[2] == -2.0 and info[1] == 9.0


@pytest.mark.parametrize("m", [1, 5, 255, 256, 257, 1000, 8192])
def test_truncate_random_against_oracle(hp, m):
    from oracle import pod
    rng = np.random.default_rng(m)
    lam = np.sort(np.exp(-rng.uniform(0, 30, m)))[::-1].copy()
    s = np.sqrt(lam)
    for N_target in sorted({0, m // 3, m // 2, m - 1, m}):
        t_hi = np.sum(lam[N_target - 1:]) if N_target > 0 else np.inf
        t_lo = np.sum(lam[N_target:])
        eps = math.sqrt(1.01 * t_lo) if N_target == 0 else math.sqrt(0.5 * (t_lo + t_hi))
        N, _ = hp.hapod_truncate(torch.tensor(lam, device="cuda"), eps)
        assert N == pod.truncation_rank(s, eps) == N_target


def test_truncate_empty(hp):
    N, _ = hp.hapod_truncate(torch.zeros(0, dtype=torch.float64, device="cuda"), 1.0)
    assert N == 0


# -------------------------------------------------------------------- lift ---
# (4096, 96, 81) and (2048, 200, 171): FP64 on the unguarded (dense) lift,
# whose operand runs past the padded row width (columns >= N) re-read the
# row's last run; one and two column tiles
@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-13), ("fp32", 1e-5), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("n,m,N", [(1, 1, 1), (100, 7, 3), (4097, 130, 129), (300, 256, 200), (64, 40, 0),
                                   (4096, 96, 81), (2048, 200, 171)])
def test_lift_against_numpy(hp, prec, rtol, n, m, N):
    rng = np.random.default_rng(n + m + N)
    S = rng.standard_normal((n, m))
    if prec != "fp64":
        S = S.astype(np.float32).astype(np.float64)
    V = rng.standard_normal((m, m))
    lam = np.exp(-np.arange(m) / 7.0) + 0.1
    Sd = dev_colmajor(S, ELEM[prec])
    for root in [False, True]:
        out = hp.hapod_lift(prec, Sd, dev_colmajor(V), N,
                            lam=torch.tensor(lam, device="cuda") if root else None)
        ref = S @ V[:, :N] / (np.sqrt(lam[:N]) if root else 1.0)
        if N == 0:
            assert host(out).shape == (n, 0)
            continue
        scale = np.abs(S).sum(axis=1).max() * np.abs(V[:, :N]).max() / (math.sqrt(lam.min()) if root else 1.0)
        assert np.abs(host(out) - ref).max() <= rtol * max(scale, 1e-300)


# ------------------------------------------------------------------ reorth ---
@pytest.mark.parametrize("N", [17, 90, 128, 300, 1024])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_reorth(hp, prec, tol, N):
    """Cholesky blocked in 16-row panels with both triangles in LDS (N <= 128:
    a partial panel, and eight whole ones) and in place in global memory
    (above), up to the 1024-column limit."""
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((5000, N)))
    U = Q + 1e-5 * rng.standard_normal(Q.shape)
    Ud = dev_colmajor(U, ELEM[prec])
    bad = hp.hapod_reorth(prec, Ud)
    R = host(Ud)
    assert bad == 0
    # after the second pass every entry of Q^T Q - I carries the rounding of
    # a length-n dot product (about sqrt(n) u_p for the FP64 Gram, the FP32
    # storage of Q for the FP32 form) plus that of the N-term triangular
    # solve and product (about N u_p): bound 4 (sqrt(n) + N) u_p in FP64; the
    # FP32 form's entries are rounded to FP32 after a FP64 factorisation, so
    # 16 sqrt(N) u_32 (each entry of Q one rounding, N terms per column norm)
    n = U.shape[0]
    bound = (4.0 * (math.sqrt(n) + N) * 2.0 ** -53) if prec == "fp64" else 16.0 * math.sqrt(N) * 2.0 ** -24
    err = np.abs(R.T @ R - np.eye(N)).max()
    print(f"  reorth {prec} N={N}: max|Q^T Q - I| = {err:.3e} (bound {bound:.3e})")
    assert err <= bound
    from oracle import metrics
    assert metrics.subspace_error(np.linalg.qr(U)[0], R, N) <= 1e3 * tol


@pytest.mark.parametrize("N", [40, 200])
def test_reorth_dependent_column(hp, N):
    """A column equal to an earlier one has no positive pivot: reported, left
    as it is, and the others come out orthonormal."""
    rng = np.random.default_rng(3)
    U = np.linalg.qr(rng.standard_normal((3000, N)))[0] + 1e-6 * rng.standard_normal((3000, N))
    U[:, 7] = U[:, 3]
    Ud = dev_colmajor(U)
    bad = hp.hapod_reorth("fp64", Ud)
    R = host(Ud)
    assert bad == 1
    keep = [c for c in range(N) if c != 7]
    assert np.abs(R[:, keep].T @ R[:, keep] - np.eye(N - 1)).max() <= 1e-13


# ---------------------------------------------------------------- node POD ---
def prescribed_svd(n, m, sigma, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, len(sigma))))
    W, _ = np.linalg.qr(rng.standard_normal((m, len(sigma))))
    return (U * sigma) @ W.T


# m = 100, 200, 250: every eigenpair from the Householder reduction (one
# workgroup); 300, 450: Krylov steps, a matrix alone above 224 columns on the
# cooperative multi-workgroup kernel (16 workgroups up to 320 columns, 32
# above)
@pytest.mark.parametrize("n,m", [(8, 3), (64, 16), (33, 33), (16, 40), (500, 100), (4096, 64), (600, 200),
                                 (500, 250), (700, 300), (900, 450)])
def test_node_pod_against_svd_oracle(hp, n, m):
    from oracle import metrics, pod
    r = min(n, m)
    sigma = 10.0 * 0.6 ** np.arange(r)
    S = prescribed_svd(n, m, sigma, n + m)
    k = min(r - 1, 5)
    eps = math.sqrt(0.5 * (np.sum(sigma[k:] ** 2) + np.sum(sigma[k + 1:] ** 2)))
    s_ref, U_ref = pod.pod(S, eps)
    s, U = hp.hapod_node_pod("fp64", dev_colmajor(S), eps)
    assert len(s) == len(s_ref) == k + 1
    np.testing.assert_allclose(s, s_ref, rtol=1e-10)
    assert metrics.subspace_error(U_ref, host(U), len(s)) < 1e-9
    assert metrics.orthonormality_error(host(U)) < 1e-9
    s2, W = hp.hapod_node_pod("fp64", dev_colmajor(S), eps, scaled=True)
    np.testing.assert_allclose(host(W), host(U) * s, rtol=0, atol=1e-12 * sigma[0])


@pytest.mark.parametrize("n,m,k", [(4096, 96, 80), (2048, 200, 170)])
def test_node_pod_dense_batch_lift(hp, n, m, k):
    """FP64 nodes whose lift takes the unguarded loads (n a multiple of 128,
    m of 8) at ranks above 64, one and two column tiles: ranks, sigma and
    modes against the SVD oracle within the method of snapshots' own error
    (eigenvalues to about m u sigma_1^2, Rem. 2.3), scaled against unscaled
    modes."""
    from oracle import metrics, pod
    r = min(n, m)
    sigma = 10.0 * 0.98 ** np.arange(r)
    S = prescribed_svd(n, m, sigma, n + m)
    eps = math.sqrt(0.5 * (np.sum(sigma[k:] ** 2) + np.sum(sigma[k + 1:] ** 2)))
    s_ref, U_ref = pod.pod(S, eps)
    s, U = hp.hapod_node_pod("fp64", dev_colmajor(S), eps)
    assert len(s) == len(s_ref) == k + 1
    floor = 64 * m * np.finfo(float).eps * sigma[0] ** 2  # eigenvalue error allowance
    np.testing.assert_allclose(s, s_ref, rtol=0, atol=floor / s_ref[-1])
    gap = sigma[k] ** 2 - sigma[k + 1] ** 2  # at the truncation
    assert metrics.subspace_error(U_ref, host(U), len(s)) < floor / gap
    assert metrics.orthonormality_error(host(U)) < 1e-9
    s2, W = hp.hapod_node_pod("fp64", dev_colmajor(S), eps, scaled=True)
    np.testing.assert_allclose(host(W), host(U) * s, rtol=0, atol=1e-12 * sigma[0])


@pytest.mark.parametrize("n,m", [(1000, 129), (4099, 200), (3000, 256), (5003, 130)])
def test_node_pod_split_bf16_one_256_tile(hp, n, m):
    """Split-BF16 nodes of 129..256 columns run their Gram as one 256-column
    tile staged from their own FP32 columns (odd row counts: unaligned
    column starts and a ragged last row block).  Against the SVD oracle on
    the FP32-rounded input: sigma within the Gram perturbation bound
    4 sqrt(n) u_p sigma_1^2 / sigma_k (u_p = 2^-17 for the split products),
    the resolved leading modes' span, the rank within one."""
    from oracle import metrics, pod
    sigma = 10.0 * 0.8 ** np.arange(m)
    S = prescribed_svd(n, m, sigma, n + m).astype(np.float32).astype(np.float64)
    eps = math.sqrt(np.sum(sigma[30:] ** 2)) * 1.0001
    s_ref, U_ref = pod.pod(S, eps)
    s, U = hp.hapod_node_pod("bf16x3", dev_colmajor(S, torch.float32), eps)
    assert abs(len(s) - len(s_ref)) <= 1
    up = 2.0 ** -17
    k = min(len(s), len(s_ref))
    tol = 4.0 * math.sqrt(n) * up * s_ref[0] ** 2 / s_ref[:k]
    assert np.all(np.abs(s[:k] - s_ref[:k]) <= tol)
    r = metrics.resolved_rank(s_ref, len(s), up, 1e-2)
    assert r >= 8
    assert metrics.subspace_error(U_ref, host(U).astype(np.float64), r) <= 1e-2


@pytest.mark.parametrize("m", [200, 250])
def test_node_pod_exact_multiplicity(hp, m):
    """A lone node of 129..256 columns needs every eigenpair (the
    Householder reduction); G = 4 I (every eigenvalue repeated) is already
    tridiagonal, so every reflector is the identity (a Krylov run would break
    down at every step): all m modes, sigma = 2, the span of the inputs."""
    from oracle import metrics
    n = 256
    S = np.zeros((n, m))
    S[np.arange(m), np.arange(m)] = 2.0
    s, U = hp.hapod_node_pod("fp64", dev_colmajor(S), 1.0)
    assert len(s) == m
    np.testing.assert_allclose(s, 2.0, rtol=1e-13)
    Uh = host(U)
    assert metrics.subspace_error(np.eye(n)[:, :m], Uh, m) < 1e-12
    assert metrics.orthonormality_error(Uh) < 1e-12


def test_node_pod_passthrough(hp):
    S = np.random.default_rng(0).standard_normal((50, 7))
    s, U = hp.hapod_node_pod("fp64", dev_colmajor(S), 0.0)
    np.testing.assert_array_equal(s, np.ones(7))
    np.testing.assert_array_equal(host(U), S)


def test_node_pod_nan_is_numeric_error(hp):
    S = np.ones((40, 4))
    S[3, 2] = np.nan
    with pytest.raises(hp.HapodError) as e:
        hp.hapod_node_pod("fp64", dev_colmajor(S), 0.1)
    assert e.value.status == 5


# ----------------------------------------------------- wide eigensolver -----
def test_eigh_wide_leading_pairs(hp):
    """m above the one-workgroup Jacobi limit: Lanczos path."""
    m = 1200
    lam = 0.9 ** np.arange(m)
    G0 = prescribed(m, lam, 11)
    G0 = 0.5 * (G0 + G0.T)
    lam_g, V, steps = hp.hapod_eigh(dev_colmajor(G0))
    lam_g, V = host(lam_g), host(V)
    b = int(np.count_nonzero(lam_g))
    print(f"wide eigh: block {b}, steps {steps}")
    r = min(b, 300)
    assert r >= 250
    np.testing.assert_allclose(lam_g[:r], lam[:r], rtol=0, atol=1e-13)
    Vr = V[:, :r]
    assert np.abs(G0 @ Vr - Vr * lam_g[:r]).max() <= 1e-12
    # a backward-stable eigensolver leaves |v_i . v_j| ~ u ||G|| / |lambda_i - lambda_j|
    L = lam_g[:r]
    gap = np.abs(L[:, None] - L[None, :]) + np.eye(r)
    assert np.all(np.abs(Vr.T @ Vr - np.eye(r)) <= 64 * m * U64 * L[0] / gap + 1e-15)
    assert np.all(lam_g[b:] == 0.0)


def test_node_pod_wide(hp):
    from oracle import metrics, pod
    n, m, r = 3000, 600, 200
    sigma = 10.0 * 0.9 ** np.arange(r)
    S = prescribed_svd(n, m, sigma, 5)
    k = 50
    eps = math.sqrt(0.5 * (np.sum(sigma[k:] ** 2) + np.sum(sigma[k + 1:] ** 2)))
    s_ref, U_ref = pod.pod(S, eps)
    s, U = hp.hapod_node_pod("fp64", dev_colmajor(S), eps)
    assert len(s) == len(s_ref) == k + 1
    np.testing.assert_allclose(s, s_ref, rtol=1e-10)
    assert metrics.subspace_error(U_ref, host(U), len(s)) < 1e-9
