"""hapod_gram_noalloc (the Gram entry point for callers that cannot allocate)
against hapod_gram, through the C ABI: the same G = S^T S within the
rounding of a different row chunking, bitwise on exactly representable data,
two calls in a row (the second smaller, so stale contents of the shared
scratch array would show), no device memory mapped by the calls, and the
size limit rejected on the host.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import dev_colmajor  # noqa: E402

U = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -24}
DT = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.float32}


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_05210_amd as m
    return m


def both(hp, prec, S):
    Sd = dev_colmajor(S, DT[prec])
    m = S.shape[1]
    G_ref = hp.hapod_gram(prec, Sd)
    G = hp.colmajor(m, m, torch.float64, fill=float("nan"))
    hp.hapod_gram_noalloc(prec, Sd, G)
    torch.cuda.synchronize()
    return G.cpu().numpy(), G_ref.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_hapod_gram_twice(hp, prec):
    print(f"no-alloc gram {prec}", flush=True)
    rng = np.random.default_rng(7)
    # first call: 300000 x 200 (row chunks capped), second: 5000 x 37
    for n, m in ((300000, 200), (5000, 37)):
        S = rng.standard_normal((n, m))
        if prec != "fp64":
            S = S.astype(np.float32).astype(np.float64)
        G, G_ref = both(hp, prec, S)
        A = np.abs(S)
        bound = 2.0 * n * U[prec] * (A.T @ A)
        assert np.all(np.isfinite(G))
        assert np.all(np.abs(G - G_ref) <= bound), (prec, n, m, np.max(np.abs(G - G_ref) / bound))
        assert np.array_equal(G, G.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_exact_on_integers(hp, prec):
    """|x| <= 32, n = 12000: every partial sum is an integer below 2^24, exact
    in every form; the noalloc Gram equals the integer Gram and hapod_gram's
    bit for bit (two calls, the second narrower and shorter)."""
    rng = np.random.default_rng(3)
    for n, m in ((12000, 256), (3000, 129)):
        S = rng.integers(-32, 33, size=(n, m)).astype(np.float64)
        G, G_ref = both(hp, prec, S)
        exact = S.T @ S
        assert np.array_equal(G, exact), prec
        assert np.array_equal(G_ref, exact), prec


def test_noalloc_maps_no_device_memory(hp):
    rng = np.random.default_rng(5)
    S = dev_colmajor(rng.standard_normal((200000, 256)))
    G = hp.colmajor(256, 256, torch.float64)
    hp.hapod_gram_noalloc("fp64", S, G)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        hp.hapod_gram_noalloc("fp64", S, G)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)


def test_noalloc_limits(hp):
    S = dev_colmajor(np.ones((100, 257)))
    G = hp.colmajor(257, 257, torch.float64)
    with pytest.raises(hp.HapodError) as ei:
        hp.hapod_gram_noalloc("fp64", S, G)
    assert ei.value.status == 8
    assert "256" in hp.hapod_last_error()
    # n = 0 gives G = 0
    Z = dev_colmajor(np.zeros((0, 40)))
    G0 = hp.colmajor(40, 40, torch.float64, fill=7.0)
    hp.hapod_gram_noalloc("fp64", Z, G0)
    torch.cuda.synchronize()
    assert torch.count_nonzero(G0).item() == 0
