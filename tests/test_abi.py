"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and its host-side plan logic (Def. 3.1 validation, levels,
|S~_alpha|, Thm. 3.5 tolerances) matches the oracle.  No device calls."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import tolerances, tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hapod.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(hapod_[a-z_]+)\s*\(", txt))
    return sorted(n for n in names if n not in ("hapod_leaf_fn",))


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ["hapod_plan", "hapod_node_pod", "hapod_run", "hapod_modes", "hapod_gram",
                 "hapod_eigh", "hapod_truncate", "hapod_lift", "hapod_reorth"]:
        assert must in names


def test_library_exports_every_declared_function():
    hp = pytest.importorskip("paper_1607_05210_amd")
    import ctypes
    lib = ctypes.CDLL(hp.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    assert sorted(header_functions()) == sorted(hp.EXPORTED)


TREES = [
    (synth.star_tree(4), [64] * 4 + [0], 1e-6, 0.75, ()),
    (synth.star_tree(64), [128] * 64 + [0], 1e-5, 0.75, ()),
    ([4, 4, 5, 6, 6, 6, -1], [3, 5, 7, 11, 0, 0, 0], 0.1, 0.5, ()),
    (synth.balanced_tree(1024, 3), [16 + (i % 240) for i in range(1024)] + [0] * 33, 1e-3, 0.75, ()),
    ([-1], [9], 0.5, 0.3, ()),
]


@pytest.mark.parametrize("case", range(len(TREES)))
def test_plan_matches_oracle(case):
    hp = pytest.importorskip("paper_1607_05210_amd")
    parent, cols, eps_star, omega, _ = TREES[case]
    plan = hp.Plan(parent, cols, 100, eps_star, omega)
    eps, lev, acc = plan.query()
    assert list(lev) == tree.levels(parent)
    assert list(acc) == tree.acc_counts(parent, cols)
    ref = tolerances.hapod_tolerances(parent, cols, eps_star, omega)
    np.testing.assert_allclose(eps, ref, rtol=1e-15, atol=0)


def test_plan_chain_with_zero_overrides():
    hp = pytest.importorskip("paper_1607_05210_amd")
    parent, chunk = synth.chain_tree(6)
    cols = [10] * len(parent)
    betas = [b for b in chunk if b != 0]
    ov = [-1.0] * len(parent)
    for b in betas:
        ov[b] = 0.0
    plan = hp.Plan(parent, cols, 50, 1e-3, 0.75, eps_override=ov)
    eps, lev, acc = plan.query()
    ref = tolerances.hapod_tolerances(parent, cols, 1e-3, 0.75, zero_nodes=betas)
    np.testing.assert_allclose(eps, ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("parent", [[1, 0], [-1, -1], [3, -1, 1, 0], [5, -1], [0, -1]])
def test_plan_rejects_invalid_trees(parent):
    hp = pytest.importorskip("paper_1607_05210_amd")
    with pytest.raises(hp.HapodError) as e:
        hp.Plan(parent, [1] * len(parent), 10, 1e-3, 0.5)
    assert e.value.status == 2


@pytest.mark.parametrize("eps_star,omega,n", [(-1.0, 0.5, 10), (1.0, 1.5, 10), (1.0, -0.1, 10), (1.0, 0.5, 0)])
def test_plan_rejects_invalid_arguments(eps_star, omega, n):
    hp = pytest.importorskip("paper_1607_05210_amd")
    with pytest.raises(hp.HapodError) as e:
        hp.Plan(synth.star_tree(2), [3, 3, 0], n, eps_star, omega)
    assert e.value.status == 1


def test_modes_before_run_is_a_state_error():
    hp = pytest.importorskip("paper_1607_05210_amd")
    plan = hp.Plan(synth.star_tree(2), [3, 3, 0], 10, 1e-3, 0.5)
    with pytest.raises(hp.HapodError) as e:
        plan.node_stats()
    assert e.value.status == 6


def test_plan_rejects_bad_leaf_rows():
    hp = pytest.importorskip("paper_1607_05210_amd")
    with pytest.raises(hp.HapodError) as e:
        hp.Plan(synth.star_tree(2), [3, 3, 0], 10, 1e-3, 0.5, leaf_rows=[5, 11, 0])
    assert e.value.status == 1
    hp.Plan(synth.star_tree(2), [3, 3, 0], 10, 1e-3, 0.5, leaf_rows=[5, 10, 0])


def test_header_declares_the_next_rows():
    names = header_functions()
    for must in ["hapod_right_vectors", "hapod_node_pod_qr"]:
        assert must in names


@pytest.mark.parametrize("kw", [
    {"prec": "fp32", "block_gram": True},
    {"prec": "bf16x3", "block_gram": True},
    {"prec": "fp32", "qr_pod": True},
    {"prec": "bf16x3", "qr_pod": True},
    {"prec": "fp64", "qr_pod": True, "right_vectors": True},
])
def test_plan_rejects_option_combinations(kw):
    """Host-side plan rules: the block-structured Gram and the QR route need
    the FP64 form; the QR route keeps no right singular vectors."""
    hp = pytest.importorskip("paper_1607_05210_amd")
    with pytest.raises(hp.HapodError):
        hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5, **kw)


def test_plan_accepts_the_fp64_options():
    hp = pytest.importorskip("paper_1607_05210_amd")
    hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5, prec="fp64", qr_pod=True, block_gram=True)
    hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5, prec="fp64", right_vectors=True)


def test_right_vectors_before_a_run_is_an_error():
    hp = pytest.importorskip("paper_1607_05210_amd")
    plan = hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5, prec="fp64", right_vectors=True)
    with pytest.raises(hp.HapodError):
        plan.right_vectors()


@pytest.mark.parametrize("kw", [{"prec": "fp32", "sketch_cols": 256}, {"sketch_cols": 100},
                                {"sketch_cols": 1024}, {"sketch_cols": 256, "right_vectors": True}])
def test_plan_rejects_bad_sketch_options(kw):
    """The sketched route is FP64 only, keeps no right singular vectors, and
    its width is whole 128-column tiles up to 512."""
    hp = pytest.importorskip("paper_1607_05210_amd")
    with pytest.raises(hp.HapodError) as e:
        hp.Plan(synth.star_tree(2), [64, 64, 0], 1000, 1e-3, 0.5, **kw)
    assert e.value.status == 1


@pytest.mark.parametrize("field,value", [("leaf_layout", 2), ("leaf_layout", -1), ("leaf_passthrough", 2)])
def test_plan_rejects_bad_leaf_options(field, value):
    """leaf_layout and leaf_passthrough are 0 or 1 (checked at the C-ABI)."""
    import ctypes as C
    hp = pytest.importorskip("paper_1607_05210_amd")
    parent = (C.c_int32 * 3)(*synth.star_tree(2))
    cols = (C.c_int64 * 3)(4, 4, 0)
    tree = hp.HapodTree(3, parent, cols, 64, None)
    opts = hp.HapodOptions()
    opts.prec = 0
    setattr(opts, field, value)
    h = C.c_void_p()
    assert hp._lib.hapod_plan(C.byref(tree), 1e-3, 0.5, C.byref(opts), C.byref(h)) == 1  # HAPOD_E_INVALID
    setattr(opts, field, 1)
    assert hp._lib.hapod_plan(C.byref(tree), 1e-3, 0.5, C.byref(opts), C.byref(h)) == 0
    hp._lib.hapod_destroy(h)


def test_to_blocks_layout():
    """to_blocks: element (r, j) of an n x m matrix at [r // 128, j, r % 128],
    rows past n zero (CPU tensors)."""
    hp = pytest.importorskip("paper_1607_05210_amd")
    import torch
    S = torch.arange(300 * 3, dtype=torch.float64).reshape(3, 300).t()  # column-major 300 x 3
    B = hp.to_blocks(S)
    assert B.shape == (3, 3, 128) and B.is_contiguous()
    for r in (0, 127, 128, 255, 256, 299):
        for j in range(3):
            assert B[r // 128, j, r % 128] == S[r, j]
    assert not B[2, :, 300 - 256:].any()


def test_plan_time_memory_cap():
    """A cap below the leaf level's scratch (needed whatever the ranks) fails
    at plan time with HAPOD_E_NOMEM; a cap above it is accepted and the
    worst case a run may need is reported."""
    hp = pytest.importorskip("paper_1607_05210_amd")
    parent, cols = synth.star_tree(64), [128] * 64 + [0]
    with pytest.raises(hp.HapodError) as e:
        hp.Plan(parent, cols, 1 << 20, 1e-5, 0.75, mem_cap_bytes=1 << 20)
    assert e.value.status == 3
    plan = hp.Plan(parent, cols, 1 << 20, 1e-5, 0.75, mem_cap_bytes=16 << 30)
    worst, peak = plan.workspace()
    # at least the 64 leaves' outputs (2^20 x 128 doubles each) plus the root's
    # 8192-wide output, and nothing measured before a run
    assert worst >= 65 * (1 << 20) * 128 * 8
    assert peak == 0
    # the FP32 form stores half the bytes
    w32, _ = hp.Plan(parent, cols, 1 << 20, 1e-5, 0.75, prec="fp32").workspace()
    assert w32 < worst


def test_route_before_a_run_is_a_state_error():
    hp = pytest.importorskip("paper_1607_05210_amd")
    plan = hp.Plan(synth.star_tree(2), [4, 4, 0], 64, 1e-3, 0.5)
    with pytest.raises(hp.HapodError) as e:
        plan.route(-1)
    assert e.value.status == 6
