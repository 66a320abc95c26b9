"""Seeded synthetic snapshot sets shaped like the HAPOD paper's workloads.

This module is shared by the CPU oracle (``oracle/``) and by the GPU path's
tests and benchmark.  It holds only data recipes: grids, coefficient draws,
the sinusoid and Gaussian-bump families, and the tree shapes of the benchmark
workloads.  It contains none of the method's arithmetic (no Gram matrix, no
eigensolve, no truncation, no lift).

Recipes (the paper's own datasets are not reproducible here, so these stand in
for them):

* grid: ``x_i = i / (n + 1)``, ``i = 1..n`` -- interior points of (0, 1).
* sinusoid family: column ``j`` is
  ``sum_{k=1..K} exp(-k / tau) * c_jk * sqrt(2) * sin(k * pi * x_i)``
  plus i.i.d. Gaussian noise of standard deviation ``noise_std``;
  ``c_jk ~ N(0, 1)`` drawn as ``C = rng.standard_normal((m, K))`` (row j is
  snapshot j), then the noise as ``rng.standard_normal((m, n)).T * noise_std``,
  with ``rng = numpy.random.default_rng(seed)`` (PCG64).
* Gaussian bumps: ``s_j(x_i) = exp(-(x_i - c_j)^2 / (2 w_j^2))`` with
  ``(u, v) = rng.random((m, 2))`` per column, ``c_j = u``,
  ``w_j = wmin + (wmax - wmin) * v``.

* uneven leaves: per-leaf heights, widths and family (sinusoid or bumps),
  evaluated on the global grid; rows past a leaf's height are zero.
* chain chunks: chunk ``l`` (0-based) of an incremental (chain) workload is
  ``bumps(n, cols, seed + l)``.
* relative tolerances: where a workload fixes the accuracy relative to the
  data, ``eps* = rel * sqrt(E ||s||^2)`` with the expected squared norm of a
  snapshot taken analytically from the generator (bumps: ``r w sqrt(pi)``
  for r grid rows and width w, interior approximation; sinusoid:
  ``r sum_k exp(-2k/tau) + r noise_std^2``).

The benchmark builds its large device-resident inputs from the same
coefficient draws (made here, on the host) and the same formulas.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "grid",
    "sinusoid_coeffs",
    "sinusoid_dense_factors",
    "sinusoid",
    "bump_params",
    "bumps",
    "uneven_leaf_specs",
    "uneven_leaf",
    "chain_chunk",
    "bump_mean_energy",
    "sinusoid_mean_energy",
    "uneven_mean_energy",
    "star_tree",
    "chain_tree",
    "balanced_tree",
    "Workload",
    "WORKLOADS",
    "UNEVEN_SPECS",
]


# --------------------------------------------------------------------------
# grids and coefficient draws
# --------------------------------------------------------------------------
def grid(n: int) -> np.ndarray:
    """Interior uniform grid ``x_i = i/(n+1)``, i = 1..n (float64)."""
    return np.arange(1, n + 1, dtype=np.float64) / float(n + 1)


def sinusoid_coeffs(m: int, K: int, seed: int) -> np.ndarray:
    """``C`` of shape (m, K): row j holds the coefficients of snapshot j."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, K))


def sinusoid_dense_factors(n: int, K: int, tau: float):
    """Return ``(Phi, decay)`` with ``Phi[i, k-1] = sqrt(2) sin(k pi x_i)`` and
    ``decay[k-1] = exp(-k/tau)``: the noise-free data is
    ``Phi @ (C * decay).T``."""
    x = grid(n)
    k = np.arange(1, K + 1, dtype=np.float64)
    phi = math.sqrt(2.0) * np.sin(np.pi * np.outer(x, k))
    decay = np.exp(-k / float(tau))
    return phi, decay


def sinusoid(n: int, m: int, K: int, tau: float, noise_std: float, seed: int,
             dtype=np.float64) -> np.ndarray:
    """Dense ``n x m`` snapshot matrix (Fortran order) of the sinusoid family."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, K))
    phi, decay = sinusoid_dense_factors(n, K, tau)
    S = phi @ (C * decay).T
    if noise_std > 0.0:
        S = S + rng.standard_normal((m, n)).T * noise_std
    return np.asfortranarray(S.astype(dtype, copy=False))


def bump_params(m: int, seed: int, wmin: float = 0.01, wmax: float = 0.05):
    """Centres and widths of ``m`` Gaussian bumps."""
    rng = np.random.default_rng(seed)
    u = rng.random((m, 2))
    return u[:, 0].copy(), wmin + (wmax - wmin) * u[:, 1]


def bumps(n: int, m: int, seed: int, wmin: float = 0.01, wmax: float = 0.05,
          dtype=np.float64) -> np.ndarray:
    """Dense ``n x m`` Gaussian-bump snapshot matrix (Fortran order)."""
    c, w = bump_params(m, seed, wmin, wmax)
    x = grid(n)
    S = np.exp(-np.subtract.outer(x, c) ** 2 / (2.0 * w * w))
    return np.asfortranarray(S.astype(dtype, copy=False))


# --------------------------------------------------------------------------
# uneven leaves: per-leaf heights, widths and families on one global grid
# --------------------------------------------------------------------------
def uneven_leaf_specs(num_leaves: int, seed: int, rows_range, cols_range):
    """Per-leaf (rows, cols, family, seed): rows ~ U{rows_range}, cols ~
    U{cols_range}, family 0 = sinusoid, 1 = Gaussian bumps (Bernoulli 1/2)."""
    rng = np.random.default_rng(seed)
    rows = rng.integers(rows_range[0], rows_range[1] + 1, num_leaves)
    cols = rng.integers(cols_range[0], cols_range[1] + 1, num_leaves)
    fam = rng.integers(0, 2, num_leaves)
    seeds = rng.integers(0, 2 ** 31 - 1, num_leaves)
    return [dict(rows=int(r), cols=int(c), family=int(f), seed=int(z))
            for r, c, f, z in zip(rows, cols, fam, seeds)]


def uneven_leaf(spec, n: int, K: int = 400, tau: float = 20.0, noise_std: float = 1e-10,
                dtype=np.float64) -> np.ndarray:
    """The first ``spec['rows']`` rows (of n on the grid x_i = i/(n+1)) of the
    leaf's snapshots; rows beyond are zero by definition.  Fortran order."""
    r, m = spec["rows"], spec["cols"]
    x = grid(n)[:r]
    rng = np.random.default_rng(spec["seed"])
    if spec["family"] == 0:
        C = rng.standard_normal((m, K))
        k = np.arange(1, K + 1, dtype=np.float64)
        S = (math.sqrt(2.0) * np.sin(np.pi * np.outer(x, k))) @ (C * np.exp(-k / tau)).T
        if noise_std > 0:
            S = S + rng.standard_normal((m, r)).T * noise_std
    else:
        u = rng.random((m, 2))
        c, w = u[:, 0], 0.01 + 0.04 * u[:, 1]
        S = np.exp(-np.subtract.outer(x, c) ** 2 / (2.0 * w * w))
    return np.asfortranarray(S.astype(dtype, copy=False))


def chain_chunk(n: int, cols: int, seed: int, chunk: int, dtype=np.float64) -> np.ndarray:
    """Chunk ``chunk`` of a chain workload: Gaussian bumps with seed+chunk."""
    return bumps(n, cols, seed + chunk, dtype=dtype)


def bump_mean_energy(rows: int, wmin: float = 0.01, wmax: float = 0.05) -> float:
    """E||s||^2 of a bump over ``rows`` grid rows: rows * E[w] * sqrt(pi)."""
    return rows * 0.5 * (wmin + wmax) * math.sqrt(math.pi)


def sinusoid_mean_energy(rows: int, K: int, tau: float, noise_std: float = 0.0) -> float:
    """E||s||^2 of a sinusoid snapshot over ``rows`` grid rows."""
    k = np.arange(1, K + 1, dtype=np.float64)
    return rows * float(np.exp(-2.0 * k / tau).sum()) + rows * noise_std ** 2


def uneven_mean_energy(specs, K: int = 400, tau: float = 20.0, noise_std: float = 1e-10) -> float:
    """Column-weighted mean of E||s||^2 over uneven leaves."""
    tot = 0.0
    cols = 0
    for sp in specs:
        e = (sinusoid_mean_energy(sp["rows"], K, tau, noise_std) if sp["family"] == 0
             else bump_mean_energy(sp["rows"]))
        tot += e * sp["cols"]
        cols += sp["cols"]
    return tot / max(cols, 1)


# --------------------------------------------------------------------------
# tree shapes (parent arrays; the root has parent -1)
# --------------------------------------------------------------------------
def star_tree(num_leaves: int):
    """Distributed HAPOD: leaves 0..L-1, root L."""
    return [num_leaves] * num_leaves + [-1]


def chain_tree(num_chunks: int):
    """Incremental HAPOD with ``num_chunks`` data chunks.

    Node ids: alpha_1..alpha_L are 0..L-1 (alpha_L = root), beta_1..beta_{L-1}
    are L..2L-2.  alpha_1 is a leaf holding chunk 0; beta_l holds chunk l and
    is a child of alpha_{l+1}, together with alpha_l.
    Returns ``(parent, chunk_of_leaf)`` where ``chunk_of_leaf`` maps leaf node
    id to chunk index.
    """
    L = num_chunks
    parent = [0] * (2 * L - 1)
    for l in range(L):          # alpha_{l+1}
        parent[l] = l + 1 if l + 1 < L else -1
    for l in range(1, L):       # beta_l -> alpha_{l+1}
        parent[L + l - 1] = l
    chunk = {0: 0}
    for l in range(1, L):
        chunk[L + l - 1] = l
    return parent, chunk


def balanced_tree(num_leaves: int, depth: int):
    """Balanced tree over ``num_leaves`` leaves with ``depth`` levels and
    arity ``ceil(num_leaves ** (1/(depth-1)))`` (leaves are level 1).
    Leaves are 0..num_leaves-1; inner nodes follow level by level; the root
    is last."""
    if depth < 2:
        raise ValueError("depth must be >= 2")
    arity = int(math.ceil(num_leaves ** (1.0 / (depth - 1)) - 1e-12))
    parent = []
    level_nodes = list(range(num_leaves))
    parent.extend([None] * num_leaves)
    next_id = num_leaves
    while len(level_nodes) > 1:
        groups = [level_nodes[i:i + arity] for i in range(0, len(level_nodes), arity)]
        new_nodes = []
        for g in groups:
            nid = next_id
            next_id += 1
            parent.append(None)
            for c in g:
                parent[c] = nid
            new_nodes.append(nid)
        level_nodes = new_nodes
    parent[level_nodes[0]] = -1
    return parent


# --------------------------------------------------------------------------
# the benchmark workloads
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    leaf_cols: tuple
    family: str            # "sinusoid", "bumps", "mixed"
    eps_star: float
    omega: float
    K: int = 0
    tau: float = 0.0
    noise_std: float = 0.0
    seed: int = 0
    precision: str = "fp64"
    tree: str = "star"
    extra: dict = field(default_factory=dict)

    @property
    def num_snapshots(self) -> int:
        return int(sum(self.leaf_cols))


_CHAIN_N = 1 << 22
_UNEVEN_N = 1 << 20
UNEVEN_SPECS = uneven_leaf_specs(1024, 5, (1 << 16, 1 << 20), (16, 256))

WORKLOADS = {
    # n=4096, 4 leaves x 64 columns, star tree, sinusoid K=200, tau=10
    "star4096x256": Workload("star4096x256", 4096, (64,) * 4, "sinusoid",
                             1e-6, 0.75, K=200, tau=10.0, noise_std=1e-10),
    # n=2^20, 64 leaves x 128 columns, star tree, sinusoid K=400, tau=20
    "star1Mx8192": Workload("star1Mx8192", 1 << 20, (128,) * 64, "sinusoid",
                            1e-5, 0.75, K=400, tau=20.0, noise_std=1e-10),
    # n=2^22 FP32, 256 chunks x 128 Gaussian bumps, chain tree (incremental
    # HAPOD), eps* = 1e-3 sqrt(E||s||^2), device memory capped at 16 GiB
    "chain4Mx32768": Workload("chain4Mx32768", _CHAIN_N, (128,) * 256, "bumps",
                              1e-3 * math.sqrt(bump_mean_energy(_CHAIN_N)), 0.75, seed=7,
                              precision="fp32", tree="chain",
                              extra={"mem_cap": 16 << 30, "rel": 1e-3}),
    # 1024 uneven leaves (rows U{2^16..2^20}, cols U{16..256}, sinusoid or
    # bumps) on one 2^20 grid, balanced 3-level tree (arity 32), leaves run
    # in waves of 256, eps* = 1e-3 sqrt(E||s||^2)
    "uneven1024": Workload("uneven1024", _UNEVEN_N, tuple(sp["cols"] for sp in UNEVEN_SPECS), "mixed",
                           1e-3 * math.sqrt(uneven_mean_energy(UNEVEN_SPECS)), 0.75, K=400, tau=20.0,
                           noise_std=1e-10, seed=5, precision="bf16x3", tree="balanced3",
                           extra={"leaf_wave": 256, "rel": 1e-3}),
}
