"""HAPOD of the noise-free sinusoid family, evaluated in coefficient space.

On the grid x_i = i/(n+1) the vectors
``phi_k[i] = sqrt(2/(n+1)) sin(k pi x_i)``, k = 1..n, are exactly orthonormal
(discrete sine transform of type I).  The noise-free sinusoid snapshots are
therefore ``S = Phi B`` with ``Phi`` (n x K) having orthonormal columns and
``B = sqrt(n+1) diag(exp(-k/tau)) C^T`` (K x m).

POD is equivariant under isometries: the singular values of ``Phi B`` are
those of ``B`` and its left singular vectors are ``Phi`` times those of ``B``
(Def. 2.1).  Every node of the HAPOD recursion (Def. 3.2) inherits this, so
HAPOD(Phi B) = Phi HAPOD(B) node by node.  Running the literal recursion on the
K-row matrix B therefore gives the exact HAPOD of an n-row problem, and rows of
the modes are materialised only where they are compared.

Additive noise E moves every singular value by at most ||E||_2 (Weyl).
"""
from __future__ import annotations

import math

import numpy as np

from . import hapod as _hapod


def sine_basis_rows(rows, n, K) -> np.ndarray:
    """Rows ``rows`` (0-based) of Phi (n x K)."""
    x = (np.asarray(rows, dtype=np.float64) + 1.0) / float(n + 1)
    k = np.arange(1, K + 1, dtype=np.float64)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(x, k))


def coefficient_matrix(C, n, tau) -> np.ndarray:
    """B = sqrt(n+1) diag(exp(-k/tau)) C^T, shape K x m."""
    C = np.asarray(C, dtype=np.float64)
    K = C.shape[1]
    decay = np.exp(-np.arange(1, K + 1, dtype=np.float64) / float(tau))
    return math.sqrt(n + 1.0) * (decay[:, None] * C.T)


def hapod_coeff(parent, leaf_coeffs, eps):
    """Literal HAPOD on the K-row coefficient blocks; returns ``{node: (sigma,
    U_B)}`` with U_B of shape K x N.  Modes in the original space are
    ``sine_basis_rows(rows, n, K) @ U_B``."""
    return _hapod.hapod(parent, leaf_coeffs, eps)


def weyl_noise_bound(n, m, noise_std, t=6.0) -> float:
    """High-probability bound on ||E||_2 for an n x m Gaussian matrix with
    i.i.d. N(0, noise_std^2) entries: noise_std (sqrt(n) + sqrt(m) + t)."""
    return noise_std * (math.sqrt(n) + math.sqrt(m) + t)
