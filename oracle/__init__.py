"""CPU FP64 oracle of the Hierarchical Approximate POD (Himpe, Leibner, Rave).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may import or
run anything in this package.  The GPU library never calls it, and the two
share no code: no kernels, headers, helpers, tables or pre/post-processing.
Both sides only take their inputs from :mod:`synth`.

What it computes, in plain NumPy float64, following the paper's definitions
rather than any optimisation of them:

* :mod:`oracle.tree`       -- rooted trees, leaves, nodes below, levels (Def. 3.1)
* :mod:`oracle.tolerances` -- local tolerances eps(alpha) (Thm. 3.5, Sec. 3.2)
* :mod:`oracle.pod`        -- POD(S, eps) by a thin SVD of the snapshot matrix
                              (Def. 2.1, Def. 2.5, Thm. 2.4)
* :mod:`oracle.hapod`      -- the literal node-by-node recursion (Def. 3.2)
* :mod:`oracle.metrics`    -- projection errors, subspace errors, theorem checks
                              (Thm. 3.3, 3.4, 3.5)
* :mod:`oracle.coeff`      -- the same HAPOD evaluated in the coefficient space
                              of an orthonormal sine basis (exact for the
                              noise-free sinusoid family)

Every function is pinned in ``tests/test_oracle_*.py`` against closed forms,
brute force on tiny inputs, special cases and the paper's inequalities.
"""
from . import tree, tolerances, pod, hapod, metrics, coeff  # noqa: F401
