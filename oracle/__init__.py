"""CPU oracle for the composite spectral direct solver (Gillman & Martinsson).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and it imports nothing from the library.

Everything here is plain, slow, FP64 NumPy/SciPy written from the paper:

* ``oracle.hps``   -- sections 2-5: nodes, leaf DtN (section 3), merge
  (section 4, eq:U_parent and eq:merge), Algorithms 1 and 2, post-processing
  (section 5.3), the interface-source extension used by iterative
  refinement (derived from eq:premerge with a non-zero third block row), and
  body loads A u = g (leaf particular solutions whose fluxes ride the same
  recursion).
* ``oracle.brute`` -- a brute-force global collocation solve (every leaf's
  interior collocation equations plus flux matching on every interior edge, in
  one dense system) and the dense interface system built from leaf DtNs; both
  pin Remark 5.1 (the merges are exact).
* ``oracle.mlp``   -- FP64 forward/backward of the leaf-DtN surrogate network.
* ``oracle.hbs``   -- sections 6-7: HBS matrices on a uniform binary tree (brute-force
  compression with nested orthonormal bases, the telescoping factorization and product,
  Algorithms 3 and 4) and thin factors of low-rank matrices.

Parity status: every function is pinned by tests under ``tests/`` except the
surrogate network's *target quality*, which the paper does not cover ("parity
unpinned" for the learned map itself; its gradients are pinned by central
finite differences).
"""
