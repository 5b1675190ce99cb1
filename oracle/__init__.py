"""Plain FP64 CPU oracle for the hierarchical interpolative factorization
for elliptic PDEs (HIF-DE; Ho and Ying, "Hierarchical Interpolative
Factorization for Elliptic Operators: Differential Equations").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It
shares no code with the HIP path.

The oracle follows the paper step by step, in the paper's order and
notation, with slow, obvious code:

* ``problem``  - the five/seven-point discretization (Sections 3.1, 3.2).
* ``tree``     - cells, separators and edge/face groups per level
                 (Sections 3.1, 4.1, 4.2, 4.3).
* ``hifde``    - sparse elimination (Lemma 2.1), the interpolative
                 decomposition (Lemma 2.2, Corollary 2.3), skeletonization
                 (Lemma 2.4), the level loop (Algorithm 4.1) and the
                 application of F and F^{-1} (the factored form of the
                 generalized LDL decomposition).
* ``pcg``      - conjugate gradients preconditioned by F^{-1} (Section 5).
* ``errest``   - the power-iteration error estimates e_a and e_s (Section 5).
* ``mlp``      - forward/backward of the small rank-prediction network
                 (not in the paper; see its module docstring).

Parity status of each function is stated in its docstring ("pinned by ..."
or "parity unpinned").
"""
