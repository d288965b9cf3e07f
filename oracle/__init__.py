"""CPU oracle of the WENO-ZN scheme -- TEST INFRASTRUCTURE ONLY.

A plain, slow C++ implementation written from the paper (arXiv 2004.07954) and
pinned by the tests in ``tests/test_oracle_*.py`` to what the paper and the
mathematics fix.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it.  The HIP library never depends on it.

Parity status: every oracle function is pinned (see the tests); none is
"parity unpinned" except the Euler runs with shocks, which have no exact solution
and are checked only through invariants (conservation, symmetry, positivity).
"""
