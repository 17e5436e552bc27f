"""Plain FP64 CPU oracle for the RIOT inner loop of incremental 4D-Var.

TEST INFRASTRUCTURE ONLY. Nothing in the product library imports, links or
executes this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark call it. It shares no code with the HIP path:
the two meet only through the seeded draws of the ``synthetic`` package and
through plain arrays passed between them by the tests.

Everything is written for clarity, not speed, in NumPy float64 (LAPACK via
``numpy.linalg`` for the few library steps). Each function cites the part of
Bousserez, Guerrette & Henze (arXiv 1906.01413) that it follows.

Parity status: every function here is pinned by a CPU test against something
other than itself (closed forms, invariants, brute force, published test
vectors); the pins are listed in tests/test_oracle_*.py.
"""
