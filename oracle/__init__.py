"""Plain, slow, FP64 CPU oracle for RPCholesky- and KRILL-preconditioned CG.

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The GPU library never
calls into it and shares no code with it: the two sides meet only through the
seeded synthetic inputs in ``synth`` (which hold none of the method's
arithmetic) and through the written sampling rules restated in each module.

Modules (each function cites the passage of the paper it follows):

* ``rng``        -- SplitMix64, used as a counter-based generator (published
                    definition: Steele, Lea & Flood, OOPSLA 2014).
* ``kernels``    -- kernel entries by direct differences, dense kernel blocks,
                    the matrix-free product (problem statement, Sec. 2.1).
* ``rpcholesky`` -- blocked RPCholesky (Appendix A, Alg. 3) and the
                    Nystrom preconditioner in SVD form (Alg. 1).
* ``krill``      -- centres, sparse sign embedding and KRILL (Alg. 2).
* ``pcg``        -- textbook preconditioned CG with zero start and a
                    relative-residual stop (Sec. 3, eq. psd_system).
* ``direct``     -- dense Cholesky solves used as pins (Sec. 2.1.1).
* ``predict``    -- prediction functions of full-data and restricted KRR
                    (Sec. 2, Sec. 2.2) and SMAPE (Sec. 4.1).

Parity status: every function here is pinned by tests under ``tests/``
(``test_oracle_*``) against closed forms, brute force or invariants; none is
"parity unpinned".
"""
