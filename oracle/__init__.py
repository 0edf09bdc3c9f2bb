"""FP64 CPU oracle for the weighted multiplicative-update NMF hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and shares no code with it: the two meet only at the seeded inputs
of ``paper_2309_04623_amd.synth``.

Contents (each function cites the passage of arXiv:2309.04623 it follows):

* ``prng``   -- counter-based SplitMix64 uniform init (Sec. 2, random init).
* ``nmf64``  -- staging, objective (Eq. 2), H- and W-rules (Eq. 3), basis
                build, per-frame projection (Sec. 4.1, target modelling) and
                subtraction (Sec. 1 / 4.1).
* ``nnls``   -- exact weighted non-negative least squares (brute force over
                supports for K <= 4, and an active-set solver), the limit the
                projection iteration must reach.
* ``mlp64``  -- FP64 forward/backward of the warm-start MLP.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
