"""Plain FP64 CPU oracle for DAMF (Deng et al., KDD 2023, arXiv 2306.08967).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under ``oracle/``; only the test suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library: it reads the same seeded inputs (``workloads``) and nothing else.

Every function is written from the paper's definitions, slowly and literally,
in float64:

* ``graph``   edge-set semantics of an edit batch, net change of A, canonical CSR
* ``factor``  t-SVD of A (Sec. 4.1, the t-SVD embedding equation) by dense
              LAPACK SVD, and the randomized t-SVD used at initialisation
              (Appendix A, Algorithm 3)
* ``update``  the space-projection update for edge changes (Sec. 4.3,
              Theorem 2; Algorithm 1, UpdateEmbeddingE; Sec. 4.5 Steps 1-3),
              generalised from one edge to a block of edges, plus the paper's
              one-edge X-form procedure for cross-checking
* ``ppr``     Personalized PageRank (Sec. 4.4, the PPR series) by power
              iteration, and the residual-push procedure whose invariant the
              dynamic enhancement maintains
* ``model``   the DAMF driver (Algorithm 2, edge branch) in explicit form

Pins (the tests under ``tests/test_oracle_*.py``) tie each function to facts
other than itself: brute-force set semantics, dense SVD, Theorem 2 at every
step, exactness when rank(A) <= d, closed forms of PPR on cycles and
complete graphs, the alpha = 1 ablation.
"""
